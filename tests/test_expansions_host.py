"""The generated expansion code (the GPU kernels' arithmetic, built here for
the host with T = double) against the oracle's independent formulas."""
import ctypes
import math
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1310_4502_amd", "csrc")


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    gen = os.path.join(CSRC, "generated", "expansions.h")
    subprocess.run([sys.executable, os.path.join(CSRC, "gen_expansions.py"), gen], check=True)
    out = str(tmp_path_factory.mktemp("shim") / "libshim.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
                    "-I", os.path.dirname(gen), os.path.join(ROOT, "tests", "host", "expansions_shim.cpp"),
                    "-o", out], check=True)
    L = ctypes.CDLL(out)
    for f in ("shim_fwd", "shim_sink", "shim_cell", "shim_p2m", "shim_m2m", "shim_m2mT",
              "shim_p2mT"):
        getattr(L, f).restype = None
    i32 = ctypes.c_int
    L.shim_fwd.argtypes = [i32, i32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]
    L.shim_sink.argtypes = [i32, i32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
    L.shim_cell.argtypes = [i32, i32, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
    L.shim_p2m.argtypes = [ctypes.c_int] + [ctypes.c_double] * 4 + [ctypes.c_void_p]
    L.shim_m2m.argtypes = [ctypes.c_int, ctypes.c_void_p] + [ctypes.c_double] * 3 + [ctypes.c_void_p]
    L.shim_m2mT.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p] + [ctypes.c_double] * 3 + \
        [ctypes.c_void_p]
    L.shim_p2mT.argtypes = [ctypes.c_int, ctypes.c_void_p] + [ctypes.c_double] * 3 + [ctypes.c_void_p]
    return L


def P(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def weights(orc, p):
    return np.array([(-1.0) ** (a + b + c) / (math.factorial(a) * math.factorial(b) * math.factorial(c))
                     for a, b, c in orc.multi_indices(p)])


@pytest.mark.parametrize("p", range(9))
@pytest.mark.parametrize("kernel,eps", [("plummer", 0.0), ("plummer", 0.4), ("k1", 2.5)])
def test_forward_matches_oracle(orc, shim, p, kernel, eps):
    """Plummer, and K1 with a kernel radius that half of the evaluation points
    fall inside (the quartic radial functions) and half outside (Newtonian)."""
    rng = np.random.default_rng(p)
    pts = rng.random((30, 3)) - 0.5
    m = rng.random(30)
    M = orc.p2m(p, pts, m, np.zeros(3))
    Mw = M * weights(orc, p)
    k1 = int(kernel == "k1")
    inside = 0
    for k in range(8):
        R = rng.normal(size=3) * (3 if k % 2 == 0 else 0.8)
        inside += int(np.dot(R, R) < eps * eps) if k1 else 0
        out = np.zeros(4)
        shim.shim_fwd(p, k1, P(Mw), P(R), eps * eps, P(out))
        a, phi = orc.m2p(p, M, R, eps, kernel=kernel)
        assert np.allclose(-out[:3], a, rtol=1e-12, atol=1e-14 * np.abs(a).max())
        assert abs(out[3] - phi) <= 1e-12 * abs(phi)
    if k1:
        assert 0 < inside < 8, inside


@pytest.mark.parametrize("p", range(9))
def test_adjoint_parts_match_oracle_derivatives(orc, shim, p):
    rng = np.random.default_rng(100 + p)
    idx = {a: i for i, a in enumerate(orc.multi_indices(p + 2))}
    al = orc.multi_indices(p)
    Mw = rng.normal(size=len(al))
    E = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    for kernel, eps, scale in (("plummer", 0.0, 2.5), ("plummer", 0.3, 2.5), ("k1", 1.5, 0.5),
                               ("k1", 0.6, 2.5)):
        # K1 at 0.5 x N(0,1) inside a radius of 1.5, at 2.5 x N(0,1) mostly outside 0.6
        k1 = int(kernel == "k1")
        R = rng.normal(size=3) * scale
        b = rng.normal(size=3)
        D = orc.derivs(p + 2, R, eps, kernel=kernel)
        # sink part: g_l = sum_k b_k sum_alpha Mw[alpha] d^(alpha+e_k+e_l) G
        ref = np.zeros(3)
        for l in range(3):
            for k in range(3):
                for s, a in enumerate(al):
                    t = tuple(a[q] + E[k][q] + E[l][q] for q in range(3))
                    ref[l] += b[k] * Mw[s] * D[idx[t]]
        g = np.zeros(3)
        shim.shim_sink(p, k1, P(Mw), P(R), eps * eps, P(b), P(g))
        assert np.allclose(g, ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())
        # cell part: row[alpha] += sum_k b_k d^(alpha+e_k) G
        refc = np.array([sum(b[k] * D[idx[tuple(a[q] + E[k][q] for q in range(3))]] for k in range(3))
                         for a in al])
        row = np.full(len(al), 0.25)
        shim.shim_cell(p, k1, P(R), eps * eps, P(b), P(row))
        assert np.allclose(row - 0.25, refc, rtol=1e-11, atol=1e-13 * np.abs(refc).max())


@pytest.mark.parametrize("p", [0, 3, 8])
def test_p2m_m2m_match_oracle(orc, shim, p):
    rng = np.random.default_rng(7)
    pts = rng.random((20, 3)) * 0.5
    m = rng.random(20)
    c = np.array([0.25, 0.25, 0.25])
    ref = orc.p2m(p, pts, m, c)
    got = np.zeros(orc.nm(p))
    for N in range(p + 1):
        off = N * (N + 1) * (N + 2) // 6
        acc = np.zeros((N + 1) * (N + 2) // 2)
        for j in range(20):
            d = pts[j] - c
            shim.shim_p2m(N, d[0], d[1], d[2], m[j], P(acc))
        got[off:off + len(acc)] = acc
    # the same monomials; the oracle's sum is compensated, the generated
    # code's plain (20 terms)
    assert np.allclose(got, ref, rtol=0, atol=1e-15 * np.abs(ref).max())
    parent = np.array([0.5, 0.5, 0.5])
    refp = orc.m2m(p, ref, c - parent)
    gotp = np.zeros(orc.nm(p))
    for N in range(p + 1):
        off = N * (N + 1) * (N + 2) // 6
        acc = np.zeros((N + 1) * (N + 2) // 2)
        shim.shim_m2m(N, P(ref), *(c - parent), P(acc))
        gotp[off:off + len(acc)] = acc
    assert np.allclose(gotp, refp, rtol=1e-14, atol=1e-15 * np.abs(refp).max())


@pytest.mark.parametrize("p", [0, 2, 5, 8])
def test_m2m_transpose_is_the_adjoint_of_the_oracle_m2m(orc, shim, p):
    """The generated transpose of the re-centring (the adjoint's downward
    pass) satisfies <Mbar, m2m(M)> = <m2mT(Mbar), M> with the oracle's own
    re-centring, for random moments and cotangents: it is the exact transpose
    of the linear map, not only of the GPU's version of it."""
    rng = np.random.default_rng(11 + p)
    nm = orc.nm(p)
    shift = np.array([0.13, -0.07, 0.21])
    for _ in range(3):
        M = rng.standard_normal(nm)
        Mb = rng.standard_normal(nm)
        lhs = float(np.dot(Mb, orc.m2m(p, M, shift)))
        got = np.zeros(nm)
        for N in range(p + 1):
            off = N * (N + 1) * (N + 2) // 6
            acc = np.zeros((N + 1) * (N + 2) // 2)
            shim.shim_m2mT(p, N, P(Mb), *shift, P(acc))
            got[off:off + len(acc)] = acc
        rhs = float(np.dot(got, M))
        scale = float(np.abs(Mb).sum() * np.abs(orc.m2m(p, np.abs(M), np.abs(shift))).max())
        assert abs(lhs - rhs) <= 1e-13 * scale, (lhs, rhs, scale)


@pytest.mark.parametrize("p", [0, 1, 4, 8])
def test_p2m_transpose_is_the_gradient_of_the_oracle_p2m(orc, shim, p):
    """The generated moment-to-particle transpose returns, for a unit mass at
    offset d, the mass cotangent <Mbar, P2M(d)> and the position cotangent
    grad_d <Mbar, P2M(d)>, both from the oracle's own P2M (the gradient by a
    fourth-order central difference)."""
    rng = np.random.default_rng(23 + p)
    nm = orc.nm(p)
    zero = np.zeros(3)
    for _ in range(3):
        Mb = rng.standard_normal(nm)
        d = rng.uniform(-0.4, 0.4, 3)
        g = np.zeros(4)
        shim.shim_p2mT(p, P(Mb), *d, P(g))

        def f(x):
            return float(np.dot(Mb, orc.p2m(p, x[None, :], np.ones(1), zero)))

        assert abs(g[3] - f(d)) <= 1e-14 * max(1.0, np.abs(Mb).sum())
        h = 1e-3
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            fd = (8 * (f(d + e) - f(d - e)) - (f(d + 2 * e) - f(d - 2 * e))) / (12 * h)
            assert abs(g[k] - fd) <= 1e-8 * max(1.0, np.abs(Mb).sum()), (k, g[k], fd)
