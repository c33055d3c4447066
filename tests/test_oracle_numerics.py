"""Pins of the oracle's arithmetic: direct sum, Green's-function derivatives,
moments, the cell-body expansion and the whole treecode.

Each check compares with something the oracle's own code does not compute:
exact rational differentiation, long-double brute force, Newton's third law,
closed forms (two bodies, a point mass at a cell centre, the Plummer sphere),
harmonicity, convergence in p, and the claim of the Error Analysis section's
p8err figure.
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_1310_4502_amd import workloads as W


# ---------------------------------------------------------------- direct sum
def test_direct_bruteforce_longdouble(orc):
    rng = np.random.default_rng(11)
    n = 48
    pos = rng.random((n, 3))
    mass = rng.random(n) + 0.1
    eps = 0.01
    acc, pot = orc.direct(pos, mass, eps)
    P = pos.astype(np.longdouble)
    M = mass.astype(np.longdouble)
    for i in range(n):
        r = P - P[i]
        s = np.sum(r * r, axis=1) + np.longdouble(eps) ** 2
        w = M / s ** np.longdouble(1.5)
        w[i] = 0
        a = np.sum(w[:, None] * r, axis=0)
        ph = -np.sum(np.where(np.arange(n) == i, 0, M / np.sqrt(s)))
        assert np.allclose(acc[i], a.astype(np.float64), rtol=1e-14, atol=1e-14 * np.abs(a).max())
        assert abs(pot[i] - float(ph)) <= 1e-14 * abs(float(ph))


def test_direct_newton_third_law(orc):
    w = W.make("plummer1m", n=3000)
    acc, _ = orc.direct(w.pos, w.mass, w.eps)
    net = np.linalg.norm(np.sum(w.mass[:, None] * acc, axis=0))
    scale = np.sum(w.mass * np.linalg.norm(acc, axis=1))
    assert net <= 1e-12 * scale


def test_direct_two_body_and_eps_zero_coincident(orc):
    pos = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0]])
    mass = np.array([2.0, 5.0])
    eps = 1.0
    acc, pot = orc.direct(pos, mass, eps)
    s = 25.0 + 1.0
    assert np.allclose(acc[0], 5.0 * np.array([3, 4, 0]) / s ** 1.5, rtol=1e-15)
    assert np.allclose(acc[1], -2.0 * np.array([3, 4, 0]) / s ** 1.5, rtol=1e-15)
    assert np.allclose(pot, [-5 / np.sqrt(s), -2 / np.sqrt(s)], rtol=1e-15)
    # coincident points with eps = 0 are skipped, not infinite
    pos = np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5], [0.0, 0.5, 0.5]])
    acc, pot = orc.direct(pos, np.ones(3), 0.0)
    assert np.all(np.isfinite(acc)) and np.allclose(acc[0], [-4.0, 0, 0])


# ------------------------------------------------ derivatives of softened G
def _exact_derivs(order, R, eps2):
    """d^alpha G, G = -s^(-1/2), s = |R|^2 + eps2, by repeated exact
    differentiation of terms c X^i Y^j Z^k s^(-(2m+1)/2) with rationals.
    R and eps2 are chosen so that s is a perfect square."""
    X = [Fraction(v) for v in R]
    s = X[0] ** 2 + X[1] ** 2 + X[2] ** 2 + Fraction(eps2)
    rs = Fraction(int(round(float(s) ** 0.5)))
    assert rs * rs == s
    memo = {(0, 0, 0): {(0, 0, 0, 0): Fraction(-1)}}

    def diff(terms, ax):
        out = {}
        for (i, j, k, m), c in terms.items():
            e = [i, j, k]
            if e[ax] > 0:
                e2 = list(e)
                e2[ax] -= 1
                key = (*e2, m)
                out[key] = out.get(key, 0) + c * e[ax]
            e3 = list(e)
            e3[ax] += 1
            key = (*e3, m + 1)
            out[key] = out.get(key, 0) - c * (2 * m + 1)
        return out

    def get(a, b, c):
        if (a, b, c) in memo:
            return memo[(a, b, c)]
        if a > 0:
            t = diff(get(a - 1, b, c), 0)
        elif b > 0:
            t = diff(get(a, b - 1, c), 1)
        else:
            t = diff(get(a, b, c - 1), 2)
        memo[(a, b, c)] = t
        return t

    vals = []
    for n in range(order + 1):
        for a in range(n, -1, -1):
            for b in range(n - a, -1, -1):
                c = n - a - b
                v = Fraction(0)
                for (i, j, k, m), co in get(a, b, c).items():
                    v += co * X[0] ** i * X[1] ** j * X[2] ** k / rs ** (2 * m + 1)
                vals.append(v)
    return vals


@pytest.mark.parametrize("R,eps2", [((1, 2, 2), 0), ((2, 3, 6), 0), ((1, 2, 2), 16),
                                    ((-2, 3, -6), 0), ((0.5, 1.5, -1), 0.5)])
def test_derivs_exact(orc, R, eps2):
    order = 10
    got = orc.derivs(order, np.array(R, dtype=float), np.sqrt(eps2))
    ref = _exact_derivs(order, R, Fraction(eps2).limit_denominator() if eps2 else 0)
    ref = np.array([float(v) for v in ref])
    scale = np.abs(ref).max()
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-13 * scale)


def test_derivs_harmonic(orc):
    # eps = 0: G = -1/r is harmonic, so every derivative has zero Laplacian;
    # with eps > 0 the Laplacian of G is 3 eps^2 s^(-5/2).
    idx = {a: i for i, a in enumerate(orc.multi_indices(12))}
    rng = np.random.default_rng(3)
    for _ in range(5):
        R = rng.normal(size=3) * 2
        d = orc.derivs(12, R, 0.0)
        for (a, b, c), i in idx.items():
            if a + b + c > 10:
                continue
            lap = d[idx[(a + 2, b, c)]] + d[idx[(a, b + 2, c)]] + d[idx[(a, b, c + 2)]]
            mag = abs(d[idx[(a + 2, b, c)]]) + abs(d[idx[(a, b + 2, c)]]) + abs(d[idx[(a, b, c + 2)]])
            assert abs(lap) <= 1e-12 * mag + 1e-300
        eps = 0.7
        d = orc.derivs(2, R, eps)
        s = R @ R + eps * eps
        lap = d[idx[(2, 0, 0)]] + d[idx[(0, 2, 0)]] + d[idx[(0, 0, 2)]]
        mag = abs(d[idx[(2, 0, 0)]]) + abs(d[idx[(0, 2, 0)]]) + abs(d[idx[(0, 0, 2)]])
        assert abs(lap - 3 * eps * eps * s ** -2.5) <= 1e-14 * mag


# ------------------------------------------------------------ moments / M2M
def test_p2m_m2m_identity(orc):
    rng = np.random.default_rng(5)
    for p in (2, 5, 8):
        pts = rng.random((50, 3)) * 0.25
        m = rng.random(50)
        child = np.array([0.125, 0.125, 0.125])
        parent = np.array([0.25, 0.25, 0.25])
        Mc = orc.p2m(p, pts, m, child)
        Mp = orc.p2m(p, pts, m, parent)
        Mt = orc.m2m(p, Mc, child - parent)
        assert np.allclose(Mt, Mp, rtol=1e-14, atol=1e-14 * np.abs(Mp).max())
    # dyadic masses: the monopole is exact
    m = np.full(64, 1.0 / 64)
    M = orc.p2m(3, rng.random((64, 3)), m, np.zeros(3))
    assert M[0] == 1.0


def test_p2m_sum_does_not_grow_with_count(orc):
    """Moments of 2^16 particles against long-double sums of the same
    monomials: the oracle's compensated sum leaves only the rounding of the
    terms themselves (random in sign, ~u S / sqrt(N) for S the sum of the
    term magnitudes), where a plain running sum would drift by ~u S sqrt(N)."""
    rng = np.random.default_rng(6)
    n = 1 << 16
    pts = rng.random((n, 3))
    m = np.full(n, 1.0 / n)
    c = np.array([0.5, 0.5, 0.5])
    p = 4
    M = orc.p2m(p, pts, m, c)
    d = (pts - c).astype(np.longdouble)
    u = np.finfo(np.float64).eps / 2
    for s, (a, b, cc) in enumerate(orc.multi_indices(p)):
        terms = np.longdouble(1.0 / n) * d[:, 0] ** a * d[:, 1] ** b * d[:, 2] ** cc
        exact = terms.sum()
        S = float(np.abs(terms).sum())
        assert abs(float(M[s] - exact)) <= u * abs(float(exact)) + 0.05 * u * S, (a, b, cc)


# ------------------------------------------------------- cell-body expansion
@pytest.mark.parametrize("p", [0, 1, 2, 4, 6, 8])
@pytest.mark.parametrize("eps", [0.0, 0.3])
def test_m2p_point_mass_closed_form(orc, p, eps):
    # a single particle at the cell centre: all moments but M_0 vanish and the
    # expansion must equal the softened point-mass field for every p.
    M = orc.p2m(p, np.array([[0.5, 0.5, 0.5]]), np.array([0.7]), np.array([0.5, 0.5, 0.5]))
    R = np.array([1.3, -2.1, 0.4])
    a, phi = orc.m2p(p, M, R, eps)
    s = R @ R + eps * eps
    assert np.allclose(a, -0.7 * R / s ** 1.5, rtol=1e-15, atol=0)
    assert abs(phi + 0.7 / np.sqrt(s)) <= 1e-15 * 0.7 / np.sqrt(s)


def test_m2p_convergence_in_p(orc):
    # a fixed cluster at distance R: the error falls with p (roughly like
    # (b/R)^(p+1)) until FP64 round-off.
    rng = np.random.default_rng(9)
    pts = rng.random((200, 3)) - 0.5
    m = np.full(200, 1.0 / 200)
    x = np.array([3.0, 1.0, -0.5])
    eps = 1e-3
    r = x - pts
    s = np.sum(r * r, axis=1) + eps * eps
    exact = -np.sum(m[:, None] * r / s[:, None] ** 1.5, axis=0)
    errs = []
    for p in range(0, 11):
        M = orc.p2m(p, pts, m, np.zeros(3))
        a, _ = orc.m2p(p, M, x, eps)
        errs.append(np.linalg.norm(a - exact) / np.linalg.norm(exact))
    errs = np.array(errs)
    bmax = np.sqrt(np.max(np.sum(pts * pts, axis=1)))
    ratio = bmax / np.linalg.norm(x)
    for p in range(0, 11):
        assert errs[p] <= 5 * ratio ** (p + 1)
    assert np.all(errs[1:] < errs[:-1])
    assert errs[10] < 1e-5 * errs[0]


def test_p8err_claim(orc):
    """Error Analysis section, figure p8err: for 512 particles uniform in a
    unit cube, a single p = 8 expansion at distance r = 4 is more accurate
    than single-precision direct summation over the same particles."""
    rng = np.random.default_rng(2013)
    worse = 0
    trials = 20
    for _ in range(trials):
        pts = rng.random((512, 3)) - 0.5
        m = np.full(512, 1.0 / 512)
        d = rng.normal(size=3)
        x = 4.0 * d / np.linalg.norm(d)
        r = x - pts
        s = np.sum(r * r, axis=1)
        exact = -np.sum(m[:, None] * r / s[:, None] ** 1.5, axis=0)
        r32 = x.astype(np.float32) - pts.astype(np.float32)
        s32 = np.sum(r32 * r32, axis=1, dtype=np.float32)
        acc32 = np.zeros(3, np.float32)
        for j in range(512):
            acc32 -= np.float32(m[j]) * r32[j] / (s32[j] * np.sqrt(s32[j]))
        e32 = np.linalg.norm(acc32.astype(np.float64) - exact) / np.linalg.norm(exact)
        M = orc.p2m(8, pts, m, np.zeros(3))
        a8, _ = orc.m2p(8, M, x, 0.0)
        e8 = np.linalg.norm(a8 - exact) / np.linalg.norm(exact)
        worse += e8 >= e32
    assert worse <= 1, f"p=8 less accurate than FP32 direct in {worse}/{trials}"


# -------------------------------------------------------------- whole treecode
def test_tree_theta_to_zero_is_direct(orc):
    w = W.make("clustered4m", n=2000)
    t = orc.Tree(w.pos, n_leaf=8, n_group=32)
    t.build_lists(1e-6)
    assert t.counts()["n_m2p"] == 0
    t.compute_moments(w.pos, w.mass, 3)
    acc, pot, cnt = t.eval(w.pos, w.mass, w.eps)
    ad, pd = orc.direct(w.pos, w.mass, w.eps)
    assert np.linalg.norm(acc - ad) / np.linalg.norm(ad) < 1e-14
    assert np.linalg.norm(pot - pd) / np.linalg.norm(pd) < 1e-14
    assert cnt[0] == w.n * w.n and cnt[1] == 0


@pytest.mark.parametrize("p,tol", [(2, 3e-3), (4, 4e-4), (6, 6e-5), (8, 1e-5)])
def test_tree_error_falls_with_p(orc, p, tol):
    w = W.make("plummer1m", n=6000)
    t = orc.Tree(w.pos, n_leaf=16, n_group=64, box=w.box)
    t.build_lists(0.5)
    t.compute_moments(w.pos, w.mass, p)
    acc, _, cnt = t.eval(w.pos, w.mass, w.eps)
    ad, _ = orc.direct(w.pos, w.mass, w.eps)
    err = np.linalg.norm(acc - ad) / np.linalg.norm(ad)
    assert err < tol
    assert cnt[1] > 0


def test_tree_plummer_closed_form(orc):
    """Plummer sphere (a = 1/16, truncated at 0.5, renormalised): the mean
    radial acceleration in shells follows -M(<r)/r^2 and the potential
    follows the truncated closed form, to the sampling noise."""
    n = 1 << 15
    a, rmax = 1.0 / 16, 0.5
    pos = W.plummer(n, 21, a=a, rmax=rmax)
    mass = np.full(n, 1.0 / n)
    t = orc.Tree(pos, box=np.array([0, 0, 0, 1.0]))
    t.build_lists(0.5)
    t.compute_moments(pos, mass, 4)
    acc, pot, _ = t.eval(pos, mass, 1e-4)
    d = pos - 0.5
    r = np.linalg.norm(d, axis=1)
    ar = np.sum(acc * d, axis=1) / r
    Mt = rmax ** 3 / (rmax ** 2 + a * a) ** 1.5
    menc = r ** 3 / (r * r + a * a) ** 1.5 / Mt
    phi = (-1 / np.sqrt(r * r + a * a) + 1 / np.sqrt(rmax ** 2 + a * a) - Mt / rmax) / Mt
    edges = np.quantile(r, np.linspace(0.05, 0.95, 10))
    for lo_, hi_ in zip(edges[:-1], edges[1:]):
        sel = (r >= lo_) & (r < hi_)
        assert abs(np.mean(ar[sel]) / np.mean(-menc[sel] / r[sel] ** 2) - 1) < 0.03
        assert abs(np.mean(pot[sel]) / np.mean(phi[sel]) - 1) < 0.01


def test_tree_absum_brute_force(orc):
    """The per-sink sum of term magnitudes: with theta -> 0 every term is a
    pair, so it equals sum_j m_j |r_ij| (r^2 + eps^2)^(-3/2) by brute force;
    with expansions it is at least |a| (triangle inequality)."""
    rng = np.random.default_rng(21)
    n = 500
    pos = rng.random((n, 3))
    mass = rng.random(n) + 0.1
    eps = 0.01
    t = orc.Tree(pos, 8, 16)
    t.build_lists(1e-6, 0)
    t.compute_moments(pos, mass, 2)
    acc, ab, cs = t.eval_abs(pos, mass, eps, cond=True)
    # each particle's distance from the centre of its sink group
    cells = t.cells()
    _, perm = t.keys()
    gof = t.group_of()
    gcent = cells["centre"][t.groups()]
    off = np.empty(n)
    off[perm] = np.linalg.norm(pos[perm] - gcent[gof], axis=1)
    for i in range(0, n, 37):
        r = pos - pos[i]
        d = np.sqrt(np.sum(r * r, axis=1))
        term = mass * d * (d * d + eps * eps) ** -1.5
        term[i] = 0.0
        assert abs(ab[i] - term.sum()) <= 1e-13 * term.sum()
        with np.errstate(divide="ignore", invalid="ignore"):
            w = np.where(term > 0, 1.0 + (off[i] + off) / d, 0.0)
        assert abs(cs[i] - (term * w).sum()) <= 1e-13 * (term * w).sum()
    t.build_lists(0.6, 0)
    acc, ab = t.eval_abs(pos, mass, eps)
    a0, _, _ = t.eval(pos, mass, eps)
    assert np.array_equal(acc, a0)
    assert np.all(ab >= np.linalg.norm(acc, axis=1) * (1 - 1e-12))
