"""Pins of the oracle's reverse derivatives (VJP) of the force evaluation.

The paper has no adjoint; the definition used is the VJP of the map
positions -> accelerations with the tree topology (membership, centres,
b_max, lists) held fixed. Pinned by central finite differences in FP64,
translation invariance, and the theta -> 0 reduction to the direct sum.
"""
import numpy as np
import pytest

from paper_1310_4502_amd import workloads as W


def _loss_direct(orc, pos, mass, eps, abar):
    a, _ = orc.direct(pos, mass, eps)
    return float(np.sum(a * abar))


def test_direct_vjp_translation_invariance(orc):
    w = W.make("plummer1m", n=500)
    abar = W.cotangent(w.n, 1)
    xb, _ = orc.direct_vjp(w.pos, w.mass, w.eps, abar)
    scale = np.sum(np.abs(xb))
    assert np.linalg.norm(np.sum(xb, axis=0)) <= 1e-12 * scale


def test_direct_vjp_fd(orc):
    rng = np.random.default_rng(3)
    n = 40
    pos = rng.random((n, 3))
    mass = rng.random(n) + 0.5
    eps = 0.05
    abar = rng.normal(size=(n, 3))
    xb, mb = orc.direct_vjp(pos, mass, eps, abar)
    h = 1e-6
    for k in range(0, n, 7):
        for d in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[k, d] += h
            pm[k, d] -= h
            fd = (_loss_direct(orc, pp, mass, eps, abar) - _loss_direct(orc, pm, mass, eps, abar)) / (2 * h)
            assert abs(fd - xb[k, d]) <= 1e-6 * max(1.0, abs(fd))
        mp, mm = mass.copy(), mass.copy()
        mp[k] += h
        mm[k] -= h
        fd = (_loss_direct(orc, pos, mp, eps, abar) - _loss_direct(orc, pos, mm, eps, abar)) / (2 * h)
        assert abs(fd - mb[k]) <= 1e-6 * max(1.0, abs(fd))
    # row selection gives the same rows
    rows = np.array([3, 17, 31])
    xr, mr = orc.direct_vjp(pos, mass, eps, abar, rows=rows)
    assert np.array_equal(xr, xb[rows]) and np.array_equal(mr, mb[rows])


def _tree_loss(orc, t, pos, mass, eps, abar, p):
    t.compute_moments(pos, mass, p)
    a, _, _ = t.eval(pos, mass, eps)
    return float(np.sum(a * abar))


@pytest.mark.parametrize("p,theta,direct_max", [(2, 0.5, 0), (4, 0.6, 0), (6, 0.5, 8)])
def test_tree_vjp_fd_topology_frozen(orc, p, theta, direct_max):
    w = W.make("clustered4m", n=600)
    t = orc.Tree(w.pos, n_leaf=8, n_group=32)
    t.build_lists(theta, direct_max)
    assert t.counts()["n_m2p"] > 0
    abar = W.cotangent(w.n, 5)
    eps = 1e-3
    t.compute_moments(w.pos, w.mass, p)
    xb, mb = t.vjp(w.pos, w.mass, eps, abar)
    rng = np.random.default_rng(6)
    h = 1e-6
    for k in rng.choice(w.n, 12, replace=False):
        for d in range(3):
            pp, pm = w.pos.copy(), w.pos.copy()
            pp[k, d] += h
            pm[k, d] -= h
            fd = (_tree_loss(orc, t, pp, w.mass, eps, abar, p) -
                  _tree_loss(orc, t, pm, w.mass, eps, abar, p)) / (2 * h)
            assert abs(fd - xb[k, d]) <= 1e-5 * max(abs(fd), np.abs(xb).max() * 1e-3), (k, d)
        mp, mm = w.mass.copy(), w.mass.copy()
        mp[k] += h
        mm[k] -= h
        fd = (_tree_loss(orc, t, w.pos, mp, eps, abar, p) -
              _tree_loss(orc, t, w.pos, mm, eps, abar, p)) / (2 * h)
        assert abs(fd - mb[k]) <= 1e-5 * max(abs(fd), np.abs(mb).max() * 1e-3)
    # a uniform translation of all positions moves nothing but the fixed
    # centres' relative geometry; with theta -> 0 there is no expansion at all
    # and the tree VJP equals the direct-sum VJP (next test).


def test_tree_vjp_theta_zero_is_direct(orc):
    w = W.make("plummer1m", n=700)
    t = orc.Tree(w.pos, n_leaf=8, n_group=16, box=w.box)
    t.build_lists(1e-6)
    t.compute_moments(w.pos, w.mass, 2)
    abar = W.cotangent(w.n, 8)
    xb, mb = t.vjp(w.pos, w.mass, w.eps, abar)
    xd, md = orc.direct_vjp(w.pos, w.mass, w.eps, abar)
    assert np.linalg.norm(xb - xd) <= 1e-13 * np.linalg.norm(xd)
    assert np.linalg.norm(mb - md) <= 1e-13 * np.linalg.norm(md)
