"""Pins of the oracle's error-bound lists (absolute-error acceptance with the
expansion order chosen per interaction; Multipole Error Bounds section).

The decisive check is against the mathematics, not against the oracle's own
formula: with eps = 0, for every accepted (group, cell, order q) the true
error of the order-q expansion of that cell, at every sink of the group, is
computed from the cell's particles directly and must not exceed the
tolerance. The limits tol -> infinity (every separated cell at order 0) and
tol -> 0 (nothing accepted: the direct sum) are checked as well.
"""
import numpy as np
import pytest

from paper_1310_4502_amd import workloads as W


def _exact_field(xs, src, m):
    """Unsoftened field at points xs of point masses m at src (FP64)."""
    r = src[None, :, :] - xs[:, None, :]
    d = np.sqrt(np.einsum("ijk,ijk->ij", r, r))
    return np.einsum("ij,ijk->ik", m[None, :] / d ** 3, r)


def _cell_particles(ot, cell):
    cells = ot.cells()
    _, perm = ot.keys()
    f, c = int(cells["first"][cell]), int(cells["count"][cell])
    return perm[f:f + c]


@pytest.mark.parametrize("name,n,tol", [("plummer1m", 3000, 1e-3), ("clustered4m", 4000, 1e-4),
                                        ("uniform4k", None, 3e-3)])
def test_every_accepted_interaction_meets_tol(orc, name, n, tol):
    w = W.make(name, n=n)
    p_max = 8
    ot = orc.Tree(w.pos, 16, 64, w.box)
    ot.build_lists_err(w.mass, tol, p_max, 0)
    ot.compute_moments(w.pos, w.mass, p_max)
    po, pl, mo, ml = ot.lists()
    q = ot.m2p_orders()
    assert q.shape == ml.shape and q.min() >= 0 and q.max() <= p_max
    M = ot.moments()
    cells = ot.cells()
    groups = ot.groups()
    _, perm = ot.keys()
    rng = np.random.default_rng(0)
    checked = 0
    worst = 0.0
    for g in rng.choice(len(groups), size=min(40, len(groups)), replace=False):
        gc = groups[g]
        f, c = int(cells["first"][gc]), int(cells["count"][gc])
        sinks = perm[f:f + c]
        xs = w.pos[sinks]
        for e in range(mo[g], mo[g + 1]):
            cell, qq = int(ml[e]), int(q[e])
            src = _cell_particles(ot, cell)
            exact = _exact_field(xs, w.pos[src], w.mass[src])
            centre = cells["centre"][cell]
            approx = np.stack([orc.m2p(qq, M[cell][:orc.nm(qq)], x - centre, 0.0)[0]
                               for x in xs])
            err = np.linalg.norm(approx - exact, axis=1).max()
            worst = max(worst, err / tol)
            assert err <= tol * (1 + 1e-9) + 1e-12 * np.abs(exact).max()
            checked += 1
    assert checked > 100
    assert worst > 1e-4  # the bound is not vacuous: some interactions come near it


def test_huge_tol_is_monopole_of_separated_cells(orc):
    w = W.make("plummer1m", n=2000)
    ot = orc.Tree(w.pos, 16, 64, w.box)
    ot.build_lists_err(w.mass, 1e300, 8, 0)
    q = ot.m2p_orders()
    assert q.size > 0 and np.all(q == 0)
    # every M2P cell is separated from its group: d = |c_g - c_c| - b_g > b_c
    po, pl, mo, ml = ot.lists()
    cells = ot.cells()
    groups = ot.groups()
    for g in range(len(groups)):
        gc = groups[g]
        for e in range(mo[g], mo[g + 1]):
            c = ml[e]
            d = np.linalg.norm(cells["centre"][gc] - cells["centre"][c]) - cells["bmax"][gc]
            assert d > cells["bmax"][c]


def test_tiny_tol_is_direct_sum(orc):
    w = W.make("plummer1m", n=1500)
    eps = 1e-3
    ot = orc.Tree(w.pos, 8, 32, w.box)
    ot.build_lists_err(w.mass, 1e-300, 8, 0)
    ot.compute_moments(w.pos, w.mass, 8)
    a, _, cnt = ot.eval(w.pos, w.mass, eps)
    ad, _ = orc.direct(w.pos, w.mass, eps)
    # only cells of zero extent (all particles at the centre) may be accepted,
    # and their monopole is exact; everything else is a pair interaction
    assert np.linalg.norm(a - ad) <= 1e-12 * np.linalg.norm(ad)


def test_orders_fall_with_distance(orc):
    """Along one group's list, a farther cell of the same size never needs a
    higher order (the bound decreases with d at fixed b and count)."""
    w = W.make("uniform4k")
    ot = orc.Tree(w.pos, 16, 64, w.box)
    ot.build_lists_err(w.mass, 1e-4, 8, 0)
    po, pl, mo, ml = ot.lists()
    q = ot.m2p_orders()
    cells = ot.cells()
    groups = ot.groups()
    for g in range(0, len(groups), 7):
        gc = groups[g]
        es = np.arange(mo[g], mo[g + 1])
        if es.size < 2:
            continue
        c = ml[es]
        d = np.linalg.norm(cells["centre"][c] - cells["centre"][gc], axis=1)
        key = np.stack([cells["bmax"][c], cells["count"][c]], 1)
        for k in np.unique(key, axis=0):
            sel = np.all(key == k, axis=1)
            if sel.sum() < 2:
                continue
            o = np.argsort(d[sel])
            assert np.all(np.diff(q[es][sel][o].astype(int)) <= 0)


def test_errmac_vjp_matches_fd(orc):
    """The oracle's VJP with per-entry orders against central differences of
    its own evaluation on the same lists (topology frozen)."""
    w = W.make("clustered4m", n=600)
    eps = 1e-2
    ot = orc.Tree(w.pos, 8, 32, w.box)
    ot.build_lists_err(w.mass, 1e-3, 6, 0)
    assert np.unique(ot.m2p_orders()).size >= 2
    abar = W.cotangent(w.n, 3)
    ot.compute_moments(w.pos, w.mass, 6)
    xb, mb = ot.vjp(w.pos, w.mass, eps, abar)
    v = np.random.default_rng(1).normal(size=w.pos.shape)
    h = 1e-6

    def L(x):
        ot.compute_moments(x, w.mass, 6)
        a, _, _ = ot.eval(x, w.mass, eps, with_pot=False)
        return float((a * abar).sum())

    def cd(hh):
        return (L(w.pos + hh * v) - L(w.pos - hh * v)) / (2 * hh)

    fd = (4 * cd(h) - cd(2 * h)) / 3  # Richardson: the h^2 term cancels
    an = float((xb * v).sum())
    assert abs(an - fd) <= 1e-8 * abs(fd)
