"""Helpers shared by the GPU parity tests (GPU tree vs oracle tree)."""
import numpy as np
import torch

import oracle


def to_dev(w):
    pos = torch.from_numpy(np.ascontiguousarray(w.pos)).cuda()
    mass = torch.from_numpy(np.ascontiguousarray(w.mass)).cuda()
    return pos, mass


def build_both(w, theta=None, direct_max=None, p=None, groups=None, cells=None, lists=True):
    from paper_1310_4502_amd.binding import Tree
    pos, mass = to_dev(w)
    gt = Tree(pos, w.n_leaf, w.n_group, w.box)
    ot = oracle.Tree(w.pos, w.n_leaf, w.n_group, w.box)
    th = w.theta if theta is None else theta
    dm = w.direct_max if direct_max is None else direct_max
    pp = w.p if p is None else p
    if lists:
        gt.build_interaction_lists(th, dm)
        ot.build_lists(th, dm, groups=groups)
    gt.compute_moments(pos, mass, pp)
    return gt, ot, pos, mass, pp


def assert_tree_equal(gt, ot):
    gk, gp = gt.keys()
    ok, op = ot.keys()
    assert np.array_equal(gk, ok), "sorted keys differ"
    assert np.array_equal(gp.astype(np.int64), op), "permutation differs"
    assert np.array_equal(gt.root(), ot.root())
    gc, oc = gt.cells(), ot.cells()
    assert len(gc["key"]) == len(oc["key"]), (len(gc["key"]), len(oc["key"]))
    for f in ("level", "key", "first", "count", "parent", "child_first", "n_child", "is_leaf"):
        a, b = gc[f].astype(np.int64), oc[f].astype(np.int64)
        if f == "child_first":
            a = np.where(gc["n_child"] > 0, a, -1)
            b = np.where(oc["n_child"] > 0, b, -1)
        assert np.array_equal(a, b), f"cell field {f} differs"
    assert np.array_equal(gc["centre"], oc["centre"]), "centres differ"
    assert np.array_equal(gc["bmax"], oc["bmax"]), "b_max differs"
    assert np.array_equal(gt.groups().astype(np.int64), ot.groups()), "groups differ"
    return gc, oc


def assert_lists_equal(gt, ot, groups=None):
    gpo, gpl, gmo, gml = gt.lists()
    opo, opl, omo, oml = ot.lists()
    if groups is None:
        assert np.array_equal(gpo, opo) and np.array_equal(gmo, omo), "list offsets differ"
        assert np.array_equal(gpl, opl), "P2P lists differ"
        assert np.array_equal(gml, oml), "M2P lists differ"
    else:
        for g in groups:
            assert np.array_equal(gpl[gpo[g]:gpo[g + 1]], opl[opo[g]:opo[g + 1]]), g
            assert np.array_equal(gml[gmo[g]:gmo[g + 1]], oml[omo[g]:omo[g + 1]]), g


def assert_moments_close(gm, om, count):
    """FP64 moments from re-centred children vs direct sums: 1e-13 relative to
    the cell's largest moment, times sqrt(count / 64) above 64 particles (the
    expected growth of rounding differences between two summation orders)."""
    scale = np.maximum(np.abs(om).max(axis=1), 1e-300)
    tol = 1e-13 * np.maximum(1.0, np.sqrt(np.asarray(count, dtype=np.float64) / 64.0))
    err = np.abs(gm - om).max(axis=1) / scale
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, (bad[:5], err[bad[:5]], tol[bad[:5]])


def rel_rms(a, ref):
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def sinks_of_groups(ot, groups):
    """Caller indices of every particle in the given group ordinals."""
    _, perm = ot.keys()
    gof = ot.group_of()
    sel = np.isin(gof, np.asarray(groups))
    return np.sort(perm[sel])
