"""Parity at the benchmark workloads' full sizes, in the configuration bench.py
times: the whole tree (keys, order, cells, centres, b_max, groups) bit-exact
against the oracle; lists bit-exact and moments close on sampled groups;
accelerations on every sink of the sampled groups against the oracle
treecode, and on sampled sinks against direct summation; for the 2^24
Zel'dovich field also the adjoint (directional FD of the FP64 forward with
the topology frozen, and direct-sum VJP rows), error-bound lists, and the
field wrapped into a periodic cube with and without background
subtraction."""
import sys
import time

import numpy as np
import pytest
import torch

import oracle
from paper_1310_4502_amd import workloads as W
from paper_1310_4502_amd.binding import HOT_FP64, HOT_MIXED, Tree
from gpu_util import (SINK_TOL_FP64, SINK_TOL_MIXED, KAPPA_C_FP64, KAPPA_C_MIXED, assert_sinks,
                      assert_sinks_kappa, assert_lists_equal, assert_moments_close, assert_tree_equal,
                      rel_rms, to_dev)

pytestmark = pytest.mark.gpu

# workload -> (n_leaf, n_group, direct_max) as timed by bench.py
BENCH = {"plummer1m": (16, 256, 16), "clustered4m": (16, 256, 32), "zeldovich16m": (16, 96, 64),
         "clustered16m": (16, 256, 32)}


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _check(name, n_groups_sample, n_direct):
    t0 = time.time()
    w = W.make(name)
    n_leaf, n_group, dmax = BENCH[name]
    pos, mass = to_dev(w)
    gt = Tree(pos, n_leaf, n_group, w.box)
    gt.build_interaction_lists(w.theta, dmax)
    gt.compute_moments(pos, mass, w.p)
    ga, _, st = gt.eval_forces(pos, mass, w.eps, HOT_MIXED, stats=True)
    ga = ga.cpu().numpy()
    _log(f"{name}: N={w.n} gpu done {time.time() - t0:.1f}s")
    ot = oracle.Tree(w.pos, n_leaf, n_group, w.box)
    assert_tree_equal(gt, ot)
    _log(f"{name}: tree bit-exact {time.time() - t0:.1f}s")
    G = ot.counts()["n_groups"]
    groups = W.sample_indices(G, n_groups_sample, 77)
    ot.build_lists(w.theta, dmax, groups=groups)
    assert_lists_equal(gt, ot, groups=groups)
    po, pl, mo, ml = ot.lists()
    cells = np.unique(np.concatenate([ml[mo[g]:mo[g + 1]] for g in groups] +
                                     [np.arange(0, ot.counts()["n_cells"], 997)]))
    ot.compute_moments(w.pos, w.mass, w.p, cells=cells)
    gm = gt.moments()[cells]
    om = ot.moments()[cells]
    assert_moments_close(gm, om, gt.cells()["count"][cells], log=_log)
    _log(f"{name}: lists + moments ok {time.time() - t0:.1f}s")
    _, perm = ot.keys()
    sinks = np.sort(perm[np.isin(ot.group_of(), groups)])
    oa, ab, cs = ot.eval_abs(w.pos, w.mass, w.eps, sinks=sinks, cond=True)
    e_tree = rel_rms(ga[sinks], oa)
    ds = W.sample_indices(w.n, n_direct, 102)
    ad, _ = oracle.direct(w.pos, w.mass, w.eps, sinks=ds)
    e_dir = rel_rms(ga[ds], ad)
    _log(f"{name}: vs oracle treecode {e_tree:.3e} ({len(sinks)} sinks), vs direct {e_dir:.3e} "
         f"({n_direct} sinks) {time.time() - t0:.1f}s")
    assert e_tree <= 1e-5
    assert_sinks_kappa(ga[sinks], oa, cs, KAPPA_C_MIXED, "mixed")
    assert e_dir <= 1e-3
    return w, gt, pos, mass


@pytest.mark.parametrize("name,ng,nd", [("plummer1m", 64, 16384), ("clustered4m", 48, 8192),
                                        ("clustered16m", 24, 4096)])
def test_forward_full_size(name, ng, nd):
    _check(name, ng, nd)


def test_zeldovich16m_forward_and_adjoint():
    w, gt, pos, mass = _check("zeldovich16m", 24, 4096)
    abar = torch.from_numpy(W.cotangent(w.n, 404)).cuda()
    xbar, _ = gt.eval_forces_adjoint(pos, mass, w.eps, abar, HOT_MIXED)
    xb = xbar.cpu().numpy()
    # direct-sum VJP rows: the tree adjoint approximates them at the expansion's accuracy
    rows = W.sample_indices(w.n, 1024, 405)
    xd, _ = oracle.direct_vjp(w.pos, w.mass, w.eps, abar.cpu().numpy(), rows=rows)
    e_rows = rel_rms(xb[rows], xd)
    # directional derivative of the FP64 forward with the topology frozen
    v = torch.from_numpy(np.random.default_rng(8).normal(size=(w.n, 3))).cuda() * 1e-3

    def L(x):
        gt.compute_moments(x, mass, w.p)
        a, _, _ = gt.eval_forces(x, mass, w.eps, HOT_FP64)
        return (a * abar).sum().item()

    h = 1e-4
    d1 = (L(pos + h * v) - L(pos - h * v)) / (2 * h)
    d2 = (L(pos + 2 * h * v) - L(pos - 2 * h * v)) / (4 * h)
    fd = (4 * d1 - d2) / 3
    an = float((xbar * v).sum())
    gt.compute_moments(pos, mass, w.p)
    _log(f"zeldovich16m adjoint: vs direct VJP rows {e_rows:.3e}; directional {an:.9e} vs FD {fd:.9e}")
    assert e_rows <= 1e-3
    assert abs(an - fd) <= 1e-4 * abs(fd)


@pytest.mark.parametrize("name,tol", [("clustered4m", 1e-4), ("zeldovich16m", 1e-3)])
def test_error_bound_lists_full_size(name, tol):
    """Error-bound lists at full size: lists and per-entry orders bit-exact on
    sampled groups, accelerations on their sinks against the oracle treecode."""
    t0 = time.time()
    w = W.make(name)
    n_leaf, n_group, dmax = BENCH[name]
    pos, mass = to_dev(w)
    gt = Tree(pos, n_leaf, n_group, w.box)
    gt.build_interaction_lists_err(mass, tol, w.p, dmax)
    gt.compute_moments(pos, mass, w.p)
    ga, _, _ = gt.eval_forces(pos, mass, w.eps, HOT_MIXED)
    ga = ga.cpu().numpy()
    gq = gt.m2p_orders()
    _log(f"{name} err lists: gpu done {time.time() - t0:.1f}s, orders "
         f"{np.bincount(gq, minlength=w.p + 1).tolist()}")
    ot = oracle.Tree(w.pos, n_leaf, n_group, w.box)
    G = ot.counts()["n_groups"]
    groups = W.sample_indices(G, 24, 78)
    ot.build_lists_err(w.mass, tol, w.p, dmax, groups=groups)
    assert_lists_equal(gt, ot, groups=groups)
    oq = ot.m2p_orders()
    _, _, gmo, _ = gt.lists()
    _, _, omo, oml = ot.lists()
    for g in groups:
        assert np.array_equal(gq[gmo[g]:gmo[g + 1]], oq[omo[g]:omo[g + 1]]), g
    cells = np.unique(np.concatenate([oml[omo[g]:omo[g + 1]] for g in groups]))
    ot.compute_moments(w.pos, w.mass, w.p, cells=cells)
    _, perm = ot.keys()
    sinks = np.sort(perm[np.isin(ot.group_of(), groups)])
    oa, ab, cs = ot.eval_abs(w.pos, w.mass, w.eps, sinks=sinks, cond=True)
    e_tree = rel_rms(ga[sinks], oa)
    _log(f"{name} err lists: vs oracle treecode {e_tree:.3e} ({len(sinks)} sinks) "
         f"{time.time() - t0:.1f}s")
    assert e_tree <= 1e-5
    assert_sinks_kappa(ga[sinks], oa, cs, KAPPA_C_MIXED, "mixed")


@pytest.mark.parametrize("mode", ["theta", "bs", "err"])
def test_periodic_full_size(mode):
    """The 2^24 Zel'dovich field wrapped into the unit cube, which is the
    periodic cell (theta lists, theta lists with background subtraction, and
    error-bound lists at tolerance 1e-3; direct_max as bench.py uses for
    each): lists, images, and for background subtraction the flags and
    boxes, for error-bound lists the orders, bit-exact on sampled groups;
    accelerations on their sinks against the oracle treecode on the same
    lists (FP64 and mixed); for the theta lists with and without
    subtraction the adjoint against a directional finite difference of the
    FP64 forward with the topology frozen."""
    t0 = time.time()
    w = W.make("zeldovich16m")
    n_leaf, n_group, dmax = BENCH["zeldovich16m"]
    bs = mode == "bs"
    if bs:
        dmax = 0
    w.pos = np.ascontiguousarray(w.pos % 1.0)
    w.box = (0.0, 0.0, 0.0, 1.0)
    pos, mass = to_dev(w)
    gt = Tree(pos, n_leaf, n_group, w.box)
    if bs:
        gt.build_interaction_lists_periodic_bs(w.theta, dmax, 3)
    elif mode == "err":
        gt.build_interaction_lists_periodic_err(mass, 1e-3, w.p, dmax)
    else:
        gt.build_interaction_lists_periodic(w.theta, dmax)
    gt.compute_moments(pos, mass, w.p)
    g32 = gt.eval_forces(pos, mass, w.eps, HOT_MIXED)[0].cpu().numpy()
    g64 = gt.eval_forces(pos, mass, w.eps, HOT_FP64)[0].cpu().numpy()
    _log(f"periodic {mode}: gpu done {time.time() - t0:.1f}s")
    ot = oracle.Tree(w.pos, n_leaf, n_group, w.box)
    G = ot.counts()["n_groups"]
    groups = W.sample_indices(G, 16, 79)
    if bs:
        ot.build_lists_periodic_bs(w.theta, dmax, width=3, groups=groups)
    elif mode == "err":
        ot.build_lists_periodic_err(w.mass, 1e-3, w.p, dmax, groups=groups)
    else:
        ot.build_lists_periodic(w.theta, dmax, groups=groups)
    assert_lists_equal(gt, ot, groups=groups)
    gpo, _, gmo, _ = gt.lists()
    opo, _, omo, oml = ot.lists()
    gpi, gmi = gt.list_images()
    opi, omi = ot.list_images()
    if bs:
        gboff, gbox, gsg, gsub = gt.background()
        oboff, obox, osg, osub = ot.background()
    if mode == "err":
        gq, oq = gt.m2p_orders(), ot.m2p_orders()
    for g in groups:
        if mode == "err":
            assert np.array_equal(gq[gmo[g]:gmo[g + 1]], oq[omo[g]:omo[g + 1]]), g
        assert np.array_equal(gpi[gpo[g]:gpo[g + 1]], opi[opo[g]:opo[g + 1]]), g
        assert np.array_equal(gmi[gmo[g]:gmo[g + 1]], omi[omo[g]:omo[g + 1]]), g
        if bs:
            assert np.array_equal(gsub[gmo[g]:gmo[g + 1]], osub[omo[g]:omo[g + 1]]), g
            assert np.array_equal(gbox[gboff[g]:gboff[g + 1]], obox[oboff[g]:oboff[g + 1]]), g
            assert np.array_equal(gsg[gboff[g]:gboff[g + 1]], osg[oboff[g]:oboff[g + 1]]), g
    cells = np.unique(np.concatenate([oml[omo[g]:omo[g + 1]] for g in groups] + [np.zeros(1, int)]))
    ot.compute_moments(w.pos, w.mass, w.p, cells=cells)
    _, perm = ot.keys()
    sinks = np.sort(perm[np.isin(ot.group_of(), groups)])
    oa, ab, cs = ot.eval_abs(w.pos, w.mass, w.eps, sinks=sinks, cond=True)
    e64, e32 = rel_rms(g64[sinks], oa), rel_rms(g32[sinks], oa)
    kap = ab / np.linalg.norm(oa, axis=1)
    s32 = float(np.linalg.norm(g32[sinks] - oa) / np.linalg.norm(ab))
    _log(f"periodic {mode}: vs oracle treecode fp64 {e64:.3e} mixed {e32:.3e} ({len(sinks)} sinks) "
         f"{time.time() - t0:.1f}s; cancellation |terms|/|a| median {np.median(kap):.1f} "
         f"p99 {np.percentile(kap, 99):.1f} max {kap.max():.1f}; mixed error / term scale {s32:.2e}")
    assert e64 <= 1e-10
    assert_sinks_kappa(g64[sinks], oa, cs, KAPPA_C_FP64, "fp64")
    # the mixed error measured against the scale of the terms it is summed
    # from: without subtraction the near-uniform field's net force is a small
    # remainder of large contributions (cancellation factor above), so FP32
    # rounding of those terms weighs more against |a|; with subtraction the
    # terms are perturbations and the plain relative bound holds as well
    assert_sinks_kappa(g32[sinks], oa, cs, KAPPA_C_MIXED, "mixed")
    assert s32 <= 1e-6
    if bs:
        assert e32 <= 1e-5
    if mode == "err":
        return
    abar = torch.from_numpy(W.cotangent(w.n, 406)).cuda()
    xbar, _ = gt.eval_forces_adjoint(pos, mass, w.eps, abar, HOT_FP64)
    v = torch.from_numpy(np.random.default_rng(9).normal(size=(w.n, 3))).cuda() * 1e-3

    def L(x):
        gt.compute_moments(x, mass, w.p)
        a, _, _ = gt.eval_forces(x, mass, w.eps, HOT_FP64)
        return (a * abar).sum().item()

    h = 1e-4
    d1 = (L(pos + h * v) - L(pos - h * v)) / (2 * h)
    d2 = (L(pos + 2 * h * v) - L(pos - 2 * h * v)) / (4 * h)
    fd = (4 * d1 - d2) / 3
    an = float((xbar * v).sum())
    _log(f"periodic {mode} adjoint at 2^24: directional {an:.9e} vs FD {fd:.9e}")
    assert abs(an - fd) <= 1e-4 * abs(fd)
