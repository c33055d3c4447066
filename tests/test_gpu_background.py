"""GPU background subtraction on periodic lists against the oracle: lists,
images, subtraction flags and boxes bit-exact; forces against the oracle
treecode on the same lists (FP64 and mixed precision) and against the Ewald
direct sum; the gain the method is for (more accurate than the unsubtracted
lists at the same order in near-uniform volumes, far less FP32 rounding
there, and so fewer interactions at equal accuracy); the adjoint against the
oracle's VJP and finite differences; and the entry point's checks."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1310_4502_amd.binding import HOT_FP64, HOT_MIXED, HotError, Tree
from gpu_util import (SINK_TOL_FP64, SINK_TOL_MIXED, KAPPA_C_FP64, KAPPA_C_MIXED, assert_sinks,
                      assert_sinks_kappa, assert_lists_equal, rel_rms)

pytestmark = pytest.mark.gpu

BOX = np.array([0.0, 0.0, 0.0, 1.0])


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _lattice(n1, amp, seed):
    g = (np.arange(n1) + 0.5) / n1
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    x = (x + amp / n1 * np.random.default_rng(seed).standard_normal(x.shape)) % 1.0
    return x, np.full(x.shape[0], 1.0 / x.shape[0])


def _clustered(n, width, seed):
    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.random((n // 2, 3)),
                        (0.3 + width * rng.standard_normal((n - n // 2, 3))) % 1.0])
    return x, np.full(n, 1.0 / n)


CASES = [
    # kind, size, amplitude / width, p, theta, direct_max, n_leaf, n_group, neighbourhood
    ("lattice", 16, 0.05, 6, 0.6, 0, 16, 64, 3),
    ("lattice", 24, 0.3, 4, 0.5, 8, 8, 32, 5),
    ("clustered", 12000, 0.04, 6, 0.5, 0, 8, 32, 3),  # straddling leaves and octants
    ("clustered", 6000, 0.02, 8, 0.6, 16, 4, 16, 7),
]


def _pos(kind, size, a):
    return _lattice(size, a, 3) if kind == "lattice" else _clustered(size, a, 11)


@pytest.mark.parametrize("kind,size,a,p,theta,dmax,n_leaf,n_group,width", CASES)
def test_bs_lists_boxes_and_forces(kind, size, a, p, theta, dmax, n_leaf, n_group, width):
    pos_np, mass_np = _pos(kind, size, a)
    n = pos_np.shape[0]
    eps = 1e-3
    pos = torch.from_numpy(pos_np).cuda()
    mass = torch.from_numpy(mass_np).cuda()
    gt = Tree(pos, n_leaf, n_group, BOX)
    ot = oracle.Tree(pos_np, n_leaf, n_group, BOX)
    gt.build_interaction_lists_periodic_bs(theta, dmax, width)
    ot.build_lists_periodic_bs(theta, dmax, width=width)
    assert_lists_equal(gt, ot)
    gpi, gmi = gt.list_images()
    opi, omi = ot.list_images()
    assert np.array_equal(gpi, opi) and np.array_equal(gmi, omi), "images differ"
    goff, gbox, gsg, gsub = gt.background()
    ooff, obox, osg, osub = ot.background()
    assert np.array_equal(goff, ooff), "box offsets differ"
    assert np.array_equal(gbox, obox), "boxes differ"
    assert np.array_equal(gsg, osg) and np.array_equal(gsub, osub), "signs or flags differ"
    _log(kind, n, "M2P", len(gmi), "subtracted", int(gsub.sum()), "boxes", len(gsg),
         "with +1", int((gsg > 0).sum()))
    if kind == "clustered" and width == 3:
        assert (gsg > 0).any()
    gt.compute_moments(pos, mass, p)
    ot.compute_moments(pos_np, mass_np, p)
    ts = np.sort(np.random.default_rng(2).choice(n, 512, replace=False))
    oa, ab, cs = ot.eval_abs(pos_np, mass_np, eps, sinks=ts, cond=True)
    g64, _, _ = gt.eval_forces(pos, mass, eps, HOT_FP64)
    g32, _, _ = gt.eval_forces(pos, mass, eps, HOT_MIXED)
    e64 = rel_rms(g64.cpu().numpy()[ts], oa)
    e32 = rel_rms(g32.cpu().numpy()[ts], oa)
    _log("vs oracle treecode: fp64", e64, "mixed", e32)
    assert e64 <= 1e-11 and e32 <= 1e-5
    assert_sinks_kappa(g64.cpu().numpy()[ts], oa, cs, KAPPA_C_FP64, "fp64")
    assert_sinks_kappa(g32.cpu().numpy()[ts], oa, cs, KAPPA_C_MIXED, "mixed")


def test_bs_gain_in_near_uniform_volume():
    """A perturbed lattice: at the same theta and order the subtracted lists
    are closer to the Ewald direct sum, and their mixed-precision result is
    far closer to their FP64 one (the large cancelling cell fields are gone
    before the FP32 arithmetic)."""
    pos_np, mass_np = _lattice(32, 0.05, 7)
    n = pos_np.shape[0]
    eps, p = 1e-3, 6
    pos = torch.from_numpy(pos_np).cuda()
    mass = torch.from_numpy(mass_np).cuda()
    sinks = np.sort(np.random.default_rng(4).choice(n, 48, replace=False))
    ad = oracle.ewald_direct(pos_np, mass_np, 1.0, eps, sinks=sinks)
    res = {}
    for bs in (False, True):
        t = Tree(pos, 16, 64, BOX)
        if bs:
            t.build_interaction_lists_periodic_bs(0.6, 0)
        else:
            t.build_interaction_lists_periodic(0.6, 0)
        t.compute_moments(pos, mass, p)
        a64 = t.eval_forces(pos, mass, eps, HOT_FP64)[0].cpu().numpy()
        a32 = t.eval_forces(pos, mass, eps, HOT_MIXED)[0].cpu().numpy()
        res[bs] = (rel_rms(a64[sinks], ad), rel_rms(a32, a64))
    _log("unsubtracted: vs Ewald", res[False][0], "mixed vs fp64", res[False][1])
    _log("subtracted:   vs Ewald", res[True][0], "mixed vs fp64", res[True][1])
    assert res[True][0] <= res[False][0] / 3
    assert res[True][1] <= res[False][1] / 3


def test_bs_checks():
    pos_np, mass_np = _lattice(8, 0.2, 1)
    pos = torch.from_numpy(pos_np).cuda()
    mass = torch.from_numpy(mass_np).cuda()
    t = Tree(pos, 16, 64)  # no box given
    with pytest.raises(HotError):
        t.build_interaction_lists_periodic_bs(0.5, 0)
    t = Tree(pos, 16, 64, BOX)
    t.build_interaction_lists_periodic(0.5, 0)
    with pytest.raises(HotError):
        t.background()
    with pytest.raises(HotError):
        t.build_interaction_lists_periodic_bs(1.5, 0)
    for bad_width in (1, 4, 11):
        with pytest.raises(HotError):
            t.build_interaction_lists_periodic_bs(0.5, 0, bad_width)
    t.build_interaction_lists_periodic_bs(0.5, 0)
    assert t.counts()["n_boxes"] >= 0
    t.compute_moments(pos, mass, 4)
    with pytest.raises(HotError):
        t.eval_forces(pos, mass, 1e-3, HOT_MIXED, with_pot=True)
    a, _, _ = t.eval_forces(pos, mass, 1e-3, HOT_MIXED)
    assert torch.isfinite(a).all()
    xb, mb = t.eval_forces_adjoint(pos, mass, 1e-3, torch.zeros_like(pos), HOT_MIXED,
                                   with_mass=True)
    assert torch.all(xb == 0) and torch.all(mb == 0)


@pytest.mark.parametrize("kind,size,a,p,theta,dmax,n_leaf,n_group,width", [
    ("lattice", 12, 0.3, 6, 0.5, 0, 16, 64, 3),
    ("clustered", 1500, 0.04, 4, 0.6, 4, 8, 32, 3),   # straddling pieces
    ("clustered", 1200, 0.1, 4, 0.5, 0, 8, 32, 5),
])
def test_bs_adjoint_vs_oracle_vjp(kind, size, a, p, theta, dmax, n_leaf, n_group, width):
    """The adjoint of background-subtracted lists (subtracted moments at the
    sink, the box fields' gradients, the mean density through every mass)
    against the oracle's VJP on the same lists, and a directional finite
    difference of the FP64 forward in positions and in masses."""
    pos_np, mass_np = _pos(kind, size, a)
    if kind == "clustered":
        mass_np = mass_np * (0.5 + np.random.default_rng(3).random(mass_np.shape))
    n, eps = pos_np.shape[0], 1e-3
    pos = torch.from_numpy(pos_np).cuda()
    mass = torch.from_numpy(mass_np).cuda()
    gt = Tree(pos, n_leaf, n_group, BOX)
    ot = oracle.Tree(pos_np, n_leaf, n_group, BOX)
    gt.build_interaction_lists_periodic_bs(theta, dmax, width)
    ot.build_lists_periodic_bs(theta, dmax, width=width)
    gt.compute_moments(pos, mass, p)
    ot.compute_moments(pos_np, mass_np, p)
    abar_np = np.random.default_rng(46).standard_normal((n, 3))
    abar_np /= np.linalg.norm(abar_np)
    ox, om = ot.vjp(pos_np, mass_np, eps, abar_np)
    abar = torch.from_numpy(abar_np).cuda()
    gx64, gm64 = gt.eval_forces_adjoint(pos, mass, eps, abar, HOT_FP64, with_mass=True)
    gx, gm = gt.eval_forces_adjoint(pos, mass, eps, abar, HOT_MIXED, with_mass=True)
    r = [rel_rms(gx64.cpu().numpy(), ox), rel_rms(gm64.cpu().numpy(), om),
         rel_rms(gx.cpu().numpy(), ox), rel_rms(gm.cpu().numpy(), om)]
    _log(kind, n, "bs adjoint vs oracle VJP: fp64", r[:2], "mixed", r[2:])
    assert max(r[:2]) <= 1e-11 and max(r[2:]) <= 1e-5
    assert_sinks(gx64.cpu().numpy(), ox, SINK_TOL_FP64, "xbar fp64")
    assert_sinks(gx.cpu().numpy(), ox, SINK_TOL_MIXED, "xbar mixed")
    rng = np.random.default_rng(47)
    v = torch.from_numpy(rng.normal(size=pos_np.shape)).cuda()
    dm = torch.from_numpy(rng.normal(size=mass_np.shape) * mass_np).cuda()

    def L(x, m):
        gt.compute_moments(x, m, p)
        acc, _, _ = gt.eval_forces(x, m, eps, HOT_FP64)
        return float((acc * abar).sum())

    def cd(f, h):
        return (f(h) - f(-h)) / (2 * h)

    fx = lambda h: L(pos + h * v, mass)
    fm = lambda h: L(pos, mass + h * dm)
    fdx = (4 * cd(fx, 1e-6) - cd(fx, 2e-6)) / 3
    fdm = (4 * cd(fm, 1e-6) - cd(fm, 2e-6)) / 3
    anx, anm = float((gx64 * v).sum()), float((gm64 * dm).sum())
    _log("directional", anx, fdx, "mass", anm, fdm)
    assert abs(anx - fdx) <= 1e-6 * abs(fdx)
    assert abs(anm - fdm) <= 1e-6 * abs(fdm)


def test_bs_fewer_interactions_at_equal_accuracy():
    """The efficiency the method is for, on a near-uniform periodic field (the
    Zel'dovich recipe at 128^3, p = 8): with subtraction a larger opening
    angle reaches the accuracy that the unsubtracted lists need a smaller one
    for, so fewer interactions are evaluated. Errors against the
    unsubtracted lists at theta = 0.25 (FP64)."""
    from paper_1310_4502_amd import workloads as W
    w = W.make("zeldovich16m", n=128 ** 3)
    pos = torch.from_numpy(np.ascontiguousarray(w.pos % 1.0)).cuda()
    mass = torch.from_numpy(w.mass).cuda()

    def run(theta, bs):
        t = Tree(pos, 16, 96, BOX)
        if bs:
            t.build_interaction_lists_periodic_bs(theta, 0, 3)
        else:
            t.build_interaction_lists_periodic(theta, 0)
        t.compute_moments(pos, mass, 8)
        a, _, st = t.eval_forces(pos, mass, w.eps, HOT_FP64, stats=True)
        return a, st.p2p_pairs + st.m2p_pairs

    ref, _ = run(0.25, False)
    res = {}
    for theta, bs in ((0.4, False), (0.5, True), (0.5, False), (0.6, True)):
        a, inter = run(theta, bs)
        res[theta, bs] = (float((a - ref).norm() / ref.norm()), inter)
        _log(f"theta {theta} subtracted {bs}: rel err {res[theta, bs][0]:.3e}, "
             f"{inter:.3e} interactions")
    # same accuracy class with 1.5x - 1.7x fewer interactions
    assert res[0.5, True][0] <= 1.5 * res[0.4, False][0]
    assert res[0.5, True][1] <= 0.65 * res[0.4, False][1]
    assert res[0.6, True][0] <= res[0.5, False][0]
    assert res[0.6, True][1] <= 0.75 * res[0.5, False][1]
