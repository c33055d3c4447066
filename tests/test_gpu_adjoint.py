"""GPU adjoint (eval_forces_adjoint) vs the oracle's VJP of its treecode with
the topology frozen, vs central finite differences of the GPU's own FP64
forward, and vs the direct-sum VJP as theta -> 0."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1310_4502_amd import workloads as W
from paper_1310_4502_amd.binding import HOT_FP64, HOT_MIXED, Tree
from gpu_util import SINK_TOL_FP64, SINK_TOL_MIXED, assert_sinks, build_both, rel_rms, to_dev

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


CASES = [
    # name, n, p, theta, direct_max, n_leaf, n_group
    ("uniform4k", None, 2, 0.5, 0, 16, 64),
    ("plummer1m", 6000, 4, 0.6, 0, 16, 64),
    ("clustered4m", 5000, 6, 0.5, 24, 8, 32),
    ("plummer1m", 2500, 8, 0.5, 0, 16, 96),
]


@pytest.mark.parametrize("name,n,p,theta,dmax,n_leaf,n_group", CASES)
def test_adjoint_vs_oracle_vjp(name, n, p, theta, dmax, n_leaf, n_group):
    w = W.make(name, n=n)
    w.n_leaf, w.n_group = n_leaf, n_group
    _log("case", name, w.n, "p", p)
    gt, ot, pos, mass, p = build_both(w, theta=theta, direct_max=dmax, p=p)
    ot.compute_moments(w.pos, w.mass, p)
    abar_np = W.cotangent(w.n, 404)
    ox, om = ot.vjp(w.pos, w.mass, w.eps, abar_np)
    abar = torch.from_numpy(abar_np).cuda()
    gx64, gm64 = gt.eval_forces_adjoint(pos, mass, w.eps, abar, HOT_FP64, with_mass=True)
    e64 = rel_rms(gx64.cpu().numpy(), ox)
    m64 = rel_rms(gm64.cpu().numpy(), om)
    _log("fp64 xbar", e64, "mbar", m64)
    assert e64 <= 1e-11 and m64 <= 1e-11
    assert_sinks(gx64.cpu().numpy(), ox, SINK_TOL_FP64, "xbar fp64")
    assert_sinks(gm64.cpu().numpy(), om, SINK_TOL_FP64, "mbar fp64")
    gx, gm = gt.eval_forces_adjoint(pos, mass, w.eps, abar, HOT_MIXED, with_mass=True)
    e32 = rel_rms(gx.cpu().numpy(), ox)
    m32 = rel_rms(gm.cpu().numpy(), om)
    _log("mixed xbar", e32, "mbar", m32)
    assert e32 <= 1e-5 and m32 <= 1e-5
    _log("per-sink max xbar", assert_sinks(gx.cpu().numpy(), ox, SINK_TOL_MIXED, "xbar mixed"),
         "mbar", assert_sinks(gm.cpu().numpy(), om, SINK_TOL_MIXED, "mbar mixed"))
    # deterministic
    gx2, _ = gt.eval_forces_adjoint(pos, mass, w.eps, abar, HOT_MIXED)
    assert torch.equal(gx, gx2)


def _source_runs(ot):
    """Records per source item (a 64-particle chunk of a group) and, per
    (item, sink group) run, the number of the item's particles that lie in
    the group's P2P cells, from the oracle's lists."""
    cells = ot.cells()
    gcell = ot.groups()
    po, pl, _, _ = ot.lists()
    gf, gn = cells["first"][gcell], cells["count"][gcell]
    n = int(gn.sum())
    item_of = np.empty(n, np.int64)
    first = []
    for g in range(len(gcell)):
        for f in range(gf[g], gf[g] + gn[g], 64):
            item_of[f:min(f + 64, gf[g] + gn[g])] = len(first)
            first.append(f)
    first = np.array(first)
    eg = np.repeat(np.arange(len(gcell)), np.diff(po))
    cf, cc = cells["first"][pl], cells["count"][pl]
    nrec = np.zeros(len(first), np.int64)
    marked = {}
    for e in range(len(pl)):
        for q in range(item_of[cf[e]], item_of[cf[e] + cc[e] - 1] + 1):
            nrec[q] += 1
            lo, hi = max(cf[e], first[q]), min(cf[e] + cc[e], first[q] + 64)
            marked[(q, eg[e])] = marked.get((q, eg[e]), 0) + hi - lo
    return nrec, np.array(list(marked.values()))


def test_adjoint_source_units_and_packed_runs():
    """In a Plummer core a source item is pair-summed by thousands of sink
    groups: its records are split into several work units whose partial sums
    are added afterwards, and runs that touch at most 32 of its particles are
    swept by packed lane slices. Both must reproduce the oracle VJP."""
    w = W.make("plummer1m", n=32768)
    w.n_leaf, w.n_group = 16, 64
    gt, ot, pos, mass, p = build_both(w, theta=0.6, direct_max=16, p=4)
    nrec, marked = _source_runs(ot)
    _log("records per item: max", nrec.max(), "items with > 512:", int((nrec > 512).sum()),
         "runs with <= 32 / > 32 particles:", int((marked <= 32).sum()), int((marked > 32).sum()))
    assert nrec.max() > 2 * 512 and (marked <= 32).any() and (marked > 32).any()
    ot.compute_moments(w.pos, w.mass, p)
    abar_np = W.cotangent(w.n, 405)
    ox, om = ot.vjp(w.pos, w.mass, w.eps, abar_np)
    abar = torch.from_numpy(abar_np).cuda()
    gx64, gm64 = gt.eval_forces_adjoint(pos, mass, w.eps, abar, HOT_FP64, with_mass=True)
    e64 = rel_rms(gx64.cpu().numpy(), ox)
    m64 = rel_rms(gm64.cpu().numpy(), om)
    gx, gm = gt.eval_forces_adjoint(pos, mass, w.eps, abar, HOT_MIXED, with_mass=True)
    e32 = rel_rms(gx.cpu().numpy(), ox)
    m32 = rel_rms(gm.cpu().numpy(), om)
    _log("fp64 xbar", e64, "mbar", m64, "mixed xbar", e32, "mbar", m32)
    assert e64 <= 1e-11 and m64 <= 1e-11
    assert e32 <= 1e-5 and m32 <= 1e-5
    assert_sinks(gx64.cpu().numpy(), ox, SINK_TOL_FP64, "xbar fp64")
    assert_sinks(gx.cpu().numpy(), ox, SINK_TOL_MIXED, "xbar mixed")
    assert_sinks(gm.cpu().numpy(), om, SINK_TOL_MIXED, "mbar mixed")


def test_adjoint_directional_fd():
    """x̄ . v equals the central difference of sum abar . a along v (topology
    frozen, FP64 GPU forward), Richardson-extrapolated from h = 2e-6 and 1e-6.
    The softening is kept well above h (truncation error ~ (h/eps)^2)."""
    w = W.make("clustered4m", n=20000)
    w.eps = 1e-3
    gt, ot, pos, mass, p = build_both(w, p=4)
    abar = torch.from_numpy(W.cotangent(w.n, 7)).cuda()
    v = torch.from_numpy(np.random.default_rng(8).normal(size=(w.n, 3))).cuda()
    xbar, mbar = gt.eval_forces_adjoint(pos, mass, w.eps, abar, HOT_FP64, with_mass=True)
    h = 1e-6

    def L(x, m):
        gt.compute_moments(x, m, p)
        a, _, _ = gt.eval_forces(x, m, w.eps, HOT_FP64)
        return float((a * abar).sum())

    def cd(f, hh):
        return (f(hh) - f(-hh)) / (2 * hh)

    fx = lambda hh: L(pos + hh * v, mass)
    fd = (4 * cd(fx, h) - cd(fx, 2 * h)) / 3
    an = float((xbar * v).sum())
    _log("directional", an, fd)
    assert abs(an - fd) <= 1e-6 * abs(fd)
    u = torch.from_numpy(np.random.default_rng(9).random(w.n)).cuda()
    fm = lambda hh: L(pos, mass * (1 + hh * u))
    fdm = (4 * cd(fm, h) - cd(fm, 2 * h)) / 3
    anm = float((mbar * mass * u).sum())
    _log("directional mass", anm, fdm)
    assert abs(anm - fdm) <= 1e-6 * abs(fdm)
    gt.compute_moments(pos, mass, p)


def test_adjoint_theta_zero_is_direct_vjp():
    w = W.make("plummer1m", n=3000)
    w.n_leaf, w.n_group = 8, 32
    gt, ot, pos, mass, p = build_both(w, theta=1e-6, p=2)
    abar_np = W.cotangent(w.n, 3)
    xd, md = oracle.direct_vjp(w.pos, w.mass, w.eps, abar_np)
    gx, gm = gt.eval_forces_adjoint(pos, mass, w.eps, torch.from_numpy(abar_np).cuda(), HOT_FP64,
                                    with_mass=True)
    assert rel_rms(gx.cpu().numpy(), xd) <= 1e-12
    assert rel_rms(gm.cpu().numpy(), md) <= 1e-12
    # translation invariance of the exact pair VJP
    assert np.linalg.norm(gx.cpu().numpy().sum(axis=0)) <= 1e-10 * np.abs(xd).sum()


@pytest.mark.parametrize("eps", [1e-3, 0.0])
def test_adjoint_ties_and_big_leaf(eps):
    rng = np.random.default_rng(5)
    pos = np.concatenate([rng.random((2000, 3)), np.full((150, 3), 0.4321),
                          np.repeat(rng.random((50, 3)), 4, axis=0)])
    n = pos.shape[0]
    w = W.Workload("mix", pos, np.full(n, 1.0 / n), eps, 0.5, 3)
    gt, ot, tpos, tmass, p = build_both(w)
    ot.compute_moments(w.pos, w.mass, p)
    abar = W.cotangent(n, 11)
    ox, om = ot.vjp(w.pos, w.mass, eps, abar)
    gx, gm = gt.eval_forces_adjoint(tpos, tmass, eps, torch.from_numpy(abar).cuda(), HOT_FP64,
                                    with_mass=True)
    assert rel_rms(gx.cpu().numpy(), ox) <= 1e-11
    assert rel_rms(gm.cpu().numpy(), om) <= 1e-11


def test_torch_autograd_function():
    from paper_1310_4502_amd.binding import TreeForce
    w = W.make("plummer1m", n=4000)
    pos, mass = to_dev(w)
    t = Tree(pos, 16, 64, w.box)
    t.build_interaction_lists(0.6, 0)
    x = pos.clone().requires_grad_(True)
    acc = TreeForce.apply(x, mass, t, w.eps, 4, HOT_FP64)
    abar = torch.from_numpy(W.cotangent(w.n, 2)).cuda()
    (acc * abar).sum().backward()
    ref, _ = t.eval_forces_adjoint(pos, mass, w.eps, abar, HOT_FP64)
    assert torch.allclose(x.grad, ref, rtol=0, atol=0)


@pytest.mark.parametrize("torch_alloc", [True, False])
def test_adjoint_transposes_on_second_stream(torch_alloc):
    """The first adjoint on a tree builds the transposed lists on the
    context's second stream while the sink-side terms run on the context
    stream. With either allocator (the torch caching allocator told the
    stream, or hipMallocAsync) the first call, the call on cached lists and
    the first call after the lists are rebuilt give bit-identical results,
    in both precisions."""
    from paper_1310_4502_amd.binding import Context
    w = W.make("clustered4m", n=30000)
    w.n_leaf, w.n_group = 8, 64
    ctx = Context(0, torch.cuda.current_stream(), torch_alloc=torch_alloc)
    pos = torch.from_numpy(w.pos).cuda()
    mass = torch.from_numpy(w.mass).cuda()
    abar = torch.from_numpy(W.cotangent(w.n, 405)).cuda()
    t = Tree(pos, n_leaf=w.n_leaf, n_group=w.n_group, ctx=ctx)
    t.compute_moments(pos, mass, 4)
    for prec in (HOT_MIXED, HOT_FP64):
        t.build_interaction_lists(0.5, direct_max=24)
        side0 = ctx.n_side_allocs
        x1, m1 = t.eval_forces_adjoint(pos, mass, w.eps, abar, prec, with_mass=True)
        if torch_alloc:
            assert ctx.n_side_allocs > side0  # the transposed lists came from the second stream
        side1 = ctx.n_side_allocs
        x2, m2 = t.eval_forces_adjoint(pos, mass, w.eps, abar, prec, with_mass=True)
        assert ctx.n_side_allocs == side1  # cached: nothing on the second stream
        t.build_interaction_lists(0.5, direct_max=24)
        x3, m3 = t.eval_forces_adjoint(pos, mass, w.eps, abar, prec, with_mass=True)
        _log("prec", prec, "allocs", ctx.n_allocs, "side", ctx.n_side_allocs)
        assert torch.equal(x1, x2) and torch.equal(m1, m2)
        assert torch.equal(x1, x3) and torch.equal(m1, m3)
        assert bool(torch.isfinite(x1).all())
    t.close()
    ctx.close()


def test_adjoint_allocation_failure_on_second_stream():
    """An allocation refused while the transposed lists are being built on
    the context's second stream fails the call with HOT_E_OOM after the
    second stream has drained; everything the call allocated is freed, the
    tree stays usable, and the next adjoint equals an undisturbed context's."""
    import ctypes
    from paper_1310_4502_amd import binding
    from paper_1310_4502_amd.binding import HOT_E_OOM, HotError
    w = W.make("clustered4m", n=20000)
    pos = torch.from_numpy(w.pos).cuda()
    mass = torch.from_numpy(w.mass).cuda()
    abar = torch.from_numpy(W.cotangent(w.n, 406)).cuda()
    ref = Tree(pos, n_leaf=8, n_group=64)
    ref.compute_moments(pos, mass, 4)
    ref.build_interaction_lists(0.5, direct_max=24)
    xr, mr = ref.eval_forces_adjoint(pos, mass, w.eps, abar, HOT_MIXED, with_mass=True)

    main = torch.cuda.current_stream().cuda_stream
    state = {"fail": False, "refused": 0}
    blocks, side = {}, {}

    def _a(user, nbytes, stream):
        if stream and stream != main:
            if state["fail"]:
                state["refused"] += 1
                return None
            if stream not in side:
                side[stream] = torch.cuda.ExternalStream(stream)
            with torch.cuda.stream(side[stream]):
                t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        else:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        blocks[t.data_ptr()] = t
        return t.data_ptr()

    def _f(user, ptr, stream):
        blocks.pop(ptr, None)

    afn, ffn = binding.ALLOC_FN(_a), binding.FREE_FN(_f)
    alloc = binding._Allocator(afn, ffn, None)
    L = binding.load()
    ctx = binding.Context(0, torch.cuda.current_stream(), torch_alloc=False)
    L.hot_ctx_destroy(ctx.h)
    h = ctypes.c_void_p()
    assert L.hot_ctx_create(0, ctypes.c_void_p(main), ctypes.byref(alloc), ctypes.byref(h)) == 0
    ctx.h = h
    t = Tree(pos, n_leaf=8, n_group=64, ctx=ctx)
    t.compute_moments(pos, mass, 4)
    t.build_interaction_lists(0.5, direct_max=24)
    held = len(blocks)
    state["fail"] = True
    with pytest.raises(HotError) as e:
        t.eval_forces_adjoint(pos, mass, w.eps, abar, HOT_MIXED, with_mass=True)
    assert e.value.code == HOT_E_OOM and state["refused"] == 1
    ctx.sync()
    assert len(blocks) == held  # the failed call freed what it allocated
    state["fail"] = False
    x, m = t.eval_forces_adjoint(pos, mass, w.eps, abar, HOT_MIXED, with_mass=True)
    _log("blocks", held, len(blocks), "side streams", len(side))
    assert torch.equal(x, xr) and torch.equal(m, mr)
    t.close()
    ctx.close()
    ref.close()
