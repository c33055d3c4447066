"""eval_forces_noalloc through the C ABI: the allocation-free variant of
eval_forces (its buffers in the library's fixed device array) gives the same
accelerations and potentials as eval_forces, makes no call of the context's
allocator, and refuses what it cannot do without allocating.

Two calls in a row on different trees, the second smaller, check that the
array's leftover contents from the first call do not leak into the second.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1310_4502_amd import workloads as W
from paper_1310_4502_amd.binding import (HOT_E_CAPACITY, HOT_E_INVALID, HOT_FP64, HOT_MIXED,
                                         HotError, Tree)
from gpu_util import rel_rms, to_dev

pytestmark = pytest.mark.gpu

MAX_N = 1 << 20


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _tree(w, periodic=False, err_tol=None):
    pos, mass = to_dev(w)
    t = Tree(pos, w.n_leaf, w.n_group, w.box)
    if periodic:
        t.build_interaction_lists_periodic(w.theta, w.direct_max)
    elif err_tol is not None:
        t.build_interaction_lists_err(mass, err_tol, w.p, w.direct_max)
    else:
        t.build_interaction_lists(w.theta, w.direct_max)
    t.compute_moments(pos, mass, w.p)
    return t, pos, mass


def _both(t, pos, mass, eps, with_pot):
    ref, rpot, _ = t.eval_forces(pos, mass, eps, HOT_MIXED, with_pot=with_pot)
    acc = torch.full_like(pos, float("nan"))
    pot = torch.full((t.n,), float("nan"), dtype=torch.float64, device=pos.device) \
        if with_pot else None
    before = t.ctx.n_allocs
    t.eval_forces_noalloc(pos, mass, eps, acc, pot)
    torch.cuda.synchronize()
    assert t.ctx.n_allocs == before, "the allocation-free call used the allocator"
    return ref, rpot, acc, pot


@pytest.mark.parametrize("mode", ["theta", "err", "periodic"])
def test_noalloc_matches_eval_forces_twice(mode):
    # first call: 2^20 particles (the largest accepted), second: 20000
    cases = [("plummer1m", None), ("uniform4k", 20000)]
    if mode == "periodic":
        cases = [("plummer1m", 200000), ("uniform4k", 20000)]
    for name, n in cases:
        w = W.make(name, n=n)
        if mode == "periodic":
            w.box = (0.0, 0.0, 0.0, 1.0)
        _log(f"noalloc {mode}: {name} N={w.n} p={w.p}")
        t, pos, mass = _tree(w, periodic=mode == "periodic",
                             err_tol=1e-4 if mode == "err" else None)
        ref, rpot, acc, pot = _both(t, pos, mass, w.eps, with_pot=True)
        assert torch.equal(acc, ref), "accelerations differ from eval_forces"
        assert torch.equal(pot, rpot), "potentials differ from eval_forces"
        if w.n <= 20000:
            # and the oracle treecode on the same lists (mixed-precision bar)
            ot = oracle.Tree(w.pos, w.n_leaf, w.n_group, w.box)
            if mode == "periodic":
                ot.build_lists_periodic(w.theta, w.direct_max)
            elif mode == "err":
                ot.build_lists_err(w.mass, 1e-4, w.p, w.direct_max)
            else:
                ot.build_lists(w.theta, w.direct_max)
            ot.compute_moments(w.pos, w.mass, w.p)
            oa, _, _ = ot.eval(w.pos, w.mass, w.eps)
            e = rel_rms(acc.cpu().numpy(), oa)
            _log(f"  vs oracle treecode {e:.2e}")
            assert e <= 1e-5, e
        t.close()


def test_noalloc_refusals():
    w = W.make("uniform4k")
    t, pos, mass = _tree(w)
    acc = torch.empty_like(pos)
    with pytest.raises(HotError) as ei:
        t.eval_forces_noalloc(pos, mass, w.eps, acc, precision=HOT_FP64)
    assert ei.value.code == HOT_E_INVALID
    t.close()
    # one particle beyond the largest size
    n = MAX_N + 1
    pos = torch.from_numpy(W.uniform(n, 5)).cuda()
    mass = torch.full((n,), 1.0 / n, dtype=torch.float64, device="cuda")
    t = Tree(pos, 16, 64)
    t.build_interaction_lists(0.5, 0)
    t.compute_moments(pos, mass, 2)
    acc = torch.empty_like(pos)
    with pytest.raises(HotError) as ei:
        t.eval_forces_noalloc(pos, mass, 1e-3, acc)
    assert ei.value.code == HOT_E_CAPACITY
    t.close()
    # background-subtracted lists
    w = W.make("uniform4k")
    t, pos, mass = _tree(w)
    t.build_interaction_lists_periodic_bs(w.theta, 0, 3)
    with pytest.raises(HotError) as ei:
        t.eval_forces_noalloc(pos, mass, w.eps, torch.empty_like(pos))
    assert ei.value.code == HOT_E_INVALID
    t.close()
