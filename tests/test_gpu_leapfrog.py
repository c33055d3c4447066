"""Differentiable run: reverse-mode gradients of a 16-step KDK leapfrog over
the tree force (adjoint kernel + checkpointing every 4 steps) against central
finite differences of the FP64 path with the unperturbed run's per-step
topology replayed. Loss: mean over 3N of (x_16 - x_target)^2.

The central difference at h = 1e-6 carries an O(h^2) truncation error that
is visible (up to ~2e-4 of the RMS gradient) for particles in close
encounters in the Plummer core, so it is Richardson-extrapolated with the
difference at 2h: (4 D(h) - D(2h)) / 3."""
import sys

import numpy as np
import pytest
import torch

from paper_1310_4502_amd import leapfrog as LF
from paper_1310_4502_amd import workloads as W
from paper_1310_4502_amd.binding import HOT_FP64, HOT_MIXED

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("n,ncoord", [(1 << 14, 16), (1 << 18, 64)])
def test_leapfrog_gradient_vs_fd(n, ncoord):
    w = W.make("plummer256k", n=n)
    dt, steps, every = 1e-3, 16, 4
    x0 = torch.from_numpy(w.pos).cuda()
    v0 = torch.from_numpy(w.extra["vel"]).cuda()
    mass = torch.from_numpy(w.mass).cuda()
    rng = np.random.default_rng(505)
    xt = x0 + torch.from_numpy(0.01 * (1.0 / 16) * rng.standard_normal(w.pos.shape)).cuda()
    field = LF.ForceField(mass, w.eps, w.theta, w.p, 16, 64, 0, HOT_MIXED)
    xK, vK, ck = LF.run(field, x0, v0, dt, steps, every)
    gK = 2.0 * (xK - xt) / xK.numel()
    gx, gv = LF.grad(field, ck, dt, steps, every, gK, torch.zeros_like(vK))
    # finite differences: FP64 forces, topology of the unperturbed run
    trees, xr, _ = LF.trees_of_run(field, x0, v0, dt, steps)
    assert torch.equal(xr, xK)  # same run (deterministic)
    h = 1e-6
    idx = np.random.default_rng(506).choice(6 * n, size=ncoord, replace=False)
    fd, ad = [], []
    def central(which, i, d, hh):
        e = torch.zeros_like(x0)
        e[i, d] = hh
        if which == 0:
            xp, _ = LF.replay(field, trees, x0 + e, v0, dt, HOT_FP64)
            xm, _ = LF.replay(field, trees, x0 - e, v0, dt, HOT_FP64)
        else:
            xp, _ = LF.replay(field, trees, x0, v0 + e, dt, HOT_FP64)
            xm, _ = LF.replay(field, trees, x0, v0 - e, dt, HOT_FP64)
        # (xp - xt)^2 - (xm - xt)^2 = (xp - xm)(xp + xm - 2 xt): no cancellation of L
        return float(((xp - xm) * (xp + xm - 2 * xt)).sum()) / xK.numel() / (2 * hh)

    for q in idx:
        which, flat = divmod(int(q), 3 * n)
        i, d = divmod(flat, 3)
        fd.append((4 * central(which, i, d, h) - central(which, i, d, 2 * h)) / 3)
        ad.append(float((gx if which == 0 else gv)[i, d]))
    fd, ad = np.array(fd), np.array(ad)
    rms = np.sqrt(np.mean(fd ** 2))
    err = np.max(np.abs(ad - fd)) / rms
    _log(f"N={n}: max |g_adj - g_fd| / rms(g_fd) = {err:.3e} over {ncoord} coordinates")
    assert err <= 1e-4


def test_leapfrog_gradient_vs_oracle_replay():
    """A few coordinates of the same kind of gradient re-checked against the
    CPU oracle: the unperturbed run's per-step trees are rebuilt by the oracle
    from that run's positions, and the perturbed runs replay them with the
    oracle's FP64 treecode (moments recomputed at the replayed positions)."""
    import oracle

    n = 1 << 10
    w = W.make("plummer256k", n=n)
    dt, steps, every = 1e-3, 16, 4
    x0 = torch.from_numpy(w.pos).cuda()
    v0 = torch.from_numpy(w.extra["vel"]).cuda()
    mass = torch.from_numpy(w.mass).cuda()
    rng = np.random.default_rng(505)
    xt = x0 + torch.from_numpy(0.01 * (1.0 / 16) * rng.standard_normal(w.pos.shape)).cuda()
    field = LF.ForceField(mass, w.eps, w.theta, w.p, 16, 64, 0, HOT_MIXED)
    xK, vK, ck = LF.run(field, x0, v0, dt, steps, every)
    gK = 2.0 * (xK - xt) / xK.numel()
    gx, gv = LF.grad(field, ck, dt, steps, every, gK, torch.zeros_like(vK))
    xs, _, xr, _, _ = LF._segment(field, x0, v0, None, dt, steps, keep_trees=False)
    assert torch.equal(xr, xK)
    trees = []
    for x in xs:
        t = oracle.Tree(x.cpu().numpy(), 16, 64)
        t.build_lists(w.theta, 0)
        trees.append(t)
    m = w.mass
    xt_np = xt.cpu().numpy()

    def accel(t, x):
        t.compute_moments(x, m, w.p)
        return t.eval(x, m, w.eps, with_pot=False)[0]

    def replay(xa, va):
        x, v = xa.copy(), va.copy()
        a = accel(trees[0], x)
        for k in range(steps):
            vh = v + (0.5 * dt) * a
            x = x + dt * vh
            a = accel(trees[k + 1], x)
            v = vh + (0.5 * dt) * a
        return x

    xa0, va0 = w.pos.copy(), w.extra["vel"].copy()

    def central(which, i, d, hh):
        e = np.zeros_like(xa0)
        e[i, d] = hh
        if which == 0:
            xp, xm = replay(xa0 + e, va0), replay(xa0 - e, va0)
        else:
            xp, xm = replay(xa0, va0 + e), replay(xa0, va0 - e)
        return float(((xp - xm) * (xp + xm - 2 * xt_np)).sum()) / xK.numel() / (2 * hh)

    h = 1e-6
    idx = np.random.default_rng(507).choice(6 * n, size=2, replace=False)
    fd, ad = [], []
    for q in idx:
        which, flat = divmod(int(q), 3 * n)
        i, d = divmod(flat, 3)
        fd.append((4 * central(which, i, d, h) - central(which, i, d, 2 * h)) / 3)
        ad.append(float((gx if which == 0 else gv)[i, d]))
    fd, ad = np.array(fd), np.array(ad)
    err = np.max(np.abs(ad - fd)) / np.sqrt(np.mean(fd ** 2))
    _log(f"N={n} oracle replay: max |g_adj - g_fd| / rms(g_fd) = {err:.3e}; {ad} vs {fd}")
    assert err <= 1e-4


@pytest.mark.parametrize("lists", ["theta", "background", "error_bound"])
def test_periodic_leapfrog_gradient_vs_fd(lists):
    """The same gradient in the periodic unit cube: positions integrated
    unwrapped and wrapped for every force evaluation (some cross a face
    during the run); periodic lists (theta, theta with background
    subtraction, error-bound), their adjoint, against central differences of
    the FP64 replay with the run's topology."""
    n = 4096
    rng = np.random.default_rng(600)
    x0 = torch.from_numpy(rng.random((n, 3))).cuda()
    v0 = torch.from_numpy(0.5 * rng.standard_normal((n, 3))).cuda()
    mass = torch.full((n,), 1.0 / n, dtype=torch.float64).cuda()
    dt, steps, every = 1e-3, 16, 4
    field = LF.ForceField(mass, 1e-3, 0.5, 4, 16, 64, 0, HOT_MIXED, (0.0, 0.0, 0.0, 1.0), True,
                          background=lists == "background",
                          err_tol=1e-3 if lists == "error_bound" else None)
    xt = x0 + torch.from_numpy(0.01 * rng.standard_normal((n, 3))).cuda()
    xK, vK, ck = LF.run(field, x0, v0, dt, steps, every)
    crossed = int(((xK < 0) | (xK >= 1)).any(dim=1).sum())
    assert crossed > 0
    gK = 2.0 * (xK - xt) / xK.numel()
    gx, gv = LF.grad(field, ck, dt, steps, every, gK, torch.zeros_like(vK))
    trees, xr, _ = LF.trees_of_run(field, x0, v0, dt, steps)
    assert torch.equal(xr, xK)
    idx = np.random.default_rng(601).choice(6 * n, size=24, replace=False)
    fd, ad = [], []

    def central(which, i, d, hh):
        e = torch.zeros_like(x0)
        e[i, d] = hh
        if which == 0:
            xp, _ = LF.replay(field, trees, x0 + e, v0, dt, HOT_FP64)
            xm, _ = LF.replay(field, trees, x0 - e, v0, dt, HOT_FP64)
        else:
            xp, _ = LF.replay(field, trees, x0, v0 + e, dt, HOT_FP64)
            xm, _ = LF.replay(field, trees, x0, v0 - e, dt, HOT_FP64)
        return float(((xp - xm) * (xp + xm - 2 * xt)).sum()) / xK.numel() / (2 * hh)

    for q in idx:
        which, flat = divmod(int(q), 3 * n)
        i, d = divmod(flat, 3)
        fd.append((4 * central(which, i, d, 1e-6) - central(which, i, d, 2e-6)) / 3)
        ad.append(float((gx if which == 0 else gv)[i, d]))
    fd, ad = np.array(fd), np.array(ad)
    err = np.max(np.abs(ad - fd)) / np.sqrt(np.mean(fd ** 2))
    _log(f"periodic leapfrog ({lists}): {crossed} particles crossed a face; "
         f"max |g_adj - g_fd| / rms = {err:.3e}")
    assert err <= 1e-4
