"""Reverse pass of the checkpointed KDK leapfrog, on the CPU with a stand-in
force field whose Jacobian is known (a(x) = -k x + c x^3 per component):
the gradients must match central finite differences of the same integrator."""
import numpy as np
import pytest
import torch

from paper_1310_4502_amd import leapfrog as LF


class ToyField:
    def __init__(self, k=3.0, c=0.7):
        self.k, self.c = k, c
        self.built = 0

    def tree(self, x):
        self.built += 1
        return None

    def accel(self, t, x, precision=None):
        return -self.k * x + self.c * x ** 3

    def vjp(self, t, x, abar):
        return abar * (-self.k + 3 * self.c * x ** 2)


@pytest.mark.parametrize("steps,every", [(16, 4), (7, 3), (5, 8)])
def test_grad_matches_fd(steps, every):
    torch.manual_seed(0)
    n = 50
    x0 = torch.rand(n, 3, dtype=torch.float64)
    v0 = torch.randn(n, 3, dtype=torch.float64) * 0.3
    xt = x0 + 0.05 * torch.randn(n, 3, dtype=torch.float64)
    dt = 0.05
    f = ToyField()
    xK, vK, ck = LF.run(f, x0, v0, dt, steps, every)
    assert len(ck) == -(-steps // every) + 1
    gK = 2 * (xK - xt) / xK.numel()
    gx, gv = LF.grad(f, ck, dt, steps, every, gK, torch.zeros_like(vK))

    def loss(x, v):
        xe, _, _ = LF.run(f, x, v, dt, steps, every)
        return float(((xe - xt) ** 2).mean())

    h = 1e-6
    rng = np.random.default_rng(1)
    for _ in range(10):
        i, d = int(rng.integers(n)), int(rng.integers(3))
        for g, which in ((gx, 0), (gv, 1)):
            e = torch.zeros_like(x0)
            e[i, d] = h
            args_p = (x0 + e, v0) if which == 0 else (x0, v0 + e)
            args_m = (x0 - e, v0) if which == 0 else (x0, v0 - e)
            fd = (loss(*args_p) - loss(*args_m)) / (2 * h)
            assert abs(fd - float(g[i, d])) <= 1e-7 * max(1.0, abs(fd)) + 1e-9


def test_recompute_mismatch_is_detected():
    f = ToyField()
    x0 = torch.rand(10, 3, dtype=torch.float64)
    v0 = torch.zeros_like(x0)
    xK, vK, ck = LF.run(f, x0, v0, 0.1, 8, 4)
    x, v, a = ck[1]
    ck[1] = (x + 1e-12, v, a)  # a corrupted checkpoint
    with pytest.raises(LF.RecomputeMismatch):
        LF.grad(f, ck, 0.1, 8, 4, torch.ones_like(xK), torch.zeros_like(vK))
