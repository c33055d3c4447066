"""Differentiable kick-drift-kick leapfrog over the tree force, with step
checkpointing for the reverse pass.

Forward (K steps, dt):
    a_0 = a(x_0)
    v_h     = v_k + dt/2 a_k
    x_{k+1} = x_k + dt v_h
    a_{k+1} = a(x_{k+1})
    v_{k+1} = v_h + dt/2 a_{k+1}
a(x) is the library's force evaluation on a tree built at x (its topology is
then held fixed for the derivative). Reverse: the adjoint of every step uses
one vector-Jacobian product of a per position (K + 1 in total), each on the
tree of that position. Only every `every`-th state is kept; the reverse pass
recomputes each segment from its checkpoint, rebuilding bit-identical trees
(the whole force path is deterministic), and checks that the recomputed
segment ends exactly on the next stored checkpoint.

The paper's integrator is the symplectic comoving leapfrog (Time Integration
section); its checkpoints keep the leapfrog offset between position and
velocity. The kick-drift-kick states kept here are synchronous, so a restart
from one needs no offset.

With periodic=True the box (lo, L) is the periodic cell: positions are
integrated unwrapped, and every force evaluation sees them wrapped into the
cell (x - L floor((x - lo) / L), whose derivative is the identity almost
everywhere), on periodic lists; background=True subtracts the mean density
on them (neighbourhood of bg_width group sides). err_tol, if set, replaces
the theta test by the error-bound test (orders up to p).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Tuple

import torch

from .binding import HOT_FP64, HOT_MIXED, Tree


@dataclass
class ForceField:
    mass: torch.Tensor
    eps: float
    theta: float
    p: int
    n_leaf: int = 16
    n_group: int = 64
    direct_max: int = 0
    precision: int = HOT_MIXED
    box: Optional[tuple] = None
    periodic: bool = False
    background: bool = False
    bg_width: int = 3
    err_tol: Optional[float] = None

    def _wrap(self, x: torch.Tensor) -> torch.Tensor:
        if not self.periodic:
            return x
        lo = torch.tensor(self.box[:3], dtype=x.dtype, device=x.device)
        side = float(self.box[3])
        w = x - side * torch.floor((x - lo) / side)
        # a coordinate rounding up to lo + L lies on the cell's far face: keep it inside
        return torch.where(w >= lo + side, w - side, w).contiguous()

    def tree(self, x: torch.Tensor) -> Tree:
        if self.periodic and self.box is None:
            raise ValueError("periodic force fields need the box (lo, L) of the periodic cell")
        if self.background and (not self.periodic or self.err_tol is not None):
            raise ValueError("background subtraction needs periodic theta lists")
        t = Tree(self._wrap(x), self.n_leaf, self.n_group, self.box)
        if self.background:
            t.build_interaction_lists_periodic_bs(self.theta, self.direct_max, self.bg_width)
        elif self.periodic and self.err_tol is not None:
            t.build_interaction_lists_periodic_err(self.mass, self.err_tol, self.p, self.direct_max)
        elif self.periodic:
            t.build_interaction_lists_periodic(self.theta, self.direct_max)
        elif self.err_tol is not None:
            t.build_interaction_lists_err(self.mass, self.err_tol, self.p, self.direct_max)
        else:
            t.build_interaction_lists(self.theta, self.direct_max)
        return t

    def accel(self, t: Tree, x: torch.Tensor, precision: Optional[int] = None) -> torch.Tensor:
        xw = self._wrap(x)
        t.compute_moments(xw, self.mass, self.p)
        a, _, _ = t.eval_forces(xw, self.mass, self.eps,
                                self.precision if precision is None else precision)
        return a

    def vjp(self, t: Tree, x: torch.Tensor, abar: torch.Tensor) -> torch.Tensor:
        xw = self._wrap(x)
        t.compute_moments(xw, self.mass, self.p)
        xbar, _ = t.eval_forces_adjoint(xw, self.mass, self.eps, abar.contiguous(),
                                        self.precision)
        return xbar


class RecomputeMismatch(RuntimeError):
    pass


def _segment(field: ForceField, x, v, a, dt, n, keep_trees: bool):
    """n KDK steps from (x, v) with a = a(x); returns the per-step positions,
    trees (if kept) and the final state."""
    xs, trees = [x], []
    if a is None or keep_trees:
        t = field.tree(x)
        if a is None:
            a = field.accel(t, x)
        if keep_trees:
            trees.append(t)
    for _ in range(n):
        vh = v + (0.5 * dt) * a
        x = x + dt * vh
        t = field.tree(x)
        a = field.accel(t, x)
        v = vh + (0.5 * dt) * a
        xs.append(x)
        if keep_trees:
            trees.append(t)
    return xs, trees, x, v, a


def run(field: ForceField, x0: torch.Tensor, v0: torch.Tensor, dt: float, steps: int,
        every: int = 4):
    """Forward pass; returns (x_K, v_K, checkpoints) with checkpoints[m] =
    (x, v, a) at step m * every."""
    ckpt = []
    x, v, a = x0, v0, None
    k = 0
    while k < steps:
        n = min(every, steps - k)
        if a is None:
            a = field.accel(field.tree(x), x)
        ckpt.append((x, v, a))
        _, _, x, v, a = _segment(field, x, v, a, dt, n, keep_trees=False)
        k += n
    ckpt.append((x, v, a))
    return x, v, ckpt


def grad(field: ForceField, ckpt, dt: float, steps: int, every: int, xbar_K: torch.Tensor,
         vbar_K: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
    """Reverse pass: (dL/dx_0, dL/dv_0) given (dL/dx_K, dL/dv_K)."""
    xbar, vbar = xbar_K.clone(), vbar_K.clone()
    apend = torch.zeros_like(xbar)  # cotangent of a_{j+1} from the following first half kick
    starts = list(range(0, steps, every))
    for m in reversed(range(len(starts))):
        k0 = starts[m]
        n = min(every, steps - k0)
        x, v, a = ckpt[m]
        xs, trees, xe, ve, _ = _segment(field, x, v, a, dt, n, keep_trees=True)
        xn, vn, _ = ckpt[m + 1]
        if not (torch.equal(xe, xn) and torch.equal(ve, vn)):
            raise RecomputeMismatch(f"segment {m} recomputed to a different state")
        for j in reversed(range(n)):
            # v_{j+1} = v_h + dt/2 a_{j+1}, a_{j+1} = a(x_{j+1})
            abar = apend + (0.5 * dt) * vbar
            xbar = xbar + field.vjp(trees[j + 1], xs[j + 1], abar)
            # x_{j+1} = x_j + dt v_h ; v_h = v_j + dt/2 a_j
            vbar = vbar + dt * xbar
            apend = (0.5 * dt) * vbar
        del trees
    x0 = ckpt[0][0]
    xbar = xbar + field.vjp(field.tree(x0), x0, apend)
    return xbar, vbar


def replay(field: ForceField, trees: List[Tree], x0: torch.Tensor, v0: torch.Tensor, dt: float,
           precision: int = HOT_FP64):
    """K steps with the given trees (one per position of a reference run):
    the topology of that run is replayed, moments are recomputed at the new
    positions. Used for finite differences of the frozen-topology map."""
    x, v = x0, v0
    a = field.accel(trees[0], x, precision)
    for k in range(len(trees) - 1):
        vh = v + (0.5 * dt) * a
        x = x + dt * vh
        a = field.accel(trees[k + 1], x, precision)
        v = vh + (0.5 * dt) * a
    return x, v


def trees_of_run(field: ForceField, x0, v0, dt, steps):
    """Positions' trees of a forward run (kept for topology replay)."""
    xs, trees, x, v, _ = _segment(field, x0, v0, None, dt, steps, keep_trees=True)
    return trees, x, v
