"""ctypes binding of libhot.so (the C ABI declared in include/hot.h).

Argument marshalling only: every step of the force path runs in the HIP
library. PyTorch supplies device memory (the library's allocator callback is
backed by the torch caching allocator) and the stream (torch's current HIP
stream). If the library is missing the calls raise; there is no CPU path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhot.so")

HOT_OK, HOT_E_INVALID, HOT_E_STATE, HOT_E_OOM, HOT_E_DEVICE, HOT_E_CAPACITY = 0, -1, -2, -3, -4, -5
HOT_MIXED, HOT_FP64 = 0, 1
HOT_K1 = 16  # ORed into the precision argument: Dehnen's K1 softening
KERNELS = {"plummer": 0, "k1": HOT_K1}
_CODES = {-1: "HOT_E_INVALID", -2: "HOT_E_STATE", -3: "HOT_E_OOM", -4: "HOT_E_DEVICE",
          -5: "HOT_E_CAPACITY"}

EXPORTS = ["hot_ctx_create", "hot_ctx_destroy", "hot_last_error", "hot_sync", "tree_build",
           "tree_destroy", "compute_moments", "build_interaction_lists", "eval_forces",
           "eval_forces_adjoint", "tree_get_counts", "tree_get_root", "tree_get_keys",
           "tree_get_cells", "tree_get_groups", "tree_get_lists", "tree_get_moments",
           "tree_lookup", "build_interaction_lists_err", "tree_get_m2p_orders",
           "build_interaction_lists_periodic", "tree_get_list_images",
           "build_interaction_lists_periodic_bs", "tree_get_background",
           "build_interaction_lists_periodic_err", "eval_forces_noalloc", "hot_set_timing",
           "hot_get_timings"]

# phases of hot_get_timings, in the order of the HOT_T_* constants
PHASES = ["tree_build", "compute_moments", "build_interaction_lists", "eval_forces", "eval_p2p",
          "eval_m2p", "eval_forces_adjoint", "adj_transpose", "adj_p2p_sink", "adj_p2p_source",
          "adj_m2p_sink", "adj_m2p_cell", "adj_downward"]


class HotError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class _BuildOpts(ctypes.Structure):
    _fields_ = [("n_leaf", ctypes.c_int), ("n_group", ctypes.c_int),
                ("box", ctypes.POINTER(ctypes.c_double))]


class Stats(ctypes.Structure):
    _fields_ = [("p2p_pairs", ctypes.c_int64), ("m2p_pairs", ctypes.c_int64),
                ("ms_p2p", ctypes.c_double), ("ms_m2p", ctypes.c_double),
                ("ms_total", ctypes.c_double)]


_lib = None


def load(path: Optional[str] = None):
    """Load libhot.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library not built: {p} is missing (run paper_1310_4502_amd.build)")
    L = ctypes.CDLL(p)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.hot_ctx_create.argtypes = [i32, vp, ctypes.POINTER(_Allocator), ctypes.POINTER(vp)]
    L.hot_ctx_destroy.argtypes = [vp]
    L.hot_last_error.argtypes = [vp]
    L.hot_last_error.restype = ctypes.c_char_p
    L.hot_sync.argtypes = [vp]
    L.hot_set_timing.argtypes = [vp, i32]
    L.hot_get_timings.argtypes = [vp, vp]
    L.tree_build.argtypes = [vp, i64, vp, ctypes.POINTER(_BuildOpts), ctypes.POINTER(vp)]
    L.tree_destroy.argtypes = [vp, vp]
    L.compute_moments.argtypes = [vp, vp, vp, vp, i32]
    L.build_interaction_lists.argtypes = [vp, vp, dbl, i32]
    L.build_interaction_lists_err.argtypes = [vp, vp, vp, dbl, i32, i32]
    L.tree_get_m2p_orders.argtypes = [vp, vp, vp]
    L.build_interaction_lists_periodic.argtypes = [vp, vp, dbl, i32]
    L.tree_get_list_images.argtypes = [vp, vp, vp, vp]
    L.build_interaction_lists_periodic_bs.argtypes = [vp, vp, dbl, i32, i32]
    L.build_interaction_lists_periodic_err.argtypes = [vp, vp, vp, dbl, i32, i32]
    L.tree_get_background.argtypes = [vp, vp, vp, vp, vp, vp]
    L.eval_forces.argtypes = [vp, vp, vp, vp, dbl, i32, vp, vp, ctypes.POINTER(Stats)]
    L.eval_forces_adjoint.argtypes = [vp, vp, vp, vp, dbl, i32, vp, vp, vp]
    L.eval_forces_noalloc.argtypes = [vp, vp, vp, vp, dbl, i32, vp, vp, ctypes.POINTER(Stats)]
    L.tree_get_counts.argtypes = [vp, vp, vp]
    L.tree_get_root.argtypes = [vp, vp, vp]
    L.tree_get_keys.argtypes = [vp, vp, vp, vp]
    L.tree_get_cells.argtypes = [vp, vp] + [vp] * 10
    L.tree_get_groups.argtypes = [vp, vp, vp]
    L.tree_get_lists.argtypes = [vp, vp, vp, vp, vp, vp]
    L.tree_get_moments.argtypes = [vp, vp, vp]
    L.tree_lookup.argtypes = [vp, vp, i64, vp, vp]
    _lib = L
    return L


def _np(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dev(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    """A library context bound to one device and one HIP stream."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None,
                 torch_alloc: bool = True):
        L = load()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._blocks = {}
        self._alloc = None
        self.n_allocs = 0  # calls of the allocator callback
        self.n_side_allocs = 0  # of them, blocks first used on the library's second stream
        if torch_alloc:
            dev = torch.device("cuda", device)

            main = self.stream.cuda_stream
            side = {}

            def _a(user, nbytes, stream):
                # the block belongs to the stream that first uses it (the
                # library's second stream for the adjoint's transposed
                # lists), so that the caching allocator never hands it to
                # another stream while work queued there may still use it
                self.n_allocs += 1
                try:
                    if not stream or stream == main:
                        t = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
                    else:
                        self.n_side_allocs += 1
                        if stream not in side:
                            side[stream] = torch.cuda.ExternalStream(stream, device=dev)
                        with torch.cuda.stream(side[stream]):
                            t = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
                except RuntimeError:
                    return None
                self._blocks[t.data_ptr()] = t
                return t.data_ptr()

            def _f(user, ptr, stream):
                self._blocks.pop(ptr, None)

            self._afn, self._ffn = ALLOC_FN(_a), FREE_FN(_f)
            self._alloc = _Allocator(self._afn, self._ffn, None)
        h = ctypes.c_void_p()
        rc = L.hot_ctx_create(device, ctypes.c_void_p(self.stream.cuda_stream),
                              ctypes.byref(self._alloc) if self._alloc else None,
                              ctypes.byref(h))
        if rc != HOT_OK:
            raise HotError(rc, "hot_ctx_create failed")
        self.h = h

    def check(self, rc):
        if rc != HOT_OK:
            raise HotError(rc, load().hot_last_error(self.h).decode())

    def sync(self):
        self.check(load().hot_sync(self.h))

    def set_timing(self, on: bool = True):
        """Record HIP events around every phase of later calls (and forget
        earlier records)."""
        self.check(load().hot_set_timing(self.h, int(bool(on))))

    def timings(self):
        """{phase: ms of its most recent recorded run} (waits for the stream);
        phases not run since timing was switched on are left out."""
        out = np.empty(len(PHASES))
        self.check(load().hot_get_timings(self.h, _np(out)))
        return {k: float(v) for k, v in zip(PHASES, out) if v >= 0}

    def close(self):
        if getattr(self, "h", None):
            load().hot_ctx_destroy(self.h)
            self.h = None
            self._blocks.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_CTX = {}


def context(device: int = 0) -> Context:
    """The cached context for (device, current stream)."""
    s = torch.cuda.current_stream(device)
    key = (device, s.cuda_stream)
    if key not in _CTX:
        _CTX[key] = Context(device, s)
    return _CTX[key]


def _as_pos(pos: torch.Tensor) -> torch.Tensor:
    if pos.dtype != torch.float64 or not pos.is_cuda or pos.dim() != 2 or pos.shape[1] != 3:
        raise ValueError("pos must be a CUDA float64 tensor of shape [N, 3]")
    return pos.contiguous()


def _as_vec(m: torch.Tensor, n: int) -> torch.Tensor:
    if m.dtype != torch.float64 or not m.is_cuda or m.shape != (n,):
        raise ValueError("mass must be a CUDA float64 tensor of shape [N]")
    return m.contiguous()


class Tree:
    """A built tree (tree_build) and its state: moments, lists."""

    def __init__(self, pos: torch.Tensor, n_leaf: int = 16, n_group: int = 64,
                 box=None, ctx: Optional[Context] = None):
        pos = _as_pos(pos)
        self.ctx = ctx or context(pos.device.index or 0)
        self.n = pos.shape[0]
        opts = _BuildOpts(n_leaf, n_group, None)
        self._box = None
        if box is not None:
            self._box = (ctypes.c_double * 4)(*[float(v) for v in box])
            opts.box = ctypes.cast(self._box, ctypes.POINTER(ctypes.c_double))
        h = ctypes.c_void_p()
        self.h = None
        self.ctx.check(load().tree_build(self.ctx.h, self.n, _dev(pos), ctypes.byref(opts),
                                         ctypes.byref(h)))
        self.h = h
        self.p = None

    def close(self):
        if getattr(self, "h", None) and self.ctx.h:
            load().tree_destroy(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- the four calls of the force path
    def compute_moments(self, pos, mass, p):
        pos = _as_pos(pos)
        mass = _as_vec(mass, self.n)
        self.ctx.check(load().compute_moments(self.ctx.h, self.h, _dev(pos), _dev(mass), int(p)))
        self.p = p

    def build_interaction_lists(self, theta, direct_max=0):
        self.ctx.check(load().build_interaction_lists(self.ctx.h, self.h, float(theta),
                                                      int(direct_max)))

    def build_interaction_lists_err(self, mass, err_tol, p_max, direct_max=0):
        """Error-bound lists: each M2P entry gets the lowest order <= p_max
        whose field-error bound is at most err_tol (an acceleration)."""
        mass = _as_vec(mass, self.n)
        self.ctx.check(load().build_interaction_lists_err(self.ctx.h, self.h, _dev(mass),
                                                          float(err_tol), int(p_max),
                                                          int(direct_max)))

    def build_interaction_lists_periodic(self, theta, direct_max=0):
        """Periodic lists: the tree's root cube (given as the box) is the
        periodic cell; eval_forces adds the far replicas."""
        self.ctx.check(load().build_interaction_lists_periodic(self.ctx.h, self.h, float(theta),
                                                               int(direct_max)))

    def build_interaction_lists_periodic_err(self, mass, err_tol, p_max, direct_max=0):
        """Periodic lists with the error-bound test (per-entry orders)."""
        mass = _as_vec(mass, self.n)
        self.ctx.check(load().build_interaction_lists_periodic_err(
            self.ctx.h, self.h, _dev(mass), float(err_tol), int(p_max), int(direct_max)))

    def build_interaction_lists_periodic_bs(self, theta, direct_max=0, width=3):
        """Periodic lists with background subtraction: outside each group's
        neighbourhood (`width` group sides) the sources are matter minus the
        mean density; eval_forces adds the exact uniform-box fields."""
        self.ctx.check(load().build_interaction_lists_periodic_bs(
            self.ctx.h, self.h, float(theta), int(direct_max), int(width)))

    def background(self):
        """(box_off (G+1), boxes (B, 6) lo|hi, sign (B,), m2p_sub (M2P entries,))."""
        c = self.counts()
        off = np.empty(c["n_groups"] + 1, np.int64)
        nb = max(c["n_boxes"], 0)
        boxes = np.empty((nb, 6))
        sign = np.empty(nb, np.int8)
        sub = np.empty(max(c["n_m2p"], 0), np.int8)
        self.ctx.check(load().tree_get_background(self.ctx.h, self.h, _np(off), _np(boxes),
                                                  _np(sign), _np(sub)))
        return off, boxes, sign, sub

    def list_images(self):
        c = self.counts()
        pi = np.empty(max(c["n_p2p"], 0), np.int8)
        mi = np.empty(max(c["n_m2p"], 0), np.int8)
        self.ctx.check(load().tree_get_list_images(self.ctx.h, self.h, _np(pi), _np(mi)))
        return pi, mi

    def m2p_orders(self):
        out = np.empty(max(self.counts()["n_m2p"], 0), np.int8)
        self.ctx.check(load().tree_get_m2p_orders(self.ctx.h, self.h, _np(out)))
        return out

    def eval_forces(self, pos, mass, eps, precision=HOT_MIXED, with_pot=False, stats=False,
                    out=None, kernel="plummer"):
        """kernel: "plummer" or "k1" (Dehnen's K1 with compact support eps)."""
        precision = int(precision) | KERNELS[kernel]
        pos = _as_pos(pos)
        mass = _as_vec(mass, self.n)
        acc = out if out is not None else torch.empty_like(pos)
        pot = torch.empty(self.n, dtype=torch.float64, device=pos.device) if with_pot else None
        st = Stats() if stats else None
        self.ctx.check(load().eval_forces(self.ctx.h, self.h, _dev(pos), _dev(mass), float(eps),
                                          int(precision), _dev(acc), _dev(pot),
                                          ctypes.byref(st) if st is not None else None))
        return acc, pot, st

    def eval_forces_noalloc(self, pos, mass, eps, acc, pot=None, precision=HOT_MIXED,
                            stats=False, kernel="plummer"):
        """eval_forces into caller-allocated outputs without any device
        allocation by the library (its fixed scratch array; at most 2^20
        particles, mixed precision, no background subtraction)."""
        precision = int(precision) | KERNELS[kernel]
        pos = _as_pos(pos)
        mass = _as_vec(mass, self.n)
        if acc.dtype != torch.float64 or acc.shape != (self.n, 3) or not acc.is_contiguous():
            raise ValueError("acc must be a contiguous float64 tensor of shape [N, 3]")
        if pot is not None and (pot.dtype != torch.float64 or pot.shape != (self.n,)):
            raise ValueError("pot must be a float64 tensor of shape [N]")
        st = Stats() if stats else None
        self.ctx.check(load().eval_forces_noalloc(self.ctx.h, self.h, _dev(pos), _dev(mass),
                                                  float(eps), int(precision), _dev(acc),
                                                  _dev(pot),
                                                  ctypes.byref(st) if st is not None else None))
        return st

    def eval_forces_adjoint(self, pos, mass, eps, acc_bar, precision=HOT_MIXED, with_mass=False,
                            kernel="plummer"):
        precision = int(precision) | KERNELS[kernel]
        pos = _as_pos(pos)
        mass = _as_vec(mass, self.n)
        acc_bar = _as_pos(acc_bar)
        xbar = torch.empty_like(pos)
        mbar = torch.empty(self.n, dtype=torch.float64, device=pos.device) if with_mass else None
        self.ctx.check(load().eval_forces_adjoint(self.ctx.h, self.h, _dev(pos), _dev(mass),
                                                  float(eps), int(precision), _dev(acc_bar),
                                                  _dev(xbar), _dev(mbar)))
        return xbar, mbar

    # ---- host copies
    def counts(self):
        out = np.zeros(16, np.int64)
        self.ctx.check(load().tree_get_counts(self.ctx.h, self.h, _np(out)))
        keys = ["n", "n_cells", "n_groups", "n_leaves", "max_level", "n_p2p", "n_m2p", "p",
                "n_items", "hash_slots", "p2p_pairs", "m2p_pairs", "n_boxes", "n_leaf_list"]
        return {k: int(out[i]) for i, k in enumerate(keys)}

    def root(self):
        out = np.empty(4)
        self.ctx.check(load().tree_get_root(self.ctx.h, self.h, _np(out)))
        return out

    def keys(self):
        k = np.empty(self.n, np.uint64)
        p = np.empty(self.n, np.uint32)
        self.ctx.check(load().tree_get_keys(self.ctx.h, self.h, _np(k), _np(p)))
        return k, p

    def cells(self):
        C = self.counts()["n_cells"]
        out = dict(level=np.empty(C, np.int32), key=np.empty(C, np.uint64),
                   first=np.empty(C, np.int32), count=np.empty(C, np.int32),
                   parent=np.empty(C, np.int32), child_first=np.empty(C, np.int32),
                   n_child=np.empty(C, np.int32), is_leaf=np.empty(C, np.int32),
                   centre=np.empty((C, 3)), bmax=np.empty(C))
        self.ctx.check(load().tree_get_cells(
            self.ctx.h, self.h, _np(out["level"]), _np(out["key"]), _np(out["first"]),
            _np(out["count"]), _np(out["parent"]), _np(out["child_first"]),
            _np(out["n_child"]), _np(out["is_leaf"]), _np(out["centre"]), _np(out["bmax"])))
        return out

    def groups(self):
        G = self.counts()["n_groups"]
        g = np.empty(G, np.int32)
        self.ctx.check(load().tree_get_groups(self.ctx.h, self.h, _np(g)))
        return g

    def lists(self):
        c = self.counts()
        G = c["n_groups"]
        po, mo = np.empty(G + 1, np.int64), np.empty(G + 1, np.int64)
        pl, ml = np.empty(max(c["n_p2p"], 0), np.int32), np.empty(max(c["n_m2p"], 0), np.int32)
        self.ctx.check(load().tree_get_lists(self.ctx.h, self.h, _np(po), _np(pl), _np(mo),
                                             _np(ml)))
        return po, pl, mo, ml

    def moments(self):
        c = self.counts()
        p = c["p"]
        out = np.empty((c["n_cells"], (p + 1) * (p + 2) * (p + 3) // 6))
        self.ctx.check(load().tree_get_moments(self.ctx.h, self.h, _np(out)))
        return out

    def lookup(self, keys):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.empty(keys.shape[0], np.int32)
        self.ctx.check(load().tree_lookup(self.ctx.h, self.h, keys.shape[0], _np(keys), _np(out)))
        return out


def forces(pos: torch.Tensor, mass: torch.Tensor, eps: float, theta: float, p: int,
           precision: str = "mixed", n_leaf: int = 16, n_group: int = 64, direct_max: int = 0,
           box=None, with_pot: bool = False, periodic: bool = False):
    """One force evaluation: tree_build, compute_moments, build_interaction_lists
    (the periodic ones, with the given box as the periodic cell, if periodic),
    eval_forces. Returns (acc, pot or None, tree)."""
    t = Tree(pos, n_leaf, n_group, box)
    t.compute_moments(pos, mass, p)
    if periodic:
        t.build_interaction_lists_periodic(theta, direct_max)
    else:
        t.build_interaction_lists(theta, direct_max)
    prec = HOT_FP64 if precision == "fp64" else HOT_MIXED
    acc, pot, _ = t.eval_forces(pos, mass, eps, prec, with_pot)
    return acc, pot, t


class TreeForce(torch.autograd.Function):
    """acc = F(pos) for a fixed tree (topology held fixed); backward = the
    library's adjoint. Moments are recomputed from the given positions."""

    @staticmethod
    def forward(ctx, pos, mass, tree: Tree, eps: float, p: int, precision: int):
        tree.compute_moments(pos, mass, p)
        acc, _, _ = tree.eval_forces(pos, mass, eps, precision)
        ctx.save_for_backward(pos, mass)
        ctx.tree, ctx.eps, ctx.p, ctx.precision = tree, eps, p, precision
        return acc

    @staticmethod
    def backward(ctx, acc_bar):
        pos, mass = ctx.saved_tensors
        tree = ctx.tree
        tree.compute_moments(pos, mass, ctx.p)
        want_m = ctx.needs_input_grad[1]
        xbar, mbar = tree.eval_forces_adjoint(pos, mass, ctx.eps, acc_bar.contiguous(),
                                              ctx.precision, with_mass=want_m)
        return xbar, mbar, None, None, None, None
