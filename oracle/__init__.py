"""Python access to the CPU oracle (``liboracle.so``, built from oracle.cpp).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg are the only callers. The GPU library never
imports, links or runs anything from here, and this module never touches the
GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
FLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
         "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (IEEE FP64, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["g++", *FLAGS, _SRC, "-o", tmp], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.oracle_last_error.restype = ctypes.c_char_p
        L.oracle_tree_destroy.restype = None
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _chk(rc):
    if rc != 0:
        raise RuntimeError("oracle: " + lib().oracle_last_error().decode())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int64)


# softening kernels: Plummer, and Dehnen's compensating K1 with compact support
KERNELS = {"plummer": 0, "k1": 1}


def _kern(kernel) -> int:
    return KERNELS[kernel] if isinstance(kernel, str) else int(kernel)


def nm(p: int) -> int:
    return (p + 1) * (p + 2) * (p + 3) // 6


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(n: int) -> None:
    lib().oracle_set_num_threads(int(n))


def morton_keys(pos, box=None):
    pos = _f64(pos)
    n = pos.shape[0]
    keys = np.empty(n, np.uint64)
    ls = np.empty(4)
    b = None if box is None else _f64(box)
    _chk(lib().oracle_morton_keys(ctypes.c_int64(n), _p(pos), _p(b), _p(ls), _p(keys)))
    return keys, ls


class Tree:
    """O-T: the FP64 scalar treecode, step by step."""

    def __init__(self, pos, n_leaf=16, n_group=64, box=None):
        self._pos = _f64(pos)
        self.n = self._pos.shape[0]
        h = ctypes.c_void_p()
        b = None if box is None else _f64(box)
        _chk(lib().oracle_tree_build(ctypes.c_int64(self.n), _p(self._pos), n_leaf, n_group,
                                     _p(b), ctypes.byref(h)))
        self.h = h
        self.p = None

    def __del__(self):
        if getattr(self, "h", None):
            lib().oracle_tree_destroy(self.h)
            self.h = None

    def counts(self):
        out = np.zeros(8, np.int64)
        _chk(lib().oracle_tree_counts(self.h, _p(out)))
        return dict(n=int(out[0]), n_cells=int(out[1]), n_groups=int(out[2]),
                    n_leaves=int(out[3]), max_level=int(out[4]), n_p2p=int(out[5]),
                    n_m2p=int(out[6]))

    def root(self):
        out = np.empty(4)
        _chk(lib().oracle_tree_root(self.h, _p(out)))
        return out

    def keys(self):
        k = np.empty(self.n, np.uint64)
        perm = np.empty(self.n, np.int64)
        _chk(lib().oracle_tree_get_keys(self.h, _p(k), _p(perm)))
        return k, perm

    def cells(self):
        C = self.counts()["n_cells"]
        out = dict(level=np.empty(C, np.int32), key=np.empty(C, np.uint64),
                   first=np.empty(C, np.int64), count=np.empty(C, np.int64),
                   parent=np.empty(C, np.int64), child_first=np.empty(C, np.int64),
                   n_child=np.empty(C, np.int32), is_leaf=np.empty(C, np.int32),
                   centre=np.empty((C, 3)), bmax=np.empty(C))
        _chk(lib().oracle_tree_get_cells(
            self.h, _p(out["level"]), _p(out["key"]), _p(out["first"]), _p(out["count"]),
            _p(out["parent"]), _p(out["child_first"]), _p(out["n_child"]), _p(out["is_leaf"]),
            _p(out["centre"]), _p(out["bmax"])))
        return out

    def groups(self):
        G = self.counts()["n_groups"]
        g = np.empty(G, np.int64)
        _chk(lib().oracle_tree_get_groups(self.h, _p(g)))
        return g

    def build_lists(self, theta, direct_max=0, groups=None):
        sel = _i64(groups)
        ns = 0 if sel is None else sel.shape[0]
        _chk(lib().oracle_build_lists(self.h, ctypes.c_double(theta), int(direct_max),
                                      ctypes.c_int64(ns), _p(sel)))

    def build_lists_err(self, mass, tol, p_max, direct_max=0, groups=None):
        """Error-bound lists: every M2P entry carries the lowest order whose
        field-error bound is at most tol (see accept_order in oracle.cpp)."""
        sel = _i64(groups)
        ns = 0 if sel is None else sel.shape[0]
        _chk(lib().oracle_build_lists_err(self.h, _p(_f64(mass)), ctypes.c_double(tol),
                                          int(p_max), int(direct_max), ctypes.c_int64(ns),
                                          _p(sel)))

    def build_lists_periodic(self, theta, direct_max=0, groups=None):
        """Lists over the 125 images of the source tree (the root cube is the
        periodic cell); evaluation then adds the far replicas."""
        sel = _i64(groups)
        ns = 0 if sel is None else sel.shape[0]
        _chk(lib().oracle_build_lists_periodic(self.h, ctypes.c_double(theta), int(direct_max),
                                               ctypes.c_int64(ns), _p(sel)))

    def build_lists_periodic_err(self, mass, tol, p_max, direct_max=0, groups=None):
        """Periodic lists (as build_lists_periodic) with the error-bound test
        of build_lists_err: every M2P entry carries its order."""
        sel = _i64(groups)
        ns = 0 if sel is None else sel.shape[0]
        _chk(lib().oracle_build_lists_periodic_err(self.h, _p(_f64(mass)), ctypes.c_double(tol),
                                                   int(p_max), int(direct_max),
                                                   ctypes.c_int64(ns), _p(sel)))

    def build_lists_periodic_bs(self, theta, direct_max=0, width=3, groups=None):
        """Periodic lists with background subtraction: outside each group's
        neighbourhood (the cube of `width` times its side) the sources are
        matter minus the uniform mean density; evaluation adds the exact
        fields of the listed boxes, takes off the neighbourhood's and adds
        back the near zone's."""
        sel = _i64(groups)
        ns = 0 if sel is None else sel.shape[0]
        _chk(lib().oracle_build_lists_periodic_bs(self.h, ctypes.c_double(theta), int(direct_max),
                                                  int(width), ctypes.c_int64(ns), _p(sel)))

    def background(self):
        """(box_off (G+1), boxes (B, 6) lo|hi, sign (B,), m2p_sub (M2P entries,))."""
        c = self.counts()
        off = np.empty(c["n_groups"] + 1, np.int64)
        _chk(lib().oracle_get_background(self.h, _p(off), None, None, None))
        nb = int(off[-1])
        boxes = np.empty((nb, 6))
        sign = np.empty(nb, np.int8)
        sub = np.empty(c["n_m2p"], np.int8)
        _chk(lib().oracle_get_background(self.h, _p(off), _p(boxes), _p(sign), _p(sub)))
        return off, boxes, sign, sub

    def list_images(self):
        c = self.counts()
        pi = np.empty(c["n_p2p"], np.int8)
        mi = np.empty(c["n_m2p"], np.int8)
        _chk(lib().oracle_get_list_images(self.h, _p(pi), _p(mi)))
        return pi, mi

    def m2p_orders(self):
        out = np.empty(self.counts()["n_m2p"], np.int8)
        _chk(lib().oracle_get_m2p_orders(self.h, _p(out)))
        return out

    def group_of(self):
        out = np.empty(self.n, np.int64)
        _chk(lib().oracle_group_of(self.h, _p(out)))
        return out

    def lists(self):
        c = self.counts()
        G = c["n_groups"]
        po = np.empty(G + 1, np.int64)
        mo = np.empty(G + 1, np.int64)
        pl = np.empty(c["n_p2p"], np.int32)
        ml = np.empty(c["n_m2p"], np.int32)
        _chk(lib().oracle_get_lists(self.h, _p(po), _p(pl), _p(mo), _p(ml)))
        return po, pl, mo, ml

    def compute_moments(self, pos, mass, p, cells=None):
        pos = _f64(pos)
        mass = _f64(mass)
        sel = _i64(cells)
        ns = 0 if sel is None else sel.shape[0]
        _chk(lib().oracle_compute_moments(self.h, _p(pos), _p(mass), int(p),
                                          ctypes.c_int64(ns), _p(sel)))
        self.p = p

    def moments(self):
        C = self.counts()["n_cells"]
        out = np.empty((C, nm(self.p)))
        _chk(lib().oracle_get_moments(self.h, _p(out)))
        return out

    def eval(self, pos, mass, eps, sinks=None, with_pot=True, kernel="plummer"):
        pos = _f64(pos)
        mass = _f64(mass)
        s = _i64(sinks)
        T = self.n if s is None else s.shape[0]
        acc = np.empty((T, 3))
        pot = np.empty(T) if with_pot else None
        counts = np.zeros(2, np.int64)
        _chk(lib().oracle_eval_tree(self.h, _p(pos), _p(mass), _kern(kernel), ctypes.c_double(eps),
                                    ctypes.c_int64(0 if s is None else T), _p(s), _p(acc),
                                    _p(pot), _p(counts), None, None))
        return acc, pot, counts

    def eval_abs(self, pos, mass, eps, sinks=None, kernel="plummer", cond=False):
        """(acc, absum) or, with cond, (acc, absum, condsum): accelerations as
        eval; per sink the sum of the magnitudes of the terms that add up to
        it (pairs, expansion entries, background boxes, far replicas), so
        absum / |acc| measures cancellation; condsum weights each term by its
        condition with respect to rounding the relative coordinates from
        offsets about the sinks' group centres (see oracle_eval_tree)."""
        pos = _f64(pos)
        mass = _f64(mass)
        s = _i64(sinks)
        T = self.n if s is None else s.shape[0]
        acc = np.empty((T, 3))
        absum = np.empty(T)
        cs = np.empty(T) if cond else None
        _chk(lib().oracle_eval_tree(self.h, _p(pos), _p(mass), _kern(kernel), ctypes.c_double(eps),
                                    ctypes.c_int64(0 if s is None else T), _p(s), _p(acc),
                                    None, None, _p(absum), _p(cs)))
        return (acc, absum, cs) if cond else (acc, absum)

    def vjp(self, pos, mass, eps, abar, kernel="plummer"):
        pos = _f64(pos)
        mass = _f64(mass)
        abar = _f64(abar)
        xbar = np.empty_like(pos)
        mbar = np.empty(self.n)
        _chk(lib().oracle_tree_vjp(self.h, _p(pos), _p(mass), _kern(kernel), ctypes.c_double(eps), _p(abar),
                                   _p(xbar), _p(mbar)))
        return xbar, mbar


def direct(pos, mass, eps, sinks=None, kernel="plummer"):
    """O-D: exact softened direct sum (compensated), sinks = caller indices."""
    pos = _f64(pos)
    mass = _f64(mass)
    s = _i64(sinks)
    n = pos.shape[0]
    T = n if s is None else s.shape[0]
    acc = np.empty((T, 3))
    pot = np.empty(T)
    _chk(lib().oracle_direct(ctypes.c_int64(n), _p(pos), _p(mass), _kern(kernel), ctypes.c_double(eps),
                             ctypes.c_int64(0 if s is None else T), _p(s), _p(acc), _p(pot)))
    return acc, pot


def direct_vjp(pos, mass, eps, abar, rows=None, kernel="plummer"):
    pos = _f64(pos)
    mass = _f64(mass)
    abar = _f64(abar)
    r = _i64(rows)
    n = pos.shape[0]
    T = n if r is None else r.shape[0]
    xbar = np.empty((T, 3))
    mbar = np.empty(T)
    _chk(lib().oracle_direct_vjp(ctypes.c_int64(n), _p(pos), _p(mass), _kern(kernel), ctypes.c_double(eps),
                                 _p(abar), ctypes.c_int64(0 if r is None else T), _p(r),
                                 _p(xbar), _p(mbar)))
    return xbar, mbar


def box_field(lo, hi, x):
    """Field at points x (n, 3) of unit density filling the box [lo, hi]."""
    lo = _f64(np.asarray(lo, dtype=np.float64))
    hi = _f64(np.asarray(hi, dtype=np.float64))
    x = _f64(np.atleast_2d(x))
    out = np.empty_like(x)
    _chk(lib().oracle_box_field(_p(lo), _p(hi), ctypes.c_int64(x.shape[0]), _p(x), _p(out)))
    return out


def box_grad(lo, hi, x):
    """Gradient (n, 3, 3), [k, l] = d a_k / d x_l, of the unit-density box field."""
    lo = _f64(np.asarray(lo, dtype=np.float64))
    hi = _f64(np.asarray(hi, dtype=np.float64))
    x = _f64(np.atleast_2d(x))
    out = np.empty((x.shape[0], 3, 3))
    _chk(lib().oracle_box_grad(_p(lo), _p(hi), ctypes.c_int64(x.shape[0]), _p(x), _p(out)))
    return out


def cube_moments(p, s):
    """Raw moments (slot order) of unit density filling a cube of side s."""
    out = np.empty((p + 1) * (p + 2) * (p + 3) // 6)
    _chk(lib().oracle_cube_moments(int(p), ctypes.c_double(s), _p(out)))
    return out


def lattice_tensor(L, K, split=2.0):
    """d^gamma F(0) of the far periodic replicas, |gamma| <= K, slot order."""
    out = np.empty((K + 1) * (K + 2) * (K + 3) // 6)
    _chk(lib().oracle_lattice_tensor(ctypes.c_double(L), int(K), ctypes.c_double(split), _p(out)))
    return out


def ewald_self(L, split=2.0):
    f = lib().oracle_ewald_self
    f.restype = ctypes.c_double
    return f(ctypes.c_double(L), ctypes.c_double(split))


def ewald_direct(pos, mass, L, eps, sinks=None, with_pot=False):
    """Periodic accelerations (and potentials) by definition (near replicas
    softened, far by Ewald sums) for the selected sinks."""
    pos = _f64(pos)
    mass = _f64(mass)
    n = pos.shape[0]
    sel = _i64(sinks)
    ns = n if sel is None else sel.shape[0]
    acc = np.empty((ns, 3))
    pot = np.empty(ns) if with_pot else None
    _chk(lib().oracle_ewald_direct(ctypes.c_int64(n), _p(pos), _p(mass), ctypes.c_double(L),
                                   ctypes.c_double(eps), ctypes.c_int64(0 if sel is None else ns),
                                   _p(sel), _p(acc), _p(pot)))
    return (acc, pot) if with_pot else acc


def m2p(p, M, R, eps, kernel="plummer"):
    M = _f64(M)
    R = _f64(R)
    out = np.empty(4)
    _chk(lib().oracle_m2p(int(p), _p(M), _p(R), _kern(kernel), ctypes.c_double(eps), _p(out)))
    return out[:3], out[3]


def p2m(p, pos, mass, centre):
    pos = _f64(pos)
    mass = _f64(mass)
    c = _f64(centre)
    out = np.empty(nm(p))
    _chk(lib().oracle_p2m(int(p), ctypes.c_int64(pos.shape[0]), _p(pos), _p(mass), _p(c),
                          _p(out)))
    return out


def m2m(p, M, shift):
    M = _f64(M)
    s = _f64(shift)
    out = np.empty(nm(p))
    _chk(lib().oracle_m2m(int(p), _p(M), _p(s), _p(out)))
    return out


def derivs(order, R, eps, kernel="plummer"):
    R = _f64(R)
    out = np.empty(nm(order))
    _chk(lib().oracle_derivs(int(order), _p(R), _kern(kernel), ctypes.c_double(eps), _p(out)))
    return out


def multi_indices(p):
    """(a, b, c) for every storage slot up to order p (order, then a desc, then b desc)."""
    out = []
    for n in range(p + 1):
        for a in range(n, -1, -1):
            for b in range(n - a, -1, -1):
                out.append((a, b, n - a - b))
    return out
