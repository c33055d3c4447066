"""MI355X-native hashed oct-tree gravitational force evaluation.

The computation runs in hand-written HIP kernels (libhot.so, C ABI in
include/hot.h); this package holds the build step, a thin ctypes binding and
the seeded workload generators. Heavy imports (torch) happen only when the
binding is used.
"""
__all__ = ["binding", "workloads", "build"]


def __getattr__(name):
    if name in ("Tree", "Context", "forces", "TreeForce", "HotError", "load", "context",
                "HOT_MIXED", "HOT_FP64", "Stats"):
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
