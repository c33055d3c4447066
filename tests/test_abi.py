"""The C-ABI library: it loads, exports every call include/hot.h declares,
and rejects bad arguments without a GPU (no compute is launched here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hot.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_path():
    names = declared()
    for n in ("tree_build", "compute_moments", "build_interaction_lists", "eval_forces",
              "eval_forces_adjoint"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1310_4502_amd import binding
    L = binding.load()
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(binding.EXPORTS) == declared()


def test_null_and_bad_arguments_fail_cleanly():
    from paper_1310_4502_amd import binding
    L = binding.load()
    assert L.hot_ctx_create(0, None, None, None) == binding.HOT_E_INVALID
    assert L.hot_last_error(None) == b"null context"
    assert L.hot_sync(None) == binding.HOT_E_INVALID
    assert L.tree_build(None, 10, None, None, None) == binding.HOT_E_INVALID
    assert L.tree_destroy(None, None) == binding.HOT_E_INVALID
    assert L.hot_ctx_destroy(None) == binding.HOT_E_INVALID
    bad = binding._Allocator()
    h = ctypes.c_void_p()
    assert L.hot_ctx_create(0, None, ctypes.byref(bad), ctypes.byref(h)) == binding.HOT_E_INVALID


def test_no_device_is_an_error_not_a_crash():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1310_4502_amd import binding
    L = binding.load()
    h = ctypes.c_void_p()
    rc = L.hot_ctx_create(0, None, None, ctypes.byref(h))
    assert rc in (binding.HOT_E_INVALID, binding.HOT_E_DEVICE)
    assert not h.value
