"""The C-ABI library loads without a GPU and exports every function that
include/llr.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "llr.h")
LIB = os.path.join(ROOT, "paper_1509_08391_amd", "libllr.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(llr_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ["llr_create", "llr_add_lattice", "llr_bind_state", "llr_run", "llr_get_a", "llr_reconstruct",
                 "llr_mlp_train", "llr_mlp_predict", "llr_sweeps", "llr_approach"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libllr.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_imports_without_gpu():
    from paper_1509_08391_amd import llr
    assert llr.lib() is not None
    assert set(llr._SIGS) | {"llr_last_error", "llr_destroy"} == set(declared())


def test_null_context_is_rejected_without_a_device():
    """Entry points taking a context fail with an error status, not a fault,
    when handed none; these checks run before any HIP call."""
    from paper_1509_08391_amd import llr
    L = llr.lib()
    n = ctypes.c_longlong()
    assert L.llr_link_stats(None, None, None) < 0
    assert L.llr_stats(None, None, None, ctypes.byref(n), ctypes.byref(n)) < 0
    assert L.llr_sweeps(None, 1, 0, llr.MODE_LINK, None) < 0
    assert L.llr_class_pass(None, 1, 0, llr.MODE_LINK, 0) < 0
    assert b"context" in L.llr_last_error() or b"state" in L.llr_last_error()
