"""CPU-only checks of the C ABI: the built library loads and exports every
entry point that include/et.h declares; host-side argument checks return
ET_EINVAL without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "et.h")
LIB = os.path.join(ROOT, "paper_2103_15217_amd", "libet.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(et_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("et_tree_build", "et_list_rank", "et_lca", "et_bridges", "et_tree_free",
                 "et_strerror", "et_ctx_create", "et_ctx_status"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libet.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name


def test_host_argument_checks():
    lib = ctypes.CDLL(LIB)
    lib.et_strerror.restype = ctypes.c_char_p
    assert lib.et_strerror(-4) == b"malformed input detected on the device"
    assert lib.et_version() >= 100
    P = ctypes.c_void_p
    # null context / null out pointer are rejected before any HIP call
    lib.et_tree_build.argtypes = [P, P, ctypes.c_int32, P, P]
    assert lib.et_tree_build(None, None, 10, None, None) == -1
    out = P()
    assert lib.et_tree_build(None, None, 10, None, ctypes.byref(out)) == -1
    lib.et_list_rank.argtypes = [P, P, ctypes.c_int32, P, ctypes.c_int32, P, P]
    assert lib.et_list_rank(None, None, 5, None, 1, None, None) == -1
    lib.et_list_scan.argtypes = [P, P, P, ctypes.c_int32, P, ctypes.c_int32, P, P, P]
    assert lib.et_list_scan(None, None, None, 5, None, 1, None, None, None) == -1
    lib.et_lca.argtypes = [P, P, P, ctypes.c_int64, P, P]
    assert lib.et_lca(None, None, None, 5, None, None) == -1
    lib.et_bridges.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_int32, P, P, P]
    assert lib.et_bridges(None, None, None, 5, 5, None, None, None) == -1
    I32, I64 = ctypes.c_int32, ctypes.c_int64
    lib.et_bridges_batch.argtypes = [P, P, P, P, P, I32, I32, I32, P, I64, P, P]
    assert lib.et_bridges_batch(None, None, None, None, None, 1, 4, 8, None, 1, None, None) == -1
    assert lib.et_strerror(-5) == b"input beyond a fixed-size limit of this call"
    # one-launch small-tree batch: a null context is rejected before any HIP call
    lib.et_lca_batch_fused.argtypes = [P, P, P, I32, I64, I32, P, P, P, I64, P, P, P, P, P, P]
    assert lib.et_lca_batch_fused(None, None, None, 1, 1, 1, None, None, None, 0, None, None, None, None,
                                  None, None) == -1
    # one-launch graph batch: a null context is rejected before any HIP call
    lib.et_bridges_batch_fused.argtypes = [P, P, P, P, P, P, I32, I32, I32, I32, I32, P, I64, P, P, P]
    assert lib.et_bridges_batch_fused(None, None, None, None, None, None, 1, 4, 8, 4, 8, None, 1, None,
                                      None, None) == -1
