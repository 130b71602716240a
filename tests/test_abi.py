"""The C ABI without a GPU: the library loads, exports every function that
include/dpf.h declares, and its host-side argument checks answer without
touching a device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpf.h")
LIB = os.path.join(ROOT, "paper_2603_28203_amd", "libdpf.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dpf_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2603_28203_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for fn in ("dpf_build_ybus", "dpf_mismatch_grad", "dpf_solve_batch", "dpf_solve_workspace_bytes",
               "dpf_mismatch_grad_workspace_bytes", "dpf_last_error", "dpf_autotune_set"):
        assert fn in names


def test_every_declared_symbol_is_exported(lib):
    for fn in declared_functions():
        assert hasattr(lib, fn), fn


class _Grid(ctypes.Structure):
    _fields_ = [("n_bus", ctypes.c_int32), ("nnz", ctypes.c_int32), ("max_row_nnz", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("n_branch", ctypes.c_int32), ("from_", ctypes.c_void_p), ("to", ctypes.c_void_p),
                ("r", ctypes.c_void_p), ("x", ctypes.c_void_p), ("b", ctypes.c_void_p)]


def test_host_side_validation(lib):
    lib.dpf_last_error.restype = ctypes.c_char_p
    lib.dpf_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.dpf_version()
    # build_ybus rejects sizes before any device work
    lib.dpf_build_ybus.restype = ctypes.c_int
    nnz = ctypes.c_int32(0)
    rc = lib.dpf_build_ybus(0, 0, None, None, None, None, None, 0, None, None, None, ctypes.byref(nnz), None, None)
    assert rc == -1 and b"n_bus" in lib.dpf_last_error()
    # mismatch_grad / solve reject a null grid
    assert lib.dpf_mismatch_grad(None, 1, 1, *([None] * 12), ctypes.c_size_t(0), None) == -1
    assert lib.dpf_solve_batch(None, 1, None, None, 1, 1, *([None] * 15), ctypes.c_size_t(0), None) == -1
    assert lib.dpf_solve_series(None, 1, 1, *([None] * 3), 1, *([None] * 4), 1, *([None] * 7),
                                ctypes.c_size_t(0), None) == -1
    # workspace sizing is pure host arithmetic
    g = _Grid(9241, 41339, 10, 1, 1, 1, 0, None, None, None, None, None)
    lib.dpf_solve_workspace_bytes.restype = ctypes.c_size_t
    lib.dpf_solve_workspace_bytes.argtypes = [ctypes.POINTER(_Grid), ctypes.c_int32, ctypes.c_void_p,
                                              ctypes.c_int32, ctypes.c_int32]
    small = lib.dpf_solve_workspace_bytes(ctypes.byref(g), 1, None, 1, 9241)
    big = lib.dpf_solve_workspace_bytes(ctypes.byref(g), 1, None, 1024, 9241)
    # streaming state: 4 moments + 3 complex scratch per bus-case, plus the sliced matrix
    assert big - small >= 1023 * 9241 * (4 * 8 + 3 * 16) - 1024  # (256-byte alignment of each array)
    assert lib.dpf_solve_workspace_bytes(None, 1, None, 1, 1) == 0


def test_variant_table_and_autotune_cache(lib):
    n = lib.dpf_solve_variant_count()
    assert n >= 2
    t, k, st = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    seen_stream = False
    for i in range(n):
        assert lib.dpf_solve_variant_info(i, ctypes.byref(t), ctypes.byref(k), ctypes.byref(st)) == 0
        assert t.value % 64 == 0 and t.value <= 1024
        seen_stream |= bool(st.value)
    assert seen_stream
    assert lib.dpf_solve_variant_info(n, ctypes.byref(t), ctypes.byref(k), ctypes.byref(st)) == -1
    # the register-resident 64-thread variant cannot hold 9241 buses
    assert lib.dpf_autotune_set(9241, 0) == -1
    d = lib.dpf_solve_variant_for(9241)
    assert d >= 0
    assert lib.dpf_autotune_set(9241, d) == 0
    lib.dpf_autotune_reset()
    assert lib.dpf_solve_variant_for(14) == 0
