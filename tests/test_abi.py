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
    assert lib.dpf_solve_batch(None, 1, None, None, 1, 1, *([None] * 17), ctypes.c_size_t(0), None) == -1
    assert lib.dpf_solve_series(None, 1, 1, *([None] * 3), 1, *([None] * 4), 1, *([None] * 8),
                                ctypes.c_size_t(0), None) == -1
    assert lib.dpf_param_grad(None, 1, 1, *([None] * 3), 0, *([None] * 8), 1, None, None,
                              ctypes.c_size_t(0), None) == -1
    assert lib.dpf_dc_init(None, 1, 1, None, None, 0, None, None, ctypes.c_double(1e-12), 10, None, None,
                           None, ctypes.c_size_t(0), None) == -1
    # workspace sizing is pure host arithmetic
    g = _Grid(9241, 41339, 10, 1, 1, 1, 0, None, None, None, None, None)
    lib.dpf_dc_init_workspace_bytes.restype = ctypes.c_size_t
    assert lib.dpf_dc_init_workspace_bytes(9241, 4) >= 3 * 9241 * 4 * 8
    assert lib.dpf_dc_init_workspace_bytes(0, 4) == 0
    # invalid argument checks that need no device: a grid is passed, sizes are wrong
    gp = ctypes.byref(g)
    assert lib.dpf_param_grad(gp, 0, 9241, *([None] * 3), 0, *([None] * 8), 1, None, None,
                              ctypes.c_size_t(0), None) == -1  # B = 0
    assert lib.dpf_dc_init(gp, 1, 100, None, None, 0, None, None, ctypes.c_double(1e-12), 10, None, None,
                           None, ctypes.c_size_t(0), None) == -1  # ld < n_bus
    _ws_types(lib)
    small = lib.dpf_solve_workspace_bytes(ctypes.byref(g), 1, None, 1024, 9241, None)
    big = lib.dpf_solve_workspace_bytes(ctypes.byref(g), 1, None, 2048, 9241, None)
    # streaming state: 4 moments + 3 complex scratch per bus-case, plus the sliced matrix
    assert big - small >= 1024 * 9241 * (4 * 8 + 3 * 16) - 1024  # (256-byte alignment of each array)
    # a single item of this size is spread over many workgroups: its layout holds the same state
    assert lib.dpf_solve_workspace_bytes(ctypes.byref(g), 1, None, 1, 9241, None) >= 9241 * (4 * 8 + 3 * 16)
    assert lib.dpf_solve_workspace_bytes(None, 1, None, 1, 1, None) == 0


def test_variant_table_and_autotune_cache(lib):
    n = lib.dpf_solve_variant_count()
    assert n >= 2
    t, k, st = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    seen_stream = False
    for i in range(n):
        assert lib.dpf_solve_variant_info(i, ctypes.byref(t), ctypes.byref(k), ctypes.byref(st)) == 0
        assert t.value % 64 == 0 and t.value <= 1024  # 0 for the multi-workgroup entry
        seen_stream |= st.value == 1
        assert st.value in range(5)  # register, streaming, banded-stream, wide, paired
        assert lib.dpf_solve_variant_cases(i) >= 1
    assert seen_stream
    assert lib.dpf_solve_variant_info(n, ctypes.byref(t), ctypes.byref(k), ctypes.byref(st)) == -1
    # the register-resident 64-thread variant cannot hold 9241 buses
    assert lib.dpf_autotune_set(9241, 0) == -1
    d = lib.dpf_solve_variant_for(9241)
    assert d >= 0
    assert lib.dpf_autotune_set(9241, d) == 0
    lib.dpf_autotune_reset()
    assert lib.dpf_solve_variant_for(14) == 0
    # cases per workgroup: 1 for every variant
    kinds = []
    for i in range(n):
        lib.dpf_solve_variant_info(i, ctypes.byref(t), ctypes.byref(k), ctypes.byref(st))
        kinds.append((st.value, k.value, lib.dpf_solve_variant_cases(i)))
    assert all(c == 1 for _, _, c in kinds)
    assert lib.dpf_solve_variant_cases(n) == -1 and lib.dpf_solve_variant_cases(-1) == -1


class _Route(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("team_cap", ctypes.c_int32), ("tail_handoff", ctypes.c_int32),
                ("tail_team", ctypes.c_int32), ("tail_chunk", ctypes.c_int32), ("tail_min_items", ctypes.c_int32),
                ("tail_slice_ms", ctypes.c_double), ("tail_first_wait_s", ctypes.c_double),
                ("tail_wait_s", ctypes.c_double), ("case_order", ctypes.c_int32), ("wide_host", ctypes.c_int32),
                ("tail_device", ctypes.c_int32)]


def _ws_types(lib):
    lib.dpf_solve_workspace_bytes.restype = ctypes.c_size_t
    lib.dpf_solve_workspace_bytes.argtypes = [ctypes.POINTER(_Grid), ctypes.c_int32, ctypes.c_void_p,
                                              ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_Route)]
    lib.dpf_route_default.argtypes = [ctypes.POINTER(_Route)]
    lib.dpf_route_default.restype = None


def _default_route(lib):
    r = _Route()
    lib.dpf_route_default(ctypes.byref(r))
    return r


def test_route_defaults_and_field_checks(lib):
    """dpf_route_default fills the documented defaults, and a route with any field
    out of range sizes no workspace (the solve call returns DPF_EINVAL for it)."""
    _ws_types(lib)
    r = _default_route(lib)
    assert (r.variant, r.team_cap, r.tail_handoff, r.tail_team, r.tail_chunk, r.tail_min_items) == (-1, 0, 0, 0,
                                                                                                    128, 0)
    assert (r.tail_slice_ms, r.tail_first_wait_s, r.tail_wait_s, r.case_order, r.wide_host) == (0.0, 1.0, 5.0, 0, 0)
    assert r.tail_device == 0
    g = _Grid(9241, 41339, 10, 1, 1, 1, 0, None, None, None, None, None)
    ok = lib.dpf_solve_workspace_bytes(ctypes.byref(g), 1, None, 1024, 9241, ctypes.byref(r))
    assert ok == lib.dpf_solve_workspace_bytes(ctypes.byref(g), 1, None, 1024, 9241, None) > 0
    bad = [("variant", -2), ("variant", 10 ** 6), ("team_cap", -1), ("tail_handoff", -1), ("tail_team", -1),
           ("tail_team", 1025), ("tail_chunk", 0), ("tail_chunk", 65537), ("tail_min_items", -1),
           ("tail_slice_ms", -1.0), ("tail_slice_ms", 1001.0), ("tail_slice_ms", float("nan")),
           ("tail_first_wait_s", -1.0), ("tail_wait_s", 61.0), ("tail_first_wait_s", float("nan")),
           ("case_order", 2), ("case_order", -1), ("wide_host", 2), ("wide_host", -1),
           ("tail_device", 2), ("tail_device", -1), ("tail_device", 1)]  # 1 needs tail_team > 0
    for name, val in bad:
        rb = _default_route(lib)
        setattr(rb, name, val)
        assert lib.dpf_solve_workspace_bytes(ctypes.byref(g), 1, None, 1024, 9241, ctypes.byref(rb)) == 0, name
    # a variant that cannot hold the grid (the 64-thread register-resident one)
    rb = _default_route(lib)
    rb.variant = 0
    assert lib.dpf_solve_workspace_bytes(ctypes.byref(g), 1, None, 1024, 9241, ctypes.byref(rb)) == 0


def test_route_tail_handoff_sizes_its_own_call_only(lib):
    """A route with a tail handoff needs the larger workspace of its call (the
    paused item list, a schedule buffer and the multi-workgroup arrays); another
    call's route, the autotune cache reset and sub-grid calls are unaffected: no
    setting outlives the call that passes it."""
    _ws_types(lib)
    g = _Grid(9241, 41339, 10, 1, 1, 1, 0, None, None, None, None, None)
    lib.dpf_autotune_reset()
    band = [i for i in range(lib.dpf_solve_variant_count()) if _kind(lib, i) == 2][0]
    plain_r = _default_route(lib)
    plain_r.variant = band
    plain = lib.dpf_solve_workspace_bytes(ctypes.byref(g), 1, None, 1024, 9241, ctypes.byref(plain_r))
    hand_r = _default_route(lib)
    hand_r.variant = band
    hand_r.tail_handoff = 192
    handed = lib.dpf_solve_workspace_bytes(ctypes.byref(g), 1, None, 1024, 9241, ctypes.byref(hand_r))
    slices = (9241 + 63) // 64
    assert handed - plain >= 1024 * (4 + 6 * 8 + slices * 16)
    # the plain route still sizes the plain call after the handoff route was used
    assert lib.dpf_solve_workspace_bytes(ctypes.byref(g), 1, None, 1024, 9241, ctypes.byref(plain_r)) == plain
    # the split-kernel team size does not change the workspace
    team_r = _default_route(lib)
    team_r.variant, team_r.tail_handoff, team_r.tail_team, team_r.tail_slice_ms = band, 192, 32, 10.0
    assert lib.dpf_solve_workspace_bytes(ctypes.byref(g), 1, None, 1024, 9241, ctypes.byref(team_r)) == handed
    # sub-grids never hand over: same size with and without it
    sub = (ctypes.c_int32 * 3)(0, 5000, 9241)
    hand_r.variant = -1
    plain_r.variant = -1
    assert (lib.dpf_solve_workspace_bytes(ctypes.byref(g), 2, sub, 1024, 9241, ctypes.byref(hand_r)) ==
            lib.dpf_solve_workspace_bytes(ctypes.byref(g), 2, sub, 1024, 9241, ctypes.byref(plain_r)))


def test_bad_outage_status_is_declared():
    """An outage index that is neither -1 nor a branch index is reported per case
    (DPF_BAD_OUTAGE, status 4), and the binding exposes the same code."""
    text = open(HEADER).read()
    assert re.search(r"#define DPF_BAD_OUTAGE 4\b", text)
    from paper_2603_28203_amd import binding
    assert binding.BAD_OUTAGE == 4


def test_unfinished_status_is_declared():
    """An item of the persistent teams whose team did not assemble in time is
    reported per item (DPF_UNFINISHED, status 5), and the binding exposes it."""
    text = open(HEADER).read()
    assert re.search(r"#define DPF_UNFINISHED 5\b", text)
    from paper_2603_28203_amd import binding
    assert binding.UNFINISHED == 5


def test_wide_host_sizes_its_own_path(lib):
    """A call with a sub-grid above one workgroup's LDS sizes the persistent
    teams' arrays by default (plan tables, one barrier counter per item, member
    partials) and the multi-workgroup path's with wide_host = 1; calls whose
    sub-grids all fit are sized the same either way."""
    _ws_types(lib)
    n_big = 30000
    g = _Grid(n_big + 28, 140000, 10, 1, 1, 1, 0, None, None, None, None, None)
    sub = (ctypes.c_int32 * 4)(0, 14, n_big + 14, n_big + 28)
    teams_r = _default_route(lib)
    host_r = _default_route(lib)
    host_r.wide_host = 1
    B = 2
    wt = lib.dpf_solve_workspace_bytes(ctypes.byref(g), 3, sub, B, g.n_bus, ctypes.byref(teams_r))
    wh = lib.dpf_solve_workspace_bytes(ctypes.byref(g), 3, sub, B, g.n_bus, ctypes.byref(host_r))
    assert wt > 0 and wh > 0 and wt != wh
    items = B * 3
    # at least: moments and three complex scratch vectors per bus and case, units,
    # first tickets, barrier counters and one partial per member
    slices = 1 + (n_big + 63) // 64 + 1
    assert wt >= B * g.n_bus * (4 * 8 + 3 * 16) + items * (4 + 4 + 256) + B * (1 + min(slices - 2, 32) + 1) * 16
    small = _Grid(9241, 41339, 10, 1, 1, 1, 0, None, None, None, None, None)
    assert (lib.dpf_solve_workspace_bytes(ctypes.byref(small), 1, None, 1024, 9241, ctypes.byref(host_r)) ==
            lib.dpf_solve_workspace_bytes(ctypes.byref(small), 1, None, 1024, 9241, ctypes.byref(teams_r)))


def _kind(lib, i):
    t, k, st = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    lib.dpf_solve_variant_info(i, ctypes.byref(t), ctypes.byref(k), ctypes.byref(st))
    return st.value


# ---------------------------------------------------------------- bus ordering (host code)


def _rcm(lib, n, f, t, sub=None, group=0):
    import numpy as np
    f = np.ascontiguousarray(f, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    perm = np.full(n, -1, dtype=np.int32)
    bw = ctypes.c_int32(-1)
    so = None if sub is None else np.ascontiguousarray(sub, dtype=np.int32)
    rc = lib.dpf_order_rcm(ctypes.c_int32(n), ctypes.c_int32(len(f)), f.ctypes.data_as(ctypes.c_void_p),
                           t.ctypes.data_as(ctypes.c_void_p), ctypes.c_int32(1 if so is None else len(so) - 1),
                           None if so is None else so.ctypes.data_as(ctypes.c_void_p), ctypes.c_int32(group),
                           perm.ctypes.data_as(ctypes.c_void_p), ctypes.byref(bw))
    return rc, perm, bw.value


def test_rcm_order_is_a_small_bandwidth_permutation(lib):
    import numpy as np

    import synth
    g = synth.config1(B=1)["grid"]
    f, t = g.f, g.t
    rc, perm, bw = _rcm(lib, g.n_bus, f, t)
    assert rc == 0
    assert np.array_equal(np.sort(perm), np.arange(g.n_bus))
    inv = np.argsort(perm)
    assert bw == np.abs(inv[f] - inv[t]).max()
    assert bw < 60 < np.abs(f - t).max()  # the generator's numbering is far from banded
    # grouping by degree: each bus moves within its window; degrees sorted per window
    rc, perm2, bw2 = _rcm(lib, g.n_bus, f, t, group=128)
    assert rc == 0 and np.array_equal(np.sort(perm2), np.arange(g.n_bus))
    deg = np.bincount(np.concatenate([f, t]), minlength=g.n_bus)
    for w in range(0, g.n_bus, 128):
        d = deg[perm2[w:w + 128]]
        assert np.all(np.diff(d) >= 0)
    assert bw2 <= bw + 2 * 127


def test_rcm_order_keeps_sub_grid_ranges_and_checks_input(lib):
    import numpy as np
    # two disjoint paths numbered in a scrambled way, as sub-grids [0, 50) and [50, 120)
    rng = np.random.default_rng(0)
    a = rng.permutation(50)
    b = 50 + rng.permutation(70)
    f = np.concatenate([a[:-1], b[:-1]])
    t = np.concatenate([a[1:], b[1:]])
    rc, perm, bw = _rcm(lib, 120, f, t, sub=[0, 50, 120])
    assert rc == 0 and bw == 1
    assert set(perm[:50].tolist()) == set(range(50)) and set(perm[50:].tolist()) == set(range(50, 120))
    # errors: end out of range, bad sub_offset, negative group
    assert _rcm(lib, 120, [0, 130], [1, 2])[0] == -1
    assert _rcm(lib, 120, f, t, sub=[0, 60, 50, 120])[0] == -1
    assert _rcm(lib, 120, f, t, group=-1)[0] == -1


def test_two_over_pi_table_holds_the_binary_expansion():
    """The Payne-Hanek table of the device sin/cos is 2/pi to 1280 bits
    (checked with mpmath, independent of how the table was produced)."""
    mpmath = pytest.importorskip("mpmath")
    src = open(os.path.join(ROOT, "paper_2603_28203_amd", "csrc", "common.hpp")).read()
    body = src[src.index("kTwoOverPiBits[20] = {"):]
    body = body[:body.index("};")]
    words = [int(w, 16) for w in re.findall(r"0x([0-9A-F]{16})ULL", body)]
    assert len(words) == 20
    table = 0
    for w in words:
        table = (table << 64) | w
    mpmath.mp.prec = 1400
    ref = int(mpmath.floor(2 / mpmath.pi * mpmath.mpf(2) ** 1280))
    assert table == ref
