"""CPU sanitizer runs: the oracle's pins against an AddressSanitizer +
UndefinedBehaviorSanitizer build of the oracle, and the library's host-only code
(bus ordering, call planning and workspace layout, route checks, argument
checks) from a build of dpf.hip whose host side is sanitized, compared with the
regular library.  No GPU is involved: the functions exercised never touch a
device."""

import ctypes
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(compiler, name):
    path = subprocess.run([compiler, f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not found for {compiler}")
    return path


def _instrumented(lib):
    syms = subprocess.run(["nm", "-D", "--undefined-only", str(lib)], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms, "library is not instrumented"


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fcx-limited-range", "-fopenmp",
                           "-fPIC", "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "dpf_oracle.c"), "-o", str(lib),
                           "-lm"])
    _instrumented(lib)
    env = dict(os.environ)
    env["LD_PRELOAD"] = _runtime("gcc", "libasan.so") + ":" + _runtime("gcc", "libubsan.so")
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["DPF_ORACLE_LIB"] = str(lib)
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle.py"), "-q", "-x",
                        "-p", "no:cacheprovider", "-m", "not gpu"], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]
    assert " passed" in out and "failed" not in out


_HOST_SCRIPT = r'''
import ctypes, json, sys
import numpy as np
sys.path.insert(0, ROOT)
import synth
L = ctypes.CDLL(LIB)
L.dpf_last_error.restype = ctypes.c_char_p

class Grid(ctypes.Structure):
    _fields_ = [("n_bus", ctypes.c_int32), ("nnz", ctypes.c_int32), ("max_row_nnz", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("n_branch", ctypes.c_int32), ("f", ctypes.c_void_p), ("t", ctypes.c_void_p),
                ("r", ctypes.c_void_p), ("x", ctypes.c_void_p), ("b", ctypes.c_void_p)]

class Route(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("team_cap", ctypes.c_int32), ("tail_handoff", ctypes.c_int32),
                ("tail_team", ctypes.c_int32), ("tail_chunk", ctypes.c_int32), ("tail_min_items", ctypes.c_int32),
                ("tail_slice_ms", ctypes.c_double), ("tail_first_wait_s", ctypes.c_double),
                ("tail_wait_s", ctypes.c_double), ("case_order", ctypes.c_int32), ("wide_host", ctypes.c_int32),
                ("tail_device", ctypes.c_int32)]

L.dpf_solve_workspace_bytes.restype = ctypes.c_size_t
L.dpf_solve_workspace_bytes.argtypes = [ctypes.POINTER(Grid), ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.POINTER(Route)]
out = {}

def rcm(n, f, t, sub=None, group=0):
    f = np.ascontiguousarray(f, np.int32); t = np.ascontiguousarray(t, np.int32)
    perm = np.full(n, -1, np.int32); bw = ctypes.c_int32(-1)
    so = None if sub is None else np.ascontiguousarray(sub, np.int32)
    rc = L.dpf_order_rcm(ctypes.c_int32(n), ctypes.c_int32(len(f)), f.ctypes.data_as(ctypes.c_void_p),
                         t.ctypes.data_as(ctypes.c_void_p), ctypes.c_int32(1 if so is None else len(so) - 1),
                         None if so is None else so.ctypes.data_as(ctypes.c_void_p), ctypes.c_int32(group),
                         perm.ctypes.data_as(ctypes.c_void_p), ctypes.byref(bw))
    return [rc, perm.tolist(), bw.value]

g1 = synth.config1(B=1)["grid"]
g2 = synth.config2(B=1)["grid"]
out["rcm1"] = rcm(g1.n_bus, g1.f, g1.t, group=128)
out["rcm2"] = rcm(g2.n_bus, g2.f, g2.t, group=2560)
half = g1.n_bus // 2
keep = (g1.f < half) == (g1.t < half)
out["rcm_sub"] = rcm(g1.n_bus, g1.f[keep], g1.t[keep], sub=[0, half, g1.n_bus], group=64)
out["rcm_bad"] = rcm(10, [0, 12], [1, 2])[0]
g = Grid(9241, 41339, 10, 1, 1, 1, 0, None, None, None, None, None)
ws = []
for variant in (-1, 0, 30):
    for handoff in (0, 192):
        for team_cap in (0, 5000):
            r = Route(); L.dpf_route_default(ctypes.byref(r))
            r.variant, r.tail_handoff, r.team_cap = variant, handoff, team_cap
            for sub in (None, (ctypes.c_int32 * 4)(0, 3000, 7000, 9241)):
                ws.append(L.dpf_solve_workspace_bytes(ctypes.byref(g), 1 if sub is None else 3, sub, 1024, 9241,
                                                      ctypes.byref(r)))
out["ws"] = ws
nnz = ctypes.c_int32(0)
rc = L.dpf_build_ybus_noalloc(0, 0, None, None, None, None, None, 0, None, None, None, ctypes.byref(nnz), None, None)
out["noalloc_rc"] = [rc, L.dpf_last_error().decode()]
print("RESULT " + json.dumps(out))
'''


def test_host_code_under_asan_and_ubsan(tmp_path):
    """dpf_order_rcm, dpf_route_default, dpf_solve_workspace_bytes (call
    planning and layout for single grids and sub-grids, with and without a
    handoff, team cap or named variant) and the argument checks of
    dpf_build_ybus_noalloc, run from a build of the library whose host code has
    AddressSanitizer and UndefinedBehaviorSanitizer: no report, and the same
    results as the regular library."""
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    lib = tmp_path / "libdpf_host_san.so"
    # device code as in the regular build; the sanitizers instrument the host side only
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O3", "-g", "-std=c++17", "-fPIC", "-shared",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
                           "-Xarch_host", "-fno-omit-frame-pointer", '-DDPF_SOURCE_HASH="sanitized"',
                           os.path.join(ROOT, "paper_2603_28203_amd", "csrc", "dpf.hip"), "-o", str(lib)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    _instrumented(lib)
    script = f"ROOT = {ROOT!r}\nLIB = {str(lib)!r}\n" + _HOST_SCRIPT
    env = dict(os.environ)
    env["LD_PRELOAD"] = _runtime("/opt/rocm/llvm/bin/clang", "libclang_rt.asan-x86_64.so")
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=600)
    text = r.stdout + r.stderr
    assert r.returncode == 0, text[-3000:]
    assert "AddressSanitizer" not in text and "runtime error" not in text, text[-3000:]
    got = json.loads([ln for ln in r.stdout.splitlines() if ln.startswith("RESULT ")][0][len("RESULT "):])
    # the same script against the regular library, in this process
    ref_lib = os.path.join(ROOT, "paper_2603_28203_amd", "libdpf.so")
    if not os.path.exists(ref_lib):
        from paper_2603_28203_amd import build
        build.build()
    ns = {}
    import contextlib
    import io
    buf = io.StringIO()
    with contextlib.redirect_stdout(buf):
        exec(compile(f"ROOT = {ROOT!r}\nLIB = {ref_lib!r}\n" + _HOST_SCRIPT, "host_script", "exec"), ns)
    ref = json.loads([ln for ln in buf.getvalue().splitlines() if ln.startswith("RESULT ")][0][len("RESULT "):])
    assert got == ref
    assert got["rcm1"][0] == 0 and sorted(got["rcm1"][1]) == list(range(len(got["rcm1"][1])))
    assert got["rcm_bad"] == -1 and got["noalloc_rc"][0] == -1
    assert np.all(np.asarray(got["ws"][:4]) > 0)
