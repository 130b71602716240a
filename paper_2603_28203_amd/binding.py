"""Python binding of libdpf (include/dpf.h): argument marshalling only.

Every numerical step runs in the HIP kernels of libdpf.so; torch provides the
device memory and the current stream.  If the library is missing the import
fails loudly -- there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
import dataclasses
from dataclasses import dataclass, field

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpf.so")

DPF_OK, DPF_EINVAL, DPF_ECAP, DPF_EHIP, DPF_ENOMEM, DPF_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
CONVERGED, MAX_ITER, NONFINITE, BAD_GRID, BAD_OUTAGE, UNFINISHED = 0, 1, 2, 3, 4, 5
SCHED_CONSTANT, SCHED_PLATEAU, SCHED_STEP = 0, 1, 2
OPT_ADAM, OPT_SGD, OPT_RMSPROP = 0, 1, 2
PQ, PV, SLACK = 0, 1, 2


class DPFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libdpf error {code}: {msg}")
        self.code = code


_P = ctypes.c_void_p
_i32 = ctypes.c_int32
_f64 = ctypes.c_double


class _Grid(ctypes.Structure):
    _fields_ = [("n_bus", _i32), ("nnz", _i32), ("max_row_nnz", _i32), ("row_ptr", _P), ("col_idx", _P), ("val", _P),
                ("n_branch", _i32), ("from_", _P), ("to", _P), ("r", _P), ("x", _P), ("b", _P)]


class _Opts(ctypes.Structure):
    _fields_ = [("lr", _f64), ("beta1", _f64), ("beta2", _f64), ("eps", _f64), ("tol", _f64),
                ("max_iter", _i32), ("sched", _i32), ("factor", _f64), ("patience", _i32),
                ("threshold", _f64), ("cooldown", _i32), ("min_lr", _f64), ("sched_eps", _f64),
                ("optimizer", _i32)]


class _Route(ctypes.Structure):
    _fields_ = [("variant", _i32), ("team_cap", _i32), ("tail_handoff", _i32), ("tail_team", _i32),
                ("tail_chunk", _i32), ("tail_min_items", _i32), ("tail_slice_ms", _f64),
                ("tail_first_wait_s", _f64), ("tail_wait_s", _f64), ("case_order", _i32), ("wide_host", _i32),
                ("tail_device", _i32)]


class _Trace(ctypes.Structure):
    _fields_ = [("max_mis", _P), ("every", _i32), ("len", _i32)]


_lib = None


def lib():
    """Load libdpf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_28203_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.dpf_last_error.restype = ctypes.c_char_p
        L.dpf_version.restype = ctypes.c_char_p
        from . import build as _build
        want = "src " + _build.source_hash()
        if not L.dpf_version().decode().endswith(want):
            raise ImportError(f"{LIB_PATH} was built from other sources ({L.dpf_version().decode()}, "
                              f"expected {want}): rebuild it with `python -m paper_2603_28203_amd.build`")
        L.dpf_build_ybus.argtypes = [_i32, _i32, _P, _P, _P, _P, _P, _i32, _P, _P, _P, _P, _P, _P]
        L.dpf_build_ybus.restype = ctypes.c_int
        L.dpf_build_ybus_noalloc.argtypes = [_i32, _i32, _P, _P, _P, _P, _P, _i32, _P, _P, _P, _P, _P, _P]
        L.dpf_build_ybus_noalloc.restype = ctypes.c_int
        L.dpf_mismatch_grad.argtypes = [ctypes.POINTER(_Grid), _i32, _i32, _P, _P, _i32, _P, _P, _P, _P,
                                        _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
        L.dpf_mismatch_grad.restype = ctypes.c_int
        L.dpf_param_grad.argtypes = [ctypes.POINTER(_Grid), _i32, _i32, _P, _P, _i32, _P, _P, _P, _P, _P, _P, _P,
                                     _P, _i32, _P, _P, ctypes.c_size_t, _P]
        L.dpf_param_grad.restype = ctypes.c_int
        L.dpf_dc_init.argtypes = [ctypes.POINTER(_Grid), _i32, _i32, _P, _P, _i32, _P, _P, ctypes.c_double, _i32,
                                  _P, _P, _P, ctypes.c_size_t, _P]
        L.dpf_dc_init.restype = ctypes.c_int
        L.dpf_dc_init_workspace_bytes.argtypes = [_i32, _i32]
        L.dpf_dc_init_workspace_bytes.restype = ctypes.c_size_t
        L.dpf_mismatch_grad_workspace_bytes.argtypes = [_i32, _i32]
        L.dpf_mismatch_grad_workspace_bytes.restype = ctypes.c_size_t
        R = ctypes.POINTER(_Route)
        L.dpf_solve_batch.argtypes = [ctypes.POINTER(_Grid), _i32, _P, _P, _i32, _i32, _P, _P, _i32, _P,
                                      _P, _P, _P, _P, ctypes.POINTER(_Opts), R, _P, _P, _P, _P, _P,
                                      ctypes.POINTER(_Trace), _P, ctypes.c_size_t, _P]
        L.dpf_solve_series.argtypes = [ctypes.POINTER(_Grid), _i32, _i32, _P, _P, _i32, _P, _P, _P, _P, _i32,
                                       ctypes.POINTER(_Opts), R, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
        L.dpf_solve_series.restype = ctypes.c_int
        L.dpf_solve_series_workspace_bytes.argtypes = [ctypes.POINTER(_Grid), _i32, _i32, R]
        L.dpf_solve_series_workspace_bytes.restype = ctypes.c_size_t
        L.dpf_solve_batch.restype = ctypes.c_int
        L.dpf_solve_workspace_bytes.argtypes = [ctypes.POINTER(_Grid), _i32, _P, _i32, _i32, R]
        L.dpf_solve_workspace_bytes.restype = ctypes.c_size_t
        L.dpf_route_default.argtypes = [R]
        L.dpf_route_default.restype = None
        L.dpf_solve_max_sub_buses.restype = _i32
        L.dpf_solve_variant_count.restype = ctypes.c_int
        L.dpf_solve_variant_info.argtypes = [ctypes.c_int, _P, _P, _P]
        L.dpf_solve_variant_info.restype = ctypes.c_int
        L.dpf_solve_variant_cases.argtypes = [ctypes.c_int]
        L.dpf_solve_variant_cases.restype = ctypes.c_int
        L.dpf_solve_variant_for.argtypes = [_i32]
        L.dpf_solve_variant_for.restype = ctypes.c_int
        L.dpf_autotune_set.argtypes = [_i32, ctypes.c_int]
        L.dpf_autotune_set_items.argtypes = [_i32, ctypes.c_int64, ctypes.c_int]
        L.dpf_autotune_set_items.restype = ctypes.c_int
        L.dpf_solve_variant_for_items.argtypes = [_i32, ctypes.c_int64]
        L.dpf_solve_variant_for_items.restype = ctypes.c_int
        L.dpf_autotune_set.restype = ctypes.c_int
        L.dpf_autotune_reset.restype = None
        L.dpf_order_rcm.argtypes = [_i32, _i32, _P, _P, _i32, _P, _i32, _P, _P]
        L.dpf_order_rcm.restype = ctypes.c_int
        L.dpf_tail_split_stats.argtypes = [_P, _P]
        L.dpf_tail_split_stats.restype = None
        _lib = L
    return _lib


def _check(rc: int):
    if rc != DPF_OK:
        raise DPFError(rc, lib().dpf_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, device):
    t = torch.as_tensor(t)
    return t.to(device=device, dtype=dtype).contiguous()


@dataclass
class DeviceGrid:
    """Y-bus CSR plus branch list, resident on the GPU."""
    n_bus: int
    nnz: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    val: torch.Tensor  # complex128
    max_row_nnz: int = 0
    f: torch.Tensor | None = None
    t: torch.Tensor | None = None
    r: torch.Tensor | None = None
    x: torch.Tensor | None = None
    b: torch.Tensor | None = None
    _c: _Grid | None = field(default=None, repr=False)

    @property
    def n_branch(self) -> int:
        return 0 if self.f is None else int(self.f.numel())

    def c(self) -> _Grid:
        if self._c is None:
            nb = self.n_branch
            self._c = _Grid(self.n_bus, self.nnz, int(self.max_row_nnz), _ptr(self.row_ptr), _ptr(self.col_idx),
                            _ptr(self.val), nb,
                            _ptr(self.f) if nb else None, _ptr(self.t) if nb else None,
                            _ptr(self.r) if nb else None, _ptr(self.x) if nb else None,
                            _ptr(self.b) if nb else None)
        return self._c


def build_ybus(n_bus: int, f, t, r, x, b, device="cuda", noalloc: bool = False) -> DeviceGrid:
    """dpf_build_ybus on device copies of the branch arrays (synchronises);
    noalloc=True calls dpf_build_ybus_noalloc, whose temporaries live in the
    library's static array (the caller's outputs are still torch tensors)."""
    f, t = _dev(f, torch.int32, device), _dev(t, torch.int32, device)
    r, x, b = (_dev(v, torch.float64, device) for v in (r, x, b))
    nbr = int(f.numel())
    cap = n_bus + 2 * nbr
    row_ptr = torch.empty(n_bus + 1, dtype=torch.int32, device=device)
    col = torch.empty(max(cap, 1), dtype=torch.int32, device=device)
    val = torch.empty(max(cap, 1), dtype=torch.complex128, device=device)
    nnz = ctypes.c_int32(0)
    mrow = ctypes.c_int32(0)
    fn = lib().dpf_build_ybus_noalloc if noalloc else lib().dpf_build_ybus
    _check(fn(n_bus, nbr, _ptr(f), _ptr(t), _ptr(r), _ptr(x), _ptr(b), cap, _ptr(row_ptr), _ptr(col), _ptr(val),
              ctypes.byref(nnz), ctypes.byref(mrow), _stream()))
    k = nnz.value
    return DeviceGrid(n_bus, k, row_ptr, col[:k].clone(), val[:k].clone(), mrow.value, f, t, r, x, b)


def mismatch_grad(grid: DeviceGrid, bus_type, s_spec, vm, va, outage=None, want_dS=True, want_grad=True):
    """One forward + fused-adjoint evaluation for B cases (vm, va: [B, n] float64 on the GPU).

    Returns dict(dS [B,n] complex128 | None, loss [B], max_mis [B], g_vm, g_va [B,n] | None)."""
    dev = vm.device
    B, ld = vm.shape
    bt = _dev(bus_type, torch.int8, dev)
    s = _dev(s_spec, torch.complex128, dev)
    s_ld = 0 if s.dim() == 1 else s.shape[1]
    vm = vm.contiguous()
    va = va.contiguous()
    out = _dev(outage, torch.int32, dev) if outage is not None else None
    dS = torch.empty((B, ld), dtype=torch.complex128, device=dev) if want_dS else None
    loss = torch.empty(B, dtype=torch.float64, device=dev)
    mx = torch.empty(B, dtype=torch.float64, device=dev)
    gv = torch.empty((B, ld), dtype=torch.float64, device=dev) if want_grad else None
    ga = torch.empty((B, ld), dtype=torch.float64, device=dev) if want_grad else None
    wsb = lib().dpf_mismatch_grad_workspace_bytes(grid.n_bus, B)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    g = grid.c()
    _check(lib().dpf_mismatch_grad(ctypes.byref(g), B, ld, _ptr(bt), _ptr(s), s_ld, _ptr(out), _ptr(vm), _ptr(va),
                                   _ptr(dS), _ptr(loss), _ptr(mx), _ptr(gv), _ptr(ga), _ptr(ws), wsb, _stream()))
    return {"dS": dS, "loss": loss, "max_mis": mx, "g_vm": gv, "g_va": ga}


def param_grad(grid: DeviceGrid, bus_type, s_spec, vm, va, outage=None, want_branch=True, want_s=True):
    """dpf_param_grad: per-case gradient of the loss with respect to every
    branch's r, x, b ([B, n_branch] each) and to S_spec ([B, n] complex,
    d/dRe S + j d/dIm S).  Returns dict(loss, max_mis, g_r, g_x, g_b, g_s)."""
    dev = vm.device
    B, ld = vm.shape
    bt = _dev(bus_type, torch.int8, dev)
    s = _dev(s_spec, torch.complex128, dev)
    s_ld = 0 if s.dim() == 1 else s.shape[1]
    vm = vm.contiguous()
    va = va.contiguous()
    out = _dev(outage, torch.int32, dev) if outage is not None else None
    nb = grid.n_branch
    loss = torch.empty(B, dtype=torch.float64, device=dev)
    mx = torch.empty(B, dtype=torch.float64, device=dev)
    gr, gx, gb = ((torch.empty((B, nb), dtype=torch.float64, device=dev) for _ in range(3)) if want_branch
                  else (None, None, None))
    gs = torch.empty((B, ld), dtype=torch.complex128, device=dev) if want_s else None
    wsb = lib().dpf_mismatch_grad_workspace_bytes(grid.n_bus, B)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    g = grid.c()
    _check(lib().dpf_param_grad(ctypes.byref(g), B, ld, _ptr(bt), _ptr(s), s_ld, _ptr(out), _ptr(vm), _ptr(va),
                                _ptr(loss), _ptr(mx), _ptr(gr), _ptr(gx), _ptr(gb), max(nb, 1), _ptr(gs), _ptr(ws),
                                wsb, _stream()))
    return {"loss": loss, "max_mis": mx, "g_r": gr, "g_x": gx, "g_b": gb, "g_s": gs}


def build_dc_grid(n_bus: int, f, t, x, device="cuda") -> DeviceGrid:
    """The admittance matrix of the branches with r = 0 and b = 0, whose
    susceptance Laplacian L = -Im(Y) is the DC power flow matrix."""
    z = np.zeros(len(np.asarray(f)))
    return build_ybus(n_bus, f, t, z, x, z, device=device)


def dc_init(dc_grid: DeviceGrid, bus_type, s_spec, va, outage=None, tol: float = 1e-12, max_iter: int = 20000):
    """dpf_dc_init: DC power flow angles written into va ([B, n] float64, in
    place; slack entries are kept).  Returns dict(iters, residual)."""
    dev = va.device
    B, ld = va.shape
    if not (va.is_contiguous() and va.dtype == torch.float64):
        raise ValueError("va must be a contiguous float64 tensor (updated in place)")
    bt = _dev(bus_type, torch.int8, dev)
    s = _dev(s_spec, torch.complex128, dev)
    s_ld = 0 if s.dim() == 1 else s.shape[1]
    out = _dev(outage, torch.int32, dev) if outage is not None else None
    it = torch.empty(B, dtype=torch.int32, device=dev)
    res = torch.empty(B, dtype=torch.float64, device=dev)
    wsb = int(lib().dpf_dc_init_workspace_bytes(dc_grid.n_bus, B))
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    g = dc_grid.c()
    _check(lib().dpf_dc_init(ctypes.byref(g), B, ld, _ptr(bt), _ptr(s), s_ld, _ptr(out), _ptr(va), float(tol),
                             int(max_iter), _ptr(it), _ptr(res), _ptr(ws), wsb, _stream()))
    return {"iters": it, "residual": res}


@dataclass
class Options:
    """Optimizer settings of Algorithm 1 (optimizer + schedule + tolerance);
    optimizer = OPT_ADAM (default), OPT_SGD (momentum beta1) or OPT_RMSPROP
    (smoothing beta2)."""
    lr: float = 1e-2
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    tol: float = 1e-6
    max_iter: int = 1000
    sched: int = SCHED_CONSTANT
    factor: float = 0.1
    patience: int = 10
    threshold: float = 1e-4
    cooldown: int = 0
    min_lr: float = 0.0
    sched_eps: float = 1e-8
    optimizer: int = OPT_ADAM

    def c(self) -> _Opts:
        return _Opts(self.lr, self.beta1, self.beta2, self.eps, self.tol, int(self.max_iter), int(self.sched),
                     self.factor, int(self.patience), self.threshold, int(self.cooldown), self.min_lr,
                     self.sched_eps, int(self.optimizer))


@dataclass
class Route:
    """Per-call routing of dpf_solve_batch (dpf_route_t): kernel variant (-1 =
    autotune cache / default), team cap, and the tail settings -- handoff
    threshold, split-kernel team size, iterations and time per launch, items
    left to the multi-workgroup path, barrier wait bounds -- the case order
    (1 = descending initial max|dS|) and how sub-grids above one workgroup run
    (wide_host 0: persistent teams in the call's one launch, 1: the host-driven
    multi-workgroup path), and who plans the split-kernel tail (tail_device 0:
    the host, which blocks; 1: the device, so the call can be captured).  The
    defaults equal dpf_route_default."""
    variant: int = -1
    team_cap: int = 0
    tail_handoff: int = 0
    tail_team: int = 0
    tail_chunk: int = 128
    tail_min_items: int = 0
    tail_slice_ms: float = 0.0
    tail_first_wait_s: float = 1.0
    tail_wait_s: float = 5.0
    case_order: int = 0
    wide_host: int = 0
    tail_device: int = 0

    def c(self) -> _Route:
        return _Route(int(self.variant), int(self.team_cap), int(self.tail_handoff), int(self.tail_team),
                      int(self.tail_chunk), int(self.tail_min_items), float(self.tail_slice_ms),
                      float(self.tail_first_wait_s), float(self.tail_wait_s), int(self.case_order),
                      int(self.wide_host), int(self.tail_device))


def _route(route):
    return None if route is None else ctypes.byref(route.c())


class SolveWorkspace:
    """Reusable device workspace for dpf_solve_batch (grown on demand)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes: int, device) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != torch.device(device):
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        return self.buf


_default_ws = SolveWorkspace()


def solve_workspace_bytes(grid: DeviceGrid, B, ld=None, sub_offset=None, route: Route | None = None) -> int:
    ld = grid.n_bus if ld is None else ld
    g = grid.c()
    if sub_offset is None:
        return int(lib().dpf_solve_workspace_bytes(ctypes.byref(g), 1, None, B, ld, _route(route)))
    so = (ctypes.c_int32 * len(sub_offset))(*[int(v) for v in sub_offset])
    return int(lib().dpf_solve_workspace_bytes(ctypes.byref(g), len(sub_offset) - 1, so, B, ld, _route(route)))


def solve(grid: DeviceGrid, bus_type, s_spec, vm, va, *, opts: Options | None = None, outage=None,
          sub_offset=None, sub_offset_dev=None, adam_state=None, sched_state=None,
          workspace: SolveWorkspace | None = None, outputs=None, route: Route | None = None,
          trace_every: int = 0, trace_len: int = 0):
    """dpf_solve_batch: Adam-DPF to convergence for B cases x n_sub sub-grids.

    vm, va ([B, ld] float64, GPU) are updated in place; `route` (Route) sets this
    call's kernel choice and tail settings.  sub_offset (host sequence) gives the
    sub-grid offsets; sub_offset_dev, an int32 device tensor of the same values,
    spares the call its host-to-device copy (a call captured in a graph needs
    it).  With trace_len > 0 the result also holds "trace" ([B * n_sub,
    trace_len] float64, NaN where an item had stopped): max|dS| of iterations 0,
    trace_every, 2 trace_every, ... of this call.  Returns dict with iters,
    status, max_mis, loss ([B * n_sub], index c * n_sub + s)."""
    opts = opts or Options()
    dev = vm.device
    B, ld = vm.shape
    if not (vm.is_contiguous() and va.is_contiguous() and vm.dtype == torch.float64 and va.dtype == torch.float64):
        raise ValueError("vm and va must be contiguous float64 tensors (updated in place)")
    bt = bus_type if (torch.is_tensor(bus_type) and bus_type.dtype == torch.int8 and bus_type.device == dev) \
        else _dev(bus_type, torch.int8, dev)
    s = s_spec if (torch.is_tensor(s_spec) and s_spec.dtype == torch.complex128 and s_spec.device == dev
                   and s_spec.is_contiguous()) else _dev(s_spec, torch.complex128, dev)
    if s.dim() == 2 and s.shape[0] != B:
        raise ValueError(f"s_spec has {s.shape[0]} rows for {B} cases (pass one row per case, or a 1-D shared row)")
    s_ld = 0 if s.dim() == 1 else s.shape[1]
    out = None if outage is None else (outage if (torch.is_tensor(outage) and outage.dtype == torch.int32
                                                  and outage.device == dev) else _dev(outage, torch.int32, dev))
    if sub_offset is None:
        n_sub, so_h, so_d = 1, None, None
    else:
        so_list = [int(v) for v in (sub_offset.tolist() if torch.is_tensor(sub_offset) else sub_offset)]
        n_sub = len(so_list) - 1
        so_h = (ctypes.c_int32 * len(so_list))(*so_list)
        if sub_offset_dev is not None:
            if not (torch.is_tensor(sub_offset_dev) and sub_offset_dev.dtype == torch.int32 and
                    sub_offset_dev.device == dev and sub_offset_dev.is_contiguous() and
                    sub_offset_dev.numel() == len(so_list)):
                raise ValueError("sub_offset_dev must be a contiguous int32 tensor on vm's device, "
                                 "as long as sub_offset")
            so_d = sub_offset_dev
        else:
            so_d = torch.tensor(so_list, dtype=torch.int32, device=dev)
    items = B * n_sub
    if outputs is None:
        outputs = {"iters": torch.empty(items, dtype=torch.int32, device=dev),
                   "status": torch.empty(items, dtype=torch.int32, device=dev),
                   "max_mis": torch.empty(items, dtype=torch.float64, device=dev),
                   "loss": torch.empty(items, dtype=torch.float64, device=dev),
                   "done_ns": torch.empty(items, dtype=torch.int64, device=dev)}
    tr = None
    if trace_len:
        if "trace" not in outputs:
            outputs["trace"] = torch.full((items, int(trace_len)), float("nan"), dtype=torch.float64, device=dev)
        tr = _Trace(_ptr(outputs["trace"]), int(trace_every), int(trace_len))
    g = grid.c()
    rc = None if route is None else route.c()
    rp = None if rc is None else ctypes.byref(rc)
    wsb = int(lib().dpf_solve_workspace_bytes(ctypes.byref(g), n_sub, so_h, B, ld, rp))
    if wsb == 0:
        raise DPFError(DPF_EINVAL, "invalid sizes or route")
    ws = (workspace or _default_ws).get(wsb, dev)
    o = opts.c()
    _check(lib().dpf_solve_batch(ctypes.byref(g), n_sub, so_h, _ptr(so_d), B, ld, _ptr(bt), _ptr(s), s_ld,
                                 _ptr(out), _ptr(vm), _ptr(va), _ptr(adam_state), _ptr(sched_state),
                                 ctypes.byref(o), rp, _ptr(outputs["iters"]), _ptr(outputs["status"]),
                                 _ptr(outputs["max_mis"]), _ptr(outputs["loss"]), _ptr(outputs.get("done_ns")),
                                 None if tr is None else ctypes.byref(tr), _ptr(ws), ws.numel(), _stream()))
    if so_d is not None:
        outputs["_keep"] = so_d  # keep the device offsets alive until the stream has used them
    return outputs


SCHED_WORDS = 6


def fresh_sched_state(items: int, lr: float, device="cuda") -> torch.Tensor:
    """Per-item schedule state {t, lr, best, counters, b1^t, b2^t} of a fresh solve."""
    st = torch.zeros((items, SCHED_WORDS), dtype=torch.float64, device=device)
    st[:, 1] = lr
    st[:, 2] = float("inf")
    st[:, 4] = 1.0
    st[:, 5] = 1.0
    return st


def solve_series(grid: DeviceGrid, bus_type, s_series, vm0, va0, *, window: int = 1,
                 opts: Options | None = None, workspace: SolveWorkspace | None = None,
                 route: Route | None = None):
    """dpf_solve_series: T warm-started power flows in windows of `window` steps.

    s_series: [T, n] complex128 (GPU); vm0, va0: [n].  Returns dict with vm, va
    ([T, n] solutions) and per-step iters, status, max_mis, loss, done_ns."""
    opts = opts or Options()
    dev = s_series.device
    T, n = s_series.shape
    s = s_series.contiguous()
    bt = bus_type if (torch.is_tensor(bus_type) and bus_type.dtype == torch.int8 and bus_type.device == dev) \
        else _dev(bus_type, torch.int8, dev)
    vm0 = _dev(vm0, torch.float64, dev)
    va0 = _dev(va0, torch.float64, dev)
    vm = torch.empty((T, n), dtype=torch.float64, device=dev)
    va = torch.empty((T, n), dtype=torch.float64, device=dev)
    out = {"iters": torch.empty(T, dtype=torch.int32, device=dev),
           "status": torch.empty(T, dtype=torch.int32, device=dev),
           "max_mis": torch.empty(T, dtype=torch.float64, device=dev),
           "loss": torch.empty(T, dtype=torch.float64, device=dev),
           "done_ns": torch.empty(T, dtype=torch.int64, device=dev)}
    g = grid.c()
    rc = None if route is None else route.c()
    rp = None if rc is None else ctypes.byref(rc)
    wsb = int(lib().dpf_solve_series_workspace_bytes(ctypes.byref(g), int(window), n, rp))
    if wsb == 0:
        raise DPFError(DPF_EINVAL, "invalid sizes or route")
    ws = (workspace or _default_ws).get(wsb, dev)
    o = opts.c()
    _check(lib().dpf_solve_series(ctypes.byref(g), T, int(window), _ptr(bt), _ptr(s), n, _ptr(vm0), _ptr(va0),
                                  _ptr(vm), _ptr(va), n, ctypes.byref(o), rp, _ptr(out["iters"]),
                                  _ptr(out["status"]), _ptr(out["max_mis"]), _ptr(out["loss"]),
                                  _ptr(out["done_ns"]), _ptr(ws), ws.numel(), _stream()))
    out["vm"] = vm
    out["va"] = va
    return out


def max_sub_buses() -> int:
    return int(lib().dpf_solve_max_sub_buses())


class DPFLoss(torch.autograd.Function):
    """Per-case DPF loss whose backward is the fused adjoint of libdpf.

    forward(vm, va, grid, bus_type, s_spec, outage) -> loss [B];
    backward returns grad_out[c] * d loss_c / d(vm, va) (zeros at fixed
    coordinates), computed in the same kernel pass as the loss."""

    @staticmethod
    def forward(ctx, vm, va, grid, bus_type, s_spec, outage=None):
        r = mismatch_grad(grid, bus_type, s_spec, vm.detach(), va.detach(), outage=outage, want_dS=False,
                          want_grad=True)
        ctx.save_for_backward(r["g_vm"], r["g_va"])
        ctx.mark_non_differentiable(r["max_mis"])
        return r["loss"], r["max_mis"]

    @staticmethod
    def backward(ctx, grad_loss, grad_mx):
        gv, ga = ctx.saved_tensors
        return grad_loss[:, None] * gv, grad_loss[:, None] * ga, None, None, None, None


# ---------------------------------------------------------------- autotuner


VARIANT_KINDS = ("register", "streaming", "banded-stream", "wide", "banded-pair")
# the per-item kinds that can hand their tail over (dpf_route_t.tail_handoff)
HANDOFF_KINDS = ("streaming", "banded-stream", "banded-pair")


def variants():
    """The solve kernel variants: list of dicts (index, threads, buses_per_thread,
    kind, streaming, cases).  For a banded variant buses_per_thread counts the buses
    of one block; it serves sub-grids of bandwidth <= threads * buses_per_thread.
    `cases` is the number of cases one workgroup solves at a time (1 for every
    variant built)."""
    L = lib()
    out = []
    for i in range(L.dpf_solve_variant_count()):
        t, k, st = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        _check(L.dpf_solve_variant_info(i, ctypes.byref(t), ctypes.byref(k), ctypes.byref(st)))
        cases = L.dpf_solve_variant_cases(i)
        if cases < 0:
            _check(cases)
        out.append({"index": i, "threads": t.value, "buses_per_thread": k.value, "kind": VARIANT_KINDS[st.value],
                    "streaming": st.value != 0, "cases": cases})
    return out


def rcm_order(n_bus: int, f, t, sub_offset=None, group: int = 0):
    """dpf_order_rcm: a small-bandwidth bus numbering (reverse Cuthill-McKee),
    optionally with buses grouped by degree inside windows of ``group``.

    Returns (perm, bandwidth) with perm[k] = old index of new bus k.  Renumber a
    grid with inv = argsort(perm): branch ends become inv[f], inv[t] and every
    per-bus array a becomes a[..., perm]."""
    f = np.ascontiguousarray(f, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    perm = np.empty(int(n_bus), dtype=np.int32)
    bw = ctypes.c_int32(0)
    if sub_offset is None:
        n_sub, so = 1, None
    else:
        so_arr = np.ascontiguousarray(sub_offset, dtype=np.int32)
        n_sub, so = len(so_arr) - 1, so_arr.ctypes.data_as(ctypes.c_void_p)
    _check(lib().dpf_order_rcm(int(n_bus), len(f), f.ctypes.data_as(ctypes.c_void_p),
                               t.ctypes.data_as(ctypes.c_void_p), n_sub, so, int(group),
                               perm.ctypes.data_as(ctypes.c_void_p), ctypes.byref(bw)))
    return perm, int(bw.value)


def variant_for(n_max: int, items: int | None = None) -> int:
    """Variant index dpf_solve_batch would use (for many items, or for `items`)."""
    if items is None:
        return int(lib().dpf_solve_variant_for(int(n_max)))
    return int(lib().dpf_solve_variant_for_items(int(n_max), int(items)))


def autotune_reset():
    lib().dpf_autotune_reset()


def route_default() -> Route:
    """dpf_route_default as a Route (the library's defaults)."""
    r = _Route()
    lib().dpf_route_default(ctypes.byref(r))
    return Route(r.variant, r.team_cap, r.tail_handoff, r.tail_team, r.tail_chunk, r.tail_min_items,
                 r.tail_slice_ms, r.tail_first_wait_s, r.tail_wait_s, r.case_order, r.wide_host, r.tail_device)


def split_stats() -> dict:
    """dpf_tail_split_stats: split-kernel launches and abandoned launches so far."""
    n, ab = ctypes.c_int64(), ctypes.c_int64()
    lib().dpf_tail_split_stats(ctypes.byref(n), ctypes.byref(ab))
    return {"launches": n.value, "abandoned": ab.value}


def autotune(grid: DeviceGrid, bus_type, s_spec, vm, va, *, outage=None, sub_offset=None, opts=None,
             iters: int = 40, reps: int = 2, tie: float = 0.0, route: Route | None = None):
    """Time every kernel variant that can hold the largest sub-grid on copies of
    the real inputs (``iters`` Adam iterations, no stop test; each probe names its
    variant in its own route, with the tail handoff off) and record the fastest
    in the library's autotune cache for this size class and this number of work
    items (B x sub-grids).  Variants within a fraction ``tie`` of the fastest
    count as equal and the first of them in the table is taken, which keeps the
    choice stable under timing noise.  With a tail handoff in ``route``, a
    single-grid call chooses among the kinds that can hand over (streaming,
    banded-stream, banded-pair): the fixed-length probes cannot see the handoff.
    Returns {variant: seconds}."""
    opts = opts or Options()
    route = route or Route()
    n_max = grid.n_bus if sub_offset is None else int(max(b - a for a, b in zip(sub_offset[:-1], sub_offset[1:])))
    items = int(vm.shape[0]) * (1 if sub_offset is None else len(sub_offset) - 1)
    probe = Options(**{**opts.__dict__, "tol": 0.0, "max_iter": int(iters)})
    times = {}
    _time_variants(grid, bus_type, s_spec, vm, va, outage, sub_offset, probe, n_max, reps, times, route)
    eligible = times
    if route.tail_handoff > 0 and sub_offset is None:
        kinds = {v["index"]: v["kind"] for v in variants()}
        can = {i: t for i, t in times.items() if kinds[i] in HANDOFF_KINDS}
        eligible = can or times
    best = min(eligible.values())
    pick = min(i for i, t in eligible.items() if t <= best * (1.0 + tie))
    _check(lib().dpf_autotune_set_items(n_max, items, pick))
    return {"choice": pick, "seconds": times, "n_max": n_max, "items": items, "iters": iters}


def _time_variants(grid, bus_type, s_spec, vm, va, outage, sub_offset, probe, n_max, reps, times, route):
    for v in variants():
        if not (v["kind"].startswith("banded") or v["buses_per_thread"] == 0
                or v["threads"] * v["buses_per_thread"] >= n_max):
            continue
        rt = dataclasses.replace(route, variant=v["index"], tail_handoff=0)
        best = None
        for _ in range(reps):
            vm1, va1 = vm.clone(), va.clone()
            torch.cuda.synchronize()
            st = torch.cuda.Event(enable_timing=True)
            en = torch.cuda.Event(enable_timing=True)
            st.record()
            solve(grid, bus_type, s_spec, vm1, va1, opts=probe, outage=outage, sub_offset=sub_offset, route=rt)
            en.record()
            torch.cuda.synchronize()
            dt = st.elapsed_time(en) * 1e-3
            best = dt if best is None else min(best, dt)
        times[v["index"]] = best
