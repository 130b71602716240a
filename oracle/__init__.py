"""FP64 CPU oracle for Differentiable Power-Flow (DPF).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports or
links anything from here, and nothing here imports the GPU library.

The arithmetic lives in ``dpf_oracle.c`` (plain C, FP64, every step written
out in the paper's order); this module loads it with ctypes and adds the
Newton-Raphson reference solve (Algorithm 2), whose linear solve is a library
routine (numpy dense LU for small systems, SciPy's sparse LU otherwise).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dpf_oracle.c")
LIB = os.path.join(HERE, "libdpf_oracle.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fcx-limited-range", "-fopenmp",
          "-fPIC", "-shared"]
# the same source for the benchmark's CPU-baseline leg, optimised for the host it
# runs on (built there at run time: -march=native code may not run on another CPU);
# -ffp-contract=off keeps the arithmetic, and so the results, those of the pinned build
NATIVE_LIB = os.path.join(HERE, "libdpf_oracle_native.so")
NATIVE_CFLAGS = ["-O3", "-march=native", "-std=c11", "-ffp-contract=off", "-fcx-limited-range", "-fopenmp",
                 "-fPIC", "-shared"]

PQ, PV, SLACK = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (when forced, missing or older than its source)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def build_native() -> str:
    """Compile the oracle with NATIVE_CFLAGS for this host (always rebuilt)."""
    tmp = NATIVE_LIB + ".tmp"
    subprocess.check_call(["gcc", *NATIVE_CFLAGS, SRC, "-o", tmp, "-lm"])
    os.replace(tmp, NATIVE_LIB)
    return NATIVE_LIB


_lib = None
_native = None


def _load(native: bool = False):
    """The ctypes library of the oracle (native=True: the host-optimised build,
    compiled on first use)."""
    global _lib, _native
    if native:
        if _native is None:
            build_native()
            _native = _bind(ctypes.CDLL(NATIVE_LIB))
        return _native
    if _lib is None:
        path = os.environ.get("DPF_ORACLE_LIB")  # another build of the same source (the sanitizer test)
        if not path:
            path = build()
        _lib = _bind(ctypes.CDLL(path))
    return _lib


def _bind(lib):
    """Argument and result types of the oracle's C functions."""
    P = ctypes.c_void_p
    i32 = ctypes.c_int32
    d = ctypes.c_double
    lib.orc_ybus.argtypes = [i32, i32, P, P, P, P, P, i32, i32, P, P, P]
    lib.orc_ybus.restype = ctypes.c_int
    lib.orc_polar.argtypes = [i32, P, P, P]
    lib.orc_current.argtypes = [i32, P, P, P, P, P]
    lib.orc_mismatch.argtypes = [i32, P, P, P, P, P, P, P]
    lib.orc_residual_count.argtypes = [i32, P]
    lib.orc_residual_count.restype = i32
    lib.orc_loss_from_mismatch.argtypes = [i32, P, P, P]
    lib.orc_loss_from_mismatch.restype = d
    lib.orc_dS_dV.argtypes = [i32, P, P, P, P, P, P, P]
    lib.orc_param_grad.argtypes = [i32, i32, P, P, P, P, P, i32, P, P, P, P, P, P, P, P, P, P, P]
    lib.orc_loss_grad.argtypes = [i32, P, P, P, P, P, P, P, P, P, P]
    lib.orc_loss_grad.restype = d
    lib.orc_solve_adam.argtypes = [i32, P, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.orc_solve_adam.restype = i32
    lib.orc_solve_adam_batch.argtypes = [i32, i32, P, P, P, P, P, i32, P, P, P, P, P, P, P]
    lib.orc_num_threads.restype = i32
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _i8(a):
    return np.ascontiguousarray(a, dtype=np.int8)


@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col: np.ndarray  # int32 [nnz]
    val: np.ndarray  # complex128 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n), dtype=np.complex128)
        for i in range(self.n):
            for q in range(self.row_ptr[i], self.row_ptr[i + 1]):
                a[i, self.col[q]] += self.val[q]
        return a


class OracleError(ValueError):
    pass


def build_ybus(n_bus, f, t, r, x, b, skip: int = -1) -> CSR:
    """Bus admittance matrix, pi-model branches (Sec. 2.1); `skip` drops one
    branch entirely (the N-1 outage case)."""
    lib = _load()
    f, t, r, x, b = _i32(f), _i32(t), _f64(r), _f64(x), _f64(b)
    cap = n_bus + 2 * len(f)
    rp = np.zeros(n_bus + 1, dtype=np.int32)
    col = np.zeros(max(cap, 1), dtype=np.int32)
    val = np.zeros(max(cap, 1), dtype=np.complex128)
    nnz = lib.orc_ybus(n_bus, len(f), _p(f), _p(t), _p(r), _p(x), _p(b), int(skip), cap,
                       _p(rp), _p(col), _p(val))
    if nnz < 0:
        raise OracleError(f"orc_ybus failed with {nnz}")
    return CSR(n_bus, rp, col[:nnz].copy(), val[:nnz].copy())


def ybus_of(grid, skip: int = -1) -> CSR:
    return build_ybus(grid.n_bus, grid.f, grid.t, grid.r, grid.x, grid.b, skip)


def polar(vm, va) -> np.ndarray:
    lib = _load()
    vm, va = _f64(vm), _f64(va)
    out = np.zeros(len(vm), dtype=np.complex128)
    lib.orc_polar(len(vm), _p(vm), _p(va), _p(out))
    return out


def current(Y: CSR, V) -> np.ndarray:
    lib = _load()
    V = _c128(V)
    out = np.zeros(Y.n, dtype=np.complex128)
    lib.orc_current(Y.n, _p(Y.row_ptr), _p(Y.col), _p(Y.val), _p(V), _p(out))
    return out


def mismatch(Y: CSR, vm, va, s_spec) -> np.ndarray:
    """dS = V .* conj(Y V) - S_spec for one case."""
    lib = _load()
    vm, va, s = _f64(vm), _f64(va), _c128(s_spec)
    out = np.zeros(Y.n, dtype=np.complex128)
    lib.orc_mismatch(Y.n, _p(Y.row_ptr), _p(Y.col), _p(Y.val), _p(vm), _p(va), _p(s), _p(out))
    return out


def injections(Y: CSR, vm, va) -> np.ndarray:
    """S_calc = V .* conj(Y V)."""
    return mismatch(Y, vm, va, np.zeros(Y.n, dtype=np.complex128))


def residual_count(bus_type) -> int:
    bt = _i8(bus_type)
    return int(_load().orc_residual_count(len(bt), _p(bt)))


def loss_from_mismatch(bus_type, dS):
    lib = _load()
    bt, dS = _i8(bus_type), _c128(dS)
    mu = ctypes.c_double(0.0)
    loss = lib.orc_loss_from_mismatch(len(bt), _p(bt), _p(dS), ctypes.byref(mu))
    return float(loss), float(mu.value)


def dS_dV(Y: CSR, vm, va):
    """Algorithm 2 partial derivatives dS/d|V| and dS/dtheta in Y's pattern."""
    lib = _load()
    vm, va = _f64(vm), _f64(va)
    dvm = np.zeros(Y.nnz, dtype=np.complex128)
    dva = np.zeros(Y.nnz, dtype=np.complex128)
    lib.orc_dS_dV(Y.n, _p(Y.row_ptr), _p(Y.col), _p(Y.val), _p(vm), _p(va), _p(dvm), _p(dva))
    return dvm, dva


def loss_grad(Y: CSR, bus_type, vm, va, s_spec):
    """(loss, mu, g_vm, g_va) for one case; gradient = (2/m) J_f^T f."""
    lib = _load()
    bt, vm, va, s = _i8(bus_type), _f64(vm), _f64(va), _c128(s_spec)
    gvm = np.zeros(Y.n)
    gva = np.zeros(Y.n)
    mu = ctypes.c_double(0.0)
    loss = lib.orc_loss_grad(Y.n, _p(Y.row_ptr), _p(Y.col), _p(Y.val), _p(bt), _p(vm), _p(va),
                             _p(s), _p(gvm), _p(gva), ctypes.byref(mu))
    return float(loss), float(mu.value), gvm, gva


def param_grad(grid, bus_type, vm, va, s_spec, skip: int = -1):
    """(g_r, g_x, g_b, g_s): gradient of one case's loss with respect to every
    branch's r, x, b and to S_spec (complex: d/dRe S + j d/dIm S).  Branch `skip`
    is outaged (absent from Y; zero gradient)."""
    lib = _load()
    Y = ybus_of(grid, skip=skip)
    f, t = _i32(grid.f), _i32(grid.t)
    r, x, b = _f64(grid.r), _f64(grid.x), _f64(grid.b)
    bt, vm, va, s = _i8(bus_type), _f64(vm), _f64(va), _c128(s_spec)
    nb = len(f)
    g_r, g_x, g_b = np.zeros(nb), np.zeros(nb), np.zeros(nb)
    g_s = np.zeros(Y.n, dtype=np.complex128)
    lib.orc_param_grad(Y.n, nb, _p(f), _p(t), _p(r), _p(x), _p(b), int(skip), _p(Y.row_ptr), _p(Y.col),
                       _p(Y.val), _p(bt), _p(vm), _p(va), _p(s), _p(g_r), _p(g_x), _p(g_b), _p(g_s))
    return g_r, g_x, g_b, g_s


def dc_power_flow(grid, bus_type, s_spec, va_slack: float = 0.0, skip: int = -1):
    """DC power flow angles (the linear approximation used to start Newton-Raphson
    in Algorithm 2): L theta = Re S_spec on the non-slack buses, L the Laplacian
    of the branch susceptances 1/x (parallel branches add, branch `skip` left
    out), the slack angle fixed at va_slack.  A library sparse solve does the
    linear algebra."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    n = grid.n_bus
    keep = np.ones(len(grid.f), dtype=bool)
    if skip >= 0:
        keep[skip] = False
    f, t, w = grid.f[keep], grid.t[keep], 1.0 / grid.x[keep]
    L = sp.coo_matrix((np.concatenate([w, w, -w, -w]),
                       (np.concatenate([f, t, f, t]), np.concatenate([f, t, t, f]))), shape=(n, n)).tocsr()
    bt = np.asarray(bus_type)
    free = np.flatnonzero(bt != 2)
    slack = np.flatnonzero(bt == 2)
    theta = np.zeros(n)
    theta[slack] = va_slack
    rhs = np.asarray(s_spec).real[free] - L[free][:, slack] @ theta[slack]
    theta[free] = spla.spsolve(L[free][:, free].tocsc(), rhs)
    return theta


class _Opts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("sched", ctypes.c_int32), ("factor", ctypes.c_double),
                ("patience", ctypes.c_int32), ("threshold", ctypes.c_double),
                ("cooldown", ctypes.c_int32), ("min_lr", ctypes.c_double),
                ("sched_eps", ctypes.c_double), ("optimizer", ctypes.c_int32)]


SCHED_CONSTANT, SCHED_PLATEAU, SCHED_STEP = 0, 1, 2
OPT_ADAM, OPT_SGD, OPT_RMSPROP = 0, 1, 2


@dataclass
class AdamOptions:
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
    optimizer: int = 0  # OPT_ADAM, OPT_SGD (momentum beta1) or OPT_RMSPROP (smoothing beta2)

    def c(self) -> _Opts:
        return _Opts(self.lr, self.beta1, self.beta2, self.eps, self.tol, int(self.max_iter),
                     int(self.sched), self.factor, int(self.patience), self.threshold,
                     int(self.cooldown), self.min_lr, self.sched_eps, int(self.optimizer))


def solve_adam(Y: CSR, bus_type, s_spec, vm0, va0, opts: AdamOptions, state=None, t0: int = 0,
               native: bool = False):
    """One DPF solve (Algorithm 1 with Adam).  Returns a dict with vm, va,
    status (0 converged, 1 max_iter, 2 non-finite), iters, mu, lr, state, t.
    native=True runs the host-optimised build of the same source."""
    lib = _load(native)
    bt, s = _i8(bus_type), _c128(s_spec)
    vm, va = _f64(vm0).copy(), _f64(va0).copy()
    st = np.zeros(4 * Y.n) if state is None else _f64(state).copy()
    t = ctypes.c_int32(int(t0))
    it = ctypes.c_int32(0)
    mu = ctypes.c_double(0.0)
    lr = ctypes.c_double(0.0)
    o = opts.c()
    status = lib.orc_solve_adam(Y.n, _p(Y.row_ptr), _p(Y.col), _p(Y.val), _p(bt), _p(s),
                                _p(vm), _p(va), ctypes.byref(o), _p(st), ctypes.byref(t),
                                ctypes.byref(it), ctypes.byref(mu), ctypes.byref(lr))
    return {"vm": vm, "va": va, "status": int(status), "iters": int(it.value),
            "mu": float(mu.value), "lr": float(lr.value), "state": st, "t": int(t.value)}


def solve_adam_batch(Y: CSR, bus_type, s_spec, vm0, va0, opts: AdamOptions):
    """B independent cases on one Y.  s_spec is [n] (shared) or [B, n];
    vm0/va0 are [B, n].  Returns dict of per-case arrays."""
    lib = _load()
    bt = _i8(bus_type)
    s = _c128(s_spec)
    shared = 1 if s.ndim == 1 else 0
    vm, va = _f64(vm0).copy(), _f64(va0).copy()
    B = vm.shape[0]
    status = np.zeros(B, dtype=np.int32)
    iters = np.zeros(B, dtype=np.int32)
    mu = np.zeros(B)
    lr = np.zeros(B)
    o = opts.c()
    lib.orc_solve_adam_batch(B, Y.n, _p(Y.row_ptr), _p(Y.col), _p(Y.val), _p(bt), _p(s), shared,
                             _p(vm), _p(va), ctypes.byref(o), _p(status), _p(iters), _p(mu),
                             _p(lr))
    return {"vm": vm, "va": va, "status": status, "iters": iters, "mu": mu, "lr": lr}


def num_threads() -> int:
    return int(_load().orc_num_threads())


# ------------------------------------------------------------ Newton-Raphson


def jacobian_f(Y: CSR, bus_type, vm, va):
    """J_f of Algorithm 2 as a SciPy CSR matrix.

    Rows: [P at pv,pq ; Q at pq]; columns: [theta at pv,pq ; |V| at pq], both
    in ascending bus order within each block."""
    import scipy.sparse as sp
    bt = np.asarray(bus_type)
    pvpq = np.flatnonzero(bt != SLACK)
    pq = np.flatnonzero(bt == PQ)
    dvm, dva = dS_dV(Y, vm, va)
    rows = np.repeat(np.arange(Y.n), np.diff(Y.row_ptr))
    cols = Y.col
    n = Y.n
    dSdVa = sp.csr_matrix((dva, (rows, cols)), shape=(n, n))
    dSdVm = sp.csr_matrix((dvm, (rows, cols)), shape=(n, n))
    j11 = dSdVa.real[pvpq][:, pvpq]
    j12 = dSdVm.real[pvpq][:, pq]
    j21 = dSdVa.imag[pq][:, pvpq]
    j22 = dSdVm.imag[pq][:, pq]
    return sp.bmat([[j11, j12], [j21, j22]], format="csr"), pvpq, pq


def residual_vector(Y: CSR, bus_type, vm, va, s_spec):
    """f = [dP[pv,pq], dQ[pq]] (Algorithm 2, power mismatch)."""
    bt = np.asarray(bus_type)
    dS = mismatch(Y, vm, va, s_spec)
    return np.concatenate([dS.real[bt != SLACK], dS.imag[bt == PQ]])


def newton(Y: CSR, bus_type, s_spec, vm0, va0, tol: float = 1e-10, max_iter: int = 30):
    """Newton-Raphson power flow (Algorithm 2): solve J_f dx = -f, update
    theta[pv,pq] and |V|[pq], stop when max|f| < tol.  The linear solve is a
    library LU (dense numpy below 2000 unknowns, SciPy splu above).
    Returns dict with vm, va, iters, mu, converged, history (max|f| per step)."""
    import scipy.sparse.linalg as spla
    vm, va = _f64(vm0).copy(), _f64(va0).copy()
    hist = []
    f = residual_vector(Y, bus_type, vm, va, s_spec)
    hist.append(float(np.max(np.abs(f))) if f.size else 0.0)
    it = 0
    while hist[-1] >= tol and it < max_iter and np.isfinite(hist[-1]):
        J, pvpq, pq = jacobian_f(Y, bus_type, vm, va)
        if J.shape[0] < 2000:
            dx = np.linalg.solve(J.toarray(), -f)
        else:
            dx = spla.splu(J.tocsc()).solve(-f)
        va[pvpq] += dx[: len(pvpq)]
        vm[pq] += dx[len(pvpq):]
        f = residual_vector(Y, bus_type, vm, va, s_spec)
        hist.append(float(np.max(np.abs(f))) if f.size else 0.0)
        it += 1
    return {"vm": vm, "va": va, "iters": it, "mu": hist[-1], "converged": hist[-1] < tol,
            "history": hist}
