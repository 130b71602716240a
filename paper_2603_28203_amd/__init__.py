"""MI355X (gfx950) hot path of Differentiable Power-Flow: HIP kernels behind
the C ABI of include/dpf.h, with a thin Python binding."""

from .binding import (  # noqa: F401
    CONVERGED,
    MAX_ITER,
    NONFINITE,
    PQ,
    PV,
    SCHED_CONSTANT,
    SCHED_PLATEAU,
    SCHED_STEP,
    SLACK,
    DeviceGrid,
    DPFError,
    DPFLoss,
    Options,
    SolveWorkspace,
    build_ybus,
    fresh_sched_state,
    lib,
    max_sub_buses,
    mismatch_grad,
    solve,
    solve_workspace_bytes,
)
