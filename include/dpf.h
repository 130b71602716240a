/*
 * dpf.h -- C ABI of libdpf, an MI355X (gfx950) implementation of the hot path of
 * Differentiable Power-Flow (DPF, arXiv 2603.28203): the batched AC power
 * mismatch, the bus-type-masked squared-mismatch loss, its gradient with respect
 * to voltage magnitudes and angles, and the Adam iteration that drives the
 * mismatch to zero.
 *
 * Conventions (all entry points)
 * -----------------------------
 *  - Array arguments are DEVICE pointers owned by the caller unless marked
 *    "host".  The library keeps no pointer after a call returns.
 *  - All arithmetic is FP64.  Complex arrays are interleaved (re, im) doubles,
 *    the layout of std::complex<double> / torch.complex128.
 *  - Per-case per-bus arrays are case-major: element (case c, bus i) is at
 *    x[c * ld + i] (complex arrays: doubles 2*(c*ld+i) and 2*(c*ld+i)+1), with
 *    ld >= n_bus.
 *  - Bus types: 0 = PQ (P and Q specified), 1 = PV (P and |V| specified),
 *    2 = slack (V specified, angle 0) -- the three bus kinds of Sec. 2.1.
 *    Exactly one slack per grid (per sub-grid for concatenated grids).
 *  - Every call is ordered on `stream` (a hipStream_t; NULL = default stream)
 *    and returns after enqueueing, unless documented as synchronising.  The
 *    synchronising parts of dpf_solve_batch (multi-workgroup items, tail
 *    handoff) use one side stream per device; concurrent such calls on one
 *    device take turns.
 *  - Return value: DPF_OK (0) or a negative error code; dpf_last_error()
 *    returns a text for the calling thread's last error.  On error nothing
 *    has been enqueued, except for DPF_EHIP, which reports a HIP runtime
 *    failure (the stream may then hold partial work).
 *  - Scratch memory: the solve and the gradient evaluation take a caller
 *    workspace (query its size first); dpf_build_ybus allocates and frees its
 *    own temporaries.  Nothing else is allocated per call.
 */
#ifndef DPF_H
#define DPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DPF_OK 0
#define DPF_EINVAL (-1)      /* bad argument: null pointer, size, index, bus types */
#define DPF_ECAP (-2)        /* nnz_cap too small */
#define DPF_EHIP (-3)        /* HIP runtime error (text in dpf_last_error) */
#define DPF_ENOMEM (-4)      /* workspace too small */
#define DPF_EUNSUPPORTED (-5) /* combination of options not implemented */

#define DPF_BUS_PQ 0
#define DPF_BUS_PV 1
#define DPF_BUS_SLACK 2

/* per-case solve status (an output, not an error) */
#define DPF_CONVERGED 0
#define DPF_MAX_ITER 1
#define DPF_NONFINITE 2
#define DPF_BAD_GRID 3   /* a CSR row is longer than the grid's declared max_row_nnz */
#define DPF_BAD_OUTAGE 4 /* the case's outage index is neither -1 nor a branch index */
#define DPF_UNFINISHED 5 /* the item's team of workgroups did not assemble in time (see dpf_route_t) */

/* learning-rate schedules (Table 2 and Table 3 of the paper use the last two) */
#define DPF_SCHED_CONSTANT 0
#define DPF_SCHED_PLATEAU 1  /* reduce-on-plateau, mode min, relative threshold */
#define DPF_SCHED_STEP 2     /* lr *= factor every `patience` iterations */

/* optimizers (Sec. 6.3 names Adam, SGD and RMSprop as the searched optimizers) */
#define DPF_OPT_ADAM 0
#define DPF_OPT_SGD 1      /* momentum beta1 (0 = plain gradient descent) */
#define DPF_OPT_RMSPROP 2  /* smoothing beta2, no momentum, not centred */

/*
 * A bus admittance matrix in CSR form plus (optionally) the branch list it was
 * built from.  row_ptr/col_idx/val as produced by dpf_build_ybus: rows sorted
 * by column, the diagonal always stored.  The branch arrays are only read by
 * the N-1 outage correction and may be NULL (n_branch = 0) otherwise.
 * Several independent grids can be concatenated into one block-diagonal CSR
 * (column indices global); see `sub_offset` of dpf_solve_batch.  max_row_nnz
 * sizes the solve workspace; 0 makes the library assume the worst case (nnz).
 */
typedef struct dpf_grid {
    int32_t n_bus;
    int32_t nnz;
    int32_t max_row_nnz;    /* longest CSR row (as returned by dpf_build_ybus), or 0 if unknown */
    const int32_t *row_ptr; /* [n_bus + 1] */
    const int32_t *col_idx; /* [nnz] */
    const double *val;      /* [2 * nnz] complex */
    int32_t n_branch;
    const int32_t *from;    /* [n_branch] */
    const int32_t *to;      /* [n_branch] */
    const double *r;        /* [n_branch] series resistance (pu) */
    const double *x;        /* [n_branch] series reactance (pu) */
    const double *b;        /* [n_branch] total line charging (pu) */
} dpf_grid_t;

/*
 * Optimizer settings (Algorithm 1: optimizer + scheduler + tolerance), applied
 * on learnable entries only.  `optimizer` selects the update of a coordinate x
 * with gradient g and per-coordinate state m, s (PyTorch's definitions):
 *   DPF_OPT_ADAM (default), Kingma & Ba: m <- b1 m + (1-b1) g; s <- b2 s + (1-b2) g^2;
 *       x <- x - lr * (m/(1-b1^t)) / (sqrt(s/(1-b2^t)) + eps)
 *   DPF_OPT_SGD: m <- b1 m + g; x <- x - lr m (b1 = momentum, no dampening)
 *   DPF_OPT_RMSPROP: s <- b2 s + (1-b2) g^2; x <- x - lr g / (sqrt(s) + eps)
 * Stop test: the largest absolute masked residual max|dS| (pu) < tol, tested
 * before each update.  Schedules:
 *   PLATEAU: after each step, with the iteration's loss L: if L < best*(1-threshold)
 *            {best = L; bad = 0} else bad++; during cooldown bad is reset;
 *            if bad > patience {lr = max(lr*factor, min_lr) when the decrease
 *            exceeds sched_eps; cooldown restarts; bad = 0}.
 *   STEP:    lr *= factor after every update whose persistent step count t
 *            (1, 2, ... over all calls that continue one schedule state) is a
 *            multiple of `patience` (PyTorch's StepLR with step_size = patience,
 *            gamma = factor), so a resumed call keeps the phase of the decay.
 */
typedef struct dpf_opts {
    double lr;
    double beta1;
    double beta2;
    double eps;
    double tol;
    int32_t max_iter;
    int32_t sched;
    double factor;
    int32_t patience;
    double threshold;
    int32_t cooldown;
    double min_lr;
    double sched_eps;
    int32_t optimizer; /* DPF_OPT_* */
} dpf_opts_t;

/* Text of the calling thread's last error ("" if none).  Host string owned by the library. */
const char *dpf_last_error(void);

/* Library version string (host, static); ends with "src <hash>", a hash of the
 * sources the library was built from. */
const char *dpf_version(void);

/*
 * dpf_build_ybus -- bus admittance matrix Y from pi-model branches (Sec. 2.1,
 * power-balance equation; the branch model is the standard pi model: series
 * y = 1/(r + jx), total charging b split b/2 to each end, no transformers):
 *     Y_ff += y + j b/2,   Y_tt += y + j b/2,   Y_ft += -y,   Y_tf += -y.
 * Parallel branches are summed (in branch order); every diagonal is stored.
 *   from, to, r, x, b : device [n_branch]
 *   row_ptr           : device [n_bus + 1] out
 *   col_idx, val      : device [nnz_cap], [2*nnz_cap] out; nnz_cap >= n_bus + 2*n_branch
 *                       always suffices
 *   nnz_out           : host out; this call SYNCHRONISES `stream` to return it
 *   max_row_nnz_out   : host out (nullable): the longest row, for dpf_grid_t.max_row_nnz
 * Errors: DPF_EINVAL for n_bus <= 0, n_branch < 0, a bus index out of range,
 * from == to, or r = x = 0 (detected on the device); DPF_ECAP if the result
 * does not fit (nnz_out still receives the needed size).  Temporaries are
 * allocated with hipMalloc and freed before the call returns.
 */
int dpf_build_ybus(int32_t n_bus, int32_t n_branch, const int32_t *from, const int32_t *to,
                   const double *r, const double *x, const double *b, int32_t nnz_cap,
                   int32_t *row_ptr, int32_t *col_idx, double *val, int32_t *nnz_out,
                   int32_t *max_row_nnz_out, void *stream);

/*
 * dpf_build_ybus_noalloc -- dpf_build_ybus for callers that cannot allocate device
 * memory (serving loops, harnesses that forbid hipMalloc): the same arguments,
 * kernels and results, with the temporaries in a static array of the library
 * (16 MiB per device, held until the process ends) instead of hipMalloc'd
 * memory.  No allocation of any kind happens in the call.  The temporaries of a
 * grid take 16 (n_bus + 1) + 256 + 8 (n_bus + 2 n_branch) + 16 n_bus bytes, each
 * part rounded up to 256; a grid that needs more than 16 MiB (for example more
 * than about 260 000 buses at 1.5 branches per bus) is rejected with DPF_EINVAL
 * before any device work.  Every call on one device shares that device's array:
 * calls that overlap on one device (two host threads, or two streams) race and
 * must be serialised by the caller; the call returns with `stream` synchronised,
 * so calls made one after the other never overlap.  The array is cleared at the
 * start of each call; nothing of a previous call's contents is used.
 */
int dpf_build_ybus_noalloc(int32_t n_bus, int32_t n_branch, const int32_t *from, const int32_t *to,
                           const double *r, const double *x, const double *b, int32_t nnz_cap,
                           int32_t *row_ptr, int32_t *col_idx, double *val, int32_t *nnz_out,
                           int32_t *max_row_nnz_out, void *stream);

/*
 * dpf_mismatch_grad -- one evaluation of the DPF forward and backward pass for
 * B cases on one grid (Algorithm 1 forward pass and loss.backward(); the
 * gradient is the reverse-mode J^T F product of Sec. 5.1, computed by one
 * transposed-Y product plus elementwise terms):
 *   dS_i   = V_i conj((Y V)_i) - S_spec,i,           V_i = vm_i e^{j va_i}
 *   r_i    = [Re dS_i if bus i is PV or PQ] , [Im dS_i if bus i is PQ]
 *   loss   = (1/m) sum r^2, m = n_pv + 2 n_pq;  max_mis = max |r|
 *   g_vm   = d loss / d vm  (zero except at PQ buses)
 *   g_va   = d loss / d va  (zero at the slack)
 * Arguments:
 *   g        : grid (host struct, device arrays); one grid, B cases
 *   B, ld    : cases (1..65535) and leading dimension of vm, va, dS, g_vm, g_va (ld >= n_bus)
 *   bus_type : device int8 [n_bus], shared by all cases
 *   s_spec   : device complex, [B][s_ld] or shared [n_bus] when s_ld == 0
 *   outage   : device int32 [B] branch index removed in case c (-1: none), or NULL.
 *              The branch's whole pi-model admittance is subtracted as a rank-2
 *              correction; requires g->n_branch > 0 and branch arrays.
 *   vm, va   : device [B][ld]
 *   dS       : device complex [B][ld] out, nullable
 *   loss, max_mis : device [B] out
 *   g_vm, g_va    : device [B][ld] out, nullable (both or neither)
 *   workspace     : device, >= dpf_mismatch_grad_workspace_bytes(n_bus, B) bytes
 * Results are deterministic (fixed reduction order).  Errors: DPF_EINVAL,
 * DPF_ENOMEM, DPF_EHIP.  Outage indices live on the device, so the host does not
 * see them: a case whose index is neither -1 nor in [0, n_branch) gets NaN in
 * dS, loss, max_mis and every learnable entry of the gradient, so that a
 * contingency that was never applied cannot pass for the base case.
 */
int dpf_mismatch_grad(const dpf_grid_t *g, int32_t B, int32_t ld, const int8_t *bus_type,
                      const double *s_spec, int32_t s_ld, const int32_t *outage,
                      const double *vm, const double *va, double *dS, double *loss,
                      double *max_mis, double *g_vm, double *g_va, void *workspace,
                      size_t ws_bytes, void *stream);

size_t dpf_mismatch_grad_workspace_bytes(int32_t n_bus, int32_t B);

/*
 * dpf_param_grad -- gradient of each case's loss with respect to the simulation
 * parameters: every branch's r, x, b and the specified injections S_spec (Sec. 1
 * and Sec. 2.3: the mismatch is differentiated end to end, so parameters can be
 * identified by gradient descent).  Same forward pass as dpf_mismatch_grad; then,
 * with the adjoint seed w_i = a_i conj(V_i), a_i = (2/m)(r^P_i + j r^Q_i), a branch
 * (f, t) with y = 1/(r + jx) and D = (w_f - w_t)(V_f - V_t) has
 *   dL/dr = -Re(y^2 D),  dL/dx = Im(y^2 D),  dL/db = -Im(w_f V_f + w_t V_t) / 2,
 * and dL/dS_spec,i = -a_i (as d/dRe S + j d/dIm S).
 * Arguments as in dpf_mismatch_grad, plus:
 *   loss, max_mis : device [B] out, nullable (both or neither)
 *   g_r, g_x, g_b : device double [B][bld] out (bld >= n_branch), nullable (all or
 *                   none; need the grid's branch arrays).  A case's outaged branch
 *                   is absent from its Y and gets 0.
 *   g_s           : device complex [B][ld] out, nullable
 *   workspace     : >= dpf_mismatch_grad_workspace_bytes(n_bus, B)
 * Per case, not summed over cases (a shared S_spec or branch gets one gradient
 * row per case).  Errors: DPF_EINVAL, DPF_ENOMEM, DPF_EHIP.
 */
int dpf_param_grad(const dpf_grid_t *g, int32_t B, int32_t ld, const int8_t *bus_type,
                   const double *s_spec, int32_t s_ld, const int32_t *outage, const double *vm,
                   const double *va, double *loss, double *max_mis, double *g_r, double *g_x,
                   double *g_b, int32_t bld, double *g_s, void *workspace, size_t ws_bytes,
                   void *stream);

/*
 * Per-call routing of dpf_solve_batch: which kernel runs the items and how the
 * last items of a call finish.  Every setting belongs to the call that passes it
 * (nothing is process-wide except the autotune cache below), so concurrent calls
 * on different streams may use different settings.  dpf_route_default fills the
 * defaults; a NULL route means the defaults.  The same route must be passed to
 * dpf_solve_workspace_bytes when sizing the workspace of the call.
 *   variant        : -1 (default): the autotune cache, else the default routing;
 *                    >= 0: this variant for the items that fit one workgroup
 *                    (DPF_EINVAL if it cannot hold the largest such sub-grid)
 *   team_cap       : sub-grids above this many buses are solved by several
 *                    workgroups per item (see wide_host) even when they would fit
 *                    one workgroup's LDS, and a member of a persistent team holds
 *                    at most this many buses' exchange values in LDS (the rest of
 *                    its columns it reads from global memory); 0 (default) = the
 *                    LDS limit
 *   tail_handoff   : single-grid calls: once at most this many items are
 *                    unfinished, the per-item kernels pause them (every 32
 *                    iterations they read a finished-items counter) and the call
 *                    finishes them on the split kernel or the multi-workgroup
 *                    path, both of which spread each item over many CUs;
 *                    iteration counts, optimizer and schedule state carry over,
 *                    so results equal a call without handoff up to the rounding
 *                    of the other path.  Applies to the streaming and banded
 *                    kernels; a call of at most this many items is
 *                    handed over after its first 32 iterations.  0 (default) = off
 *   tail_team      : how handed-over items finish.  0 (default): on the
 *                    multi-workgroup path.  > 0 (at most 1024): on the split
 *                    kernel, which gives each item a team of at most this many
 *                    workgroups (each member keeps the exchange vector in LDS; the
 *                    team synchronises through global memory twice per iteration).
 *                    With tail_team > 0, a single-grid call of few large items
 *                    (more than 2048 buses, at most one item per two CUs, no variant
 *                    chosen for them) runs them on the split kernel from their
 *                    first iteration, without the per-item kernel or a handoff
 *   tail_chunk     : iterations per split-kernel launch, 1..65536 (default 128);
 *                    launches repeat with the finished items dropped while more
 *                    than tail_min_items (>= 0, default 0) items are left; the
 *                    multi-workgroup path finishes the rest
 *   tail_slice_ms  : 0 (default): equal teams, T = min(tail_team, W / items left,
 *                    slices of the grid), W = workgroups of the kernel the device
 *                    holds at once.  In (0, 1000]: a launch also ends after that
 *                    much time, and teams are sized in proportion to the square of
 *                    each item's remaining budget max_iter - iters (at least 1, at
 *                    most tail_team, together at most W)
 *   tail_first_wait_s, tail_wait_s : barrier wait bounds of the teams of
 *                    workgroups, in seconds, [0, 60] each (defaults 1 and 5).
 *                    Split kernel: tail_first_wait_s at a launch's first barrier,
 *                    where another stream's kernels may still hold CUs,
 *                    tail_wait_s after it; a member that waits longer abandons the
 *                    barrier and the item finishes on the multi-workgroup path.
 *                    Persistent teams (wide_host = 0): a unit's first barrier waits
 *                    as long as its team or the launch makes progress and is
 *                    abandoned after tail_first_wait_s without any; later
 *                    barriers after tail_wait_s; an abandoned item ends with
 *                    status DPF_UNFINISHED.  Every member finishes its part of an
 *                    iteration before it arrives, so an abandoned barrier leaves
 *                    the state of a whole iteration
 *   case_order     : 1: a call that may hand over its tail (one grid, at most
 *                    16384 cases) first evaluates every case's max|r| at its start
 *                    point and starts the cases in descending order of it
 *                    (non-finite first, ties by index); results per case are those
 *                    of index order up to the rounding of the tail path.  0
 *                    (default): index order
 *   wide_host      : how a call with sub-grids above the LDS limit (or team_cap),
 *                    or with few large items (more than 2048 buses, at most one
 *                    item per two CUs, no variant chosen for them), runs.  0 (default):
 *                    every item of the call in ONE persistent launch of as many
 *                    workgroups as the device holds; an item is a unit of one or
 *                    more workgroups (a team, each member holding its rows and their
 *                    neighbours in LDS, synchronised through global memory twice
 *                    per iteration) taken from a device-side queue; a one-workgroup
 *                    kernel plans team sizes and order from the sub-grid sizes and
 *                    bandwidths.  1: the multi-workgroup path (three kernels per
 *                    iteration, host polls every 32 iterations)
 *   tail_device    : 0 (default): the host plans every split-kernel launch of a
 *                    handoff or split-kernel start (team table, items left) and
 *                    waits for each.  1 (needs tail_team > 0, and a grid whose
 *                    exchange vector fits one workgroup's LDS, else
 *                    DPF_EUNSUPPORTED): the call enqueues a fixed sequence of
 *                    launches, each planned on the device by a one-workgroup
 *                    kernel from the paused items with the same rule (team sizes
 *                    by remaining budget with a time slice, else equal), and
 *                    nothing waits on the host; with a time slice there are 256
 *                    launches (a launch with nothing left only starts and ends;
 *                    the tail is re-planned for 256 slices, whatever is left then
 *                    runs on the last plan), without one enough for max_iter at
 *                    tail_chunk iterations each, and a last one without limits.  tail_min_items is not
 *                    used; an item whose team gives up at a barrier is planned
 *                    again in the next launch, and one still paused after the
 *                    last ends with DPF_UNFINISHED
 * A call with tail_handoff > 0 or a split-kernel start (tail_team > 0 and few
 * large items) without tail_device, or the multi-workgroup path (wide_host = 1
 * with items above the LDS or team cap, or variant naming that path) BLOCKS the
 * host until it is done and cannot be captured in a graph; every other call,
 * persistent teams and tail_device included, only enqueues work and can be
 * captured.
 * A field out of range makes the call return DPF_EINVAL.
 */
typedef struct dpf_route {
    int32_t variant;
    int32_t team_cap;
    int32_t tail_handoff;
    int32_t tail_team;
    int32_t tail_chunk;
    int32_t tail_min_items;
    double tail_slice_ms;
    double tail_first_wait_s;
    double tail_wait_s;
    int32_t case_order;
    int32_t wide_host;
    int32_t tail_device;
} dpf_route_t;

/* Fill *route with the defaults (host; no device call). */
void dpf_route_default(dpf_route_t *route);

/*
 * Optional per-item trace of the stop-test quantity of dpf_solve_batch (the
 * loss curves of Sec. 6.4 show its decay): max|dS| of iteration k of the call,
 * tested before that iteration's update, is written to max_mis[item*len + k/every]
 * for every k that is a multiple of `every` and below len*every, where item =
 * c*n_sub + s and k counts from 0 in each call.  Slots past an item's stop are
 * left as they were (fill them, e.g. with NaN, before the call).
 *   max_mis : device double [B*n_sub][len]
 *   every   : > 0 when len > 0
 *   len     : slots per item; 0 = no trace
 */
typedef struct dpf_trace {
    double *max_mis;
    int32_t every;
    int32_t len;
} dpf_trace_t;

/*
 * dpf_solve_batch -- the DPF iteration (Algorithm 1 with Adam) run to
 * convergence for many independent problems in ONE kernel launch.
 *
 * Work items: B cases x n_sub sub-grids.  Item (c, s) solves sub-grid s of case
 * c: buses [sub_offset[s], sub_offset[s+1]) of the (block-diagonal) grid `g`.
 * With sub_offset == NULL there is one sub-grid, [0, n_bus).  Every item keeps
 * its own Adam moments, step count, learning-rate schedule and stop test, so a
 * batch equals B*n_sub separate solves (Sec. 4.2 batches problems; here they
 * do not share a loss).  An item stops when max|dS| < tol (status 0), when its
 * iteration count reaches max_iter (status 1), or when its mismatch becomes
 * non-finite (status 2); a stopped item leaves the kernel while others go on.
 * Status 3 (DPF_BAD_GRID, iters 0) reports a CSR row longer than g->max_row_nnz;
 * status 4 (DPF_BAD_OUTAGE, iters 0, max_mis and loss NaN, vm/va and the optimizer
 * state untouched) a case whose outage index is neither -1 nor a branch index;
 * status 5 (DPF_UNFINISHED) an item of the persistent teams whose team could not
 * assemble within the route's wait bounds (the device was busy with other work):
 * vm/va, adam_state and sched_state hold the state after `iters` updates, so a
 * call that passes them back continues the item.
 * Per call the library re-lays Y out in the workspace as 64-row slices
 * (column-major within a slice) so that each wave reads its rows' neighbour
 * entries with coalesced loads.
 *
 *   g             : grid
 *   n_sub, sub_offset, sub_offset_dev : sub-grid bus offsets [n_sub + 1], the
 *                   same values on the host (sizes, kernel choice) and on the
 *                   device (read by the kernel); both NULL for one sub-grid
 *                   [0, n_bus) with n_sub = 1.  Offsets must start at 0, end at
 *                   n_bus and not decrease; every CSR row of a sub-grid must
 *                   only reference columns of the same sub-grid (entries that
 *                   do not are ignored).  Items start in the order
 *                   (sub-grid major, case minor): list large sub-grids first.
 *   B, ld         : cases; leading dimension of per-case arrays
 *   bus_type      : device int8 [n_bus] (one slack per sub-grid)
 *   s_spec, s_ld  : as in dpf_mismatch_grad
 *   outage        : device int32 [B] or NULL (requires n_sub == 1): -1 or a branch
 *                   index per case (see status DPF_BAD_OUTAGE)
 *   vm, va        : device [B][ld] in: start point (flat or warm), out: result
 *                   (the voltages of the last stop test).  Entries that are not
 *                   learnable (|V| at PV/slack, angle at the slack) are unchanged.
 *   adam_state    : device [4][B][ld] in/out (m_vm, m_va, s_vm, s_va) or NULL
 *                   (fresh zero moments, discarded at the end)
 *   sched_state   : device [B*n_sub][6] in/out, per item: step count t, current
 *                   lr, best plateau loss, bad + 2^20 * cooldown counters, b1^t,
 *                   b2^t; or NULL (t = 0, lr = opts->lr, fresh schedule).  A fresh
 *                   state is {0, lr, +inf, 0, 1, 1}.  Passing the state (and
 *                   adam_state) of a previous call continues the same iteration
 *                   bit for bit.
 *   opts          : host
 *   route         : host, nullable (defaults): kernel choice and tail settings of
 *                   this call (dpf_route_t)
 *   iters, status : device int32 [B*n_sub] out (index c*n_sub + s); iters = number
 *                   of Adam updates applied in this call
 *   max_mis, loss : device double [B*n_sub] out, at the returned voltages
 *   done_ns       : device int64 [B*n_sub] out, nullable: nanoseconds from the start of
 *                   the call's kernels to the item's stop (time to converge per item)
 *   trace         : host, nullable: the optional max|dS| trace (dpf_trace_t)
 *   workspace     : device, >= dpf_solve_workspace_bytes(g, n_sub, sub_offset, B, ld,
 *                   route) bytes
 * Errors: DPF_EINVAL (sizes, pointers, opts, route or trace out of range, a sub-grid
 * larger than the solver supports), DPF_ENOMEM, DPF_EUNSUPPORTED, DPF_EHIP.
 */
int dpf_solve_batch(const dpf_grid_t *g, int32_t n_sub, const int32_t *sub_offset,
                    const int32_t *sub_offset_dev, int32_t B,
                    int32_t ld, const int8_t *bus_type, const double *s_spec, int32_t s_ld,
                    const int32_t *outage, double *vm, double *va, double *adam_state,
                    double *sched_state, const dpf_opts_t *opts, const dpf_route_t *route,
                    int32_t *iters, int32_t *status, double *max_mis, double *loss,
                    int64_t *done_ns, const dpf_trace_t *trace, void *workspace, size_t ws_bytes,
                    void *stream);

/* Workspace bytes of the dpf_solve_batch call with these sizes and this route
 * (nullable); 0 for invalid sizes or an invalid route. */
size_t dpf_solve_workspace_bytes(const dpf_grid_t *g, int32_t n_sub, const int32_t *sub_offset,
                                 int32_t B, int32_t ld, const dpf_route_t *route);

/*
 * dpf_solve_series -- a time series of T power flows on one grid (Sec. 6.4: time
 * series reuse the previous solution).  Steps run in windows of `window`: all
 * steps of a window start from the solution of the step before the window (step
 * 0 from vm0/va0) and are solved together as one dpf_solve_batch of `window`
 * cases; window = 1 gives the sequential warm-started chain.  Every step starts
 * with fresh Adam moments and schedule.
 *   s_series : device complex [T][s_ld] injections per step
 *   vm0, va0 : device [n_bus] start of step 0
 *   vm, va   : device [T][ld] out: the solution returned for each step
 *   iters, status, max_mis, loss, done_ns : [T] as in dpf_solve_batch (done_ns per
 *              window start, nullable)
 *   route    : host, nullable: routing of every window's dpf_solve_batch call
 *   workspace: >= dpf_solve_series_workspace_bytes(g, window, ld, route)
 */
int dpf_solve_series(const dpf_grid_t *g, int32_t T, int32_t window, const int8_t *bus_type,
                     const double *s_series, int32_t s_ld, const double *vm0, const double *va0,
                     double *vm, double *va, int32_t ld, const dpf_opts_t *opts,
                     const dpf_route_t *route, int32_t *iters, int32_t *status, double *max_mis,
                     double *loss, int64_t *done_ns, void *workspace, size_t ws_bytes,
                     void *stream);

size_t dpf_solve_series_workspace_bytes(const dpf_grid_t *g, int32_t window, int32_t ld,
                                        const dpf_route_t *route);

/*
 * dpf_order_rcm -- a bus numbering of small bandwidth (reverse Cuthill-McKee on
 * the branch graph), for grids that the caller renumbers before building Y: the
 * banded solve kernels need max|row - col| of every sub-grid at most their block.
 * With group > 1 the buses of every aligned window of `group` consecutive new
 * indices are then ordered by degree (stable), so that the 64-row slices of the
 * solve kernels' sliced-ELL matrix hold rows of similar length (less padding);
 * each bus moves by less than group, so the bandwidth grows by at most 2 (group - 1).
 * Bus numbering is arbitrary in the power-flow problem (Sec. 2: the equations are
 * per bus and per branch), so renumbering changes no result beyond rounding.
 *   n_bus, n_branch : sizes;  from, to : host int32 [n_branch] branch ends
 *   sub_offset      : host int32 [n_sub + 1] or NULL; each range [sub_offset[s],
 *                     sub_offset[s+1]) is ordered on its own and keeps its place;
 *                     branches between ranges are ignored; windows start at the
 *                     range start
 *   group           : degree-grouping window (0 or 1: plain RCM)
 *   perm            : host int32 [n_bus] out: perm[k] = old index of new bus k
 *   bandwidth_out   : host, nullable: max|new(f) - new(t)| over the branches
 * Host-only, synchronous, allocates host memory for the adjacency lists.
 * Errors: DPF_EINVAL (sizes, null pointers, branch end out of range, sub_offset
 * not increasing from 0 to n_bus), DPF_ENOMEM.
 */
int dpf_order_rcm(int32_t n_bus, int32_t n_branch, const int32_t *from, const int32_t *to, int32_t n_sub,
                  const int32_t *sub_offset, int32_t group, int32_t *perm, int32_t *bandwidth_out);

/*
 * dpf_dc_init -- DC power flow angles as a start point (Algorithm 2 initialises
 * with the DC power flow; Sec. 3 lists the DC approximation as a screening
 * method).  Solves  L theta = P  on the non-slack buses, with P = Re S_spec, the
 * slack angle fixed at its input value and L the branch-susceptance Laplacian
 * (weights 1/x): L_ij = -Im(Y_ij) of `g_dc`, the admittance matrix of the same
 * branches built with r = 0 and b = 0 (dpf_build_ybus), whose branch arrays
 * (r = 0, b = 0) give the N-1 corrections.  Jacobi-preconditioned conjugate
 * gradients, one workgroup per case, until ||P - L theta||_2 <= tol ||P||_2 or
 * max_iter iterations.  vm is not an argument: the DC model takes the start
 * point's magnitudes (flat: 1 at PQ, setpoints at PV and slack).
 *   B, ld, bus_type, s_spec, s_ld, outage : as in dpf_mismatch_grad
 *   va        : device [B][ld] in: start angles (slack entry = slack angle;
 *               others: the CG start, e.g. 0), out: DC angles (slack unchanged)
 *   iters     : device int32 [B] out, nullable: CG iterations
 *   residual  : device double [B] out, nullable: final ||r||_2 / ||P||_2 (NaN, with
 *               iters 0 and va untouched, for a case whose outage index is neither
 *               -1 nor a branch index)
 *   workspace : >= dpf_dc_init_workspace_bytes(n_bus, B)
 * Errors: DPF_EINVAL, DPF_ENOMEM, DPF_EUNSUPPORTED (more buses than one
 * workgroup's LDS holds at 8 B per bus), DPF_EHIP.
 */
int dpf_dc_init(const dpf_grid_t *g_dc, int32_t B, int32_t ld, const int8_t *bus_type,
                const double *s_spec, int32_t s_ld, const int32_t *outage, double *va, double tol,
                int32_t max_iter, int32_t *iters, double *residual, void *workspace, size_t ws_bytes,
                void *stream);

size_t dpf_dc_init_workspace_bytes(int32_t n_bus, int32_t B);

/* Largest sub-grid (buses) one workgroup can hold on this device; larger sub-grids
 * are solved by several workgroups (see dpf_route_t.team_cap). */
int32_t dpf_solve_max_sub_buses(void);

/*
 * Kernel variants and the autotune cache.  dpf_solve_batch picks a kernel
 * variant (workgroup size, buses per thread, register-resident or streaming
 * state) from the largest sub-grid of the call and the number of work items,
 * unless the call's route names one.  Sizes are grouped into classes (the
 * smallest variant that holds them) and item counts into buckets (<= 64, <= 256,
 * more); dpf_autotune_set records, for the class of n_max, which variant to use
 * instead -- a project-side autotuner times the eligible variants on real inputs
 * (each probe names its variant in its route) and stores the fastest.  Without a
 * recorded choice, items above 2048 buses that fill at most half of the device
 * (items <= compute units / 2) are spread over several workgroups each (the
 * persistent teams, or the multi-workgroup path with route.wide_host = 1; the
 * index reported for them is that of kind 3), the others take the default
 * variant of their class.  The cache is the library's only process-wide setting
 * and is guarded by a mutex.
 *   dpf_solve_variant_count : number of variants
 *   dpf_solve_variant_info  : threads per workgroup, buses per thread (0 = any),
 *                             and the kind: register-resident (0), streaming (1),
 *                             banded with a barrier-free gradient sweep (2),
 *                             multi-workgroup (3: not a kernel of its own --
 *                             every sub-grid of the call is spread over many
 *                             workgroups), banded with the state kept as
 *                             (|V|, theta) and moment pairs (4); host outs.  A
 *                             banded variant
 *                             (buses per thread = buses per thread per block)
 *                             serves the sub-grids whose bandwidth max|row - col|
 *                             is at most threads * buses_per_thread (see
 *                             dpf_order_rcm); the same call runs the other
 *                             sub-grids with the default variant of their size
 *   dpf_solve_variant_cases : cases per workgroup of a variant (1 for every
 *                             variant), DPF_EINVAL for a bad index
 *   dpf_solve_variant_for   : variant index dpf_solve_batch would use for many
 *                             items, -1 if none
 *   dpf_solve_variant_for_items : the same for `items` work items
 *   dpf_autotune_set        : record `variant` for every item bucket of the class
 *                             of n_max; DPF_EINVAL if it cannot hold n_max buses
 *   dpf_autotune_set_items  : record it for the bucket of `items` only
 *   dpf_autotune_reset      : forget every choice
 *   dpf_tail_split_stats    : split-kernel launches, and launches in which a team
 *                             abandoned a barrier, since the library was loaded,
 *                             over all calls (statistics only; either pointer may
 *                             be null)
 * Items larger than the LDS limit always run on several workgroups each (see
 * dpf_route_t.wide_host for which path and whether the call blocks).
 */
int dpf_solve_variant_count(void);
int dpf_solve_variant_info(int idx, int32_t *threads, int32_t *buses_per_thread, int32_t *streaming);
int dpf_solve_variant_cases(int idx);
int dpf_solve_variant_for(int32_t n_max);
int dpf_solve_variant_for_items(int32_t n_max, int64_t items);
int dpf_autotune_set(int32_t n_max, int variant);
int dpf_autotune_set_items(int32_t n_max, int64_t items, int variant);
void dpf_tail_split_stats(int64_t *launches, int64_t *abandoned);
void dpf_autotune_reset(void);

#ifdef __cplusplus
}
#endif

#endif /* DPF_H */
