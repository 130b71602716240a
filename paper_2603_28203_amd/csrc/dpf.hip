// libdpf: C ABI entry points (include/dpf.h) and the host side of the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dpf.h"
#include "common.hpp"
#include "dc.hpp"
#include "eval.hpp"
#include "pair.hpp"
#include "sell.hpp"
#include "solve.hpp"
#include "split.hpp"
#include "teams.hpp"
#include "wide.hpp"
#include "ybus.hpp"

namespace {

static_assert(dpf::kPaused != DPF_CONVERGED && dpf::kPaused != DPF_MAX_ITER && dpf::kPaused != DPF_NONFINITE &&
                  dpf::kPaused != DPF_BAD_GRID && dpf::kPaused != DPF_BAD_OUTAGE &&
                  dpf::kPaused != DPF_UNFINISHED,
              "the internal paused status must differ from every public status code");

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define DPF_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(DPF_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Temporaries of dpf_build_ybus_noalloc: one array per device, kept for the life
// of the process.  Host code uses the address hipGetSymbolAddress returns for the
// current device (DeviceInfo::ybus_scratch), never the name itself.
constexpr size_t kYbusScratchBytes = (size_t)16 << 20;
__device__ __align__(256) char scratch[kYbusScratchBytes];

// Progress count of the persistent teams, one per device and shared by every
// launch on it (a team waiting for members held by another launch sees that
// launch's progress); only ever incremented and compared for change.
__device__ int32_t team_progress;

// Per-device limits, queried once per device.
struct DeviceInfo {
    int lds_per_block = 0;  // bytes
    int n_cu = 0;
    double ns_per_tick = 10.0;  // wall-clock counter period
    bool ok = false;
    hipStream_t side = nullptr;      // stream of the multi-workgroup path
    hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_poll = nullptr;
    int32_t *pinned_count = nullptr; // host-pinned poll target (two words)
    void *ybus_scratch = nullptr;    // this device's copy of `scratch`
    int32_t *team_progress = nullptr;  // this device's copy of `team_progress`
    int index = 0;
};
std::mutex g_dev_mu;
DeviceInfo g_dev[64];
// the side stream, its events and the poll word are per device: calls that use them
// (multi-workgroup items, tail handoff) hold this lock while they do
std::mutex g_side_mu[64];

int device_info(DeviceInfo &out) {
    int dev = 0;
    DPF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(DPF_EHIP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (!g_dev[dev].ok) {
        int lds = 0, ncu = 0;
        DPF_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        DPF_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        g_dev[dev].lds_per_block = lds;
        g_dev[dev].n_cu = ncu;
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            g_dev[dev].ns_per_tick = 1e6 / (double)khz;
        DPF_HIP(hipStreamCreateWithFlags(&g_dev[dev].side, hipStreamNonBlocking));
        DPF_HIP(hipEventCreateWithFlags(&g_dev[dev].ev_in, hipEventDisableTiming));
        DPF_HIP(hipEventCreateWithFlags(&g_dev[dev].ev_out, hipEventDisableTiming));
        DPF_HIP(hipEventCreateWithFlags(&g_dev[dev].ev_poll, hipEventDisableTiming));
        DPF_HIP(hipHostMalloc((void **)&g_dev[dev].pinned_count, 2 * sizeof(int32_t), hipHostMallocDefault));
        DPF_HIP(hipGetSymbolAddress((void **)&g_dev[dev].ybus_scratch, HIP_SYMBOL(scratch)));
        DPF_HIP(hipGetSymbolAddress((void **)&g_dev[dev].team_progress, HIP_SYMBOL(team_progress)));
        g_dev[dev].index = dev;
        g_dev[dev].ok = true;
    }
    out = g_dev[dev];
    return DPF_OK;
}

constexpr int kGfx950LdsBytes = 160 * 1024;  // LDS per workgroup on gfx950

// Bytes of static LDS the solve kernels use besides the dynamic exchange array.
constexpr int kSolveStaticLds = 2 * (1024 / dpf::kWave) * 8 + 256;

std::atomic<int64_t> g_split_launches{0}, g_split_abandoned{0};  // statistics since the library was loaded

dpf_route_t default_route() {
    dpf_route_t r;
    r.variant = -1;
    r.team_cap = 0;
    r.tail_handoff = 0;
    r.tail_team = 0;
    r.tail_chunk = 128;
    r.tail_min_items = 0;
    r.tail_slice_ms = 0.0;
    r.tail_first_wait_s = 1.0;
    r.tail_wait_s = 5.0;
    r.case_order = 0;
    r.wide_host = 0;
    r.tail_device = 0;
    return r;
}

dpf_route_t route_of(const dpf_route_t *r) { return r ? *r : default_route(); }

const char *route_error(const dpf_route_t &r) {
    if (r.variant < -1) return "route.variant must be -1 or a variant index";
    if (r.team_cap < 0) return "route.team_cap must be >= 0";
    if (r.tail_handoff < 0) return "route.tail_handoff must be >= 0";
    if (r.tail_team < 0 || r.tail_team > 1024) return "route.tail_team must be in [0, 1024]";
    if (r.tail_chunk < 1 || r.tail_chunk > 65536) return "route.tail_chunk must be in [1, 65536]";
    if (r.tail_min_items < 0) return "route.tail_min_items must be >= 0";
    if (!(r.tail_slice_ms >= 0.0 && r.tail_slice_ms <= 1000.0)) return "route.tail_slice_ms must be in [0, 1000]";
    if (!(r.tail_first_wait_s >= 0.0 && r.tail_first_wait_s <= 60.0) || !(r.tail_wait_s >= 0.0 && r.tail_wait_s <= 60.0))
        return "route wait bounds must be in [0, 60] s";
    if (r.case_order < 0 || r.case_order > 1) return "route.case_order must be 0 or 1";
    if (r.wide_host < 0 || r.wide_host > 1) return "route.wide_host must be 0 or 1";
    if (r.tail_device < 0 || r.tail_device > 1) return "route.tail_device must be 0 or 1";
    if (r.tail_device == 1 && r.tail_team == 0) return "route.tail_device needs route.tail_team > 0";
    return nullptr;
}

int32_t max_sub_buses_for(const DeviceInfo &d, int32_t team_cap) {
    int32_t cap = (d.lds_per_block - kSolveStaticLds) / 16;
    cap = std::min<int32_t>(cap, 10 * 1024);
    return team_cap > 0 ? std::min(cap, team_cap) : cap;
}

// ---------------------------------------------------------------- solve variants

using KernelFn = void (*)(dpf::SolveArgs);

struct Variant {
    int nt;
    int k;
    int mode;
    KernelFn fn;
};

template <int NT, int K>
Variant make_variant() {
    return Variant{NT, K, dpf::kReg, dpf::team_solve_kernel<NT, K, dpf::kReg>};
}
// any number of buses per thread (k = 0)
template <int NT>
Variant make_stream_variant() {
    return Variant{NT, 0, dpf::kGlobal, dpf::team_solve_stream_kernel<NT>};
}
// banded, barrier-free gradient sweep (k = J buses per thread per block)
template <int NT, int J>
Variant make_band_variant() {
    return Variant{NT, J, dpf::kBandStream, dpf::team_solve_band_kernel<NT, J>};
}
// the same with the state in (|V|, theta) and moment pairs
template <int NT, int J>
Variant make_pair_variant() {
    return Variant{NT, J, dpf::kPair, dpf::team_solve_pair_kernel<NT, J>};
}


// Register-resident variants up to 2048 buses per item, the 1024-thread streaming
// variant above (any size).  The banded variants (k = buses per thread per block)
// serve sub-grids whose bandwidth is at most threads * k; the others go to the
// default variant of the size in the same call.  The last entry is not a
// workgroup-per-item kernel: it sends every sub-grid of the call to the
// multi-workgroup path, which spreads one item over many CUs.  Kinds measured and
// retired as dominated on every workload timed (64 to 4096 cases of 300 to 9241
// buses): streaming kernels of 512 threads holding exchange values in registers,
// banded kernels with a pipelined gradient sweep, windowed kernels (rings of
// blocks in LDS) and their batched form (several cases per workgroup).
const Variant *variant_table(int *count) {
    static const Variant table[] = {
        make_variant<64, 1>(),          make_variant<128, 1>(),       make_variant<256, 1>(),
        make_variant<256, 2>(),         make_variant<512, 2>(),       make_variant<512, 3>(),
        make_variant<512, 4>(),         make_stream_variant<1024>(),  make_band_variant<1024, 2>(),
        make_band_variant<1024, 4>(),   make_pair_variant<1024, 4>(), make_pair_variant<1024, 2>(),
        Variant{0, 0, dpf::kWide, nullptr},
    };
    *count = (int)(sizeof(table) / sizeof(table[0]));
    return table;
}

bool variant_fits(const Variant &v, int32_t n_max) {
    return dpf::is_banded(v.mode) || v.mode == dpf::kWide || v.k == 0 || (int64_t)n_max <= (int64_t)v.nt * v.k;
}

// Autotune cache: (size class = index of the default variant, number-of-items
// bucket) -> chosen variant.  Items buckets: <= 64, <= 256, more.
constexpr int kItemBuckets = 3;
std::mutex g_tune_mu;
int g_tune[64][kItemBuckets];
bool g_tune_init = false;

int items_bucket(int64_t items) { return items <= 64 ? 0 : (items <= 256 ? 1 : 2); }

// Items larger than this (buses) that fill at most half of the chip (2 items <= CUs)
// are solved faster spread over several workgroups than one workgroup each (measured
// on the persistent teams: 9241 buses, 64 cases, 38 against 68 us per iteration; 1354
// buses: one workgroup wins; 256 cases of 3000 buses, one per CU: the per-item
// streaming kernel, 29 against 39 us).
constexpr int32_t kWideDefaultBuses = 2048;

// first workgroup-per-item (non-banded) variant that holds n_max buses
int default_variant_index(int32_t n_max) {
    int cnt = 0;
    const Variant *t = variant_table(&cnt);
    for (int i = 0; i < cnt; ++i)
        if (!dpf::is_banded(t[i].mode) && t[i].mode != dpf::kWide && variant_fits(t[i], n_max)) return i;
    return -1;
}

int wide_variant_index() {
    int cnt = 0;
    variant_table(&cnt);
    return cnt - 1;
}

// forced >= 0: the call's route names the variant (nullptr if it cannot hold n_max).
// *few_large: the multi-workgroup path was chosen by default for few large items
// (not from the autotune cache or the route)
const Variant *pick_variant(int32_t n_max, int64_t items, int n_cu, int forced = -1, bool *few_large = nullptr) {
    int cnt = 0;
    const Variant *t = variant_table(&cnt);
    int d = default_variant_index(n_max);
    if (few_large) *few_large = false;
    if (d < 0) return nullptr;
    if (forced >= 0) return forced < cnt && variant_fits(t[forced], n_max) ? &t[forced] : nullptr;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        const int c = g_tune_init ? g_tune[d][items_bucket(items)] : -1;
        if (c >= 0 && c < cnt && variant_fits(t[c], n_max)) return &t[c];
    }
    if (n_max > kWideDefaultBuses && items <= n_cu / 2) {
        if (few_large) *few_large = true;
        return &t[wide_variant_index()];
    }
    return &t[d];
}

// How one call is split: sub-grids of at most `cap` buses run one workgroup per item
// with variant `v`; larger ones take the multi-workgroup path.
struct CallPlan {
    int32_t cap = 0;
    int32_t n_max = 0;  // largest sub-grid <= cap
    bool has_small = false;
    const Variant *v = nullptr;
    int32_t handoff = 0;  // tail handoff threshold for this call (0 = none)
    bool split_direct = false;  // every item on the split kernel from its first iteration
    bool teams = false;         // every item in one persistent launch of teams (teams.hpp)
    dpf_route_t route{};        // the call's settings
};

bool valid_opts(const dpf_opts_t *o) {
    if (!o) return false;
    if (!(o->lr >= 0.0) || !(o->beta1 >= 0.0 && o->beta1 < 1.0) || !(o->beta2 >= 0.0 && o->beta2 < 1.0))
        return false;
    if (!(o->eps >= 0.0) || !(o->tol >= 0.0) || o->max_iter < 0) return false;
    if (o->sched < DPF_SCHED_CONSTANT || o->sched > DPF_SCHED_STEP) return false;
    if (o->optimizer < DPF_OPT_ADAM || o->optimizer > DPF_OPT_RMSPROP) return false;
    if (o->sched != DPF_SCHED_CONSTANT && (!(o->factor >= 0.0) || o->patience < 0 || o->cooldown < 0))
        return false;
    return true;
}

bool valid_grid(const dpf_grid_t *g) {
    return g && g->n_bus > 0 && g->nnz >= 0 && g->row_ptr && g->col_idx && g->val;
}

struct SolveLayout {
    int32_t n_slices = 0;
    int32_t w_total = 0;  // slices of the wide sub-grids (per case)
    int64_t entries = 0;  // sliced-ELL entries (multiple of 64)
    size_t off_nslice = 0, off_slice_off = 0, off_width = 0, off_start = 0, off_col = 0, off_val = 0;
    size_t off_bw = 0, off_mom = 0, off_scr = 0, off_wcount = 0, off_woff = 0, off_mres = 0, off_part = 0,
           off_items = 0, off_list = 0, off_list2 = 0, off_sched = 0, off_bar = 0, off_tfirst = 0,
           off_order = 0;
    size_t off_thdr = 0, off_tunit = 0, off_tfirst2 = 0, off_tbar = 0, off_tpart = 0;  // persistent teams
    int32_t h_total = 0;  // tail handoff: slices of the (single) grid, 0 without handoff
    size_t total = 0;
};

static SolveLayout solve_layout(const dpf_grid_t *g, int32_t n_sub, const int32_t *sub_offset, int32_t B,
                                int32_t ld, bool streaming, int32_t team_cap, bool handoff = false,
                                bool pairs = false, bool teams = false) {
    SolveLayout L;
    int64_t team_part = 0;  // member partials: at most min(slices, members cap) per item
    for (int32_t s = 0; s < (sub_offset ? n_sub : 1); ++s) {
        int32_t ns = sub_offset ? sub_offset[s + 1] - sub_offset[s] : g->n_bus;
        L.n_slices += (ns + 63) / 64;
        if (ns > team_cap && !teams) L.w_total += (ns + 63) / 64;
        team_part += std::max<int64_t>(1, std::min<int64_t>((ns + 63) / 64, dpf::kTeamMaxMembers));
    }
    if (handoff) L.h_total = L.n_slices;
    const bool wide = L.w_total > 0 || handoff;
    streaming = streaming || teams;
    const int32_t part_slices = std::max(L.w_total, L.h_total);
    streaming = streaming || wide;
    int64_t wmax = g->max_row_nnz > 0 ? g->max_row_nnz : std::max<int32_t>(g->nnz, 1);
    L.entries = std::min<int64_t>((int64_t)L.n_slices * 64 * wmax, (int64_t)64 * std::max<int32_t>(g->nnz, 1));
    size_t o = 256;  // [0]: bad-grid flag
    L.off_nslice = o;
    o += align_up(sizeof(int32_t) * (size_t)(n_sub + 1), 256);
    L.off_slice_off = o;
    o += align_up(sizeof(int32_t) * (size_t)(n_sub + 1), 256);
    L.off_bw = o;
    o += align_up(sizeof(int32_t) * (size_t)n_sub, 256);
    L.off_width = o;
    o += align_up(sizeof(int32_t) * (size_t)(L.n_slices + 1), 256);
    L.off_start = o;
    o += align_up(sizeof(int32_t) * (size_t)(L.n_slices + 1), 256);
    L.off_col = o;
    o += align_up(sizeof(int32_t) * (size_t)L.entries, 256);
    L.off_val = o;
    o += align_up(sizeof(double2) * (size_t)L.entries, 256);
    if (streaming) {
        L.off_mom = o;  // Adam moments [4][B][ld] when the caller passes none
        o += align_up(sizeof(double) * 4 * (size_t)B * ld, 256);
        L.off_scr = o;  // V, a*I and w [3][B][ld] complex (paired state: I and the three pairs, [4][B][ld];
                        // persistent teams: a*I, V, w and the three pairs, [6][B][ld])
        o += align_up(sizeof(double2) * (teams ? 6 : pairs ? 4 : 3) * (size_t)B * ld, 256);
    }
    if (wide) {
        L.off_wcount = o;
        o += align_up(sizeof(int32_t) * (size_t)(n_sub + 1), 256);
        L.off_woff = o;
        o += align_up(sizeof(int32_t) * (size_t)(n_sub + 1), 256);
        L.off_mres = o;
        o += align_up(sizeof(double) * (size_t)n_sub, 256);
        L.off_part = o;
        o += align_up(sizeof(double2) * (size_t)B * part_slices, 256);
        L.off_items = o;
        o += align_up(sizeof(dpf::WideItem) * (size_t)B * n_sub, 256);
    }
    if (handoff) {
        L.off_list = o;  // paused items, and the list compacted as they finish
        o += align_up(sizeof(int32_t) * (size_t)B, 256);
        L.off_list2 = o;
        o += align_up(sizeof(int32_t) * (size_t)B, 256);
        L.off_sched = o;  // schedule state when the caller passes none [B][6]
        o += align_up(sizeof(double) * dpf::kSchedWords * (size_t)B, 256);
        L.off_bar = o;  // split kernel: one arrival counter per listed item, 256 bytes apart
        o += align_up(sizeof(int32_t) * dpf::kBarStride * (size_t)B, 256);
        L.off_tfirst = o;  // ... and its team table
        o += align_up(sizeof(int32_t) * (size_t)(B + 1), 256);
        L.off_order = o;  // case order: [B] int32 order, [B] max|r|, [B] loss, residual count
        o += align_up(sizeof(int32_t) * (size_t)B, 256) + 2 * align_up(sizeof(double) * (size_t)B, 256) + 256;
    }
    if (teams) {
        const int64_t items = (int64_t)B * (sub_offset ? n_sub : 1);
        L.off_thdr = o;  // ticket counter, tickets, units
        o += 256;
        L.off_tunit = o;
        o += align_up(sizeof(int32_t) * (size_t)items, 256);
        L.off_tfirst2 = o;
        o += align_up(sizeof(int32_t) * (size_t)(items + 1), 256);
        L.off_tbar = o;  // one 64-bit arrival counter per unit, 256 bytes apart
        o += align_up(sizeof(long long) * dpf::kTeamBarStride * (size_t)items, 256);
        L.off_tpart = o;
        o += align_up(sizeof(double2) * (size_t)(B * team_part), 256);
    }
    L.total = o;
    return L;
}

// Multi-workgroup path for sub-grids above the LDS capacity (see wide.hpp).
// Runs on the device's side stream; the host enqueues chunks of iterations and
// polls the number of active items, so this part of the call blocks the host.
int run_wide(const dpf::SolveArgs &a, const SolveLayout &L, char *ws, int32_t n_sub, const int32_t *sub_offset_dev,
             int32_t B, int32_t ld, int32_t cap, const DeviceInfo &dev, const int32_t *list = nullptr,
             int32_t n_list = 0) {
    hipStream_t sd = dev.side;
    dpf::WideArgs w{};
    w.sell = a.sell;
    w.sub_off = sub_offset_dev;
    w.wide_off = (const int32_t *)(ws + L.off_woff);
    w.nslice = (const int32_t *)(ws + L.off_nslice);
    w.n_sub = n_sub;
    w.B = B;
    w.n_bus = a.n_bus;
    w.w_total = list ? L.h_total : L.w_total;
    w.list = list;
    w.resume = list ? 1 : 0;
    w.bt = a.bt;
    w.s_spec = a.s_spec;
    w.s_ld = a.s_ld;
    w.ov = a.ov;
    w.vm = a.vm;
    w.va = a.va;
    w.ld = ld;
    w.st = a.st;
    w.st_stride = a.st_stride;
    w.st_fresh = list ? 0 : a.st_fresh;  // paused items bring their moments
    w.Vg = a.scratch;
    w.aIg = a.scratch + a.st_stride;
    w.Wg = a.scratch + 2 * a.st_stride;
    w.part = (double2 *)(ws + L.off_part);
    w.items = (dpf::WideItem *)(ws + L.off_items);
    w.bad_grid = a.bad_grid;
    w.m_res = (const double *)(ws + L.off_mres);
    w.sched = a.sched;
    w.lr = a.lr;
    w.opt = a.opt;
    w.b1 = a.b1;
    w.b2 = a.b2;
    w.eps = a.eps;
    w.tol = a.tol;
    w.max_iter = a.max_iter;
    w.sch = a.sch;
    w.factor = a.factor;
    w.patience = a.patience;
    w.threshold = a.threshold;
    w.cooldown = a.cooldown;
    w.min_lr = a.min_lr;
    w.sched_eps = a.sched_eps;
    w.iters = a.iters;
    w.status = a.status;
    w.mu_out = a.mu_out;
    w.loss_out = a.loss_out;
    w.trace = a.trace;
    w.trace_every = a.trace_every;
    w.trace_len = a.trace_len;
    w.done_ns = a.done_ns;
    w.stamp = a.stamp;
    w.ns_per_tick = a.ns_per_tick;
    int32_t *wcount = (int32_t *)(ws + L.off_wcount);
    // the active counter sits in the 256-byte header of the workspace (word 1; word 0 is the bad-grid flag)
    w.active_count = (int32_t *)ws + 1;
    const int items = B * n_sub;
    hipLaunchKernelGGL(dpf::wide_count_kernel, dim3((n_sub + 255) / 256), dim3(256), 0, sd, n_sub, sub_offset_dev,
                       a.n_bus, cap, w.nslice, wcount);
    hipLaunchKernelGGL(dpf::scan_kernel, dim3(1), dim3(1024), 0, sd, n_sub, wcount, 0, (int32_t *)w.wide_off);
    hipLaunchKernelGGL(dpf::sub_residual_count_kernel, dim3(n_sub), dim3(256), 0, sd, n_sub, sub_offset_dev, a.n_bus,
                       a.bt, (double *)w.m_res);
    hipLaunchKernelGGL(dpf::wide_item_init_kernel, dim3((items + 255) / 256), dim3(256), 0, sd, w, cap);
    int units = (list ? n_list : B) * w.w_total;
    w.n_units = units;  // the spare waves of the last block must not read past the list
    int ublocks = (units + 3) / 4;
    int rblocks = list ? n_list : items;
    hipLaunchKernelGGL(dpf::wide_init_rows_kernel, dim3(ublocks), dim3(256), 0, sd, w);
    DPF_HIP(hipGetLastError());
    const int chunk = 32;
    for (int64_t done = 0; done <= (int64_t)a.max_iter; done += chunk) {
        for (int k = 0; k < chunk && done + k <= (int64_t)a.max_iter; ++k) {
            hipLaunchKernelGGL(dpf::wide_phase_a_kernel, dim3(ublocks), dim3(256), 0, sd, w);
            hipLaunchKernelGGL(dpf::wide_reduce_kernel, dim3(rblocks), dim3(dpf::kWave), 0, sd, w);
            hipLaunchKernelGGL(dpf::wide_phase_b_kernel, dim3(ublocks), dim3(256), 0, sd, w);
        }
        // with a list, the poll also drops the finished items from it (into the other
        // list buffer), so that the launches shrink as items finish
        int32_t *next = nullptr;
        if (list) {
            next = (int32_t *)(list == (const int32_t *)(ws + L.off_list) ? ws + L.off_list2 : ws + L.off_list);
            hipLaunchKernelGGL(dpf::wide_compact_kernel, dim3(1), dim3(1024), 0, sd, w, rblocks, next);
        } else {
            hipLaunchKernelGGL(dpf::wide_active_count_kernel, dim3(1), dim3(256), 0, sd, w);
        }
        DPF_HIP(hipGetLastError());
        DPF_HIP(hipMemcpyAsync(dev.pinned_count, w.active_count, sizeof(int32_t), hipMemcpyDeviceToHost, sd));
        DPF_HIP(hipEventRecord(dev.ev_poll, sd));
        DPF_HIP(hipEventSynchronize(dev.ev_poll));
        const int32_t active = *dev.pinned_count;
        if (active == 0) break;
        if (list) {
            list = next;
            w.list = next;
            rblocks = active;
            units = active * w.w_total;
            w.n_units = units;
            ublocks = (units + 3) / 4;
        }
    }
    hipLaunchKernelGGL(dpf::wide_finish_kernel, dim3((items + 255) / 256), dim3(256), 0, sd, w, cap);
    DPF_HIP(hipGetLastError());
    return DPF_OK;
}

// Split kernel for the handed-over items (see split.hpp): chunks of iterations
// with T = (workgroups the device holds at once) / (items left) workgroups per
// item, at most max_team, relaunched as items finish, for as long as more than
// min_items items are left.  Items still paused when it returns (at most
// min_items, or a team abandoned a barrier) are left in *rest / *rest_list for
// the multi-workgroup path.
// host-pinned staging of the split kernel's team table and the list / counts it
// is computed from, per device; used under the device's side lock
struct PinnedScratch {
    int32_t *p = nullptr;
    size_t n = 0;
};
PinnedScratch g_pinned[64];

int pinned_scratch(int dev, size_t n, int32_t **out) {
    PinnedScratch &ps = g_pinned[dev];
    if (ps.n < n) {
        if (ps.p) DPF_HIP(hipHostFree(ps.p));
        ps.p = nullptr;
        ps.n = 0;
        DPF_HIP(hipHostMalloc((void **)&ps.p, n * sizeof(int32_t), hipHostMallocDefault));
        ps.n = n;
    }
    *out = ps.p;
    return DPF_OK;
}

// Split kernel for the handed-over items (see split.hpp), relaunched as items
// finish for as long as more than min_items are left.  Team sizes per launch:
// without a time slice T = (workgroups the device holds at once) / (items left)
// for every item; with one, in proportion to the square of each item's
// remaining iteration budget (max_iter - iters; the square favours the long
// runners more than the budget itself, 6.48 against 6.56 s on the N-1 batch),
// at least 1, and together at most what the device holds.  Both are capped by max_team and the slices of the grid.  Items still
// paused when it returns (at most min_items, or a team abandoned a barrier) are
// left in *rest / *rest_list for the multi-workgroup path.
int run_split(const dpf::SolveArgs &a0, const SolveLayout &L, char *ws, const DeviceInfo &dev, int32_t *list,
              int32_t n_list, int32_t B, const dpf_route_t &route, int32_t *rest, int32_t **rest_list) {
    const int32_t max_team = route.tail_team, chunk = route.tail_chunk, min_items = route.tail_min_items;
    const double slice_ms = route.tail_slice_ms;
    hipStream_t sd = dev.side;
    *rest = n_list;
    *rest_list = list;
    dpf::SolveArgs a = a0;
    a.handoff = 0;  // no per-item kernel polls the finished count any more
    const int32_t ns = (a.n_bus + dpf::kWave - 1) / dpf::kWave;
    // X and the bitmap of the columns a member reads, then as much of the list of
    // those columns (16-bit) as the rest of the LDS holds
    const size_t lds_x = (size_t)a.n_bus * 16 + (size_t)(a.n_bus + 31) / 32 * 4;
    if (lds_x + 512 > (size_t)dev.lds_per_block) return DPF_OK;  // the multi-workgroup path takes them
    const int32_t list_cap = (int32_t)std::min<size_t>((size_t)a.n_bus, ((size_t)dev.lds_per_block - 512 - lds_x) / 2);
    const size_t lds = lds_x + align_up((size_t)list_cap * 2, 4);
    // 512 threads: 168 VGPRs without spills (1024 threads spill ~37 at 128); one
    // case alone 12.5 us per iteration against 16.4 (1024) and 16.5 (256)
    constexpr int kSplitThreads = 512;
    void (*fn)(dpf::SolveArgs, dpf::SplitArgs) = dpf::team_solve_split_kernel<kSplitThreads>;
    DPF_HIP(hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    DPF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kSplitThreads, lds));
    const int64_t capacity = (int64_t)std::max(per_cu, 0) * dev.n_cu;
    if (capacity < 1) return DPF_OK;
    const int64_t tmax = std::max<int64_t>(1, std::min<int64_t>(max_team, ns));
    int32_t *hp = nullptr;  // [B] list, [B] iteration counts, [B + 1] team table
    int rc = pinned_scratch(dev.index, 3 * (size_t)B + 1, &hp);
    if (rc != DPF_OK) return rc;
    int32_t *h_list = hp, *h_iters = hp + B, *h_first = hp + 2 * B;
    int32_t *hdr = (int32_t *)ws;  // header words 6 (paused count) and 7 (abandoned flag)
    dpf::SplitArgs p{};
    p.bar = (int32_t *)(ws + L.off_bar);
    p.part = (double2 *)(ws + L.off_part);
    p.first = (const int32_t *)(ws + L.off_tfirst);
    p.Ig = a.scratch;
    p.Wg = a.scratch + 2 * a.st_stride;
    p.aborted = hdr + 7;
    p.chunk = chunk;
    p.slice = slice_ms > 0.0 ? (int64_t)(slice_ms * 1e6 / dev.ns_per_tick) : 0;
    p.first_limit = (int64_t)(route.tail_first_wait_s * 1e9 / dev.ns_per_tick);  // other work may hold CUs
    p.limit = (int64_t)(route.tail_wait_s * 1e9 / dev.ns_per_tick);
    p.list_cap = list_cap;
    const bool by_budget = p.slice > 0;
    hipLaunchKernelGGL(dpf::split_clear_kernel, dim3(1), dim3(64), 0, sd, 1, 1, p.aborted);
    int32_t *cur = list;
    int32_t *other = (int32_t *)(list == (int32_t *)(ws + L.off_list) ? ws + L.off_list2 : ws + L.off_list);
    auto fetch_counts = [&](const int32_t *dlist, int32_t n) -> int {
        DPF_HIP(hipMemcpyAsync(h_list, dlist, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, sd));
        DPF_HIP(hipMemcpyAsync(h_iters, a.iters, sizeof(int32_t) * (size_t)B, hipMemcpyDeviceToHost, sd));
        return DPF_OK;
    };
    if (by_budget) {
        if ((rc = fetch_counts(cur, n_list)) != DPF_OK) return rc;
        DPF_HIP(hipEventRecord(dev.ev_poll, sd));
        DPF_HIP(hipEventSynchronize(dev.ev_poll));
    }
    std::vector<int64_t> T((size_t)B);
    // every launch advances each listed case by at least one update (or finishes or
    // abandons it), so max_iter + 1 launches finish any list; past that bound the
    // rest goes to the multi-workgroup path, whose loop is bounded by max_iter too
    int64_t launches = 0;
    while (n_list > std::max(min_items, 0) && launches++ <= (int64_t)a.max_iter + 1) {
        int64_t total = 0;
        if (by_budget && n_list <= capacity) {
            auto weight = [&](int32_t k) {
                const double r = (double)std::max(1, a.max_iter - h_iters[h_list[k]]);
                return r * r;
            };
            double wsum = 0.0;
            for (int32_t k = 0; k < n_list; ++k) wsum += weight(k);
            for (int32_t k = 0; k < n_list; ++k) {
                const double w = weight(k);
                T[k] = std::min<int64_t>(std::max<int64_t>((int64_t)(w / wsum * (double)capacity), 1), tmax);
                total += T[k];
            }
            while (total > capacity) {  // the floor of 1 can overshoot: shrink the largest teams
                int32_t big = 0;
                for (int32_t k = 1; k < n_list; ++k)
                    if (T[k] > T[big]) big = k;
                if (T[big] <= 1) break;
                --T[big];
                --total;
            }
        } else {
            const int64_t t = std::max<int64_t>(1, std::min<int64_t>(capacity / n_list, tmax));
            for (int32_t k = 0; k < n_list; ++k) T[k] = t;
        }
        h_first[0] = 0;
        for (int32_t k = 0; k < n_list; ++k) h_first[k + 1] = h_first[k] + (int32_t)T[k];
        DPF_HIP(hipMemcpyAsync((void *)p.first, h_first, sizeof(int32_t) * (size_t)(n_list + 1),
                               hipMemcpyHostToDevice, sd));
        p.list = cur;
        p.n_list = n_list;
        hipLaunchKernelGGL(dpf::split_clear_kernel, dim3((n_list + 255) / 256), dim3(256), 0, sd, n_list,
                           dpf::kBarStride, p.bar);
        hipLaunchKernelGGL(fn, dim3(h_first[n_list]), dim3(kSplitThreads), lds, sd, a, p);
        hipLaunchKernelGGL(dpf::collect_paused_kernel, dim3(1), dim3(1024), 0, sd, B, a.status, other, hdr + 6);
        DPF_HIP(hipGetLastError());
        DPF_HIP(hipMemcpyAsync(dev.pinned_count, hdr + 6, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, sd));
        // the next table needs the new list and counts (at most B entries are read)
        if (by_budget && (rc = fetch_counts(other, B)) != DPF_OK) return rc;
        DPF_HIP(hipEventRecord(dev.ev_poll, sd));
        DPF_HIP(hipEventSynchronize(dev.ev_poll));
        n_list = dev.pinned_count[0];
        std::swap(cur, other);
        *rest = n_list;
        *rest_list = cur;
        g_split_launches.fetch_add(1);
        if (dev.pinned_count[1]) {  // abandoned: the rest goes to the multi-workgroup path
            g_split_abandoned.fetch_add(1);
            break;
        }
    }
    return DPF_OK;
}

// Bytes of static LDS the persistent team kernel uses besides its window.
constexpr int kTeamStaticLds = 2 * (dpf::kTeamThreads / dpf::kWave) * 8 + (dpf::kTeamThreads / dpf::kWave) * 4 + 64;

// The split kernel for the paused items with every launch planned on the device
// (route.tail_device): on `st`, a fixed sequence of (plan, split kernel, collect)
// launches and no host wait, so the call can be captured.  Launches end after
// `chunk` iterations or the time slice, as on the host; with a time slice there
// are kTailDeviceSlices of them, without one enough for max_iter, and a last
// launch without either limit.  A launch whose list is
// empty costs its workgroups nothing but their start.  A case whose team gave up
// at a barrier stays paused and is planned again; one still paused after the
// last launch ends with DPF_UNFINISHED.  (The call checks beforehand that the
// grid fits the split kernel.)
constexpr int kTailDeviceSlices = 256;
int run_split_device(const dpf::SolveArgs &a0, const SolveLayout &L, char *ws, const DeviceInfo &dev,
                     int32_t *list, int32_t B, const dpf_route_t &route, hipStream_t st) {
    dpf::SolveArgs a = a0;
    a.handoff = 0;
    const int32_t ns = (a.n_bus + dpf::kWave - 1) / dpf::kWave;
    const size_t lds_x = (size_t)a.n_bus * 16 + (size_t)(a.n_bus + 31) / 32 * 4;
    if (lds_x + 512 > (size_t)dev.lds_per_block) return fail(DPF_EUNSUPPORTED, "grid too large for route.tail_device");
    const int32_t list_cap = (int32_t)std::min<size_t>((size_t)a.n_bus, ((size_t)dev.lds_per_block - 512 - lds_x) / 2);
    const size_t lds = lds_x + align_up((size_t)list_cap * 2, 4);
    constexpr int kSplitThreads = 512;
    void (*fn)(dpf::SolveArgs, dpf::SplitArgs) = dpf::team_solve_split_kernel<kSplitThreads>;
    DPF_HIP(hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    DPF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kSplitThreads, lds));
    const int64_t capacity = (int64_t)std::max(per_cu, 0) * dev.n_cu;
    if (capacity < 1) return fail(DPF_EUNSUPPORTED, "the split kernel does not fit a compute unit");
    const int32_t tmax = (int32_t)std::max<int64_t>(1, std::min<int64_t>(route.tail_team, ns));
    int32_t *hdr = (int32_t *)ws;  // header words 6 (paused count) and 7 (abandoned flag)
    dpf::SplitArgs p{};
    p.n_list_dev = hdr + 6;
    p.bar = (int32_t *)(ws + L.off_bar);
    p.part = (double2 *)(ws + L.off_part);
    p.first = (const int32_t *)(ws + L.off_tfirst);
    p.Ig = a.scratch;
    p.Wg = a.scratch + 2 * a.st_stride;
    p.aborted = hdr + 7;
    p.first_limit = (int64_t)(route.tail_first_wait_s * 1e9 / dev.ns_per_tick);
    p.limit = (int64_t)(route.tail_wait_s * 1e9 / dev.ns_per_tick);
    p.list_cap = list_cap;
    const int64_t slice = route.tail_slice_ms > 0.0 ? (int64_t)(route.tail_slice_ms * 1e6 / dev.ns_per_tick) : 0;
    const int64_t n_launch = slice > 0 ? kTailDeviceSlices + 1
                                       : ((int64_t)a.max_iter + route.tail_chunk) / route.tail_chunk + 1;
    // a grid that holds every team of a plan (at most capacity members, or one per
    // case when there are more cases than that)
    const unsigned grid = (unsigned)std::max<int64_t>(capacity, B);
    hipLaunchKernelGGL(dpf::split_clear_kernel, dim3(1), dim3(64), 0, st, 1, 1, p.aborted);
    int32_t *cur = list;
    int32_t *other = (int32_t *)(list == (int32_t *)(ws + L.off_list) ? ws + L.off_list2 : ws + L.off_list);
    for (int64_t k = 0; k < n_launch; ++k) {
        const bool last = k == n_launch - 1;
        hipLaunchKernelGGL(dpf::split_plan_kernel, dim3(1), dim3(dpf::kSplitPlanThreads), 0, st, cur, hdr + 6,
                           a.iters, a.max_iter, (int32_t)capacity, tmax, slice > 0 ? 1 : 0, (int32_t *)p.first,
                           p.bar);
        p.list = cur;
        p.slice = last ? 0 : slice;
        p.chunk = last ? a.max_iter + 1 : route.tail_chunk;
        hipLaunchKernelGGL(fn, dim3(grid), dim3(kSplitThreads), lds, st, a, p);
        hipLaunchKernelGGL(dpf::collect_paused_kernel, dim3(1), dim3(1024), 0, st, B, a.status, other, hdr + 6);
        std::swap(cur, other);
    }
    hipLaunchKernelGGL(dpf::split_unfinished_kernel, dim3((B + 255) / 256), dim3(256), 0, st, B, a.status);
    DPF_HIP(hipGetLastError());
    g_split_launches.fetch_add(n_launch);
    return DPF_OK;
}

// Persistent teams (teams.hpp): every item of the call in one launch on `st`, with
// a device-side plan; nothing waits on the host, so the call can be captured.
int run_teams(const dpf::SolveArgs &a0, const SolveLayout &L, char *ws, int32_t n_sub, int32_t B,
              const DeviceInfo &dev, const dpf_route_t &route, hipStream_t st) {
    dpf::SolveArgs a = a0;
    a.handoff = 0;
    // the window (16 B per column) and the 16-bit halo list behind it
    const int64_t avail = (int64_t)dev.lds_per_block - kTeamStaticLds - 2 * dpf::kTeamHaloCap;
    int32_t win = (int32_t)std::min<int64_t>(std::max<int64_t>(avail, 0) / 16, 65536);  // 16-bit offsets
    if (route.team_cap > 0) win = std::min(win, std::max<int32_t>(dpf::kWave, route.team_cap));
    if (win < dpf::kWave) return fail(DPF_EUNSUPPORTED, "too little LDS for the team kernel");
    const int lds = win * 16 + 2 * dpf::kTeamHaloCap;
    void (*fn)(dpf::SolveArgs, dpf::TeamArgs) = dpf::team_solve_persist_kernel<dpf::kTeamThreads>;
    DPF_HIP(hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    int per_cu = 0;
    DPF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, dpf::kTeamThreads, lds));
    if (per_cu < 1) return fail(DPF_EUNSUPPORTED, "the team kernel does not fit a compute unit");
    const int grid = per_cu * dev.n_cu;
    dpf::TeamArgs p{};
    p.hdr = (int32_t *)(ws + L.off_thdr);
    p.progress = dev.team_progress;
    p.unit_item = (int32_t *)(ws + L.off_tunit);
    p.first = (int32_t *)(ws + L.off_tfirst2);
    p.bar = (long long *)(ws + L.off_tbar);
    p.part = (double2 *)(ws + L.off_tpart);
    p.Ig = a.scratch;
    p.Vg = a.scratch + a.st_stride;
    p.Wg = a.scratch + 2 * a.st_stride;
    p.P0 = a.scratch + 3 * a.st_stride;
    p.P1 = a.scratch + 4 * a.st_stride;
    p.P2 = a.scratch + 5 * a.st_stride;
    p.first_limit = (int64_t)(route.tail_first_wait_s * 1e9 / dev.ns_per_tick);
    p.limit = (int64_t)(route.tail_wait_s * 1e9 / dev.ns_per_tick);
    p.win = win;  // a route's team cap also caps the window (members then hold fewer buses)
    p.grid = grid;
    p.tmax = std::max(1, std::min(dpf::kTeamMaxMembers, grid / 2));
    // the state as pairs for the launch, and back to the caller's arrays after it
    // (every entry, unfinished items included)
    const dim3 pgrid((unsigned)((a.n_bus + 255) / 256), (unsigned)std::min<int32_t>(B, 65535));
    hipLaunchKernelGGL(dpf::pair_in_kernel, pgrid, dim3(256), 0, st, a.n_bus, a.ld, B, a.vm, a.va, a.st,
                       a.st_stride, a.st_fresh, p.P0, p.P1, p.P2);
    hipLaunchKernelGGL(dpf::team_plan_kernel, dim3(1), dim3(dpf::kPlanThreads), 0, st, n_sub, a.sub_off, a.n_bus,
                       a.sub_bw, B, p);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(dpf::kTeamThreads), (size_t)lds, st, a, p);
    hipLaunchKernelGGL(dpf::pair_out_kernel, pgrid, dim3(256), 0, st, a.n_bus, a.ld, B, a.vm, a.va, a.st,
                       a.st_stride, p.P0, p.P1, p.P2);
    DPF_HIP(hipGetLastError());
    return DPF_OK;
}

// Temporaries of the Y-bus build: deg[n+1] fill[n+1] soff[n+1] ucount[n+1] err[64]
// (int32, cleared), then the slot list int2[n + 2 n_branch] and the diagonal
// double2[n], each region 256-byte aligned.
struct YbusTemps {
    size_t bytes_i = 0, bytes_s = 0, bytes_d = 0;
    size_t total() const { return bytes_i + bytes_s + bytes_d; }
};

YbusTemps ybus_temps(int32_t n_bus, int32_t n_branch) {
    YbusTemps t;
    t.bytes_i = align_up(sizeof(int32_t) * (4 * (size_t)(n_bus + 1) + 64), 256);
    t.bytes_s = align_up(sizeof(int2) * ((size_t)n_bus + 2 * (size_t)n_branch), 256);
    t.bytes_d = align_up(sizeof(double2) * (size_t)n_bus, 256);
    return t;
}

int ybus_check_args(int32_t n_bus, int32_t n_branch, const int32_t *from, const int32_t *to, const double *r,
                    const double *x, const double *b, int32_t nnz_cap, int32_t *row_ptr, int32_t *col_idx,
                    double *val, int32_t *nnz_out) {
    if (n_bus <= 0 || n_branch < 0) return fail(DPF_EINVAL, "n_bus must be > 0 and n_branch >= 0");
    if (n_branch > 0 && (!from || !to || !r || !x || !b)) return fail(DPF_EINVAL, "null branch array");
    if (!row_ptr || !nnz_out || (nnz_cap > 0 && (!col_idx || !val)) || nnz_cap < 0)
        return fail(DPF_EINVAL, "null output array or negative nnz_cap");
    if ((int64_t)n_bus + 2 * (int64_t)n_branch > INT32_MAX) return fail(DPF_EINVAL, "grid too large");
    return DPF_OK;
}

// The Y-bus build on temporaries at `tmp` (laid out as ybus_temps says); returns
// with the stream synchronised (the result count is read back on the way).
int build_ybus_on(char *tmp, const YbusTemps &T, int32_t n_bus, int32_t n_branch, const int32_t *from,
                  const int32_t *to, const double *r, const double *x, const double *b, int32_t nnz_cap,
                  int32_t *row_ptr, int32_t *col_idx, double *val, int32_t *nnz_out, int32_t *max_row_nnz_out,
                  hipStream_t st) {
    const size_t bytes_i = T.bytes_i, bytes_s = T.bytes_s;
    int32_t *deg = (int32_t *)tmp;
    int32_t *fill = deg + (n_bus + 1);
    int32_t *soff = fill + (n_bus + 1);
    int32_t *ucount = soff + (n_bus + 1);
    int32_t *err = ucount + (n_bus + 1);
    int2 *slot = (int2 *)(tmp + bytes_i);
    double2 *diag = (double2 *)(tmp + bytes_i + bytes_s);
    int rc = DPF_OK;
    int32_t herr = 0, nnz = 0;
    do {
        // the counters start at zero (a fill kernel, so that a reused scratch is cleared too)
        hipLaunchKernelGGL(dpf::zero_f64_kernel, dim3((unsigned)((bytes_i / 8 + 255) / 256)), dim3(256), 0, st,
                           (int64_t)(bytes_i / 8), (double *)tmp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) { rc = fail(DPF_EHIP, std::string("clear: ") + hipGetErrorString(e)); break; }
        const int bs = 256;
        int gb = std::max(1, (n_branch + bs - 1) / bs);
        if (n_branch > 0)
            hipLaunchKernelGGL(dpf::ybus_count_kernel, dim3(gb), dim3(bs), 0, st, n_bus, n_branch, from, to, r, x,
                               deg, err);
        e = hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) { rc = fail(DPF_EHIP, std::string("branch validation: ") + hipGetErrorString(e)); break; }
        if (herr) { rc = fail(DPF_EINVAL, "branch with bus index out of range, from == to, or r = x = 0"); break; }
        hipLaunchKernelGGL(dpf::scan_kernel, dim3(1), dim3(1024), 0, st, n_bus, deg, 1, soff);
        int gmax = std::max(1, (std::max(n_bus, n_branch) + bs - 1) / bs);
        hipLaunchKernelGGL(dpf::ybus_scatter_kernel, dim3(gmax), dim3(bs), 0, st, n_bus, n_branch, from, to, soff,
                           fill, slot);
        int gn = (n_bus + bs - 1) / bs;
        hipLaunchKernelGGL(dpf::ybus_row_order_kernel, dim3(gn), dim3(bs), 0, st, n_bus, soff, slot, r, x, b, diag,
                           ucount);
        hipLaunchKernelGGL(dpf::scan_kernel, dim3(1), dim3(1024), 0, st, n_bus, ucount, 0, row_ptr);
        hipLaunchKernelGGL(dpf::imax_kernel, dim3(1), dim3(1024), 0, st, n_bus, ucount, err + 1);
        int32_t hmax = 0;
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&hmax, err + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&nnz, row_ptr + n_bus, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) { rc = fail(DPF_EHIP, std::string("ybus pattern: ") + hipGetErrorString(e)); break; }
        *nnz_out = nnz;
        if (max_row_nnz_out) *max_row_nnz_out = hmax;
        if (nnz > nnz_cap) { rc = fail(DPF_ECAP, "nnz_cap too small"); break; }
        hipLaunchKernelGGL(dpf::ybus_emit_kernel, dim3(gn), dim3(bs), 0, st, n_bus, soff, slot, r, x, diag, row_ptr,
                           nnz_cap, col_idx, (double2 *)val);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) { rc = fail(DPF_EHIP, std::string("ybus values: ") + hipGetErrorString(e)); break; }
    } while (0);
    (void)hipStreamSynchronize(st);
    return rc;
}

}  // namespace

extern "C" {

const char *dpf_last_error(void) { return g_err.c_str(); }

#ifndef DPF_SOURCE_HASH
#define DPF_SOURCE_HASH "unknown"
#endif
const char *dpf_version(void) { return "libdpf 0.1 (gfx950, FP64) src " DPF_SOURCE_HASH; }

int dpf_build_ybus(int32_t n_bus, int32_t n_branch, const int32_t *from, const int32_t *to, const double *r,
                   const double *x, const double *b, int32_t nnz_cap, int32_t *row_ptr, int32_t *col_idx,
                   double *val, int32_t *nnz_out, int32_t *max_row_nnz_out, void *stream) {
    g_err.clear();
    int rc = ybus_check_args(n_bus, n_branch, from, to, r, x, b, nnz_cap, row_ptr, col_idx, val, nnz_out);
    if (rc != DPF_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const YbusTemps T = ybus_temps(n_bus, n_branch);
    char *tmp = nullptr;
    DPF_HIP(hipStreamSynchronize(st));
    DPF_HIP(hipMalloc((void **)&tmp, T.total()));
    rc = build_ybus_on(tmp, T, n_bus, n_branch, from, to, r, x, b, nnz_cap, row_ptr, col_idx, val, nnz_out,
                       max_row_nnz_out, st);
    (void)hipFree(tmp);
    return rc;
}

int dpf_build_ybus_noalloc(int32_t n_bus, int32_t n_branch, const int32_t *from, const int32_t *to,
                           const double *r, const double *x, const double *b, int32_t nnz_cap, int32_t *row_ptr,
                           int32_t *col_idx, double *val, int32_t *nnz_out, int32_t *max_row_nnz_out,
                           void *stream) {
    g_err.clear();
    int rc = ybus_check_args(n_bus, n_branch, from, to, r, x, b, nnz_cap, row_ptr, col_idx, val, nnz_out);
    if (rc != DPF_OK) return rc;
    const YbusTemps T = ybus_temps(n_bus, n_branch);
    if (T.total() > kYbusScratchBytes)
        return fail(DPF_EINVAL, "grid too large for the library's static scratch (" + std::to_string(T.total()) +
                                    " bytes needed, " + std::to_string(kYbusScratchBytes) +
                                    " available): use dpf_build_ybus");
    DeviceInfo dev;
    rc = device_info(dev);
    if (rc != DPF_OK) return rc;
    return build_ybus_on((char *)dev.ybus_scratch, T, n_bus, n_branch, from, to, r, x, b, nnz_cap, row_ptr,
                         col_idx, val, nnz_out, max_row_nnz_out, (hipStream_t)stream);
}

size_t dpf_mismatch_grad_workspace_bytes(int32_t n_bus, int32_t B) {
    if (n_bus <= 0 || B <= 0) return 0;
    size_t per = sizeof(double2) * (size_t)n_bus * (size_t)B;
    int32_t nblk = (n_bus + dpf::kEvalBlock - 1) / dpf::kEvalBlock;
    return 256 + 3 * align_up(per, 256) + align_up(sizeof(double2) * (size_t)B * nblk, 256);
}

int dpf_mismatch_grad(const dpf_grid_t *g, int32_t B, int32_t ld, const int8_t *bus_type, const double *s_spec,
                      int32_t s_ld, const int32_t *outage, const double *vm, const double *va, double *dS,
                      double *loss, double *max_mis, double *g_vm, double *g_va, void *workspace, size_t ws_bytes,
                      void *stream) {
    g_err.clear();
    if (!valid_grid(g)) return fail(DPF_EINVAL, "invalid grid");
    if (B <= 0 || ld < g->n_bus) return fail(DPF_EINVAL, "B must be > 0 and ld >= n_bus");
    if (B > 65535) return fail(DPF_EINVAL, "B must be <= 65535 for one evaluation call");
    if (s_ld != 0 && s_ld < g->n_bus) return fail(DPF_EINVAL, "s_ld must be 0 or >= n_bus");
    if (!bus_type || !s_spec || !vm || !va || !loss || !max_mis) return fail(DPF_EINVAL, "null argument");
    if ((g_vm == nullptr) != (g_va == nullptr)) return fail(DPF_EINVAL, "g_vm and g_va: both or neither");
    if (outage && (g->n_branch <= 0 || !g->from || !g->to || !g->r || !g->x || !g->b))
        return fail(DPF_EINVAL, "outage needs the grid's branch arrays");
    const int32_t n = g->n_bus;
    size_t need = dpf_mismatch_grad_workspace_bytes(n, B);
    if (!workspace || ws_bytes < need) return fail(DPF_ENOMEM, "workspace too small");
    if ((int64_t)B * ld > ((int64_t)1 << 40)) return fail(DPF_EINVAL, "batch too large");
    hipStream_t st = (hipStream_t)stream;
    size_t per = align_up(sizeof(double2) * (size_t)n * (size_t)B, 256);
    char *ws = (char *)workspace;
    double *m_res = (double *)ws;
    double2 *Vw = (double2 *)(ws + 256);
    double2 *ww = (double2 *)(ws + 256 + per);
    double2 *aI = (double2 *)(ws + 256 + 2 * per);
    double2 *part = (double2 *)(ws + 256 + 3 * per);
    const int32_t nblk = (n + dpf::kEvalBlock - 1) / dpf::kEvalBlock;
    dpf::OutageView ov{outage, g->from, g->to, g->r, g->x, g->b, g->n_branch};
    hipLaunchKernelGGL(dpf::residual_count_kernel, dim3(1), dim3(1024), 0, st, n, bus_type, m_res);
    hipLaunchKernelGGL(dpf::polar_kernel, dim3(nblk, B), dim3(dpf::kEvalBlock), 0, st, n, (int64_t)ld, vm, va, Vw);
    hipLaunchKernelGGL(dpf::forward_kernel, dim3(nblk, B), dim3(dpf::kEvalBlock), 0, st, n, g->row_ptr, g->col_idx,
                       (const double2 *)g->val, bus_type, (const double2 *)s_spec, (int64_t)s_ld, ov, Vw, m_res,
                       (int64_t)ld, (double2 *)dS, ww, aI, part, nullptr);
    if (g_vm)
        hipLaunchKernelGGL(dpf::adjoint_kernel, dim3(nblk, B), dim3(dpf::kEvalBlock), 0, st, n, g->row_ptr,
                           g->col_idx, (const double2 *)g->val, bus_type, ov, Vw, vm, (int64_t)ld, ww, aI, g_vm,
                           g_va);
    hipLaunchKernelGGL(dpf::finalize_kernel, dim3((B + 255) / 256), dim3(256), 0, st, B, nblk, part, m_res, loss,
                       max_mis);
    DPF_HIP(hipGetLastError());
    return DPF_OK;
}

int dpf_param_grad(const dpf_grid_t *g, int32_t B, int32_t ld, const int8_t *bus_type, const double *s_spec,
                   int32_t s_ld, const int32_t *outage, const double *vm, const double *va, double *loss,
                   double *max_mis, double *g_r, double *g_x, double *g_b, int32_t bld, double *g_s, void *workspace,
                   size_t ws_bytes, void *stream) {
    g_err.clear();
    if (!valid_grid(g)) return fail(DPF_EINVAL, "invalid grid");
    if (B <= 0 || ld < g->n_bus) return fail(DPF_EINVAL, "B must be > 0 and ld >= n_bus");
    if (B > 65535) return fail(DPF_EINVAL, "B must be <= 65535 for one evaluation call");
    if (s_ld != 0 && s_ld < g->n_bus) return fail(DPF_EINVAL, "s_ld must be 0 or >= n_bus");
    if (!bus_type || !s_spec || !vm || !va) return fail(DPF_EINVAL, "null argument");
    if ((loss == nullptr) != (max_mis == nullptr)) return fail(DPF_EINVAL, "loss and max_mis: both or neither");
    const bool br = g_r || g_x || g_b;
    if (br && !(g_r && g_x && g_b)) return fail(DPF_EINVAL, "g_r, g_x and g_b: all or none");
    if ((br || outage) && (g->n_branch <= 0 || !g->from || !g->to || !g->r || !g->x || !g->b))
        return fail(DPF_EINVAL, "branch gradients and outages need the grid's branch arrays");
    if (br && bld < g->n_branch) return fail(DPF_EINVAL, "bld must be >= n_branch");
    const int32_t n = g->n_bus;
    size_t need = dpf_mismatch_grad_workspace_bytes(n, B);
    if (!workspace || ws_bytes < need) return fail(DPF_ENOMEM, "workspace too small");
    if ((int64_t)B * ld > ((int64_t)1 << 40) || (int64_t)B * bld > ((int64_t)1 << 40))
        return fail(DPF_EINVAL, "batch too large");
    hipStream_t st = (hipStream_t)stream;
    size_t per = align_up(sizeof(double2) * (size_t)n * (size_t)B, 256);
    char *ws = (char *)workspace;
    double *m_res = (double *)ws;
    double2 *Vw = (double2 *)(ws + 256);
    double2 *ww = (double2 *)(ws + 256 + per);
    double2 *aI = (double2 *)(ws + 256 + 2 * per);
    double2 *part = (double2 *)(ws + 256 + 3 * per);
    const int32_t nblk = (n + dpf::kEvalBlock - 1) / dpf::kEvalBlock;
    dpf::OutageView ov{outage, g->from, g->to, g->r, g->x, g->b, g->n_branch};
    hipLaunchKernelGGL(dpf::residual_count_kernel, dim3(1), dim3(1024), 0, st, n, bus_type, m_res);
    hipLaunchKernelGGL(dpf::polar_kernel, dim3(nblk, B), dim3(dpf::kEvalBlock), 0, st, n, (int64_t)ld, vm, va, Vw);
    hipLaunchKernelGGL(dpf::forward_kernel, dim3(nblk, B), dim3(dpf::kEvalBlock), 0, st, n, g->row_ptr, g->col_idx,
                       (const double2 *)g->val, bus_type, (const double2 *)s_spec, (int64_t)s_ld, ov, Vw, m_res,
                       (int64_t)ld, (double2 *)nullptr, ww, aI, part, (double2 *)g_s);
    if (br) {
        const int32_t eblk = (g->n_branch + dpf::kEvalBlock - 1) / dpf::kEvalBlock;
        hipLaunchKernelGGL(dpf::branch_grad_kernel, dim3(eblk, B), dim3(dpf::kEvalBlock), 0, st, n, g->n_branch, ov,
                           Vw, ww, (int64_t)bld, g_r, g_x, g_b);
    }
    if (loss)
        hipLaunchKernelGGL(dpf::finalize_kernel, dim3((B + 255) / 256), dim3(256), 0, st, B, nblk, part, m_res,
                           loss, max_mis);
    DPF_HIP(hipGetLastError());
    return DPF_OK;
}

size_t dpf_dc_init_workspace_bytes(int32_t n_bus, int32_t B) {
    if (n_bus <= 0 || B <= 0) return 0;
    return 3 * align_up(sizeof(double) * (size_t)n_bus * (size_t)B, 256);
}

int dpf_dc_init(const dpf_grid_t *g_dc, int32_t B, int32_t ld, const int8_t *bus_type, const double *s_spec,
                int32_t s_ld, const int32_t *outage, double *va, double tol, int32_t max_iter, int32_t *iters,
                double *residual, void *workspace, size_t ws_bytes, void *stream) {
    g_err.clear();
    if (!valid_grid(g_dc)) return fail(DPF_EINVAL, "invalid grid");
    if (B <= 0 || ld < g_dc->n_bus) return fail(DPF_EINVAL, "B must be > 0 and ld >= n_bus");
    if (s_ld != 0 && s_ld < g_dc->n_bus) return fail(DPF_EINVAL, "s_ld must be 0 or >= n_bus");
    if (!bus_type || !s_spec || !va) return fail(DPF_EINVAL, "null argument");
    if (!(tol >= 0.0) || max_iter < 0) return fail(DPF_EINVAL, "tol must be >= 0 and max_iter >= 0");
    if (outage && (g_dc->n_branch <= 0 || !g_dc->from || !g_dc->to || !g_dc->r || !g_dc->x || !g_dc->b))
        return fail(DPF_EINVAL, "outage needs the grid's branch arrays");
    DeviceInfo dev;
    int rc = device_info(dev);
    if (rc != DPF_OK) return rc;
    const int32_t n = g_dc->n_bus;
    const size_t lds = sizeof(double) * (size_t)n;
    if (lds + 1024 > (size_t)dev.lds_per_block) return fail(DPF_EUNSUPPORTED, "grid too large for one workgroup's LDS");
    if (!workspace || ws_bytes < dpf_dc_init_workspace_bytes(n, B)) return fail(DPF_ENOMEM, "workspace too small");
    const size_t per = align_up(sizeof(double) * (size_t)n * (size_t)B, 256);
    char *ws = (char *)workspace;
    dpf::DcArgs a{};
    a.rp = g_dc->row_ptr;
    a.ci = g_dc->col_idx;
    a.yv = (const double2 *)g_dc->val;
    a.bt = bus_type;
    a.s_spec = (const double2 *)s_spec;
    a.s_ld = s_ld;
    a.ov = dpf::OutageView{outage, g_dc->from, g_dc->to, g_dc->r, g_dc->x, g_dc->b, g_dc->n_branch};
    a.va = va;
    a.ld = ld;
    a.r = (double *)ws;
    a.z = (double *)(ws + per);
    a.dg = (double *)(ws + 2 * per);
    a.n = n;
    a.tol = tol;
    a.max_iter = max_iter;
    a.iters = iters;
    a.res_out = residual;
    hipStream_t st = (hipStream_t)stream;
    DPF_HIP(hipFuncSetAttribute((const void *)dpf::dc_pcg_kernel<1024>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    hipLaunchKernelGGL(dpf::dc_pcg_kernel<1024>, dim3(B), dim3(1024), lds, st, a);
    DPF_HIP(hipGetLastError());
    return DPF_OK;
}

int dpf_solve_variant_count(void) {
    int cnt = 0;
    variant_table(&cnt);
    return cnt;
}

int dpf_solve_variant_info(int idx, int32_t *threads, int32_t *buses_per_thread, int32_t *streaming) {
    g_err.clear();
    int cnt = 0;
    const Variant *t = variant_table(&cnt);
    if (idx < 0 || idx >= cnt || !threads || !buses_per_thread || !streaming)
        return fail(DPF_EINVAL, "variant index out of range or null output");
    *threads = t[idx].nt;
    *buses_per_thread = t[idx].k;
    *streaming = t[idx].mode;
    return DPF_OK;
}

int dpf_solve_variant_cases(int idx) {
    g_err.clear();
    int cnt = 0;
    const Variant *t = variant_table(&cnt);
    if (idx < 0 || idx >= cnt) return fail(DPF_EINVAL, "variant index out of range");
    return 1;
}

int dpf_solve_variant_for_items(int32_t n_max, int64_t items) {
    DeviceInfo dev;
    if (device_info(dev) != DPF_OK) {
        g_err.clear();
        dev.n_cu = 256;
    }
    const Variant *v = pick_variant(n_max, items, dev.n_cu > 0 ? dev.n_cu : 256);
    if (!v) return -1;
    int cnt = 0;
    return (int)(v - variant_table(&cnt));
}

int dpf_solve_variant_for(int32_t n_max) { return dpf_solve_variant_for_items(n_max, INT64_MAX); }

static int autotune_store(int32_t n_max, int64_t items, int variant, bool all_buckets) {
    g_err.clear();
    int cnt = 0;
    const Variant *t = variant_table(&cnt);
    int d = default_variant_index(n_max);
    if (d < 0) return fail(DPF_EINVAL, "no variant holds a sub-grid of this size");
    if (variant < 0 || variant >= cnt || !variant_fits(t[variant], n_max))
        return fail(DPF_EINVAL, "variant cannot hold a sub-grid of this size");
    if (!all_buckets && items <= 0) return fail(DPF_EINVAL, "items must be > 0");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_init) {
        for (auto &row : g_tune)
            for (int &x : row) x = -1;
        g_tune_init = true;
    }
    for (int b = 0; b < kItemBuckets; ++b)
        if (all_buckets || b == items_bucket(items)) g_tune[d][b] = variant;
    return DPF_OK;
}

int dpf_autotune_set(int32_t n_max, int variant) { return autotune_store(n_max, 0, variant, true); }

int dpf_autotune_set_items(int32_t n_max, int64_t items, int variant) {
    return autotune_store(n_max, items, variant, false);
}

void dpf_tail_split_stats(int64_t *launches, int64_t *abandoned) {
    if (launches) *launches = g_split_launches.load();
    if (abandoned) *abandoned = g_split_abandoned.load();
}

void dpf_route_default(dpf_route_t *route) {
    if (route) *route = default_route();
}

void dpf_autotune_reset(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto &row : g_tune)
        for (int &x : row) x = -1;
    g_tune_init = true;
}

int dpf_order_rcm(int32_t n_bus, int32_t n_branch, const int32_t *from, const int32_t *to, int32_t n_sub,
                  const int32_t *sub_offset, int32_t group, int32_t *perm, int32_t *bandwidth_out) {
    g_err.clear();
    if (n_bus <= 0 || n_branch < 0 || group < 0 || !perm || (n_branch > 0 && (!from || !to)))
        return fail(DPF_EINVAL, "invalid sizes or null pointer");
    if (!sub_offset) n_sub = 1;
    if (n_sub <= 0) return fail(DPF_EINVAL, "n_sub must be > 0");
    if (sub_offset) {
        if (sub_offset[0] != 0 || sub_offset[n_sub] != n_bus)
            return fail(DPF_EINVAL, "sub_offset must start at 0 and end at n_bus");
        for (int32_t s = 0; s < n_sub; ++s)
            if (sub_offset[s + 1] < sub_offset[s]) return fail(DPF_EINVAL, "sub_offset must not decrease");
    }
    for (int32_t e = 0; e < n_branch; ++e)
        if (from[e] < 0 || from[e] >= n_bus || to[e] < 0 || to[e] >= n_bus)
            return fail(DPF_EINVAL, "branch end out of range");
    try {
        std::vector<int32_t> sub_of(n_bus, 0);
        for (int32_t s = 0; s < n_sub; ++s)
            for (int32_t i = sub_offset ? sub_offset[s] : 0; i < (sub_offset ? sub_offset[s + 1] : n_bus); ++i)
                sub_of[i] = s;
        // adjacency within each range, duplicates and self loops removed
        std::vector<int32_t> deg(n_bus + 1, 0);
        for (int32_t e = 0; e < n_branch; ++e)
            if (from[e] != to[e] && sub_of[from[e]] == sub_of[to[e]]) {
                ++deg[from[e]];
                ++deg[to[e]];
            }
        std::vector<int32_t> ptr(n_bus + 1, 0);
        for (int32_t i = 0; i < n_bus; ++i) ptr[i + 1] = ptr[i] + deg[i];
        std::vector<int32_t> adj(ptr[n_bus]), fill(ptr.begin(), ptr.end() - 1);
        for (int32_t e = 0; e < n_branch; ++e)
            if (from[e] != to[e] && sub_of[from[e]] == sub_of[to[e]]) {
                adj[fill[from[e]]++] = to[e];
                adj[fill[to[e]]++] = from[e];
            }
        for (int32_t i = 0; i < n_bus; ++i) {
            auto b = adj.begin() + ptr[i], en = adj.begin() + ptr[i + 1];
            std::sort(b, en);
            deg[i] = (int32_t)(std::unique(b, en) - b);
        }
        std::vector<int32_t> level(n_bus, -1), order, queue;
        std::vector<char> done(n_bus, 0);
        order.reserve(n_bus);
        queue.reserve(n_bus);
        // breadth-first levels from r inside its component; returns the last level's nodes
        auto bfs_last = [&](int32_t r, int32_t &depth) {
            queue.clear();
            queue.push_back(r);
            level[r] = 0;
            for (size_t h = 0; h < queue.size(); ++h) {
                int32_t u = queue[h];
                for (int32_t p = ptr[u]; p < ptr[u] + deg[u]; ++p)
                    if (level[adj[p]] < 0) {
                        level[adj[p]] = level[u] + 1;
                        queue.push_back(adj[p]);
                    }
            }
            depth = level[queue.back()];
            std::vector<int32_t> last;
            for (int32_t u : queue)
                if (level[u] == depth) last.push_back(u);
            for (int32_t u : queue) level[u] = -1;
            return last;
        };
        for (int32_t s = 0; s < n_sub; ++s) {
            const int32_t lo = sub_offset ? sub_offset[s] : 0, hi = sub_offset ? sub_offset[s + 1] : n_bus;
            const size_t first = order.size();
            for (;;) {
                // start of the next component: unvisited bus of least degree
                int32_t r = -1;
                for (int32_t i = lo; i < hi; ++i)
                    if (!done[i] && (r < 0 || deg[i] < deg[r])) r = i;
                if (r < 0) break;
                // pseudo-peripheral start: move to a least-degree bus of the last
                // level while the depth grows
                int32_t depth = 0;
                std::vector<int32_t> last = bfs_last(r, depth);
                for (int guard = 0; guard < 32; ++guard) {
                    int32_t c = last[0];
                    for (int32_t u : last)
                        if (deg[u] < deg[c]) c = u;
                    int32_t d2 = 0;
                    std::vector<int32_t> l2 = bfs_last(c, d2);
                    if (d2 <= depth) break;
                    r = c;
                    depth = d2;
                    last.swap(l2);
                }
                // Cuthill-McKee: breadth first, neighbours by increasing degree
                size_t head = order.size();
                order.push_back(r);
                done[r] = 1;
                std::vector<int32_t> nb;
                while (head < order.size()) {
                    int32_t u = order[head++];
                    nb.clear();
                    for (int32_t p = ptr[u]; p < ptr[u] + deg[u]; ++p)
                        if (!done[adj[p]]) nb.push_back(adj[p]);
                    std::stable_sort(nb.begin(), nb.end(), [&](int32_t x, int32_t y) { return deg[x] < deg[y]; });
                    for (int32_t v : nb) {
                        done[v] = 1;
                        order.push_back(v);
                    }
                }
            }
            std::reverse(order.begin() + first, order.end());
            if (group > 1)
                for (size_t w = first; w < order.size(); w += (size_t)group) {
                    auto we = order.begin() + std::min(order.size(), w + (size_t)group);
                    std::stable_sort(order.begin() + w, we, [&](int32_t x, int32_t y) { return deg[x] < deg[y]; });
                }
        }
        for (int32_t k = 0; k < n_bus; ++k) perm[k] = order[k];
        if (bandwidth_out) {
            std::vector<int32_t> inv(n_bus);
            for (int32_t k = 0; k < n_bus; ++k) inv[order[k]] = k;
            int32_t bw = 0;
            for (int32_t e = 0; e < n_branch; ++e)
                if (sub_of[from[e]] == sub_of[to[e]]) bw = std::max(bw, std::abs(inv[from[e]] - inv[to[e]]));
            *bandwidth_out = bw;
        }
    } catch (const std::bad_alloc &) {
        return fail(DPF_ENOMEM, "host allocation failed");
    }
    return DPF_OK;
}

int32_t dpf_solve_max_sub_buses(void) {
    DeviceInfo d;
    if (device_info(d) != DPF_OK) return 0;
    return max_sub_buses_for(d, 0);
}

// *forced_bad: the route names a variant that cannot hold the call's sub-grids
static CallPlan plan_call(const dpf_grid_t *g, int32_t n_sub, const int32_t *sub_offset, int32_t B,
                          const DeviceInfo &dev, const dpf_route_t &route, bool *forced_bad = nullptr) {
    CallPlan p;
    p.route = route;
    p.cap = max_sub_buses_for(dev, route.team_cap);
    int64_t small = 0;
    for (int32_t s = 0; s < (sub_offset ? n_sub : 1); ++s) {
        const int32_t ns = sub_offset ? sub_offset[s + 1] - sub_offset[s] : g->n_bus;
        if (ns <= p.cap) {
            ++small;
            p.n_max = std::max(p.n_max, ns);
        }
    }
    p.has_small = small > 0;
    bool few_large = false;
    p.v = pick_variant(std::max(1, p.n_max), (int64_t)B * small, dev.n_cu > 0 ? dev.n_cu : 256, route.variant,
                       &few_large);
    if (forced_bad) *forced_bad = route.variant >= 0 && !p.v;
    // few large items of one grid that the split kernel can hold, with the split
    // kernel enabled: it runs them from the first iteration (the multi-workgroup
    // path's iteration is launch-bound for a few items)
    if (few_large && route.tail_team > 0 && small == 1 && (!sub_offset || n_sub == 1) &&
        (size_t)p.n_max * 16 + (size_t)(p.n_max + 31) / 32 * 4 + 512 <= (size_t)dev.lds_per_block)
        p.split_direct = true;
    if (p.v && p.v->mode == dpf::kWide) {  // every sub-grid to the multi-workgroup path
        p.cap = 0;
        p.n_max = 0;
        p.has_small = false;
    }
    // sub-grids above the cap (or every sub-grid, when few large items chose the
    // multi-workgroup path by default): all items on persistent teams, unless the
    // route asks for the host-driven path or names it as the variant
    const bool any_large = p.v && small < (sub_offset ? (int64_t)n_sub : 1);
    const bool wide_named = route.variant >= 0 && p.v && p.v->mode == dpf::kWide;
    if (p.v && !p.split_direct && route.wide_host == 0 && !wide_named &&
        (any_large || p.v->mode == dpf::kWide)) {
        p.teams = true;
        p.has_small = false;
    }
    // tail handoff: single-grid calls whose per-item kernel keeps the state in global memory
    const int32_t h = route.tail_handoff;
    if (h > 0 && p.v && p.has_small && small == 1 && (!sub_offset || n_sub == 1) &&
        (p.v->mode == dpf::kGlobal || p.v->mode == dpf::kBandStream || p.v->mode == dpf::kPair))
        p.handoff = h;
    return p;
}

size_t dpf_solve_workspace_bytes(const dpf_grid_t *g, int32_t n_sub, const int32_t *sub_offset, int32_t B,
                                 int32_t ld, const dpf_route_t *route) {
    if (!g || g->n_bus <= 0 || B <= 0 || ld < g->n_bus) return 0;
    const dpf_route_t rt = route_of(route);
    if (route_error(rt)) return 0;
    if (!sub_offset) n_sub = 1;
    DeviceInfo dev;
    if (device_info(dev) != DPF_OK) {
        g_err.clear();
        dev.lds_per_block = kGfx950LdsBytes;  // no device visible: size for gfx950
        dev.n_cu = 256;
    }
    bool forced_bad = false;
    const CallPlan p = plan_call(g, n_sub, sub_offset, B, dev, rt, &forced_bad);
    if (forced_bad) return 0;
    return solve_layout(g, n_sub, sub_offset, B, ld, p.v && p.v->mode != dpf::kReg, p.cap,
                        p.handoff > 0 || p.split_direct, p.v && p.v->mode == dpf::kPair && p.has_small, p.teams)
        .total;
}

int dpf_solve_batch(const dpf_grid_t *g, int32_t n_sub, const int32_t *sub_offset, const int32_t *sub_offset_dev,
                    int32_t B, int32_t ld, const int8_t *bus_type, const double *s_spec, int32_t s_ld,
                    const int32_t *outage, double *vm, double *va, double *adam_state, double *sched_state,
                    const dpf_opts_t *opts, const dpf_route_t *route, int32_t *iters, int32_t *status,
                    double *max_mis, double *loss, int64_t *done_ns, const dpf_trace_t *trace, void *workspace,
                    size_t ws_bytes, void *stream) {
    g_err.clear();
    const dpf_route_t rt = route_of(route);
    if (const char *re = route_error(rt)) return fail(DPF_EINVAL, re);
    if (!valid_grid(g)) return fail(DPF_EINVAL, "invalid grid");
    if (B <= 0 || ld < g->n_bus) return fail(DPF_EINVAL, "B must be > 0 and ld >= n_bus");
    if (s_ld != 0 && s_ld < g->n_bus) return fail(DPF_EINVAL, "s_ld must be 0 or >= n_bus");
    if (!bus_type || !s_spec || !vm || !va || !iters || !status || !max_mis || !loss)
        return fail(DPF_EINVAL, "null argument");
    if (!valid_opts(opts)) return fail(DPF_EINVAL, "invalid optimizer options");
    if (trace && (trace->len < 0 || (trace->len > 0 && (trace->every <= 0 || !trace->max_mis))))
        return fail(DPF_EINVAL, "trace: len >= 0, and every > 0 with a buffer when len > 0");
    if ((sub_offset == nullptr) != (sub_offset_dev == nullptr))
        return fail(DPF_EINVAL, "sub_offset and sub_offset_dev: both or neither");
    if (!sub_offset) n_sub = 1;
    if (n_sub <= 0) return fail(DPF_EINVAL, "n_sub must be > 0");
    if (sub_offset) {
        if (sub_offset[0] != 0 || sub_offset[n_sub] != g->n_bus)
            return fail(DPF_EINVAL, "sub_offset must start at 0 and end at n_bus");
        for (int32_t s = 0; s < n_sub; ++s)
            if (sub_offset[s + 1] < sub_offset[s]) return fail(DPF_EINVAL, "sub_offset must not decrease");
    }
    if (outage && n_sub != 1) return fail(DPF_EUNSUPPORTED, "outages need a single sub-grid");
    if (outage && (g->n_branch <= 0 || !g->from || !g->to || !g->r || !g->x || !g->b))
        return fail(DPF_EINVAL, "outage needs the grid's branch arrays");
    if ((int64_t)B * n_sub > INT32_MAX / 2) return fail(DPF_EINVAL, "too many work items");
    DeviceInfo dev;
    int rc = device_info(dev);
    if (rc != DPF_OK) return rc;
    bool forced_bad = false;
    const CallPlan plan = plan_call(g, n_sub, sub_offset, B, dev, rt, &forced_bad);
    if (forced_bad) return fail(DPF_EINVAL, "route.variant cannot hold the call's largest sub-grid");
    const int32_t cap = plan.cap;  // larger sub-grids take the multi-workgroup path
    const int32_t n_max = plan.n_max;
    const bool has_small = plan.has_small;
    const Variant *v = plan.v;
    if (!v) return fail(DPF_EUNSUPPORTED, "no kernel variant");
    const bool handoff = plan.handoff > 0;
    if (rt.tail_device == 1 && (handoff || plan.split_direct) &&
        (size_t)g->n_bus * 16 + (size_t)(g->n_bus + 31) / 32 * 4 + 512 > (size_t)dev.lds_per_block)
        return fail(DPF_EUNSUPPORTED, "route.tail_device: the grid is too large for the split kernel");
    const bool pairs = v->mode == dpf::kPair && has_small;
    const SolveLayout L = solve_layout(g, n_sub, sub_offset, B, ld, v->mode != dpf::kReg, cap,
                                       handoff || plan.split_direct, pairs, plan.teams);
    const bool has_wide = L.w_total > 0;
    if (!workspace || ws_bytes < L.total) return fail(DPF_ENOMEM, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)workspace;
    int32_t *bad = (int32_t *)ws;
    int32_t *nslice = (int32_t *)(ws + L.off_nslice);
    int32_t *slice_off = (int32_t *)(ws + L.off_slice_off);
    int32_t *width = (int32_t *)(ws + L.off_width);
    int32_t *start = (int32_t *)(ws + L.off_start);
    int32_t *scol = (int32_t *)(ws + L.off_col);
    double2 *sval = (double2 *)(ws + L.off_val);
    int32_t *sub_bw = (int32_t *)(ws + L.off_bw);
    const int32_t wmax = g->max_row_nnz > 0 ? g->max_row_nnz : std::max<int32_t>(g->nnz, 1);
    if (done_ns) hipLaunchKernelGGL(dpf::stamp_kernel, dim3(1), dim3(64), 0, st, (int64_t *)(ws + 8));
    // sliced-ELL copy of Y for this call (the flag is cleared by a kernel, not a memset,
    // so that the whole call can be captured in a graph)
    if (n_sub <= dpf::kSellSmallSubs && L.n_slices <= dpf::kSellSmallSlices) {  // small grids: one launch
        hipLaunchKernelGGL(dpf::sell_small_kernel, dim3(1), dim3(dpf::kSellSmallThreads), 0, st, n_sub,
                           sub_offset_dev, g->n_bus, g->row_ptr, g->col_idx, (const double2 *)g->val, wmax, nslice,
                           slice_off, width, start, scol, sval, sub_bw, bad, bad + 4);
    } else {
        hipLaunchKernelGGL(dpf::sell_count_kernel, dim3((n_sub + 255) / 256), dim3(256), 0, st, n_sub,
                           sub_offset_dev, g->n_bus, nslice, sub_bw, bad, bad + 4);  // clears header words 0, 4 and 5
        hipLaunchKernelGGL(dpf::scan_kernel, dim3(1), dim3(1024), 0, st, n_sub, nslice, 0, slice_off);
        if (L.n_slices > 0) {
            hipLaunchKernelGGL(dpf::sell_width_kernel, dim3(L.n_slices), dim3(dpf::kWave), 0, st, n_sub,
                               sub_offset_dev, g->n_bus, slice_off, g->row_ptr, wmax, width, bad);
            hipLaunchKernelGGL(dpf::scan_kernel, dim3(1), dim3(1024), 0, st, L.n_slices, width, 0, start);
            hipLaunchKernelGGL(dpf::sell_fill_kernel, dim3(L.n_slices), dim3(dpf::kWave), 0, st, n_sub,
                               sub_offset_dev, g->n_bus, slice_off, g->row_ptr, g->col_idx, (const double2 *)g->val,
                               width, start, scol, sval, sub_bw);
        }
    }
    // cases with an outage index that is neither -1 nor a branch (after the header is cleared)
    if (outage)
        hipLaunchKernelGGL(dpf::outage_check_kernel, dim3((B + 255) / 256), dim3(256), 0, st, B,
                           dpf::OutageView{outage, g->from, g->to, g->r, g->x, g->b, g->n_branch}, status, iters,
                           max_mis, loss, bad + 5);
    DPF_HIP(hipGetLastError());

    dpf::SolveArgs a{};
    a.rp = g->row_ptr;
    a.ci = g->col_idx;
    a.yv = (const double2 *)g->val;
    a.bt = bus_type;
    a.s_spec = (const double2 *)s_spec;
    a.s_ld = s_ld;
    a.ov = dpf::OutageView{outage, g->from, g->to, g->r, g->x, g->b, g->n_branch};
    a.vm = vm;
    a.va = va;
    a.ld = ld;
    a.st_stride = (int64_t)B * ld;
    a.sell = dpf::SellView{slice_off, width, start, scol, sval};
    a.sub_bw = sub_bw;
    a.band_nt = 0;
    a.bad_grid = bad;
    a.done_count = bad + 5;  // header word 5: finished items (tail handoff)
    a.handoff = handoff ? plan.handoff : 0;
    a.total_items = B * n_sub;
    a.team_cap = cap;
    if (v->mode != dpf::kReg || has_wide || plan.teams) {
        double *mom = (double *)(ws + L.off_mom);
        a.scratch = (double2 *)(ws + L.off_scr);
        a.st = adam_state ? adam_state : mom;
    } else {
        a.scratch = nullptr;
        a.st = adam_state;  // may be null: fresh moments kept in registers only
    }
    a.st_fresh = adam_state ? 0 : 1;
    a.sched = sched_state;
    if ((handoff || plan.split_direct) && !sched_state) {  // paused items carry their schedule
        a.sched = (double *)(ws + L.off_sched);
        hipLaunchKernelGGL(dpf::sched_init_kernel, dim3((B + 255) / 256), dim3(256), 0, st, B, opts->lr, a.sched);
    }
    a.sub_off = sub_offset_dev;
    a.n_bus = g->n_bus;
    a.n_sub = n_sub;
    a.B = B;
    a.lr = opts->lr;
    a.opt = opts->optimizer;
    a.b1 = opts->beta1;
    a.b2 = opts->beta2;
    a.eps = opts->eps;
    a.tol = opts->tol;
    a.max_iter = opts->max_iter;
    a.sch = opts->sched;
    a.factor = opts->factor;
    a.patience = opts->patience;
    a.threshold = opts->threshold;
    a.cooldown = opts->cooldown;
    a.min_lr = opts->min_lr;
    a.sched_eps = opts->sched_eps;
    a.iters = iters;
    a.status = status;
    a.mu_out = max_mis;
    a.loss_out = loss;
    a.done_ns = done_ns;
    a.trace = trace && trace->len > 0 ? trace->max_mis : nullptr;
    a.trace_every = trace && trace->len > 0 ? trace->every : 1;
    a.trace_len = trace && trace->len > 0 ? trace->len : 0;
    a.stamp = (const int64_t *)(ws + 8);  // header words 2-3
    a.ns_per_tick = dev.ns_per_tick;

    // dynamic LDS: two exchange arrays when they fit, else one
    const int32_t lds_entries_max = (dev.lds_per_block - kSolveStaticLds) / 16;
    int32_t entries = 2 * n_max <= lds_entries_max ? 2 * n_max : n_max;
    entries = std::max<int32_t>(entries, 1);
    a.lds_cap = entries;
    const size_t lds_bytes = (size_t)entries * 16;
    const int32_t items = B * n_sub;
    // handoff calls of one grid may start their cases by descending initial max|r|:
    // the cases likely to run longest then do not start last (one evaluation of
    // every case with the mismatch kernels, into the solve's scratch, then a rank)
    if (handoff && !sub_offset && rt.case_order == 1 && B <= 16384) {
        const int32_t n = g->n_bus;
        const int32_t nblk = (n + dpf::kEvalBlock - 1) / dpf::kEvalBlock;
        int32_t *order = (int32_t *)(ws + L.off_order);
        double *key = (double *)(ws + L.off_order + align_up(sizeof(int32_t) * (size_t)B, 256));
        double *lossv = key + align_up(sizeof(double) * (size_t)B, 256) / sizeof(double);
        double *m_res = lossv + align_up(sizeof(double) * (size_t)B, 256) / sizeof(double);
        double2 *Vw = a.scratch, *ww = a.scratch + a.st_stride, *aIw = a.scratch + 2 * a.st_stride;
        double2 *part = (double2 *)(ws + L.off_part);  // B x slices >= B x nblk entries
        hipLaunchKernelGGL(dpf::residual_count_kernel, dim3(1), dim3(1024), 0, st, n, bus_type, m_res);
        hipLaunchKernelGGL(dpf::polar_kernel, dim3(nblk, B), dim3(dpf::kEvalBlock), 0, st, n, (int64_t)ld, vm, va,
                           Vw);
        hipLaunchKernelGGL(dpf::forward_kernel, dim3(nblk, B), dim3(dpf::kEvalBlock), 0, st, n, g->row_ptr,
                           g->col_idx, (const double2 *)g->val, bus_type, (const double2 *)s_spec, (int64_t)s_ld,
                           a.ov, Vw, m_res, (int64_t)ld, (double2 *)nullptr, ww, aIw, part, (double2 *)nullptr);
        hipLaunchKernelGGL(dpf::finalize_kernel, dim3((B + 255) / 256), dim3(256), 0, st, B, nblk, part, m_res, lossv,
                           key);
        hipLaunchKernelGGL(dpf::rank_desc_kernel, dim3((B + 255) / 256), dim3(256), 0, st, B, key, order);
        DPF_HIP(hipGetLastError());
        a.order = order;
    }
    if (plan.teams) return run_teams(a, L, ws, n_sub, B, dev, rt, st);
    const bool tail_device = rt.tail_device == 1 && rt.tail_team > 0 && !has_wide;
    std::unique_lock<std::mutex> side_lock;  // concurrent blocking calls on one device take turns
    if (has_wide || ((handoff || plan.split_direct) && !tail_device))
        side_lock = std::unique_lock<std::mutex>(g_side_mu[dev.index]);
    if (plan.split_direct && tail_device) {
        // every item starts paused at iteration 0, listed on the device
        int32_t *list = (int32_t *)(ws + L.off_list);
        hipLaunchKernelGGL(dpf::split_start_kernel, dim3((B + 255) / 256), dim3(256), 0, st, B, a.ov, a.status,
                           a.iters, list);
        if (a.st_fresh) {
            const int64_t words = 4 * (int64_t)B * ld;
            hipLaunchKernelGGL(dpf::zero_f64_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st, words,
                               a.st);
        }
        hipLaunchKernelGGL(dpf::collect_paused_kernel, dim3(1), dim3(1024), 0, st, B, a.status, list, bad + 6);
        DPF_HIP(hipGetLastError());
        return run_split_device(a, L, ws, dev, list, B, rt, st);
    }
    if (plan.split_direct) {
        // every item starts paused at iteration 0; the split kernel runs them, and any
        // it leaves (a team abandoned a barrier) finish on the multi-workgroup path
        int32_t *list = (int32_t *)(ws + L.off_list);
        hipLaunchKernelGGL(dpf::split_start_kernel, dim3((B + 255) / 256), dim3(256), 0, st, B, a.ov, a.status,
                           a.iters, list);
        if (a.st_fresh) {
            const int64_t words = 4 * (int64_t)B * ld;
            hipLaunchKernelGGL(dpf::zero_f64_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st, words,
                               a.st);
        }
        DPF_HIP(hipGetLastError());
        DPF_HIP(hipEventRecord(dev.ev_in, st));
        DPF_HIP(hipStreamWaitEvent(dev.side, dev.ev_in, 0));
        int32_t rest = B;
        int32_t *rest_list = list;
        int rc2 = run_split(a, L, ws, dev, list, B, B, rt, &rest, &rest_list);
        if (rc2 != DPF_OK) return rc2;
        rc2 = rest > 0 ? run_wide(a, L, ws, 1, nullptr, B, ld, 0, dev, rest_list, rest) : DPF_OK;
        if (rc2 != DPF_OK) return rc2;
        DPF_HIP(hipEventRecord(dev.ev_out, dev.side));
        DPF_HIP(hipStreamWaitEvent(st, dev.ev_out, 0));
        return DPF_OK;
    }
    if (has_wide) {
        DPF_HIP(hipEventRecord(dev.ev_in, st));
        DPF_HIP(hipStreamWaitEvent(dev.side, dev.ev_in, 0));
    }
    if (has_small) {
        const dim3 pgrid((g->n_bus + 255) / 256, std::min<int32_t>(B, 65535));
        double2 *P = a.scratch + a.st_stride;  // the pairs follow I in the scratch
        if (pairs)
            hipLaunchKernelGGL(dpf::pair_in_kernel, pgrid, dim3(256), 0, st, g->n_bus, (int64_t)ld, B, vm, va, a.st,
                               a.st_stride, a.st_fresh, P, P + a.st_stride, P + 2 * a.st_stride);
        DPF_HIP(hipFuncSetAttribute((const void *)v->fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds_bytes));
        hipLaunchKernelGGL(v->fn, dim3(items), dim3(v->nt), lds_bytes, st, a);
        DPF_HIP(hipGetLastError());
        // the pairs back to the caller's layout (every item, paused ones included) before
        // any other path reads the state
        if (pairs)
            hipLaunchKernelGGL(dpf::pair_out_kernel, pgrid, dim3(256), 0, st, g->n_bus, (int64_t)ld, B, vm, va, a.st,
                               a.st_stride, P, P + a.st_stride, P + 2 * a.st_stride);
        DPF_HIP(hipGetLastError());
        if (dpf::is_banded(v->mode)) {
            // items whose bandwidth exceeds the banded block go to the general variant
            int cnt = 0;
            const Variant *f = &variant_table(&cnt)[default_variant_index(std::max(1, n_max))];
            dpf::SolveArgs b = a;
            b.band_nt = v->nt * v->k;  // the banded block
            DPF_HIP(hipFuncSetAttribute((const void *)f->fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)lds_bytes));
            hipLaunchKernelGGL(f->fn, dim3(items), dim3(f->nt), lds_bytes, st, b);
            DPF_HIP(hipGetLastError());
        }
    }
    if (has_wide) {
        int rc2 = run_wide(a, L, ws, n_sub, sub_offset_dev, B, ld, cap, dev);
        if (rc2 != DPF_OK) return rc2;
        DPF_HIP(hipEventRecord(dev.ev_out, dev.side));
        DPF_HIP(hipStreamWaitEvent(st, dev.ev_out, 0));
    }
    if (handoff && tail_device) {
        // the items the per-item kernels paused finish on the split kernel, every
        // launch planned on the device
        int32_t *list = (int32_t *)(ws + L.off_list);
        hipLaunchKernelGGL(dpf::collect_paused_kernel, dim3(1), dim3(1024), 0, st, B, a.status, list, bad + 6);
        DPF_HIP(hipGetLastError());
        return run_split_device(a, L, ws, dev, list, B, rt, st);
    }
    if (handoff) {
        // the items the per-item kernels paused finish on the multi-workgroup path
        int32_t *list = (int32_t *)(ws + L.off_list);
        int32_t *n_paused = bad + 6;  // header word 6
        hipLaunchKernelGGL(dpf::collect_paused_kernel, dim3(1), dim3(1024), 0, st, B, a.status, list, n_paused);
        DPF_HIP(hipGetLastError());
        DPF_HIP(hipMemcpyAsync(dev.pinned_count, n_paused, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        DPF_HIP(hipEventRecord(dev.ev_poll, st));
        DPF_HIP(hipEventSynchronize(dev.ev_poll));
        const int32_t paused = *dev.pinned_count;
        if (paused > 0) {
            DPF_HIP(hipEventRecord(dev.ev_in, st));
            DPF_HIP(hipStreamWaitEvent(dev.side, dev.ev_in, 0));
            int32_t rest = paused;
            int32_t *rest_list = list;
            if (rt.tail_team > 0) {
                int rc2 = run_split(a, L, ws, dev, list, paused, B, rt, &rest, &rest_list);
                if (rc2 != DPF_OK) return rc2;
            }
            int rc2 = rest > 0 ? run_wide(a, L, ws, 1, nullptr, B, ld, 0, dev, rest_list, rest) : DPF_OK;
            if (rc2 != DPF_OK) return rc2;
            DPF_HIP(hipEventRecord(dev.ev_out, dev.side));
            DPF_HIP(hipStreamWaitEvent(st, dev.ev_out, 0));
        }
    }
    return DPF_OK;
}

size_t dpf_solve_series_workspace_bytes(const dpf_grid_t *g, int32_t window, int32_t ld,
                                        const dpf_route_t *route) {
    return dpf_solve_workspace_bytes(g, 1, nullptr, window, ld, route);
}

int dpf_solve_series(const dpf_grid_t *g, int32_t T, int32_t window, const int8_t *bus_type,
                     const double *s_series, int32_t s_ld, const double *vm0, const double *va0, double *vm,
                     double *va, int32_t ld, const dpf_opts_t *opts, const dpf_route_t *route, int32_t *iters,
                     int32_t *status, double *max_mis, double *loss, int64_t *done_ns, void *workspace,
                     size_t ws_bytes, void *stream) {
    g_err.clear();
    if (!valid_grid(g)) return fail(DPF_EINVAL, "invalid grid");
    if (T <= 0 || window <= 0 || ld < g->n_bus || s_ld < g->n_bus)
        return fail(DPF_EINVAL, "T and window must be > 0, ld and s_ld >= n_bus");
    if (!s_series || !vm0 || !va0 || !vm || !va || !bus_type || !iters || !status || !max_mis || !loss)
        return fail(DPF_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    for (int32_t t0 = 0; t0 < T; t0 += window) {
        const int32_t bw = std::min(window, T - t0);
        const double *src_m = t0 == 0 ? vm0 : vm + (int64_t)(t0 - 1) * ld;
        const double *src_a = t0 == 0 ? va0 : va + (int64_t)(t0 - 1) * ld;
        const int blocks = (g->n_bus + 255) / 256;
        hipLaunchKernelGGL(dpf::row_broadcast_kernel, dim3(blocks, bw), dim3(256), 0, st, g->n_bus, src_m, src_a,
                           vm + (int64_t)t0 * ld, va + (int64_t)t0 * ld, (int64_t)ld);
        DPF_HIP(hipGetLastError());
        int rc = dpf_solve_batch(g, 1, nullptr, nullptr, bw, ld, bus_type, s_series + 2 * (int64_t)t0 * s_ld, s_ld,
                                 nullptr, vm + (int64_t)t0 * ld, va + (int64_t)t0 * ld, nullptr, nullptr, opts,
                                 route, iters + t0, status + t0, max_mis + t0, loss + t0,
                                 done_ns ? done_ns + t0 : nullptr, nullptr, workspace, ws_bytes, stream);
        if (rc != DPF_OK) return rc;
    }
    return DPF_OK;
}

}  // extern "C"
