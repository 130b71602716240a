// Multi-workgroup solve for sub-grids larger than one CU's LDS ("wide" items).
//
// An iteration is three kernels over 64-row slices (one wave per slice of an
// item, any number of CUs per item):
//   wide_phase_a : I = Y V (global V), residual, seed -> w, a*I; per-slice loss
//                  and max partials (fixed reduction order)
//   wide_reduce  : one wave per item: loss, max|r|, stop test, Adam step count,
//                  learning-rate schedule -- the item's scalar state
//   wide_phase_b : h = Y^T w, gradient, Adam, new V
// Kernel boundaries order the global exchange vectors V and w between
// neighbouring slices.  Retired items are skipped by all three kernels.  The
// host enqueues chunks of iterations and polls the number of active items.
#pragma once

#include "../../include/dpf.h"
#include "common.hpp"
#include "eval.hpp"
#include "sell.hpp"

namespace dpf {

// scalar state of one item (indexed like the outputs: c * n_sub + s)
struct WideItem {
    double t, lr, best, b1t, b2t, loss, mu, lr_use;
    int64_t done;  // wall clock when the item stopped
    int32_t bad, cool, iters, status, active, owned;  // owned: run (and reported) by this path
};

struct WideArgs {
    SellView sell;
    const int32_t *sub_off;       // device [n_sub + 1] or null
    const int32_t *wide_off;      // [n_sub + 1] prefix of slices over wide sub-grids
    const int32_t *nslice;        // [n_sub] slices per sub-grid
    int32_t n_sub, B, n_bus, w_total;  // w_total = slices of all wide sub-grids (per case)
    const int8_t *bt;
    const double2 *s_spec;
    int64_t s_ld;
    OutageView ov;
    double *vm, *va;
    int64_t ld;
    double *st;          // moments [4][B][ld]
    int64_t st_stride;   // B * ld
    int32_t st_fresh;
    double2 *Vg, *Wg, *aIg;  // [B][ld] complex each
    double2 *part;       // [B][w_total] (loss partial, max partial)
    WideItem *items;     // [B * n_sub]
    const int32_t *bad_grid;  // set when a row exceeded the declared width bound
    const double *m_res; // [n_sub] residual count per sub-grid
    double *sched;       // caller schedule state or null
    double lr, b1, b2, eps, tol;
    int32_t opt;  // DPF_OPT_*
    int32_t max_iter, sch;
    double factor;
    int32_t patience;
    double threshold;
    int32_t cooldown;
    double min_lr, sched_eps;
    int32_t *iters, *status;
    double *mu_out, *loss_out;
    double *trace;       // per item [trace_len], max|r| every trace_every iterations, or null
    int32_t trace_every, trace_len;
    int32_t *active_count;
    int64_t *done_ns;
    const int64_t *stamp;
    double ns_per_tick;
    // tail handoff (single grid): the items listed here were paused by the per-item
    // kernels (status kPaused) and continue from their state and iteration count
    const int32_t *list;  // [n_list] item indices, or null: every wide item
    int32_t resume;
    int32_t n_units;      // (n_list, or B) * w_total: one wave per unit
};

struct WideUnit {
    int c, s, lo, hi, g, ws;  // case, sub-grid, row range, global slice, wide slice index
};

__device__ __forceinline__ WideUnit wide_unit(const WideArgs &a, int u) {
    WideUnit w;
    const int k = u / a.w_total;
    w.ws = u - k * a.w_total;
    w.c = a.list ? a.list[k] : k;  // with a list the call has one sub-grid: item index = case
    w.s = find_sub(w.ws, a.n_sub, a.wide_off);
    w.lo = a.sub_off ? a.sub_off[w.s] : 0;
    w.hi = a.sub_off ? a.sub_off[w.s + 1] : a.n_bus;
    w.g = a.sell.slice_off[w.s] + (w.ws - a.wide_off[w.s]);
    return w;
}

// residual counts m per sub-grid (one workgroup per sub-grid)
__global__ __launch_bounds__(256) void sub_residual_count_kernel(int32_t n_sub, const int32_t *__restrict__ sub_off,
                                                                 int32_t n_bus, const int8_t *__restrict__ bt,
                                                                 double *__restrict__ m_res) {
    __shared__ int part[256 / kWave];
    int s = blockIdx.x;
    int lo = sub_off ? sub_off[s] : 0, hi = sub_off ? sub_off[s + 1] : n_bus;
    int cnt = 0;
    for (int i = lo + (int)threadIdx.x; i < hi; i += 256) {
        int8_t t = bt[i];
        cnt += t == kPQ ? 2 : (t == kPV ? 1 : 0);
    }
    cnt = wave_isum(cnt);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) m_res[s] = (double)(part[0] + part[1] + part[2] + part[3]);
}

// slice counts restricted to wide sub-grids (n_s > cap)
__global__ void wide_count_kernel(int32_t n_sub, const int32_t *__restrict__ sub_off, int32_t n_bus, int32_t cap,
                                  const int32_t *__restrict__ nslice, int32_t *__restrict__ wcount) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sub) return;
    int lo = sub_off ? sub_off[s] : 0, hi = sub_off ? sub_off[s + 1] : n_bus;
    wcount[s] = (hi - lo) > cap ? nslice[s] : 0;
}

__global__ void wide_item_init_kernel(WideArgs a, int32_t cap) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.B * a.n_sub) return;
    int s = idx % a.n_sub;
    int lo = a.sub_off ? a.sub_off[s] : 0, hi = a.sub_off ? a.sub_off[s + 1] : a.n_bus;
    WideItem it{};
    it.active = (hi - lo) > cap ? 1 : 0;  // only wide items are run here
    if (a.resume) it.active = a.status[idx] == kPaused ? 1 : 0;
    // a bad outage index (one sub-grid: item = case) was reported by the prologue
    if (a.ov.outage && outage_index_bad(a.ov.outage[idx], a.ov.n_branch)) it.active = 0;
    it.owned = it.active;
    it.iters = a.resume && it.active ? a.iters[idx] : 0;
    it.t = 0.0;
    it.lr = a.lr;
    it.best = __longlong_as_double(0x7ff0000000000000LL);
    it.b1t = 1.0;
    it.b2t = 1.0;
    it.status = DPF_MAX_ITER;
    if (it.active && a.sched) {
        const double *ss = a.sched + 6 * (int64_t)idx;
        it.t = ss[0];
        it.lr = ss[1];
        it.best = ss[2];
        const int packed = (int)ss[3];
        it.bad = packed & 0xFFFFF;
        it.cool = packed >> 20;
        it.b1t = ss[4];
        it.b2t = ss[5];
    }
    if (it.active && *a.bad_grid) {  // see DPF_BAD_GRID (the schedule is written back unchanged)
        it.active = 0;
        it.status = DPF_BAD_GRID;
        it.iters = 0;
    }
    it.lr_use = it.lr;
    a.items[idx] = it;
}

// V = vm e^{j va} for every row of the wide items; fresh moments cleared
__global__ __launch_bounds__(256) void wide_init_rows_kernel(WideArgs a) {
    int u = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (u >= a.n_units) return;
    WideUnit w = wide_unit(a, u);
    int r = w.lo + (w.ws - a.wide_off[w.s]) * kWave + (threadIdx.x & (kWave - 1));
    if (r >= w.hi) return;
    const int64_t o = (int64_t)w.c * a.ld + r;
    double sn, cs;
    fast_sincos(a.va[o], sn, cs);
    const double m = a.vm[o];
    a.Vg[o] = make_double2(m * cs, m * sn);
    if (a.st_fresh) {
        a.st[o] = 0.0;
        a.st[a.st_stride + o] = 0.0;
        a.st[2 * a.st_stride + o] = 0.0;
        a.st[3 * a.st_stride + o] = 0.0;
    }
}

__device__ __forceinline__ double2 wide_outage_term(const WideArgs &a, int c, int r, const double2 *Zc) {
    if (!a.ov.outage) return make_double2(0.0, 0.0);
    const int32_t k = a.ov.outage[c];
    if ((uint32_t)k >= (uint32_t)a.ov.n_branch) return make_double2(0.0, 0.0);
    const int32_t f = a.ov.from[k], t = a.ov.to[k];
    if (r != f && r != t) return make_double2(0.0, 0.0);
    if ((uint32_t)f >= (uint32_t)a.n_bus || (uint32_t)t >= (uint32_t)a.n_bus || f == t) return make_double2(0.0, 0.0);
    return outage_term(a.ov, k, r, Zc[f], Zc[t], f, t);
}

__global__ __launch_bounds__(256) void wide_phase_a_kernel(WideArgs a) {
    int u = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (u >= a.n_units) return;
    WideUnit w = wide_unit(a, u);
    const int idx = w.c * a.n_sub + w.s;
    if (!a.items[idx].active) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int r = w.lo + (w.ws - a.wide_off[w.s]) * kWave + lane;
    const double2 *Vc = a.Vg + (int64_t)w.c * a.ld;
    double lsum = 0.0, lmax = 0.0;
    if (r < w.hi) {
        const int wdt = a.sell.width[w.g];
        const int base = a.sell.start[w.g] * kWave + lane;
        double2 acc = make_double2(0.0, 0.0);
        acc = sell_row<4, true>(a.sell.val, a.sell.col, base, wdt, r - w.lo, [&](int j) { return Vc[w.lo + j]; }, acc);
        acc = csub(acc, wide_outage_term(a, w.c, r, Vc));
        const int8_t tk = a.bt[r];
        const double2 v = Vc[r];
        const double2 d = csub(cmulc(v, acc), a.s_spec[(int64_t)w.c * a.s_ld + r]);
        const double rP = tk != kSlack ? d.x : 0.0;
        const double rQ = tk == kPQ ? d.y : 0.0;
        lsum = rP * rP + rQ * rQ;
        lmax = fmax(fabs(rP), fabs(rQ));
        const double mm = a.m_res[w.s];
        const double sc = mm > 0.0 ? 2.0 / mm : 0.0;
        const double2 av = make_double2(sc * rP, sc * rQ);
        const int64_t o = (int64_t)w.c * a.ld + r;
        a.Wg[o] = cmulc(av, v);
        a.aIg[o] = cmul(av, acc);
    }
    lsum = wave_sum(lsum);
    lmax = wave_max(lmax);
    if (lane == 0) a.part[(int64_t)w.c * a.w_total + w.ws] = make_double2(lsum, lmax);
}

// one wave per item (per listed item)
__global__ __launch_bounds__(kWave) void wide_reduce_kernel(WideArgs a) {
    const int idx = a.list ? a.list[blockIdx.x] : blockIdx.x;
    WideItem it = a.items[idx];
    if (!it.active) return;
    const int c = idx / a.n_sub, s = idx - c * a.n_sub;
    const int lane = threadIdx.x;
    const int s0 = a.wide_off[s], ns = a.wide_off[s + 1] - s0;
    double ls = 0.0, lm = 0.0;
    for (int k = lane; k < ns; k += kWave) {
        double2 p = a.part[(int64_t)c * a.w_total + s0 + k];
        ls += p.x;
        lm = fmax(lm, p.y);
    }
    ls = wave_sum(ls);
    lm = wave_max(lm);
    if (lane != 0) return;
    const double mm = a.m_res[s];
    it.loss = mm > 0.0 ? ls / mm : 0.0;
    it.mu = isnan(ls) ? ls : lm;
    if (a.trace_len > 0 && it.iters % a.trace_every == 0 && it.iters / a.trace_every < a.trace_len)
        a.trace[(int64_t)idx * a.trace_len + it.iters / a.trace_every] = it.mu;
    if (!(isfinite(it.loss) && isfinite(it.mu))) {
        it.status = DPF_NONFINITE;
        it.active = 0;
        it.done = wall_clock64();
    } else if (it.mu < a.tol) {
        it.status = DPF_CONVERGED;
        it.active = 0;
        it.done = wall_clock64();
    } else if (it.iters >= a.max_iter) {
        it.status = DPF_MAX_ITER;
        it.active = 0;
        it.done = wall_clock64();
    } else {
        // this iteration's update uses the current lr; the schedule step after it
        it.t += 1.0;
        it.b1t *= a.b1;
        it.b2t *= a.b2;
        it.lr_use = it.lr;
        it.iters += 1;
        if (a.sch == DPF_SCHED_PLATEAU) {
            if (it.loss < it.best * (1.0 - a.threshold)) {
                it.best = it.loss;
                it.bad = 0;
            } else {
                it.bad += 1;
            }
            if (it.cool > 0) {
                it.cool -= 1;
                it.bad = 0;
            }
            if (it.bad > a.patience) {
                double nl = it.lr * a.factor;
                if (nl < a.min_lr) nl = a.min_lr;
                if (it.lr - nl > a.sched_eps) it.lr = nl;
                it.cool = a.cooldown;
                it.bad = 0;
            }
        } else if (a.sch == DPF_SCHED_STEP) {
            // keyed on the persistent step count, as in the per-item kernels
            if (a.patience > 0 && ((int64_t)it.t % a.patience) == 0) it.lr = it.lr * a.factor;
        }
    }
    a.items[idx] = it;
}

__global__ __launch_bounds__(256) void wide_phase_b_kernel(WideArgs a) {
    int u = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (u >= a.n_units) return;
    WideUnit w = wide_unit(a, u);
    const int idx = w.c * a.n_sub + w.s;
    const WideItem &it = a.items[idx];
    if (!it.active) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int r = w.lo + (w.ws - a.wide_off[w.s]) * kWave + lane;
    if (r >= w.hi) return;
    const double2 *Wc = a.Wg + (int64_t)w.c * a.ld;
    const int wdt = a.sell.width[w.g];
    const int base = a.sell.start[w.g] * kWave + lane;
    double2 h = make_double2(0.0, 0.0);
    h = sell_row<4, true>(a.sell.val, a.sell.col, base, wdt, r - w.lo, [&](int j) { return Wc[w.lo + j]; }, h);
    h = csub(h, wide_outage_term(a, w.c, r, Wc));
    const int64_t o = (int64_t)w.c * a.ld + r;
    const double2 ai = a.aIg[o];
    const double2 G = make_double2(ai.x + h.x, ai.y - h.y);
    const double2 v = a.Vg[o];
    const int8_t tk = a.bt[r];
    const double lr = it.lr_use;
    const double bc1 = 1.0 - it.b1t, bc2 = 1.0 - it.b2t;
    double vmi = a.vm[o], vai = a.va[o];
    if (tk == kPQ) {
        const double g = (G.x * v.x + G.y * v.y) / vmi;
        double mv = a.st[o], sv = a.st[2 * a.st_stride + o];
        vmi = opt_update(a.opt, lr, a.b1, a.b2, a.eps, bc1, bc2, vmi, g, mv, sv);
        a.vm[o] = vmi;
        a.st[o] = mv;
        a.st[2 * a.st_stride + o] = sv;
    }
    if (tk != kSlack) {
        const double g = G.y * v.x - G.x * v.y;
        double ma = a.st[a.st_stride + o], sa = a.st[3 * a.st_stride + o];
        vai = opt_update(a.opt, lr, a.b1, a.b2, a.eps, bc1, bc2, vai, g, ma, sa);
        a.va[o] = vai;
        a.st[a.st_stride + o] = ma;
        a.st[3 * a.st_stride + o] = sa;
    }
    double sn, cs;
    fast_sincos(vai, sn, cs);
    a.Vg[o] = make_double2(vmi * cs, vmi * sn);
}

// number of active wide items (one workgroup)
__global__ __launch_bounds__(256) void wide_active_count_kernel(WideArgs a) {
    __shared__ int part[256 / kWave];
    int cnt = 0;
    for (int i = threadIdx.x; i < a.B * a.n_sub; i += 256) cnt += a.items[i].active;
    cnt = wave_isum(cnt);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) *a.active_count = part[0] + part[1] + part[2] + part[3];
}

// the still active entries of a list of n items (one workgroup), written to out;
// their number goes to *a.active_count
__global__ __launch_bounds__(1024) void wide_compact_kernel(WideArgs a, int32_t n, int32_t *__restrict__ out) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int32_t idx = a.list[i];
        if (a.items[idx].active) out[atomicAdd(&cnt, 1)] = idx;
    }
    __syncthreads();
    if (threadIdx.x == 0) *a.active_count = cnt;
}

// outputs of the wide items
__global__ void wide_finish_kernel(WideArgs a, int32_t cap) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.B * a.n_sub) return;
    WideItem it = a.items[idx];
    if (!it.owned) return;
    a.iters[idx] = it.iters;
    a.status[idx] = it.status;
    a.mu_out[idx] = it.mu;
    a.loss_out[idx] = it.loss;
    if (a.done_ns) a.done_ns[idx] = (int64_t)((double)(it.done - *a.stamp) * a.ns_per_tick);
    if (a.sched) {
        double *ss = a.sched + 6 * (int64_t)idx;
        ss[0] = it.t;
        ss[1] = it.lr;
        ss[2] = it.best;
        ss[3] = (double)(it.bad + (it.cool << 20));
        ss[4] = it.b1t;
        ss[5] = it.b2t;
    }
}

}  // namespace dpf
