// Persistent DPF solve: one workgroup owns one work item (a case of a sub-grid)
// and runs the whole Adam iteration of Algorithm 1 for it inside the kernel.
//
// Why this shape on gfx950: a solve needs two grid-wide exchanges per
// iteration (the adjoint product needs every neighbour's residual seed, the next
// forward product needs every neighbour's updated voltage).  Keeping one item
// inside one workgroup turns both into LDS traffic plus workgroup barriers: the
// complex exchange vector X (16 B per bus) lives in LDS, so a sub-grid of up to
// ~10k buses fits in the 160 KB of one CU.  Converged items simply leave the
// kernel; the hardware dispatcher then starts the next item on that CU.
//
// Per iteration, for every bus i owned by the thread (i = lo + tid + k*NT):
//   A: I_i = sum_j Y_ij X_j (X = V) [- outage block];  dS_i = V_i conj(I_i) - S_i
//      r^P = [PV|PQ] Re dS, r^Q = [PQ] Im dS; loss and max|r| (workgroup reduce)
//      a_i = (2/m)(r^P + j r^Q); w_i = a_i conj(V_i); keep a_i I_i
//   stop test on max|r| (before the update, as the loop's convergence check)
//   B: h_i = sum_j Y_ij X_j (X = w; Y^T = Y) [- outage block]
//      G_i = a_i I_i + conj(h_i); g_vm = Re(conj(G) V)/vm at PQ; g_va = Im(G conj V)
//      Adam on the learnable entries; V_i = vm e^{j va}
// Two storage modes:
//   kReg    : the item's state (vm, va, Adam moments, S_spec, V, aI) stays in
//             registers for the whole solve (small sub-grids, K <= 2).
//   kGlobal : state in global memory (the caller's vm/va/adam arrays, scratch
//             for V and a*I), streamed once per iteration (large sub-grids).
// LDS is double-buffered (separate V and w arrays, 2 barriers per iteration)
// when 2n complex values fit, single-buffered (4 barriers) otherwise.
#pragma once

#include "../../include/dpf.h"
#include "common.hpp"
#include "eval.hpp"
#include "sell.hpp"

namespace dpf {

enum StoreMode {
    kReg = 0,         // state in registers
    kGlobal = 1,      // streaming: state in global memory
    kBandStream = 2,  // banded, barrier-free gradient sweep
    kWide = 3,        // the multi-workgroup path for a whole call
    kPair = 4         // banded, state kept as (|V|, theta) and moment pairs
};
__host__ __device__ constexpr bool is_banded(int mode) { return mode == kBandStream || mode == kPair; }

constexpr int kSchedWords = 6;  // per-item schedule state, see SolveArgs::sched

struct SolveArgs {
    const int32_t *rp;
    const int32_t *ci;
    const double2 *yv;
    const int8_t *bt;
    const double2 *s_spec;
    int64_t s_ld;
    OutageView ov;
    double *vm;
    double *va;
    int64_t ld;
    double *st;          // Adam moments [4][B][ld]
    int64_t st_stride;   // B * ld
    int32_t st_fresh;    // moments start at zero
    double2 *scratch;    // streaming: [3][B][ld] complex (V, a*I, w)
    double *sched;       // [items][6] (t, lr, best, bad + cooldown * 2^20, b1^t, b2^t) or null
    const int32_t *sub_off;  // device [n_sub + 1] or null
    SellView sell;           // sliced-ELL copy of Y (local columns)
    const int32_t *sub_bw;   // [n_sub] largest |row - col| of the sub-grid's matrix (local indices)
    int32_t band_nt;         // > 0: sub-grids with sub_bw <= band_nt belong to the banded kernel
    int32_t team_cap;        // items above this size belong to the multi-workgroup path
    const int32_t *bad_grid; // set when a row exceeded the declared width bound
    int32_t handoff;         // > 0: tail handoff threshold in unfinished items (see handoff_due)
    int32_t total_items;     // items of the call
    int32_t *done_count;     // items finished so far (handoff only), cleared per call
    const int32_t *order;    // [items] item taken by workgroup k, or null: workgroup k takes item k
    int32_t n_bus;
    int32_t n_sub;
    int32_t B;
    int32_t lds_cap;     // complex entries available in dynamic LDS
    double lr, b1, b2, eps, tol;
    int32_t opt;  // DPF_OPT_*
    int32_t max_iter;
    int32_t sch;
    double factor;
    int32_t patience;
    double threshold;
    int32_t cooldown;
    double min_lr;
    double sched_eps;
    int32_t *iters;
    int32_t *status;
    double *mu_out;
    double *loss_out;
    int64_t *done_ns;         // per item: ns from the call's start stamp to completion, or null
    double *trace;            // per item [trace_len]: max|r| every trace_every iterations, or null
    int32_t trace_every, trace_len;
    const int64_t *stamp;     // wall clock at the start of the call
    double ns_per_tick;
};

template <int NT>
__device__ __forceinline__ void block_reduce2(double &s, double &m, double (*red)[NT / kWave]) {
    s = wave_sum(s);
    m = wave_max(m);
    const int wv = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        red[0][wv] = s;
        red[1][wv] = m;
    }
}

template <int NT>
__device__ __forceinline__ void block_reduce2_finish(double &s, double &m, double (*red)[NT / kWave]) {
    s = 0.0;
    m = 0.0;
#pragma unroll
    for (int k = 0; k < NT / kWave; ++k) {
        s += red[0][k];
        m = fmax(m, red[1][k]);
    }
    s = uniform(s);  // every lane read the same partials
    m = uniform(m);
}

// Per-item step count and learning-rate schedule, kept across calls in
// SolveArgs::sched as {t, lr, best, bad + cooldown * 2^20, b1^t, b2^t}.
struct ItemSched {
    double t_step, lr, best, b1t, b2t;
    int bad, cool;
};

__device__ __forceinline__ ItemSched load_item_sched(const SolveArgs &a, int out_idx) {
    ItemSched s{0.0, a.lr, __longlong_as_double(0x7ff0000000000000LL), 1.0, 1.0, 0, 0};
    if (a.sched) {
        const double *ss = a.sched + kSchedWords * (int64_t)out_idx;
        s.t_step = ss[0];
        s.lr = ss[1];
        s.best = ss[2];
        const int packed = (int)ss[3];
        s.bad = packed & 0xFFFFF;
        s.cool = packed >> 20;
        s.b1t = ss[4];
        s.b2t = ss[5];
    }
    return s;
}

// scheduler step after an optimizer step (uniform across the workgroup; s.t_step
// already counts that step): PyTorch's reduce-on-plateau (mode min, relative
// threshold) or StepLR.  StepLR decays after every `patience`-th update of the
// item's persistent step count, so a call resumed from its schedule state keeps
// the phase of the decay (PyTorch's StepLR counts scheduler steps across epochs
// the same way).
__device__ __forceinline__ void sched_step(const SolveArgs &a, ItemSched &s, double loss) {
    if (a.sch == DPF_SCHED_PLATEAU) {
        if (loss < s.best * (1.0 - a.threshold)) {
            s.best = loss;
            s.bad = 0;
        } else {
            s.bad += 1;
        }
        if (s.cool > 0) {
            s.cool -= 1;
            s.bad = 0;
        }
        if (s.bad > a.patience) {
            double nl = s.lr * a.factor;
            if (nl < a.min_lr) nl = a.min_lr;
            if (s.lr - nl > a.sched_eps) s.lr = nl;
            s.cool = a.cooldown;
            s.bad = 0;
        }
    } else if (a.sch == DPF_SCHED_STEP) {
        if (a.patience > 0 && ((int64_t)s.t_step % a.patience) == 0) s.lr = s.lr * a.factor;
    }
}

// Tail handoff.  Early retirement leaves the last items of a batch alone on
// their CUs, one workgroup each; once at most a.handoff items of the call are
// unfinished, the per-item kernels stop them (status kPaused, state in global
// memory, schedule in a.sched) and the host finishes them on the multi-workgroup
// path, which spreads every item over many CUs.  Checked every 32 iterations;
// thread 0 reads the counter and the decision reaches the workgroup through LDS.
__device__ __forceinline__ bool handoff_due(const SolveArgs &a, int it, int *flag) {
    if (a.handoff <= 0 || it == 0 || (it & 31) != 0) return false;
    if (threadIdx.x == 0)
        *flag = a.total_items - __hip_atomic_load(a.done_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <=
                a.handoff;
    __syncthreads();
    return *flag != 0;
}

// optional trace of the stop-test quantity: max|r| of iteration `it` of this call
// (tested before its update) goes to slot it / trace_every when it is a multiple
// of trace_every and the slot exists; one thread writes (thread 0 of `writer`)
__device__ __forceinline__ void trace_mu(const SolveArgs &a, bool writer, int out_idx, int it, double mu) {
    if (a.trace_len > 0 && writer && threadIdx.x == 0 && it % a.trace_every == 0 && it / a.trace_every < a.trace_len)
        a.trace[(int64_t)out_idx * a.trace_len + it / a.trace_every] = mu;
}

// per-item results and the schedule state, written by one thread
__device__ __forceinline__ void finish_item(const SolveArgs &a, int out_idx, int it, int stat, double mu, double loss,
                                            const ItemSched &s) {
    if (a.handoff > 0 && stat != kPaused) atomicAdd(a.done_count, 1);
    a.iters[out_idx] = it;
    a.status[out_idx] = stat;
    a.mu_out[out_idx] = mu;
    a.loss_out[out_idx] = loss;
    if (a.done_ns) a.done_ns[out_idx] = (int64_t)((double)(wall_clock64() - *a.stamp) * a.ns_per_tick);
    if (a.sched) {
        double *ss = a.sched + kSchedWords * (int64_t)out_idx;
        ss[0] = s.t_step;
        ss[1] = s.lr;
        ss[2] = s.best;
        ss[3] = (double)(s.bad + (s.cool << 20));
        ss[4] = s.b1t;
        ss[5] = s.b2t;
    }
}

// residual count m = n_pv + 2 n_pq of buses [lo, hi) (workgroup reduction)
template <int NT>
__device__ __forceinline__ double residual_count(const int8_t *__restrict__ bt, int lo, int hi,
                                                 double (*red)[NT / kWave]) {
    double cnt = 0.0, dummy = 0.0;
    for (int i = lo + (int)threadIdx.x; i < hi; i += NT) {
        const int8_t t = bt[i];
        cnt += t == kPQ ? 2.0 : (t == kPV ? 1.0 : 0.0);
    }
    block_reduce2<NT>(cnt, dummy, red);
    __syncthreads();
    block_reduce2_finish<NT>(cnt, dummy, red);
    __syncthreads();
    return cnt;
}

// the N-1 branch of case c as local bus indices and its pi-model blocks
// (of = ot = -1 when the case has no outage inside [lo, hi)); bad: the index is
// neither -1 nor a branch index, and the kernels leave the case alone (the call's
// prologue, outage_check_kernel, reports it)
struct Rank2 {
    int of, ot;
    double2 oy, oyd;
    bool bad;
};

__device__ __forceinline__ Rank2 outage_of_case(const OutageView &ov, int c, int lo, int hi) {
    Rank2 r{-1, -1, make_double2(0.0, 0.0), make_double2(0.0, 0.0), false};
    if (ov.outage) {
        const int32_t k = ov.outage[c];
        r.bad = outage_index_bad(k, ov.n_branch);
        if ((uint32_t)k < (uint32_t)ov.n_branch) {
            const int32_t f = ov.from[k], t = ov.to[k];
            if (f >= lo && f < hi && t >= lo && t < hi && f != t) {
                r.of = f - lo;
                r.ot = t - lo;
                double2 ysh;
                branch_admittance(ov.r[k], ov.x[k], ov.b[k], r.oy, ysh);
                r.oyd = cadd(r.oy, ysh);
            }
        }
    }
    return r;
}

template <int NT, int K, int MODE>
__global__ __launch_bounds__(NT) void team_solve_kernel(SolveArgs a) {
    extern __shared__ double2 X[];
    __shared__ double red[2][NT / kWave];
    constexpr bool REG = MODE == kReg;

    const int tid = threadIdx.x;
    const int item = a.order ? a.order[blockIdx.x] : (int)blockIdx.x;
    const int sidx = item / a.B;
    const int c = item - sidx * a.B;
    const int lo = a.sub_off ? a.sub_off[sidx] : 0;
    const int hi = a.sub_off ? a.sub_off[sidx + 1] : a.n_bus;
    const int n = hi - lo;
    const int out_idx = c * a.n_sub + sidx;
    if (n > a.team_cap) return;  // handled by the multi-workgroup path
    if (a.band_nt > 0 && a.sub_bw[sidx] <= a.band_nt) return;  // handled by the banded kernel
    if (n < 0 || n > NT * K || n > a.lds_cap || *a.bad_grid) {  // see DPF_BAD_GRID
        if (tid == 0) {
            a.status[out_idx] = DPF_BAD_GRID;
            a.iters[out_idx] = 0;
        }
        return;
    }
    const int slice0 = a.sell.slice_off[sidx];
    const int lane = tid & (kWave - 1);
    const bool dbl = 2 * n <= a.lds_cap;
    double2 *Xv = X;
    double2 *Xw = dbl ? X + n : X;

    // step count and schedule (a resumed solve continues them)
    ItemSched sc = load_item_sched(a, out_idx);

    const double m_res = residual_count<NT>(a.bt, lo, hi, red);
    const double two_over_m = m_res > 0.0 ? 2.0 / m_res : 0.0;

    // N-1 outage of this case (only meaningful for a single sub-grid)
    const Rank2 r2 = outage_of_case(a.ov, c, lo, hi);
    if (r2.bad) return;  // reported by the call's prologue
    const int of = r2.of, ot = r2.ot;
    const double2 oy = r2.oy, oyd = r2.oyd;

    const int64_t cb = (int64_t)c * a.ld;
    const int64_t sb = (int64_t)c * a.s_ld;
    double *vm_c = a.vm + cb;
    double *va_c = a.va + cb;
    double *mv_c = a.st + cb;
    double *ma_c = a.st + a.st_stride + cb;
    double *sv_c = a.st + 2 * a.st_stride + cb;
    double *sa_c = a.st + 3 * a.st_stride + cb;
    double2 *Vg = a.scratch ? a.scratch + cb : nullptr;
    double2 *aIg = a.scratch ? a.scratch + a.st_stride + cb : nullptr;

    // Per-bus registers.  kReg keeps the whole item state; kGlobal keeps only
    // `hold` (w or the new V across the single-buffer barrier).
    constexpr int KR = REG ? K : 1;
    double2 V[KR], aI[KR], Sr[KR];
    double vmr[KR], var_[KR], mvr[KR], mar[KR], svr[KR], sar[KR];
    int8_t ty[KR];
    double2 hold[K];

#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = lo + tid + k * NT;
        hold[k] = make_double2(0.0, 0.0);
        if (REG) {
            ty[k % KR] = kSlack;
            V[k % KR] = aI[k % KR] = Sr[k % KR] = make_double2(0.0, 0.0);
            vmr[k % KR] = var_[k % KR] = mvr[k % KR] = mar[k % KR] = svr[k % KR] = sar[k % KR] = 0.0;
        }
        if (i < hi) {
            const double vmi = vm_c[i], vai = va_c[i];
            double sn, cs;
            fast_sincos(vai, sn, cs);
            const double2 v = make_double2(vmi * cs, vmi * sn);
            if (REG) {
                ty[k % KR] = a.bt[i];
                V[k % KR] = v;
                vmr[k % KR] = vmi;
                var_[k % KR] = vai;
                Sr[k % KR] = a.s_spec[sb + i];
                if (!a.st_fresh) {
                    mvr[k % KR] = mv_c[i];
                    mar[k % KR] = ma_c[i];
                    svr[k % KR] = sv_c[i];
                    sar[k % KR] = sa_c[i];
                }
            } else {
                Vg[i] = v;
                if (a.st_fresh) {
                    mv_c[i] = 0.0;
                    ma_c[i] = 0.0;
                    sv_c[i] = 0.0;
                    sa_c[i] = 0.0;
                }
            }
            Xv[i - lo] = v;
        }
    }
    __syncthreads();

    int it = 0, stat = DPF_MAX_ITER;
    double mu = 0.0, loss = 0.0;
    __shared__ int pause_flag;
    for (;; ++it) {
        if (!REG && handoff_due(a, it, &pause_flag)) {
            stat = kPaused;
            break;
        }
        // ---------------- phase A: forward product, residual, loss, seed
        double lsum = 0.0, lmax = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = lo + tid + k * NT;
            if (i < hi) {
                const int8_t tk = REG ? ty[k % KR] : a.bt[i];
                const int il = i - lo;
                const int gsl = __builtin_amdgcn_readfirstlane(slice0 + (il >> 6));
                const int wdt = a.sell.width[gsl];
                const int base = a.sell.start[gsl] * kWave + lane;
                double2 acc = make_double2(0.0, 0.0);
                acc = sell_row<4, true>(a.sell.val, a.sell.col, base, wdt, il, [&](int j) { return Xv[j]; }, acc);
                if (il == of) acc = csub(acc, csub(cmul(oyd, Xv[of]), cmul(oy, Xv[ot])));
                else if (il == ot) acc = csub(acc, csub(cmul(oyd, Xv[ot]), cmul(oy, Xv[of])));
                const double2 v = REG ? V[k % KR] : Xv[il];
                const double2 s = REG ? Sr[k % KR] : a.s_spec[sb + i];
                const double2 d = csub(cmulc(v, acc), s);
                const double rP = tk != kSlack ? d.x : 0.0;
                const double rQ = tk == kPQ ? d.y : 0.0;
                lsum += rP * rP + rQ * rQ;
                lmax = fmax(lmax, fmax(fabs(rP), fabs(rQ)));
                const double2 av = make_double2(two_over_m * rP, two_over_m * rQ);
                const double2 w = cmulc(av, v);
                if (REG) aI[k % KR] = cmul(av, acc);
                else aIg[i] = cmul(av, acc);
                if (dbl) Xw[il] = w;
                else hold[k] = w;
            }
        }
        block_reduce2<NT>(lsum, lmax, red);
        __syncthreads();
        if (!dbl) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int i = lo + tid + k * NT;
                if (i < hi) Xw[i - lo] = hold[k];
            }
        }
        block_reduce2_finish<NT>(lsum, lmax, red);
        loss = m_res > 0.0 ? lsum / m_res : 0.0;
        mu = isnan(lsum) ? lsum : lmax;
        trace_mu(a, true, out_idx, it, mu);
        if (!dbl) __syncthreads();  // w fully in X before phase B reads it
        if (!(isfinite(loss) && isfinite(mu))) {
            stat = DPF_NONFINITE;
            break;
        }
        if (mu < a.tol) {
            stat = DPF_CONVERGED;
            break;
        }
        if (it >= a.max_iter) {
            stat = DPF_MAX_ITER;
            break;
        }

        // ---------------- phase B: adjoint product, gradient, Adam
        sc.t_step += 1.0;
        sc.b1t *= a.b1;
        sc.b2t *= a.b2;
        const double bc1 = 1.0 - sc.b1t;
        const double bc2 = 1.0 - sc.b2t;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = lo + tid + k * NT;
            if (i < hi) {
                const int8_t tk = REG ? ty[k % KR] : a.bt[i];
                const int il = i - lo;
                const int gsl = __builtin_amdgcn_readfirstlane(slice0 + (il >> 6));
                const int wdt = a.sell.width[gsl];
                const int base = a.sell.start[gsl] * kWave + lane;
                double2 h = make_double2(0.0, 0.0);
                h = sell_row<4, true>(a.sell.val, a.sell.col, base, wdt, il, [&](int j) { return Xw[j]; }, h);
                if (il == of) h = csub(h, csub(cmul(oyd, Xw[of]), cmul(oy, Xw[ot])));
                else if (il == ot) h = csub(h, csub(cmul(oyd, Xw[ot]), cmul(oy, Xw[of])));
                double2 v, ai;
                double vmi, vai, mv = 0.0, ma = 0.0, sv = 0.0, sa = 0.0;
                if (REG) {
                    v = V[k % KR];
                    ai = aI[k % KR];
                    vmi = vmr[k % KR];
                    vai = var_[k % KR];
                    mv = mvr[k % KR];
                    ma = mar[k % KR];
                    sv = svr[k % KR];
                    sa = sar[k % KR];
                } else {
                    v = Vg[i];
                    ai = aIg[i];
                    vmi = vm_c[i];
                    vai = va_c[i];
                }
                const double2 G = make_double2(ai.x + h.x, ai.y - h.y);
                if (tk == kPQ) {
                    if (!REG) {
                        mv = mv_c[i];
                        sv = sv_c[i];
                    }
                    const double g = (G.x * v.x + G.y * v.y) / vmi;
                    vmi = opt_update(a.opt, sc.lr, a.b1, a.b2, a.eps, bc1, bc2, vmi, g, mv, sv);
                    if (!REG) {
                        vm_c[i] = vmi;
                        mv_c[i] = mv;
                        sv_c[i] = sv;
                    }
                }
                if (tk != kSlack) {
                    if (!REG) {
                        ma = ma_c[i];
                        sa = sa_c[i];
                    }
                    const double g = G.y * v.x - G.x * v.y;
                    vai = opt_update(a.opt, sc.lr, a.b1, a.b2, a.eps, bc1, bc2, vai, g, ma, sa);
                    if (!REG) {
                        va_c[i] = vai;
                        ma_c[i] = ma;
                        sa_c[i] = sa;
                    }
                }
                double sn, cs;
                fast_sincos(vai, sn, cs);
                v = make_double2(vmi * cs, vmi * sn);
                if (REG) {
                    V[k % KR] = v;
                    vmr[k % KR] = vmi;
                    var_[k % KR] = vai;
                    mvr[k % KR] = mv;
                    mar[k % KR] = ma;
                    svr[k % KR] = sv;
                    sar[k % KR] = sa;
                } else {
                    Vg[i] = v;
                }
                if (dbl) Xv[il] = v;
                else hold[k] = v;
            }
        }
        // ---------------- schedule step (uniform across the workgroup)
        sched_step(a, sc, loss);
        if (!dbl) {
            __syncthreads();
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int i = lo + tid + k * NT;
                if (i < hi) Xv[i - lo] = hold[k];
            }
        }
        __syncthreads();
    }

    // ---------------- write back
    if (REG) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = lo + tid + k * NT;
            if (i < hi) {
                if (ty[k % KR] == kPQ) vm_c[i] = vmr[k % KR];
                if (ty[k % KR] != kSlack) va_c[i] = var_[k % KR];
                if (!a.st_fresh) {
                    mv_c[i] = mvr[k % KR];
                    ma_c[i] = mar[k % KR];
                    sv_c[i] = svr[k % KR];
                    sa_c[i] = sar[k % KR];
                }
            }
        }
    }
    if (tid == 0) finish_item(a, out_idx, it, stat, mu, loss, sc);
}

// Streaming variant for large sub-grids.  Every per-bus value lives in global
// memory (the caller's vm/va/Adam arrays and the scratch arrays a*I and w) and
// is streamed once per iteration, with a runtime loop over any number of buses
// per thread.  With the single-buffered LDS exchange, w goes through the scratch
// array W and the new V is rebuilt from |V| and theta (both L2-resident), which
// keeps the register count low enough for 1024-thread workgroups; the per-bus
// address arithmetic is re-derived inside the iteration (opaque_index) instead
// of being kept live.
__device__ __forceinline__ uint32_t opaque_index(uint32_t i) {
    asm volatile("" : "+v"(i));
    return i;
}

template <int NT>
__global__ __launch_bounds__(NT) void team_solve_stream_kernel(SolveArgs a) {
    extern __shared__ double2 X[];
    __shared__ double red[2][NT / kWave];

    const int tid = threadIdx.x;
    const int item = a.order ? a.order[blockIdx.x] : (int)blockIdx.x;
    const int sidx = item / a.B;
    const int c = item - sidx * a.B;
    const int lo = a.sub_off ? a.sub_off[sidx] : 0;
    const int hi = a.sub_off ? a.sub_off[sidx + 1] : a.n_bus;
    const int n = hi - lo;
    const int out_idx = c * a.n_sub + sidx;
    if (n > a.team_cap) return;  // handled by the multi-workgroup path
    if (a.band_nt > 0 && a.sub_bw[sidx] <= a.band_nt) return;  // handled by the banded kernel
    if (n < 0 || n > a.lds_cap || *a.bad_grid) {  // see DPF_BAD_GRID
        if (tid == 0) {
            a.status[out_idx] = DPF_BAD_GRID;
            a.iters[out_idx] = 0;
        }
        return;
    }
    const int slice0 = a.sell.slice_off[sidx];
    const int lane = tid & (kWave - 1);
    const bool dbl = 2 * n <= a.lds_cap;
    double2 *Xv = X;
    double2 *Xw = dbl ? X + n : X;

    // step count and schedule (a resumed solve continues them)
    ItemSched sc = load_item_sched(a, out_idx);

    const double m_res = residual_count<NT>(a.bt, lo, hi, red);
    const double two_over_m = m_res > 0.0 ? 2.0 / m_res : 0.0;

    // N-1 outage of this case (only meaningful for a single sub-grid)
    const Rank2 r2 = outage_of_case(a.ov, c, lo, hi);
    if (r2.bad) return;  // reported by the call's prologue
    const int of = r2.of, ot = r2.ot;
    const double2 oy = r2.oy, oyd = r2.oyd;

    const int64_t cb = (int64_t)c * a.ld;
    const int64_t sb = (int64_t)c * a.s_ld;
    double2 *__restrict__ Wg = a.scratch + 2 * a.st_stride + cb;
    double *__restrict__ vm_c = a.vm + cb;
    double *__restrict__ va_c = a.va + cb;
    double *__restrict__ mv_c = a.st + cb;
    double *__restrict__ ma_c = a.st + a.st_stride + cb;
    double *__restrict__ sv_c = a.st + 2 * a.st_stride + cb;
    double *__restrict__ sa_c = a.st + 3 * a.st_stride + cb;
    double2 *__restrict__ aIg = a.scratch + a.st_stride + cb;
    const double2 *__restrict__ Sc = a.s_spec + sb;
    const int32_t *__restrict__ swidth = a.sell.width;
    const int32_t *__restrict__ sstart = a.sell.start;
    const int32_t *__restrict__ scol = a.sell.col;
    const double2 *__restrict__ sval = a.sell.val;
    const int8_t *__restrict__ btp = a.bt;

    for (int i = lo + tid; i < hi; i += NT) {
        double sn, cs;
        const double vmi = vm_c[i];
        fast_sincos(va_c[i], sn, cs);
        const double2 v = make_double2(vmi * cs, vmi * sn);
        Xv[i - lo] = v;
        if (a.st_fresh) {
            mv_c[i] = 0.0;
            ma_c[i] = 0.0;
            sv_c[i] = 0.0;
            sa_c[i] = 0.0;
        }
    }
    __syncthreads();

    // bus loop of one phase
#define DPF_BUS_LOOP_BEGIN                                               \
    for (int kk = 0;; ++kk) {                                            \
        const uint32_t i = opaque_index((uint32_t)(lo + tid + kk * NT)); \
        if ((int)i >= hi) break;                                         \
        {
#define DPF_BUS_LOOP_END \
    }                    \
    }

    int it = 0, stat = DPF_MAX_ITER;
    double mu = 0.0, loss = 0.0;
    __shared__ int pause_flag;
    for (;; ++it) {
        if (handoff_due(a, it, &pause_flag)) {
            stat = kPaused;
            break;
        }
        // ---------------- phase A
        double lsum = 0.0, lmax = 0.0;
        DPF_BUS_LOOP_BEGIN
                const int il = (int)i - lo;
                // global loads of this bus first, so that they overlap the gather below
                const int8_t tk = btp[i];
                const double2 sp = Sc[i];
                const int gsl = __builtin_amdgcn_readfirstlane(slice0 + (il >> 6));
                const int wdt = swidth[gsl];
                const int base = sstart[gsl] * kWave + lane;
                double2 acc = make_double2(0.0, 0.0);
                acc = sell_row<4, false>(sval, scol, base, wdt, il, [&](int j) { return Xv[j]; }, acc);
                if (il == of) acc = csub(acc, csub(cmul(oyd, Xv[of]), cmul(oy, Xv[ot])));
                else if (il == ot) acc = csub(acc, csub(cmul(oyd, Xv[ot]), cmul(oy, Xv[of])));
                const double2 v = Xv[il];
                const double2 d = csub(cmulc(v, acc), sp);
                const double rP = tk != kSlack ? d.x : 0.0;
                const double rQ = tk == kPQ ? d.y : 0.0;
                lsum += rP * rP + rQ * rQ;
                lmax = fmax(lmax, fmax(fabs(rP), fabs(rQ)));
                const double2 av = make_double2(two_over_m * rP, two_over_m * rQ);
                aIg[i] = cmul(av, acc);
                const double2 w = cmulc(av, v);
                if (dbl) Xw[il] = w;
                else Wg[i] = w;
        DPF_BUS_LOOP_END
        block_reduce2<NT>(lsum, lmax, red);
        __syncthreads();
        if (!dbl)
            for (int i = lo + tid; i < hi; i += NT) Xw[i - lo] = Wg[i];
        block_reduce2_finish<NT>(lsum, lmax, red);
        loss = m_res > 0.0 ? lsum / m_res : 0.0;
        mu = isnan(lsum) ? lsum : lmax;
        trace_mu(a, true, out_idx, it, mu);
        if (!dbl) __syncthreads();
        if (!(isfinite(loss) && isfinite(mu))) {
            stat = DPF_NONFINITE;
            break;
        }
        if (mu < a.tol) {
            stat = DPF_CONVERGED;
            break;
        }
        if (it >= a.max_iter) {
            stat = DPF_MAX_ITER;
            break;
        }

        // ---------------- phase B
        sc.t_step += 1.0;
        sc.b1t *= a.b1;
        sc.b2t *= a.b2;
        const double bc1 = 1.0 - sc.b1t;
        const double bc2 = 1.0 - sc.b2t;
        DPF_BUS_LOOP_BEGIN
                const int il = (int)i - lo;
                // every global load of this bus first, so that they overlap the gather
                const int8_t tk = btp[i];
                const double2 ai = aIg[i];
                double vmi = vm_c[i], vai = va_c[i];
                const double mv0 = mv_c[i], sv0 = sv_c[i], ma0 = ma_c[i], sa0 = sa_c[i];
                const int gsl = __builtin_amdgcn_readfirstlane(slice0 + (il >> 6));
                const int wdt = swidth[gsl];
                const int base = sstart[gsl] * kWave + lane;
                double2 h = make_double2(0.0, 0.0);
                h = sell_row<4, false>(sval, scol, base, wdt, il, [&](int j) { return Xw[j]; }, h);
                if (il == of) h = csub(h, csub(cmul(oyd, Xw[of]), cmul(oy, Xw[ot])));
                else if (il == ot) h = csub(h, csub(cmul(oyd, Xw[ot]), cmul(oy, Xw[of])));
                const double2 G = make_double2(ai.x + h.x, ai.y - h.y);
                double2 v;
                {
                    double sn0, cs0;
                    fast_sincos(vai, sn0, cs0);
                    v = make_double2(vmi * cs0, vmi * sn0);
                }
                if (tk == kPQ) {
                    const double g = (G.x * v.x + G.y * v.y) / vmi;
                    double mv = mv0, sv = sv0;
                    vmi = opt_update(a.opt, sc.lr, a.b1, a.b2, a.eps, bc1, bc2, vmi, g, mv, sv);
                    vm_c[i] = vmi;
                    mv_c[i] = mv;
                    sv_c[i] = sv;
                }
                if (tk != kSlack) {
                    const double g = G.y * v.x - G.x * v.y;
                    double ma = ma0, sa = sa0;
                    vai = opt_update(a.opt, sc.lr, a.b1, a.b2, a.eps, bc1, bc2, vai, g, ma, sa);
                    va_c[i] = vai;
                    ma_c[i] = ma;
                    sa_c[i] = sa;
                }
                double sn, cs;
                fast_sincos(vai, sn, cs);
                v = make_double2(vmi * cs, vmi * sn);
                if (dbl) Xv[il] = v;
        DPF_BUS_LOOP_END
        sched_step(a, sc, loss);
        if (!dbl) {
            __syncthreads();
            for (int i = lo + tid; i < hi; i += NT) {
                double sn, cs;
                const double vmi = vm_c[i];
                fast_sincos(va_c[i], sn, cs);
                Xv[i - lo] = make_double2(vmi * cs, vmi * sn);
            }
        }
        __syncthreads();
    }
#undef DPF_BUS_LOOP_BEGIN
#undef DPF_BUS_LOOP_END

    if (tid == 0) finish_item(a, out_idx, it, stat, mu, loss, sc);
}

// Banded variant, for sub-grids numbered with a small bandwidth: every entry of
// the matrix has |row - col| <= NT*J in local indices (a reverse Cuthill-McKee
// numbering gives ~80 on a 9241-bus meshed grid).  Buses are processed in blocks
// of BLK = NT*J consecutive buses, thread tid owning buses s*BLK + j*NT + tid of
// block s.  The rows of block s then read the exchange vector only in blocks
// s-1, s and s+1, so the single LDS array X can go from V to w to the new V
// block by block, with one block of values held in registers instead of the
// whole sub-grid:
//   A/W sweep, step s: rows of block s gather V, form dS, the loss terms and
//       w = a conj(V); I goes to scratch for the second sweep.  After a barrier
//       the w of block s-1 replaces V there (its readers, blocks s-2..s, are done).
//   stop test on the reduced max|r|
//   gradient sweep, one pass without barriers (w stays in X throughout): rows
//       gather w, rebuild dS and a*I from I and V, form the gradient and apply
//       the optimizer step; then X is refilled with the new V from |V| and theta.
// Per bus and iteration this moves |V|, theta and the four moments once each way,
// I (16 B written, 16 B read) and the refill's |V| and theta (16 B read); there is
// no w round trip through memory.  (A pipelined gradient sweep that overwrote w
// block by block with the new V moved 16 B less but, with a barrier per block,
// ran slower: the lockstep waves stopped overlapping loads and arithmetic.)
template <int NT, int J>
__global__ __launch_bounds__(NT) void team_solve_band_kernel(SolveArgs a) {
    constexpr int BLK = NT * J;
    extern __shared__ double2 X[];
    __shared__ double red[2][NT / kWave];

    const int tid = threadIdx.x;
    const int item = a.order ? a.order[blockIdx.x] : (int)blockIdx.x;
    const int sidx = item / a.B;
    const int c = item - sidx * a.B;
    const int lo = a.sub_off ? a.sub_off[sidx] : 0;
    const int hi = a.sub_off ? a.sub_off[sidx + 1] : a.n_bus;
    const int n = hi - lo;
    const int out_idx = c * a.n_sub + sidx;
    if (n > a.team_cap) return;        // handled by the multi-workgroup path
    if (a.sub_bw[sidx] > BLK) return;  // bandwidth too large: the general kernel takes it
    if (n < 0 || n > a.lds_cap || *a.bad_grid) {  // see DPF_BAD_GRID
        if (tid == 0) {
            a.status[out_idx] = DPF_BAD_GRID;
            a.iters[out_idx] = 0;
        }
        return;
    }
    const int slice0 = a.sell.slice_off[sidx];
    const int lane = tid & (kWave - 1);

    // step count and schedule (a resumed solve continues them)
    ItemSched sc = load_item_sched(a, out_idx);

    const double m_res = residual_count<NT>(a.bt, lo, hi, red);
    const double two_over_m = m_res > 0.0 ? 2.0 / m_res : 0.0;

    // N-1 outage of this case (only meaningful for a single sub-grid)
    const Rank2 r2 = outage_of_case(a.ov, c, lo, hi);
    if (r2.bad) return;  // reported by the call's prologue
    const int of = r2.of, ot = r2.ot;
    const double2 oy = r2.oy, oyd = r2.oyd;

    const int64_t cb = (int64_t)c * a.ld;
    const int64_t sb = (int64_t)c * a.s_ld;
    double *__restrict__ vm_c = a.vm + cb;
    double *__restrict__ va_c = a.va + cb;
    double *__restrict__ mv_c = a.st + cb;
    double *__restrict__ ma_c = a.st + a.st_stride + cb;
    double *__restrict__ sv_c = a.st + 2 * a.st_stride + cb;
    double *__restrict__ sa_c = a.st + 3 * a.st_stride + cb;
    double2 *__restrict__ Ig = a.scratch + cb;  // I of the A/W sweep
    const double2 *__restrict__ Sc = a.s_spec + sb;
    const int32_t *__restrict__ swidth = a.sell.width;
    const int32_t *__restrict__ sstart = a.sell.start;
    const int32_t *__restrict__ scol = a.sell.col;
    const double2 *__restrict__ sval = a.sell.val;
    const int8_t *__restrict__ btp = a.bt;

    for (int i = lo + tid; i < hi; i += NT) {
        double sn, cs;
        const double vmi = vm_c[i];
        fast_sincos(va_c[i], sn, cs);
        X[i - lo] = make_double2(vmi * cs, vmi * sn);
        if (a.st_fresh) {
            mv_c[i] = 0.0;
            ma_c[i] = 0.0;
            sv_c[i] = 0.0;
            sa_c[i] = 0.0;
        }
    }
    __syncthreads();

    const int nb = (n + BLK - 1) / BLK;
    int it = 0, stat = DPF_MAX_ITER;
    double mu = 0.0, loss = 0.0;
    __shared__ int pause_flag;
    for (;; ++it) {
        if (handoff_due(a, it, &pause_flag)) {
            stat = kPaused;
            break;
        }
        // ---------------- A/W sweep
        double lsum = 0.0, lmax = 0.0;
        double2 hold[J];
#pragma unroll
        for (int j = 0; j < J; ++j) hold[j] = make_double2(0.0, 0.0);
        for (int s = 0; s <= nb; ++s) {
            double2 w[J];
#pragma unroll
            for (int j = 0; j < J; ++j) {
                w[j] = make_double2(0.0, 0.0);
                const int il = s * BLK + j * NT + tid;
                if (s < nb && il < n) {
                    const int i = lo + il;
                    const int8_t tk = btp[i];
                    const double2 sp = Sc[i];
                    const int gsl = __builtin_amdgcn_readfirstlane(slice0 + (il >> 6));
                    const int wdt = swidth[gsl];
                    const int base = sstart[gsl] * kWave + lane;
                    double2 acc = make_double2(0.0, 0.0);
                    acc = sell_row<4, false>(sval, scol, base, wdt, il, [&](int j) { return X[j]; }, acc);
                    if (il == of) acc = csub(acc, csub(cmul(oyd, X[of]), cmul(oy, X[ot])));
                    else if (il == ot) acc = csub(acc, csub(cmul(oyd, X[ot]), cmul(oy, X[of])));
                    const double2 v = X[il];
                    const double2 d = csub(cmulc(v, acc), sp);
                    const double rP = tk != kSlack ? d.x : 0.0;
                    const double rQ = tk == kPQ ? d.y : 0.0;
                    lsum += rP * rP + rQ * rQ;
                    lmax = fmax(lmax, fmax(fabs(rP), fabs(rQ)));
                    const double2 av = make_double2(two_over_m * rP, two_over_m * rQ);
                    Ig[i] = acc;
                    w[j] = cmulc(av, v);
                }
            }
            __syncthreads();
            if (s > 0) {
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    const int il = (s - 1) * BLK + j * NT + tid;
                    if (il < n) X[il] = hold[j];
                }
            }
#pragma unroll
            for (int j = 0; j < J; ++j) hold[j] = w[j];
        }
        block_reduce2<NT>(lsum, lmax, red);
        __syncthreads();
        block_reduce2_finish<NT>(lsum, lmax, red);
        loss = m_res > 0.0 ? lsum / m_res : 0.0;
        mu = isnan(lsum) ? lsum : lmax;
        trace_mu(a, true, out_idx, it, mu);
        if (!(isfinite(loss) && isfinite(mu))) {
            stat = DPF_NONFINITE;
            break;
        }
        if (mu < a.tol) {
            stat = DPF_CONVERGED;
            break;
        }
        if (it >= a.max_iter) {
            stat = DPF_MAX_ITER;
            break;
        }

        // ---------------- B/U sweep
        sc.t_step += 1.0;
        sc.b1t *= a.b1;
        sc.b2t *= a.b2;
        const double bc1 = 1.0 - sc.b1t;
        const double bc2 = 1.0 - sc.b2t;
        // one barrier-free pass (w stays in X throughout), then the new V is
        // rebuilt from |V| and theta in a refill pass
        for (int s = 0; s < nb; ++s) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int il = s * BLK + j * NT + tid;
                if (il < n) {
                    const int i = lo + il;
                    // every global load of this bus first, so that they overlap the gather
                    const int8_t tk = btp[i];
                    const double2 I = Ig[i];
                    const double2 sp = Sc[i];
                    double vmi = vm_c[i], vai = va_c[i];
                    const double mv0 = mv_c[i], sv0 = sv_c[i], ma0 = ma_c[i], sa0 = sa_c[i];
                    const int gsl = __builtin_amdgcn_readfirstlane(slice0 + (il >> 6));
                    const int wdt = swidth[gsl];
                    const int base = sstart[gsl] * kWave + lane;
                    double2 h = make_double2(0.0, 0.0);
                    h = sell_row<4, false>(sval, scol, base, wdt, il, [&](int j) { return X[j]; }, h);
                    if (il == of) h = csub(h, csub(cmul(oyd, X[of]), cmul(oy, X[ot])));
                    else if (il == ot) h = csub(h, csub(cmul(oyd, X[ot]), cmul(oy, X[of])));
                    double2 v;
                    {
                        double sn0, cs0;
                        fast_sincos(vai, sn0, cs0);
                        v = make_double2(vmi * cs0, vmi * sn0);
                    }
                    // the seed of the A/W sweep, rebuilt from I and the same V
                    const double2 d = csub(cmulc(v, I), sp);
                    const double rP = tk != kSlack ? d.x : 0.0;
                    const double rQ = tk == kPQ ? d.y : 0.0;
                    const double2 ai = cmul(make_double2(two_over_m * rP, two_over_m * rQ), I);
                    const double2 G = make_double2(ai.x + h.x, ai.y - h.y);
                    if (tk == kPQ) {
                        const double g = (G.x * v.x + G.y * v.y) / vmi;
                        double mv = mv0, sv = sv0;
                        vmi = opt_update(a.opt, sc.lr, a.b1, a.b2, a.eps, bc1, bc2, vmi, g, mv, sv);
                        vm_c[i] = vmi;
                        mv_c[i] = mv;
                        sv_c[i] = sv;
                    }
                    if (tk != kSlack) {
                        const double g = G.y * v.x - G.x * v.y;
                        double ma = ma0, sa = sa0;
                        vai = opt_update(a.opt, sc.lr, a.b1, a.b2, a.eps, bc1, bc2, vai, g, ma, sa);
                        va_c[i] = vai;
                        ma_c[i] = ma;
                        sa_c[i] = sa;
                    }
                }
            }
        }
        __syncthreads();
        for (int i = lo + tid; i < hi; i += NT) {
            double sn, cs;
            const double vmi = vm_c[i];
            fast_sincos(va_c[i], sn, cs);
            X[i - lo] = make_double2(vmi * cs, vmi * sn);
        }
        sched_step(a, sc, loss);
        __syncthreads();
    }

    if (tid == 0) finish_item(a, out_idx, it, stat, mu, loss, sc);
}

// start point of every step of a time-series window: rows [0, gridDim.y) of dst
// receive the source voltages
__global__ void row_broadcast_kernel(int32_t n, const double *__restrict__ src_m, const double *__restrict__ src_a,
                                     double *__restrict__ dst_m, double *__restrict__ dst_a, int64_t ld) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double m = src_m[i], v = src_a[i];
    dst_m[blockIdx.y * ld + i] = m;
    dst_a[blockIdx.y * ld + i] = v;
}

// default schedule state {t, lr, best, bad + cooldown * 2^20, b1^t, b2^t} of B items
__global__ void sched_init_kernel(int32_t B, double lr, double *__restrict__ sched) {
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= B) return;
    double *ss = sched + kSchedWords * (int64_t)c;
    ss[0] = 0.0;
    ss[1] = lr;
    ss[2] = __longlong_as_double(0x7ff0000000000000LL);
    ss[3] = 0.0;
    ss[4] = 1.0;
    ss[5] = 1.0;
}

// indices of the paused items (one workgroup; the order of the list is free)
__global__ __launch_bounds__(1024) void collect_paused_kernel(int32_t n_items, const int32_t *__restrict__ status,
                                                              int32_t *__restrict__ list, int32_t *__restrict__ count) {
    __shared__ int n;
    if (threadIdx.x == 0) n = 0;
    __syncthreads();
    for (int32_t i = threadIdx.x; i < n_items; i += blockDim.x)
        if (status[i] == kPaused) list[atomicAdd(&n, 1)] = i;
    __syncthreads();
    if (threadIdx.x == 0) *count = n;
}

// Call prologue with an outage list: a case whose index is neither -1 nor a
// branch index is reported (status DPF_BAD_OUTAGE, no updates, NaN mismatch and
// loss) and counted as finished for the tail handoff; the kernels skip it.
__global__ void outage_check_kernel(int32_t B, OutageView ov, int32_t *__restrict__ status,
                                    int32_t *__restrict__ iters, double *__restrict__ mu,
                                    double *__restrict__ loss, int32_t *__restrict__ done_count) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= B || !outage_index_bad(ov.outage[c], ov.n_branch)) return;
    status[c] = DPF_BAD_OUTAGE;
    iters[c] = 0;
    mu[c] = __longlong_as_double(0x7ff8000000000000LL);
    loss[c] = __longlong_as_double(0x7ff8000000000000LL);
    atomicAdd(done_count, 1);
}

// Case order of a call: descending initial max|r| (NaN first, ties by index), so
// that the cases likely to run longest start first.  order[rank] = case; one
// thread per case counts the cases ahead of it (B is small enough for O(B^2)).
__global__ void rank_desc_kernel(int32_t B, const double *__restrict__ key, int32_t *__restrict__ order) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    auto k = [&](int32_t j) {
        const double x = key[j];
        return isnan(x) ? __longlong_as_double(0x7ff0000000000000LL) : x;
    };
    const double ki = k(i);
    int32_t rank = 0;
    for (int32_t j = 0; j < B; ++j) {
        const double kj = k(j);
        rank += (kj > ki || (kj == ki && j < i)) ? 1 : 0;
    }
    order[rank] = i;
}

// wall-clock stamp at the start of a solve call (for per-item completion times)
__global__ void stamp_kernel(int64_t *stamp) {
    if (threadIdx.x == 0) *stamp = wall_clock64();
}

}  // namespace dpf
