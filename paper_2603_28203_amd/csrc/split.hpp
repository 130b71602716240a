// Split solve: the last unfinished cases of a single-grid batch, each spread over
// a team of T workgroups on T CUs.
//
// Per-item kernels give every case one CU.  Once a batch has retired most of its
// cases, the few left (often the slowest: they run to the iteration cap) would
// hold a handful of CUs for thousands of iterations while the rest of the chip
// idles.  Here each of them is cut into T row ranges of whole 64-row slices, one
// workgroup per range, and the team keeps the per-item kernels' LDS gathers:
// every member holds the exchange vector X for the columns its rows reference
// (a bitmap of them follows X in LDS) and refreshes those from global memory
// after each of the two exchanges of an iteration (the adjoint product of Sec. 5.1
// needs every neighbour's seed w, the next forward product every neighbour's new V):
//   A : rows of the member: I = Y V, dS, loss terms, w = a conj(V) -> global;
//       the member's (loss sum, max|r|) partial -> global
//   -- team barrier --
//   every member sums the T partials in the same order (identical loss, max|r|
//   and stop decision in all members); X <- w of the range
//   B : rows of the member: h = Y^T w, G, optimizer step; |V|, theta, moments
//       -> global; schedule step
//   -- team barrier --
//   X <- polar(|V|, theta) of the range
// The barrier is a per-team arrival counter in global memory.  What crosses it
// (w, |V|, theta, the partials) is written and read with device-scope accesses
// (relaxed agent-scope atomics: stores write through to the device's coherence
// point, loads do not hit a possibly stale L1/L2 copy), and every thread waits
// for its own stores to complete before the team's arrival is counted.  Fences
// at agent scope would do the same for all memory, but on a chip with one L2 per
// XCD they write back and invalidate the L2 at every barrier of every member,
// which cost several times the iteration itself.  Members of one team must run
// at the same time, which the host arranges by launching at most as many
// workgroups as the device holds.
// A member that waits longer than a bound abandons the barrier (kSplitAbort in
// the counter, set by a compare-and-swap that fails if a member arrived
// meanwhile); every member then leaves at its next barrier with the item still
// paused, and the host finishes it on the multi-workgroup path.  Members finish
// their part of an iteration before they arrive, so the state left behind is
// that of a whole iteration: the start of iteration it (barrier after A, no
// update yet) or of it + 1 (barrier after B, every member's rows updated), and
// member 0 records that count with the schedule.
//
// A launch runs each listed case for at most `chunk` iterations and, when a time
// slice is set, until member 0 of its team sees the slice used up (it publishes
// that beside the team's counter before the first barrier of an iteration, so
// that every member pauses at the same point); the host then drops the finished
// cases and relaunches the rest.  Team sizes come from the host per launch
// (`first`): equal, or -- with time slices -- in proportion to the square of
// each case's remaining iteration budget, so that the cases that can still run
// longest get the most CUs.
#pragma once

#include "../../include/dpf.h"
#include "common.hpp"
#include "solve.hpp"

namespace dpf {

constexpr int32_t kSplitAbort = 1 << 30;
// one counter per 256 bytes: device-scope atomics and polls of different teams on
// one cache line serialize
constexpr int32_t kBarStride = 64;

struct SplitArgs {
    const int32_t *list;  // [n_list] paused case indices
    int32_t n_list;
    const int32_t *n_list_dev;  // the list's length in device memory (planned on the device), or null
    const int32_t *first; // [n_list + 1] first workgroup of each team (sizes <= slices of the grid)
    int32_t chunk;        // iterations per launch
    int64_t slice;        // wall-clock ticks per launch, 0 = no limit
    int32_t *bar;         // [n_list][kBarStride] arrival counters (first word of each), zero at launch
    double2 *part;        // [first[n_list]] member partials (loss sum, max|r|), team k at first[k]
    double2 *Ig;          // [B][ld] I of the A sweep
    double2 *Wg;          // [B][ld] exchanged w
    int32_t *aborted;     // set when a team abandoned a barrier
    int64_t first_limit;  // wall-clock ticks a member waits at the first barrier
    int64_t limit;        // ... and at every later one
    int32_t list_cap;     // needed-column list entries the dynamic LDS holds behind the bitmap
};

// arrival barrier of the T members of one team; false when it was abandoned
__device__ __forceinline__ bool team_barrier(int32_t *cnt, int32_t target, int64_t limit, int *flag) {
    dev_stores_done();
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t v = atomicAdd(cnt, 1) + 1;
        bool ok = (v & kSplitAbort) == 0;
        const int64_t t0 = wall_clock64();
        while (ok && v < target) {
            __builtin_amdgcn_s_sleep(1);
            v = __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v & kSplitAbort) {
                ok = false;
            } else if (v < target && wall_clock64() - t0 > limit) {
                // abandon only if no member arrived meanwhile (else poll again)
                if (atomicCAS(cnt, v, v | kSplitAbort) == v) ok = false;
            }
        }
        *flag = ok ? 1 : 0;
    }
    __syncthreads();
    return *flag != 0;
}

template <int NT>
__global__ __launch_bounds__(NT) void team_solve_split_kernel(SolveArgs a, SplitArgs p) {
    extern __shared__ double2 X[];
    __shared__ double red[2][NT / kWave];
    __shared__ int bar_flag;
    __shared__ int slice_flag;
    __shared__ int scan_part[NT / kWave];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    // a launch planned on the device has a fixed grid: workgroups past the table leave
    const int32_t n_list = p.n_list_dev ? *p.n_list_dev : p.n_list;
    if (n_list <= 0 || (int)blockIdx.x >= p.first[n_list]) return;
    int team = 0;  // largest k with first[k] <= blockIdx.x
    for (int hi_k = n_list - 1; team < hi_k;) {
        const int m = (team + hi_k + 1) >> 1;
        if (p.first[m] <= (int)blockIdx.x) team = m;
        else hi_k = m - 1;
    }
    const int T = p.first[team + 1] - p.first[team];
    const int mem = blockIdx.x - p.first[team];
    const int c = p.list[team];
    const int n = a.n_bus;
    const int ns = (n + kWave - 1) / kWave;
    const int rlo = (int)((int64_t)mem * ns / T) * kWave;
    const int rhi = min((int)((int64_t)(mem + 1) * ns / T) * kWave, n);
    const int bw = a.sub_bw[0];
    const int xlo = max(0, rlo - bw), xhi = min(n, rhi + bw);
    int32_t *cnt = p.bar + (int64_t)team * kBarStride;
    int32_t *slice_up = cnt + 1;  // member 0: this launch's time slice is used up
    double2 *part = p.part + p.first[team];
    const int64_t t_start = wall_clock64();

    if (*a.bad_grid) {  // a row longer than the declared bound (see DPF_BAD_GRID); every member leaves
        if (mem == 0 && tid == 0) {
            a.status[c] = DPF_BAD_GRID;
            a.iters[c] = 0;
        }
        return;
    }
    ItemSched sc = load_item_sched(a, c);
    const double m_res = residual_count<NT>(a.bt, 0, n, red);
    const double two_over_m = m_res > 0.0 ? 2.0 / m_res : 0.0;
    const Rank2 r2 = outage_of_case(a.ov, c, 0, n);
    if (r2.bad) return;  // reported by the call's prologue (status stays DPF_BAD_OUTAGE); every member leaves
    const int of = r2.of, ot = r2.ot;
    const double2 oy = r2.oy, oyd = r2.oyd;

    const int64_t cb = (int64_t)c * a.ld;
    double *__restrict__ vm_c = a.vm + cb;
    double *__restrict__ va_c = a.va + cb;
    double *__restrict__ mv_c = a.st + cb;
    double *__restrict__ ma_c = a.st + a.st_stride + cb;
    double *__restrict__ sv_c = a.st + 2 * a.st_stride + cb;
    double *__restrict__ sa_c = a.st + 3 * a.st_stride + cb;
    double2 *__restrict__ Ig = p.Ig + cb;
    double2 *__restrict__ Wg = p.Wg + cb;
    const double2 *__restrict__ Sc = a.s_spec + (int64_t)c * a.s_ld;
    const int32_t *__restrict__ swidth = a.sell.width;
    const int32_t *__restrict__ sstart = a.sell.start;
    const int32_t *__restrict__ scol = a.sell.col;
    const double2 *__restrict__ sval = a.sell.val;
    const int8_t *__restrict__ btp = a.bt;

    // A team of one has no partners: plain accesses, workgroup barriers only, and
    // its own sums are the totals.
    const bool solo = T == 1;
    auto ld = [&](const double *q) { return solo ? *q : ld_dev(q); };
    auto ld2 = [&](const double2 *q) { return solo ? *q : ld_dev2(q); };
    auto st = [&](double *q, double v) {
        if (solo) *q = v;
        else st_dev(q, v);
    };

    // The columns the member's rows read (its own rows, their neighbours and the
    // two buses of the outage) as a bitmap behind X: the refills below load only
    // those (on the 9241-bus grid under the degree-grouped numbering, 32% of the
    // range at 8 members, 13% at 32).
    uint32_t *need = reinterpret_cast<uint32_t *>(X + n);
    for (int k = tid; k < (n + 31) / 32; k += NT) need[k] = 0u;
    __syncthreads();
    for (int il = rlo + tid; il < rhi; il += NT) {
        const int gsl = __builtin_amdgcn_readfirstlane(il >> 6);
        const int wdt = swidth[gsl];
        const int base = sstart[gsl] * kWave + lane;
        atomicOr(need + (il >> 5), 1u << (il & 31));
        for (int q = 0; q < wdt; ++q) {
            const int cc = scol[base + q * kWave];
            atomicOr(need + (cc >> 5), 1u << (cc & 31));
        }
    }
    if (of >= 0 && tid < 2) {
        const int i = tid == 0 ? of : ot;
        atomicOr(need + (i >> 5), 1u << (i & 31));
    }
    __syncthreads();
    auto needed = [&](int i) { return (need[i >> 5] >> (i & 31)) & 1u; };

    // The same columns in increasing order as a list behind the bitmap, when they
    // fit: a refill then loads them directly instead of testing every column of
    // the range (which is several times longer).  n_need = -1: no list.
    const int nwords = (n + 31) / 32;
    uint16_t *nlist = reinterpret_cast<uint16_t *>(need + nwords);
    int n_need = -1;
    {
        const int per = (nwords + NT - 1) / NT;  // contiguous words per thread
        const int w0 = min(tid * per, nwords), w1 = min(w0 + per, nwords);
        int cnt_b = 0;
        for (int w = w0; w < w1; ++w) cnt_b += __popc(need[w]);
        int incl = cnt_b;  // inclusive scan over the wave, then over the waves
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += y;
        }
        if (lane == kWave - 1) scan_part[tid / kWave] = incl;
        __syncthreads();
        int before = 0, total = 0;
        for (int k = 0; k < NT / kWave; ++k) {
            before += k < tid / kWave ? scan_part[k] : 0;
            total += scan_part[k];
        }
        if (total <= p.list_cap) {
            int pos = before + incl - cnt_b;
            for (int w = w0; w < w1; ++w)
                for (uint32_t bits = need[w]; bits != 0u; bits &= bits - 1u)
                    nlist[pos++] = (uint16_t)(w * 32 + __ffs(bits) - 1);
            n_need = total;
        }
        __syncthreads();
    }

    // X <- V at the needed columns of the range (and the two buses of the outage,
    // which the rank-2 term of the outage rows reads, wherever they are)
    auto fill_v = [&]() {
        if (n_need >= 0) {
            for (int k = tid; k < n_need; k += NT) {
                const int i = nlist[k];
                double sn, cs;
                const double vmi = ld(vm_c + i);
                fast_sincos(ld(va_c + i), sn, cs);
                X[i] = make_double2(vmi * cs, vmi * sn);
            }
            return;
        }
        for (int i = xlo + tid; i < xhi; i += NT) {
            if (!needed(i)) continue;
            double sn, cs;
            const double vmi = ld(vm_c + i);
            fast_sincos(ld(va_c + i), sn, cs);
            X[i] = make_double2(vmi * cs, vmi * sn);
        }
        if (of >= 0 && tid < 2) {
            const int i = tid == 0 ? of : ot;
            if (i < xlo || i >= xhi) {
                double sn, cs;
                const double vmi = ld(vm_c + i);
                fast_sincos(ld(va_c + i), sn, cs);
                X[i] = make_double2(vmi * cs, vmi * sn);
            }
        }
    };
    auto fill_w = [&]() {
        if (n_need >= 0) {
            for (int k = tid; k < n_need; k += NT) {
                const int i = nlist[k];
                X[i] = ld2(Wg + i);
            }
            return;
        }
        for (int i = xlo + tid; i < xhi; i += NT)
            if (needed(i)) X[i] = ld2(Wg + i);
        if (of >= 0 && tid < 2) {
            const int i = tid == 0 ? of : ot;
            if (i < xlo || i >= xhi) X[i] = ld2(Wg + i);
        }
    };

    const int it0 = a.iters[c];  // paused cases continue their iteration count
    int it = it0, stat = kPaused, nbar = 0;
    double mu = 0.0, loss = 0.0;
    bool ok = true;
    for (;; ++it) {
        fill_v();  // X <- V (the state at the start of iteration it)
        __syncthreads();
        if (it - it0 >= p.chunk) break;  // paused again; the host relaunches
        // ---------------- A: rows of this member
        double lsum = 0.0, lmax = 0.0;
        for (int il = rlo + tid; il < rhi; il += NT) {
            const int8_t tk = btp[il];
            const double2 sp = Sc[il];
            const int gsl = __builtin_amdgcn_readfirstlane(il >> 6);
            const int wdt = swidth[gsl];
            const int base = sstart[gsl] * kWave + lane;
            double2 acc = make_double2(0.0, 0.0);
            acc = sell_row<4, true>(sval, scol, base, wdt, il, [&](int j) { return X[j]; }, acc);
            if (il == of) acc = csub(acc, csub(cmul(oyd, X[of]), cmul(oy, X[ot])));
            else if (il == ot) acc = csub(acc, csub(cmul(oyd, X[ot]), cmul(oy, X[of])));
            const double2 v = X[il];
            const double2 d = csub(cmulc(v, acc), sp);
            const double rP = tk != kSlack ? d.x : 0.0;
            const double rQ = tk == kPQ ? d.y : 0.0;
            lsum += rP * rP + rQ * rQ;
            lmax = fmax(lmax, fmax(fabs(rP), fabs(rQ)));
            Ig[il] = acc;
            const double2 w = cmulc(make_double2(two_over_m * rP, two_over_m * rQ), v);
            if (solo) Wg[il] = w;
            else st_dev2(Wg + il, w);
        }
        block_reduce2<NT>(lsum, lmax, red);
        __syncthreads();
        block_reduce2_finish<NT>(lsum, lmax, red);
        if (tid == 0 && !solo) {
            st_dev2(part + mem, make_double2(lsum, lmax));
            if (mem == 0)
                __hip_atomic_store(slice_up, p.slice > 0 && wall_clock64() - t_start >= p.slice ? 1 : 0,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (!solo) {
            ++nbar;
            ok = team_barrier(cnt, nbar * T, nbar == 1 ? p.first_limit : p.limit, &bar_flag);
            if (!ok) break;
        } else {
            __syncthreads();
        }
        // team totals: the same partials combined in the same order by every member
        // (their loads overlap the refill of X with w, which the stop test would
        // only discard)
        {
            double s = 0.0, m = 0.0;
            if (solo) {
                if (tid == 0) {  // the whole team's sums, spread over the first wave's lanes below
                    s = lsum;
                    m = lmax;
                    slice_flag = p.slice > 0 && wall_clock64() - t_start >= p.slice ? 1 : 0;
                }
            } else {
                for (int q = tid; q < T; q += NT) {
                    const double2 pp = ld_dev2(part + q);
                    s += pp.x;
                    m = fmax(m, pp.y);
                }
                // member 0 cannot rewrite the flag before every member has passed the
                // next barrier; the barriers below hand it to the whole workgroup
                if (tid == 0) slice_flag = __hip_atomic_load(slice_up, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            fill_w();
            block_reduce2<NT>(s, m, red);
            __syncthreads();
            block_reduce2_finish<NT>(s, m, red);
            __syncthreads();
            lsum = s;
            lmax = m;
        }
        loss = m_res > 0.0 ? lsum / m_res : 0.0;
        mu = isnan(lsum) ? lsum : lmax;
        trace_mu(a, mem == 0, c, it, mu);
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
        // time slice used up: paused at the start of iteration it, once this launch has
        // applied an update (so that every launch advances every unfinished case)
        if (slice_flag && it > it0) break;

        // ---------------- B: rows of this member
        sc.t_step += 1.0;
        sc.b1t *= a.b1;
        sc.b2t *= a.b2;
        const double bc1 = 1.0 - sc.b1t;
        const double bc2 = 1.0 - sc.b2t;
        for (int il = rlo + tid; il < rhi; il += NT) {
            const int8_t tk = btp[il];
            const double2 I = Ig[il];
            const double2 sp = Sc[il];
            double vmi = vm_c[il], vai = va_c[il];
            const double mv0 = mv_c[il], sv0 = sv_c[il], ma0 = ma_c[il], sa0 = sa_c[il];
            const int gsl = __builtin_amdgcn_readfirstlane(il >> 6);
            const int wdt = swidth[gsl];
            const int base = sstart[gsl] * kWave + lane;
            double2 h = make_double2(0.0, 0.0);
            h = sell_row<4, true>(sval, scol, base, wdt, il, [&](int j) { return X[j]; }, h);
            if (il == of) h = csub(h, csub(cmul(oyd, X[of]), cmul(oy, X[ot])));
            else if (il == ot) h = csub(h, csub(cmul(oyd, X[ot]), cmul(oy, X[of])));
            double2 v;
            {
                double sn0, cs0;
                fast_sincos(vai, sn0, cs0);
                v = make_double2(vmi * cs0, vmi * sn0);
            }
            const double2 d = csub(cmulc(v, I), sp);
            const double rP = tk != kSlack ? d.x : 0.0;
            const double rQ = tk == kPQ ? d.y : 0.0;
            const double2 ai = cmul(make_double2(two_over_m * rP, two_over_m * rQ), I);
            const double2 G = make_double2(ai.x + h.x, ai.y - h.y);
            if (tk == kPQ) {
                const double g = (G.x * v.x + G.y * v.y) / vmi;
                double mv = mv0, sv = sv0;
                vmi = opt_update(a.opt, sc.lr, a.b1, a.b2, a.eps, bc1, bc2, vmi, g, mv, sv);
                st(vm_c + il, vmi);
                mv_c[il] = mv;
                sv_c[il] = sv;
            }
            if (tk != kSlack) {
                const double g = G.y * v.x - G.x * v.y;
                double ma = ma0, sa = sa0;
                vai = opt_update(a.opt, sc.lr, a.b1, a.b2, a.eps, bc1, bc2, vai, g, ma, sa);
                st(va_c + il, vai);
                ma_c[il] = ma;
                sa_c[il] = sa;
            }
        }
        sched_step(a, sc, loss);
        if (!solo) ok = team_barrier(cnt, ++nbar * T, p.limit, &bar_flag);
        else __syncthreads();
        if (!ok) {
            ++it;  // the members that arrived applied this iteration's step
            break;
        }
    }

    if (mem != 0 || tid != 0) return;
    if (!ok) {
        // abandoned: the case stays paused with its current count and schedule
        *p.aborted = 1;
        stat = kPaused;
    }
    finish_item(a, c, it, stat, mu, loss, sc);
}

// a call that starts on the split kernel: every case paused at iteration 0 and
// listed in order
__global__ void split_start_kernel(int32_t B, OutageView ov, int32_t *__restrict__ status,
                                   int32_t *__restrict__ iters, int32_t *__restrict__ list) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= B) return;
    list[c] = c;
    // a case with a bad outage index keeps the prologue's status, so that it
    // drops out of the list after the first launch (its team leaves at once)
    if (ov.outage && outage_index_bad(ov.outage[c], ov.n_branch)) return;
    status[c] = kPaused;
    iters[c] = 0;
}

// fresh optimizer moments
__global__ void zero_f64_kernel(int64_t n, double *__restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

// zero n counters spaced `stride` words apart
__global__ void split_clear_kernel(int32_t n, int32_t stride, int32_t *__restrict__ bar) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) bar[(int64_t)i * stride] = 0;
}

// Team table of one split-kernel launch, planned on the device from the list of
// paused cases (*count of them) by the rule the host otherwise applies: with
// by_budget, team sizes in proportion to the square of each case's remaining
// budget max_iter - iters (at least 1, at most tmax, together at most capacity,
// the largest teams shrunk first when the floors overshoot); else equal teams
// of min(tmax, capacity / cases).  first[k] is the first workgroup of team k;
// the arrival counters of the listed teams are cleared.  One workgroup.
constexpr int kSplitPlanThreads = 1024;
__global__ __launch_bounds__(kSplitPlanThreads) void split_plan_kernel(
    const int32_t *__restrict__ list, const int32_t *__restrict__ count, const int32_t *__restrict__ iters,
    int32_t max_iter, int32_t capacity, int32_t tmax, int32_t by_budget, int32_t *__restrict__ first,
    int32_t *__restrict__ bar) {
    __shared__ double wpart[kSplitPlanThreads];
    __shared__ long long tpart[kSplitPlanThreads];
    __shared__ double sh_wsum;
    const int tid = threadIdx.x;
    const int n = *count;
    const int per = (n + kSplitPlanThreads - 1) / kSplitPlanThreads;  // contiguous cases per thread
    const int k0 = min(tid * per, n), k1 = min(k0 + per, n);
    auto weight = [&](int k) {
        const double r = (double)max(1, max_iter - iters[list[k]]);
        return r * r;
    };
    const bool budget = by_budget && n <= capacity;
    if (budget) {
        double w = 0.0;
        for (int k = k0; k < k1; ++k) w += weight(k);
        wpart[tid] = w;
        __syncthreads();
        if (tid == 0) {  // the partials in thread order: the sum of the cases in list order
            double t = 0.0;
            for (int q = 0; q < kSplitPlanThreads; ++q) t += wpart[q];
            sh_wsum = t;
        }
        __syncthreads();
    }
    // team sizes into first[k + 1], then their running sum
    long long own = 0;
    for (int k = k0; k < k1; ++k) {
        long long t;
        if (budget) t = min<long long>(max<long long>((long long)(weight(k) / sh_wsum * (double)capacity), 1), tmax);
        else t = max(1, min(capacity / max(n, 1), tmax));
        first[k + 1] = (int32_t)t;
        own += t;
    }
    tpart[tid] = own;
    __syncthreads();
    if (tid == 0) {
        long long total = 0;
        for (int q = 0; q < kSplitPlanThreads; ++q) total += tpart[q];
        while (budget && total > capacity) {  // the floor of 1 can overshoot: shrink the largest teams
            int big = 0;
            for (int k = 1; k < n; ++k)
                if (first[k + 1] > first[big + 1]) big = k;
            if (first[big + 1] <= 1) break;
            --first[big + 1];
            --total;
        }
        first[0] = 0;
    }
    __syncthreads();
    own = 0;
    for (int k = k0; k < k1; ++k) own += first[k + 1];
    tpart[tid] = own;
    __syncthreads();
    long long before = 0;
    for (int q = 0; q < tid; ++q) before += tpart[q];
    for (int k = k0; k < k1; ++k) {
        before += first[k + 1];
        first[k + 1] = (int32_t)before;
    }
    for (int k = tid; k < n; k += kSplitPlanThreads) bar[(int64_t)k * kBarStride] = 0;
}

// after the last launch planned on the device: a case still paused (its team gave
// up waiting at a barrier in every launch) ends with DPF_UNFINISHED
__global__ void split_unfinished_kernel(int32_t B, int32_t *__restrict__ status) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < B && status[c] == kPaused) status[c] = DPF_UNFINISHED;
}

}  // namespace dpf
