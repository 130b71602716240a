// Persistent teams: every item of a call in ONE launch, sub-grids larger than one
// workgroup's LDS included, with no host wait (the call only enqueues kernels and
// can be captured in a graph).
//
// The launch holds as many workgroups as the device runs at once.  Each item
// (case c, sub-grid s) is a unit of T_s tickets, T_s = 1 for sub-grids up to the
// per-member row target, else enough members that each holds its rows and both
// halos (the sub-grid's bandwidth) in LDS.  A workgroup takes the next ticket from
// a device counter, becomes member m of that ticket's unit, runs the unit to its
// end and takes another ticket.  Tickets are handed out in unit order, so at most
// one unit at a time has members waiting for the rest of its team; every other
// unit either runs complete or has not started, and the units that run finish and
// free their workgroups for the waiting team.  A team of T members therefore
// always assembles when T workgroups fit on the device (T is capped at 32 and at
// half of the launch).
//
// A member owns rows [rlo, rhi) of its sub-grid (whole 64-row slices) and keeps in
// LDS a window of the exchanged vector: its rows plus the sub-grid's bandwidth on
// each side as far as the LDS holds (the whole sub-grid when it fits).  An entry
// outside the window (a bandwidth wider than the LDS allows, or the two buses of
// an outage branch whose admittance entry the matrix does not store) is read from
// global memory instead, so every member is correct whatever the numbering; the
// plan keeps that path cold.  Per iteration (the order of Algorithm 1, the
// adjoint of Sec. 5.1, the update of Sec. 4.1):
//   X <- V of the window (global, written by the owners)
//   A : rows of the member: I = Y V (+ the rank-2 outage term), dS, loss terms,
//       a*I -> global (own rows), w = a conj(V) -> global; the member's
//       (loss sum, max|r|) -> global
//   -- team barrier --
//   every member reduces the T partials in the same fixed order (one loss,
//   max|r| and stop decision for the whole team); X <- w of the window
//   B : rows of the member: h = Y^T w, G = a*I + conj(h) with V rebuilt from
//       |V| and theta, optimizer step; |V|, theta, moments and V = polar(|V|,
//       theta) -> global; schedule step
//   -- team barrier --
// The per-bus state lives in the workspace as three 16-byte pairs (|V|, theta),
// (m_vm, m_va), (s_vm, s_va), filled from the caller's arrays before the launch and
// written back after it (pair_in_kernel / pair_out_kernel): three loads and three
// stores per bus-iteration instead of six each.
// What crosses a barrier is written and read with device-scope accesses (see
// common.hpp) and each thread waits for its stores before the arrival is counted.
// A team of one uses workgroup barriers only.
//
// Waits: the first barrier of a unit (after the members publish V of their rows)
// may wait for members still finishing other units, of this launch or of another
// persistent launch on the device that holds the CUs; it is abandoned only when
// neither the team's arrival count nor the device's progress count (bumped by
// every running unit of every launch every 64 iterations and when it ends) has
// moved for the first bound.  Later barriers, with the whole team running, use the second bound.
// An abandoned unit leaves its item with status DPF_UNFINISHED at the state of a
// whole iteration, as the split kernel's teams do.
//
// Plan (one workgroup, on the device, from the sub-grid sizes and the
// bandwidths the sliced-ELL build measured): for w = 1..8 waves of the launch's
// G workgroups, the smallest per-member row target R (a multiple of 64) whose
// team sizes sum to at most w*G members; the w with the least w*(R + kTeamRowsPerBarrier)
// wins.  Units are then ordered by per-member load, largest first (half-octave
// buckets, index order inside a bucket), so that long units start first and
// single-member units fill the gaps.  The plan changes only where and when an
// item runs, and the team size, which fixes the order in which the members'
// partial loss sums are added.
#pragma once

#include "../../include/dpf.h"
#include "common.hpp"
#include "solve.hpp"

namespace dpf {

// 1024 threads (16 waves, one workgroup per CU): ~30 VGPRs spill at the 128-register
// limit, yet an iteration runs 1.2-1.5x faster than at 512 threads without spills
// (measured on 64 cases of 9241 buses, 256 cases of 3000 and the uneven batch).
// The gathers unroll by 2 (by 4: 44 spilled registers and 5-10% slower).
constexpr int kTeamThreads = 1024;
constexpr int kPlanThreads = 256;
// members per team at most: one 9241-bus case takes 14 us per iteration on 32
// members, 19 us on 128 (more arrivals per barrier, more halo per row)
constexpr int kTeamMaxMembers = 32;
constexpr int kLoadKeys = 32;      // half-octave buckets of the per-member load
constexpr int kTeamMaxWaves = 8;
constexpr int kTeamRowsPerBarrier = 512;  // the plan's price of a barrier pair, in rows
constexpr int kTeamBarStride = 32;        // one 64-bit counter per 256 bytes
constexpr int kTeamHaloCap = 2048;        // halo columns a member's refill list holds
constexpr long long kTeamAbort = 1LL << 62;

struct TeamArgs {
    int32_t *hdr;          // [0] next ticket, [1] tickets, [2] units
    int32_t *progress;     // the device's progress count (one per device, shared by all launches)
    int32_t *unit_item;    // [items] item of each unit, in ticket order
    int32_t *first;        // [items + 1] first ticket of each unit
    long long *bar;        // [items][kTeamBarStride] arrival counter of each unit
    double2 *part;         // [tickets] member partials (loss sum, max|r|), unit u's at first[u]
    double2 *Ig, *Vg, *Wg; // [B][ld] a*I of the A sweep, V, exchanged w
    double2 *P0, *P1, *P2; // [B][ld] the state as pairs (|V|, theta), (m_vm, m_va), (s_vm, s_va)
    int64_t first_limit;   // wall-clock ticks a unit's first barrier waits without progress
    int64_t limit;         // ... and every later barrier
    int32_t win;           // complex entries of the LDS window (followed in LDS by the
                           // 16-bit halo list, kTeamHaloCap entries)
    int32_t grid;          // workgroups of the launch
    int32_t tmax;          // members per team at most
};

// members of every item of sub-grid (n buses, bandwidth bw) at row target R
__device__ __forceinline__ int team_size(int n, int bw, int R, int win, int tmax) {
    if (n <= R && n <= win) return 1;
    const int ns = (n + kWave - 1) / kWave;
    const int fit = ((win - 2 * bw) / kWave) * kWave;  // rows that fit beside both halos
    const int rs = max(min(R, fit), kWave) / kWave;     // slices per member
    const int T = (ns + rs - 1) / rs;
    return max(1, min(T, min(ns, tmax)));
}

// bucket of a per-member load of L rows: floor(2 log2 L), at most kLoadKeys - 1
__device__ __forceinline__ int load_key(int L) {
    if (L <= 1) return 0;
    const int lg = 31 - __clz(L);
    const int half = (long long)L * L >= (1LL << (2 * lg + 1)) ? 1 : 0;
    return min(kLoadKeys - 1, 2 * lg + half);
}

template <int NT>
__device__ __forceinline__ long long block_sum_ll(long long v, long long *buf) {
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) buf[threadIdx.x] += buf[threadIdx.x + o];
        __syncthreads();
    }
    const long long r = buf[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kPlanThreads) void team_plan_kernel(int32_t n_sub, const int32_t *__restrict__ sub_off,
                                                                 int32_t n_bus, const int32_t *__restrict__ sub_bw,
                                                                 int32_t B, TeamArgs p) {
    __shared__ int32_t cnt[kLoadKeys][kPlanThreads];
    __shared__ int32_t wtot[kPlanThreads / kWave][kLoadKeys];
    __shared__ long long buf[kPlanThreads];
    __shared__ int32_t sh_R;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wv = tid / kWave;
    auto n_of = [&](int s) { return sub_off ? sub_off[s + 1] - sub_off[s] : n_bus; };
    auto members = [&](int R) {
        long long m = 0;
        for (int s = tid; s < n_sub; s += kPlanThreads) m += team_size(n_of(s), sub_bw[s], R, p.win, p.tmax);
        return block_sum_ll<kPlanThreads>(m, buf) * B;
    };

    // ---- per-member row target
    const long long total = (long long)B * n_bus;
    const int rcap = max(kWave, (p.win / kWave) * kWave);
    int bestR = rcap;
    long long best = -1;
    for (int w = 1; w <= kTeamMaxWaves; ++w) {
        const long long cap_m = (long long)w * p.grid;
        const long long need = (total + cap_m - 1) / cap_m;
        int lo = (int)min<long long>(rcap, max<long long>(kWave, (need + kWave - 1) / kWave * kWave));
        int hi = rcap;
        if (members(hi) > cap_m) continue;  // not even at the largest rows
        while (lo < hi) {                   // smallest R (multiple of 64) that fits w waves
            const int mid = (lo / kWave + hi / kWave) / 2 * kWave;
            if (members(mid) <= cap_m) hi = mid;
            else lo = mid + kWave;
        }
        const long long cost = (long long)w * (hi + kTeamRowsPerBarrier);
        if (best < 0 || cost < best) {
            best = cost;
            bestR = hi;
        }
    }
    if (tid == 0) sh_R = bestR;
    __syncthreads();
    const int R = sh_R;

    // ---- units in descending per-member load (stable counting sort over the buckets)
    const int items = B * n_sub;
    const int per = (items + kPlanThreads - 1) / kPlanThreads;
    const int i0 = min(tid * per, items), i1 = min(i0 + per, items);
    auto key_of = [&](int item) {
        const int s = item / B;
        const int n = n_of(s);
        const int T = team_size(n, sub_bw[s], R, p.win, p.tmax);
        return load_key((n + T - 1) / T);
    };
    for (int b = 0; b < kLoadKeys; ++b) cnt[b][tid] = 0;
    for (int i = i0; i < i1; ++i) cnt[key_of(i)][tid] += 1;
    int c[kLoadKeys];
#pragma unroll
    for (int b = 0; b < kLoadKeys; ++b) {
        c[b] = cnt[b][tid];
        int incl = c[b];
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += y;
        }
        c[b] = incl - c[b];  // exclusive within the wave
        if (lane == kWave - 1) wtot[wv][b] = incl;
    }
    __syncthreads();
    {
        int base = 0;  // units of the buckets above b, then of the earlier waves in b
        for (int b = kLoadKeys - 1; b >= 0; --b) {
            int tot = 0, before = 0;
            for (int k = 0; k < kPlanThreads / kWave; ++k) {
                tot += wtot[k][b];
                before += k < wv ? wtot[k][b] : 0;
            }
            cnt[b][tid] = base + before;  // this thread's first slot in bucket b (own counts above)
            base += tot;
        }
    }
#pragma unroll
    for (int b = 0; b < kLoadKeys; ++b) cnt[b][tid] += c[b];
    for (int i = i0; i < i1; ++i) {
        const int k = key_of(i);
        p.unit_item[cnt[k][tid]] = i;
        cnt[k][tid] += 1;
    }
    __syncthreads();

    // ---- first ticket of each unit: exclusive scan of the team sizes in unit order
    long long own = 0;
    for (int u = i0; u < i1; ++u) {
        const int s = p.unit_item[u] / B;
        own += team_size(n_of(s), sub_bw[s], R, p.win, p.tmax);
    }
    buf[tid] = own;
    __syncthreads();
    long long before = 0;
    for (int k = 0; k < tid; ++k) before += buf[k];
    for (int u = i0; u < i1; ++u) {
        p.first[u] = (int32_t)before;
        const int s = p.unit_item[u] / B;
        before += team_size(n_of(s), sub_bw[s], R, p.win, p.tmax);
    }
    if (tid == kPlanThreads - 1) {
        p.first[items] = (int32_t)before;
        p.hdr[0] = 0;
        p.hdr[1] = (int32_t)before;
        p.hdr[2] = items;
    }
    for (int u = tid; u < items; u += kPlanThreads) p.bar[(int64_t)u * kTeamBarStride] = 0;
}

// Arrival barrier of the T members of one unit; false when it was abandoned.
// first: the unit's first barrier, which waits while the arrival count or the
// device's progress count moves and abandons after `limit` ticks without either;
// later barriers abandon after `limit` ticks.
__device__ __forceinline__ bool unit_barrier(long long *cnt, long long target, int64_t limit, bool first,
                                             const int32_t *progress, int *flag) {
    dev_stores_done();
    __syncthreads();
    if (threadIdx.x == 0) {
        long long v = (long long)atomicAdd((unsigned long long *)cnt, 1ULL) + 1;
        bool ok = (v & kTeamAbort) == 0;
        int64_t t0 = wall_clock64();
        int32_t pv = first ? __hip_atomic_load(const_cast<int32_t *>(progress), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT)
                           : 0;
        long long lv = v;
        while (ok && v < target) {
            __builtin_amdgcn_s_sleep(1);
            v = __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v & kTeamAbort) {
                ok = false;
            } else if (v < target) {
                if (first) {
                    const int32_t pg = __hip_atomic_load(const_cast<int32_t *>(progress), __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                    if (pg != pv || v != lv) {
                        pv = pg;
                        lv = v;
                        t0 = wall_clock64();
                        continue;
                    }
                }
                if (wall_clock64() - t0 > limit) {
                    // abandon only if no member arrived meanwhile (else poll again)
                    if ((long long)atomicCAS((unsigned long long *)cnt, (unsigned long long)v,
                                             (unsigned long long)(v | kTeamAbort)) == v)
                        ok = false;
                }
            }
        }
        *flag = ok ? 1 : 0;
    }
    __syncthreads();
    return *flag != 0;
}

// member `mem` of the T members of unit u
template <int NT>
__device__ __forceinline__ void team_member(const SolveArgs &a, const TeamArgs &p, int u, int mem, int T,
                                            double2 *__restrict__ X, double (*red)[NT / kWave], int *bar_flag,
                                            int *scan_part) {
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int item = p.unit_item[u];
    const int sidx = item / a.B;
    const int c = item - sidx * a.B;
    const int s0 = a.sub_off ? a.sub_off[sidx] : 0;
    const int n = (a.sub_off ? a.sub_off[sidx + 1] : a.n_bus) - s0;
    const int out_idx = c * a.n_sub + sidx;
    long long *cnt = p.bar + (int64_t)u * kTeamBarStride;
    double2 *part = p.part + p.first[u];
    int32_t *progress = p.progress;
    if (*a.bad_grid) {  // a row longer than the declared bound (see DPF_BAD_GRID)
        if (mem == 0 && tid == 0) {
            a.status[out_idx] = DPF_BAD_GRID;
            a.iters[out_idx] = 0;
        }
        return;
    }
    const Rank2 r2 = outage_of_case(a.ov, c, s0, s0 + n);
    if (r2.bad) return;  // reported by the call's prologue; every member leaves
    const int of = r2.of, ot = r2.ot;
    const double2 oy = r2.oy, oyd = r2.oyd;
    ItemSched sc = load_item_sched(a, out_idx);
    const double m_res = residual_count<NT>(a.bt, s0, s0 + n, red);
    const double two_over_m = m_res > 0.0 ? 2.0 / m_res : 0.0;

    // rows of the member and its LDS window [xlo, xlo + wn) (sub-grid-local)
    const int ns = (n + kWave - 1) / kWave;
    const int rlo = (int)((int64_t)mem * ns / T) * kWave;
    const int rhi = min((int)((int64_t)(mem + 1) * ns / T) * kWave, n);
    int xlo = 0, wn = n;
    if (n > p.win) {
        const int rows = rhi - rlo;
        const int H = rows < p.win ? min(a.sub_bw[sidx], (p.win - rows) / 2) : 0;
        xlo = max(0, rlo - H);
        wn = min(p.win, min(n, rhi + H) - xlo);
    }

    const int64_t cb = (int64_t)c * a.ld + s0;
    double2 *__restrict__ P0 = p.P0 + cb;
    double2 *__restrict__ P1 = p.P1 + cb;
    double2 *__restrict__ P2 = p.P2 + cb;
    double2 *__restrict__ Ig = p.Ig + cb;
    double2 *__restrict__ Vg = p.Vg + cb;
    double2 *__restrict__ Wg = p.Wg + cb;
    const double2 *__restrict__ Sc = a.s_spec + (int64_t)c * a.s_ld + s0;
    const int8_t *__restrict__ btp = a.bt + s0;
    const int slice0 = a.sell.slice_off[sidx];
    const int32_t *__restrict__ swidth = a.sell.width;
    const int32_t *__restrict__ sstart = a.sell.start;
    const int32_t *__restrict__ scol = a.sell.col;
    const double2 *__restrict__ sval = a.sell.val;

    // what crosses the team's barriers (V, w, the partials) is read and written
    // at device scope, 16 bytes per access, through uniform bases; a team of one
    // uses cached accesses
    const bool solo = T == 1;
    const __amdgpu_buffer_rsrc_t rV = buffer_of(Vg, (uint32_t)n * 16u);  // whole sub-grid
    const __amdgpu_buffer_rsrc_t rW = buffer_of(Wg, (uint32_t)n * 16u);
    const __amdgpu_buffer_rsrc_t rVx = buffer_of(Vg + xlo, (uint32_t)wn * 16u);  // the window
    const __amdgpu_buffer_rsrc_t rWx = buffer_of(Wg + xlo, (uint32_t)wn * 16u);
    const __amdgpu_buffer_rsrc_t rPart = buffer_of(part, (uint32_t)T * 16u);
    auto ld2 = [solo](__amdgpu_buffer_rsrc_t r, int idx) {
        return solo ? rsrc_ld2<false>(r, idx) : rsrc_ld2<true>(r, idx);
    };
    auto st2 = [solo](__amdgpu_buffer_rsrc_t r, int idx, double2 v) {
        if (solo) rsrc_st2<false>(r, idx, v);
        else rsrc_st2<true>(r, idx, v);
    };
    // exchanged value of a column: the LDS window, else the global copy behind r
    auto xat = [&, xlo, wn](int col, __amdgpu_buffer_rsrc_t r) {
        return (unsigned)(col - xlo) < (unsigned)wn ? X[col - xlo] : ld2(r, col);
    };

    // The member's own rows and the halo columns of the window they read (their
    // neighbours outside [rlo, rhi), the two buses of the outage): the refills load
    // the rows as a range and the halo columns from a 16-bit list of window offsets
    // behind X (at most kTeamHaloCap; a longer halo refills the whole window).  A
    // window is wider than what the member reads whenever the bandwidth exceeds
    // the halo its rows actually touch.  The bitmap that builds the list lives in
    // X, which is filled only after it has been read.
    uint32_t *need = reinterpret_cast<uint32_t *>(X);
    uint16_t *hlist = reinterpret_cast<uint16_t *>(X + p.win);
    const int nwords = (wn + 31) / 32;
    for (int k = tid; k < nwords; k += NT) need[k] = 0u;
    __syncthreads();
    auto mark = [&](int col) {
        const int x = col - xlo;
        if ((unsigned)x < (unsigned)wn && (col < rlo || col >= rhi)) atomicOr(need + (x >> 5), 1u << (x & 31));
    };
    for (int il = rlo + tid; il < rhi; il += NT) {
        const int gsl = __builtin_amdgcn_readfirstlane(slice0 + (il >> 6));
        const int wdt = swidth[gsl];
        const int base = sstart[gsl] * kWave + lane;
        for (int q = 0; q < wdt; ++q) mark(scol[base + q * kWave]);
    }
    if (of >= 0 && tid < 2) mark(tid == 0 ? of : ot);
    __syncthreads();
    int n_halo = 0;  // -1: more than the list holds
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
        int before = 0;
        for (int k = 0; k < NT / kWave; ++k) {
            before += k < tid / kWave ? scan_part[k] : 0;
            n_halo += scan_part[k];
        }
        if (n_halo <= kTeamHaloCap) {
            int pos = before + incl - cnt_b;
            for (int w = w0; w < w1; ++w)
                for (uint32_t bits = need[w]; bits != 0u; bits &= bits - 1u)
                    hlist[pos++] = (uint16_t)(w * 32 + __ffs(bits) - 1);
        } else {
            n_halo = -1;
        }
        __syncthreads();
    }
    const int own0 = rlo - xlo, own1 = min(rhi, xlo + wn) - xlo;  // own rows inside the window
    // The sweeps take the member's rows in chunks of NT; in chunk k wave v takes the
    // chunk's slice (v + 5k) mod 16 (a different slice order per chunk).  With a
    // fixed order, a numbering whose heavy slices recur every 512 or 1024 rows (rows
    // sorted by degree in windows of that size) gives the same waves the widest
    // slices in every chunk, and the workgroup waits for them at the sweep's end:
    // about 9% of the time of the uneven batch.
    static_assert((NT / kWave & (NT / kWave - 1)) == 0, "waves per workgroup: a power of two");
    const int nchunk = (rhi - rlo + NT - 1) / NT;
    auto row_of = [&](int k) {
        return rlo + k * NT + ((((tid / kWave) + 5 * k) & (NT / kWave - 1)) * kWave) + lane;
    };
    // X <- the columns the rows read, through resource r (window offsets)
    auto fill = [&](auto &&load) {
        if (n_halo < 0) {
            for (int k = tid; k < wn; k += NT) X[k] = load(k);
            return;
        }
        for (int k = own0 + tid; k < own1; k += NT) X[k] = load(k);
        for (int k = tid; k < n_halo; k += NT) {
            const int x = hlist[k];
            X[x] = load(x);
        }
    };

    // V of the member's rows for the team
    for (int il = rlo + tid; il < rhi; il += NT) {
        double sn, cs;
        const double2 p0 = P0[il];
        fast_sincos(p0.y, sn, cs);
        st2(rV, il, make_double2(p0.x * cs, p0.x * sn));
    }
    long long nbar = 0;
    bool ok = true;
    if (!solo) ok = unit_barrier(cnt, ++nbar * T, p.first_limit, true, progress, bar_flag);
    else __syncthreads();

    int it = 0, stat = DPF_UNFINISHED;
    double mu = 0.0, loss = 0.0;
    while (ok) {
        fill([&](int x) { return ld2(rVx, x); });
        __syncthreads();
        // ---------------- A: rows of this member
        double lsum = 0.0, lmax = 0.0;
        for (int k = 0; k < nchunk; ++k) {
            const int il = row_of(k);
            if (il >= rhi) continue;
            const int8_t tk = btp[il];
            const double2 sp = Sc[il];
            const int gsl = __builtin_amdgcn_readfirstlane(slice0 + (il >> 6));
            const int wdt = swidth[gsl];
            const int base = sstart[gsl] * kWave + lane;
            double2 acc = make_double2(0.0, 0.0);
            acc = sell_row<4, false>(sval, scol, base, wdt, il, [&](int j) { return xat(j, rV); }, acc);
            if (il == of) acc = csub(acc, csub(cmul(oyd, xat(of, rV)), cmul(oy, xat(ot, rV))));
            else if (il == ot) acc = csub(acc, csub(cmul(oyd, xat(ot, rV)), cmul(oy, xat(of, rV))));
            const double2 v = xat(il, rV);
            const double2 d = csub(cmulc(v, acc), sp);
            const double rP = tk != kSlack ? d.x : 0.0;
            const double rQ = tk == kPQ ? d.y : 0.0;
            lsum += rP * rP + rQ * rQ;
            lmax = fmax(lmax, fmax(fabs(rP), fabs(rQ)));
            Ig[il] = cmul(make_double2(two_over_m * rP, two_over_m * rQ), acc);  // a*I for the B sweep
            st2(rW, il, cmulc(make_double2(two_over_m * rP, two_over_m * rQ), v));
        }
        block_reduce2<NT>(lsum, lmax, red);
        __syncthreads();
        block_reduce2_finish<NT>(lsum, lmax, red);
        if (!solo) {
            if (tid == 0) rsrc_st2<true>(rPart, mem, make_double2(lsum, lmax));
            ok = unit_barrier(cnt, ++nbar * T, p.limit, false, progress, bar_flag);
            if (!ok) break;
            // team totals: the T partials reduced in the same order by every member
            // (their loads overlap the refill of X with w)
            double s = 0.0, m = 0.0;
            if (tid < T) {
                const double2 pp = rsrc_ld2<true>(rPart, tid);
                s = pp.x;
                m = pp.y;
            }
            fill([&](int x) { return rsrc_ld2<true>(rWx, x); });
            block_reduce2<NT>(s, m, red);
            __syncthreads();
            block_reduce2_finish<NT>(s, m, red);
            __syncthreads();
            lsum = s;
            lmax = m;
        } else {
            __syncthreads();
            fill([&](int x) { return Wg[xlo + x]; });
            __syncthreads();
        }
        loss = m_res > 0.0 ? lsum / m_res : 0.0;
        mu = isnan(lsum) ? lsum : lmax;
        trace_mu(a, mem == 0, out_idx, it, mu);
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

        // ---------------- B: rows of this member
        sc.t_step += 1.0;
        sc.b1t *= a.b1;
        sc.b2t *= a.b2;
        const double bc1 = 1.0 - sc.b1t;
        const double bc2 = 1.0 - sc.b2t;
        for (int k = 0; k < nchunk; ++k) {
            const int il = row_of(k);
            if (il >= rhi) continue;
            const int8_t tk = btp[il];
            const double2 ai = Ig[il];
            const double2 p0 = P0[il];
            double vmi = p0.x, vai = p0.y;
            const int gsl = __builtin_amdgcn_readfirstlane(slice0 + (il >> 6));
            const int wdt = swidth[gsl];
            const int base = sstart[gsl] * kWave + lane;
            double2 h = make_double2(0.0, 0.0);
            h = sell_row<4, false>(sval, scol, base, wdt, il, [&](int j) { return xat(j, rW); }, h);
            if (il == of) h = csub(h, csub(cmul(oyd, xat(of, rW)), cmul(oy, xat(ot, rW))));
            else if (il == ot) h = csub(h, csub(cmul(oyd, xat(ot, rW)), cmul(oy, xat(of, rW))));
            // V of this row, rebuilt from |V| and theta (the same bits the owner published)
            double2 v;
            {
                double sn0, cs0;
                fast_sincos(vai, sn0, cs0);
                v = make_double2(vmi * cs0, vmi * sn0);
            }
            const double2 G = make_double2(ai.x + h.x, ai.y - h.y);
            if (tk != kSlack) {
                const double2 p1 = P1[il], p2 = P2[il];
                double mv = p1.x, ma = p1.y, sv = p2.x, sa = p2.y;
                if (tk == kPQ) {
                    const double g = (G.x * v.x + G.y * v.y) / vmi;
                    vmi = opt_update(a.opt, sc.lr, a.b1, a.b2, a.eps, bc1, bc2, vmi, g, mv, sv);
                }
                const double g = G.y * v.x - G.x * v.y;
                vai = opt_update(a.opt, sc.lr, a.b1, a.b2, a.eps, bc1, bc2, vai, g, ma, sa);
                P0[il] = make_double2(vmi, vai);
                P1[il] = make_double2(mv, ma);
                P2[il] = make_double2(sv, sa);
                double sn, cs;
                fast_sincos(vai, sn, cs);
                st2(rV, il, make_double2(vmi * cs, vmi * sn));
            }
        }
        sched_step(a, sc, loss);
        ++it;
        if (mem == 0 && tid == 0 && (it & 63) == 0) atomicAdd(progress, 1);
        if (!solo) {
            ok = unit_barrier(cnt, ++nbar * T, p.limit, false, progress, bar_flag);
            if (!ok) break;  // the members that arrived applied this iteration's step
        } else {
            __syncthreads();
        }
    }
    if (mem != 0 || tid != 0) return;
    atomicAdd(progress, 1);
    finish_item(a, out_idx, it, ok ? stat : DPF_UNFINISHED, mu, loss, sc);
}

template <int NT>
__global__ __launch_bounds__(NT) void team_solve_persist_kernel(SolveArgs a, TeamArgs p) {
    extern __shared__ double2 X[];
    __shared__ double red[2][NT / kWave];
    __shared__ int bar_flag;
    __shared__ int sh_t, sh_u;
    __shared__ int scan_part[NT / kWave];
    const int tid = threadIdx.x;
    const int n_tickets = p.hdr[1];
    const int n_units = p.hdr[2];
    for (;;) {
        if (tid == 0) {
            const int t = atomicAdd(p.hdr, 1);
            int u = 0;  // largest u with first[u] <= t
            if (t < n_tickets)
                for (int hi_u = n_units - 1; u < hi_u;) {
                    const int m = (u + hi_u + 1) >> 1;
                    if (p.first[m] <= t) u = m;
                    else hi_u = m - 1;
                }
            sh_t = t;
            sh_u = u;
        }
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(sh_t), u = __builtin_amdgcn_readfirstlane(sh_u);
        __syncthreads();
        if (t >= n_tickets) break;
        team_member<NT>(a, p, u, t - p.first[u], p.first[u + 1] - p.first[u], X, red, &bar_flag, scan_part);
        __syncthreads();
    }
}

}  // namespace dpf
