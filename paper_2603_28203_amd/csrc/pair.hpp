// Banded solve with paired state: the A/W and gradient sweeps of the
// barrier-free banded kernel (team_solve_band_kernel<NT, J>), with the
// per-bus state of a case held in the workspace as three complex-sized pairs
//     P0 = (|V|, theta),  P1 = (m_vm, m_va),  P2 = (s_vm, s_va)
// instead of six separate arrays.  Same arithmetic in the same order, so the
// iterates equal the banded kernel's bit for bit.
//
// Why: the banded kernel on gfx950 is bound by the vector-memory instructions
// its waves issue per bus and the bytes they move (rocprofv3: about 37 memory
// instructions per bus-iteration, 160 bytes to and from HBM against the 96-byte
// floor).  Here a bus's state takes three 16-byte loads and three 16-byte stores
// per iteration instead of six 8-byte ones each way, and the refill of the
// exchange vector one load instead of two; the bytes are the same (5% less time
// per iteration on the N-1 batch).  Removing VALU work instead (one sincos per
// bus-iteration, Adam's bias corrections as per-iteration scalars) at the price
// of one more 16-byte store per bus was measured 3% slower.
// pair_in_kernel fills the pairs from the caller's arrays before the solve and
// pair_out_kernel writes them back after it (also for items paused for the tail
// handoff, whose state the split kernel reads from the caller's layout).
#pragma once

#include "../../include/dpf.h"
#include "common.hpp"
#include "eval.hpp"
#include "sell.hpp"
#include "solve.hpp"

namespace dpf {

// P0..P2 [B][ld] complex from vm, va and the moments st [4][B][ld] (m_vm, m_va,
// s_vm, s_va); fresh: the moments start at zero
__global__ void pair_in_kernel(int32_t n, int64_t ld, int32_t B, const double *__restrict__ vm,
                               const double *__restrict__ va, const double *__restrict__ st, int64_t stride,
                               int32_t fresh, double2 *__restrict__ P0, double2 *__restrict__ P1,
                               double2 *__restrict__ P2) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int32_t c = blockIdx.y; c < B; c += gridDim.y) {  // the grid's y extent may be below B
        const int64_t o = (int64_t)c * ld + i;
        P0[o] = make_double2(vm[o], va[o]);
        if (fresh) {
            P1[o] = make_double2(0.0, 0.0);
            P2[o] = make_double2(0.0, 0.0);
        } else {
            P1[o] = make_double2(st[o], st[stride + o]);
            P2[o] = make_double2(st[2 * stride + o], st[3 * stride + o]);
        }
    }
}

// the pairs back to vm, va and the moments (every entry: the kernel leaves the
// fixed coordinates as they came in)
__global__ void pair_out_kernel(int32_t n, int64_t ld, int32_t B, double *__restrict__ vm, double *__restrict__ va,
                                double *__restrict__ st, int64_t stride, const double2 *__restrict__ P0,
                                const double2 *__restrict__ P1, const double2 *__restrict__ P2) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int32_t c = blockIdx.y; c < B; c += gridDim.y) {
        const int64_t o = (int64_t)c * ld + i;
        const double2 p0 = P0[o], p1 = P1[o], p2 = P2[o];
        vm[o] = p0.x;
        va[o] = p0.y;
        st[o] = p1.x;
        st[stride + o] = p1.y;
        st[2 * stride + o] = p2.x;
        st[3 * stride + o] = p2.y;
    }
}

// a.scratch holds [4][B][ld] complex: I of the A/W sweep, then P0, P1, P2
template <int NT, int J>
__global__ __launch_bounds__(NT) void team_solve_pair_kernel(SolveArgs a) {
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

    ItemSched sc = load_item_sched(a, out_idx);
    const double m_res = residual_count<NT>(a.bt, lo, hi, red);
    const double two_over_m = m_res > 0.0 ? 2.0 / m_res : 0.0;
    const Rank2 r2 = outage_of_case(a.ov, c, lo, hi);
    if (r2.bad) return;  // reported by the call's prologue
    const int of = r2.of, ot = r2.ot;
    const double2 oy = r2.oy, oyd = r2.oyd;

    const int64_t cb = (int64_t)c * a.ld;
    const int64_t sb = (int64_t)c * a.s_ld;
    double2 *__restrict__ Ig = a.scratch + cb;
    double2 *__restrict__ P0 = a.scratch + a.st_stride + cb;
    double2 *__restrict__ P1 = a.scratch + 2 * a.st_stride + cb;
    double2 *__restrict__ P2 = a.scratch + 3 * a.st_stride + cb;
    const double2 *__restrict__ Sc = a.s_spec + sb;
    const int32_t *__restrict__ swidth = a.sell.width;
    const int32_t *__restrict__ sstart = a.sell.start;
    const int32_t *__restrict__ scol = a.sell.col;
    const double2 *__restrict__ sval = a.sell.val;
    const int8_t *__restrict__ btp = a.bt;

    // the exchange vector starts as V = |V| e^{j theta}
    auto refill = [&]() {
        for (int i = lo + tid; i < hi; i += NT) {
            double sn, cs;
            const double2 p = P0[i];
            fast_sincos(p.y, sn, cs);
            X[i - lo] = make_double2(p.x * cs, p.x * sn);
        }
    };
    refill();
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
        // ---------------- A/W sweep (as in team_solve_band_kernel)
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

        // ---------------- gradient sweep: one barrier-free pass (w stays in X), then
        // the new V refilled from the updated pairs
        sc.t_step += 1.0;
        sc.b1t *= a.b1;
        sc.b2t *= a.b2;
        const double bc1 = 1.0 - sc.b1t;
        const double bc2 = 1.0 - sc.b2t;
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
                    const double2 p0 = P0[i], p1 = P1[i], p2 = P2[i];
                    const int gsl = __builtin_amdgcn_readfirstlane(slice0 + (il >> 6));
                    const int wdt = swidth[gsl];
                    const int base = sstart[gsl] * kWave + lane;
                    double2 h = make_double2(0.0, 0.0);
                    h = sell_row<4, false>(sval, scol, base, wdt, il, [&](int j) { return X[j]; }, h);
                    if (il == of) h = csub(h, csub(cmul(oyd, X[of]), cmul(oy, X[ot])));
                    else if (il == ot) h = csub(h, csub(cmul(oyd, X[ot]), cmul(oy, X[of])));
                    double vmi = p0.x, vai = p0.y;
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
                    double mv = p1.x, ma = p1.y, sv = p2.x, sa = p2.y;
                    if (tk == kPQ) {
                        const double g = (G.x * v.x + G.y * v.y) / vmi;
                        vmi = opt_update(a.opt, sc.lr, a.b1, a.b2, a.eps, bc1, bc2, vmi, g, mv, sv);
                    }
                    if (tk != kSlack) {
                        const double g = G.y * v.x - G.x * v.y;
                        vai = opt_update(a.opt, sc.lr, a.b1, a.b2, a.eps, bc1, bc2, vai, g, ma, sa);
                        P0[i] = make_double2(vmi, vai);
                        P1[i] = make_double2(mv, ma);
                        P2[i] = make_double2(sv, sa);
                    }
                }
            }
        }
        __syncthreads();
        refill();
        sched_step(a, sc, loss);
        __syncthreads();
    }

    if (tid == 0) finish_item(a, out_idx, it, stat, mu, loss, sc);
}

}  // namespace dpf
