// One forward + fused-adjoint evaluation for B cases on one grid
// (dpf_mismatch_grad).  Case-major layout, one thread per (bus, case):
//
//   polar    : V = vm e^{j va}                                   -> ws.V
//   forward  : I = Y V (+ rank-2 outage term), dS = V conj(I) - S,
//              masked residual r, seed a = (2/m) r, w = a conj(V), aI = a I
//              per-block partial loss / max                        -> ws
//   adjoint  : h = Y^T w (Y symmetric: same CSR, + outage term),
//              G = aI + conj(h); g_vm = Re(conj(G) V)/vm, g_va = Im(G conj(V))
//   finalize : per-case loss = sum / m and max, fixed summation order
//
// The gradient follows from d loss = Re sum_k conj(G_k) dV_k with
// dV_k = e^{j va_k} dvm_k + j V_k dva_k (reverse mode through S = V conj(Y V)).
#pragma once

#include "common.hpp"

namespace dpf {

constexpr int kEvalBlock = 256;

struct OutageView {
    const int32_t *outage;  // [B] or null
    const int32_t *from;
    const int32_t *to;
    const double *r;
    const double *x;
    const double *b;
    int32_t n_branch;
};

// An outage index is -1 (no outage) or a branch index; anything else marks the
// case as bad (the solve reports DPF_BAD_OUTAGE, the evaluations return NaN).
__host__ __device__ __forceinline__ bool outage_index_bad(int32_t k, int32_t n_branch) {
    return k != -1 && (uint32_t)k >= (uint32_t)n_branch;
}

// Rank-2 correction: subtract branch k's pi-model block from row i of Y z.
// Y_k = [[y + ysh, -y], [-y, y + ysh]] on (f, t).
__device__ __forceinline__ double2 outage_term(const OutageView &ov, int32_t k, int32_t i, double2 zf, double2 zt,
                                               int32_t f, int32_t t) {
    double2 y, ysh;
    branch_admittance(ov.r[k], ov.x[k], ov.b[k], y, ysh);
    double2 yd = cadd(y, ysh);
    if (i == f) return csub(cmul(yd, zf), cmul(y, zt));
    return csub(cmul(yd, zt), cmul(y, zf));  // i == t
}

__global__ __launch_bounds__(1024) void residual_count_kernel(int32_t n, const int8_t *__restrict__ bt,
                                                               double *__restrict__ m_out) {
    __shared__ int part[16];
    int s = 0;
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
        int8_t t = bt[i];
        s += t == kPQ ? 2 : (t == kPV ? 1 : 0);
    }
    s = wave_isum(s);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) tot += part[w];
        *m_out = (double)tot;
    }
}

__global__ void polar_kernel(int32_t n, int64_t ld, const double *__restrict__ vm, const double *__restrict__ va,
                             double2 *__restrict__ V) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    int32_t c = blockIdx.y;
    if (i >= n) return;
    double s, co;
    fast_sincos(va[c * ld + i], s, co);
    double m = vm[c * ld + i];
    V[(int64_t)c * n + i] = make_double2(m * co, m * s);
}

__global__ __launch_bounds__(kEvalBlock) void forward_kernel(
    int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, const double2 *__restrict__ yv,
    const int8_t *__restrict__ bt, const double2 *__restrict__ s_spec, int64_t s_ld, OutageView ov,
    const double2 *__restrict__ V, const double *__restrict__ m_res, int64_t ld, double2 *__restrict__ dS,
    double2 *__restrict__ w, double2 *__restrict__ aI, double2 *__restrict__ part, double2 *__restrict__ g_s) {
    __shared__ double red[2][kEvalBlock / kWave];
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    int32_t c = blockIdx.y;
    const double2 *Vc = V + (int64_t)c * n;
    double lsum = 0.0, lmax = 0.0;
    if (i < n) {
        double2 acc = make_double2(0.0, 0.0);
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            int32_t j = ci[q];
            if ((uint32_t)j < (uint32_t)n) acc = cfma(yv[q], Vc[j], acc);
        }
        if (ov.outage) {
            int32_t k = ov.outage[c];
            if ((uint32_t)k < (uint32_t)ov.n_branch) {
                int32_t f = ov.from[k], t = ov.to[k];
                if ((i == f || i == t) && (uint32_t)f < (uint32_t)n && (uint32_t)t < (uint32_t)n)
                    acc = csub(acc, outage_term(ov, k, i, Vc[f], Vc[t], f, t));
            } else if (outage_index_bad(k, ov.n_branch)) {
                acc = make_double2(__longlong_as_double(0x7ff8000000000000LL), 0.0);  // NaN outputs
            }
        }
        double2 v = Vc[i];
        double2 s = s_spec[c * s_ld + i];
        double2 d = csub(cmulc(v, acc), s);
        int8_t ty = bt[i];
        double rP = ty != kSlack ? d.x : 0.0;
        double rQ = ty == kPQ ? d.y : 0.0;
        lsum = rP * rP + rQ * rQ;
        lmax = fmax(fabs(rP), fabs(rQ));
        double sc = 2.0 / *m_res;
        double2 a = make_double2(sc * rP, sc * rQ);
        int64_t o = (int64_t)c * n + i;
        w[o] = cmulc(a, v);
        aI[o] = cmul(a, acc);
        if (dS) dS[c * ld + i] = d;
        if (g_s) g_s[c * ld + i] = make_double2(-a.x, -a.y);  // d loss / d S_spec
    }
    lsum = wave_sum(lsum);
    lmax = wave_max(lmax);
    int wv = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        red[0][wv] = lsum;
        red[1][wv] = lmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0, m = 0.0;
        for (int k = 0; k < kEvalBlock / kWave; ++k) {
            s += red[0][k];
            m = fmax(m, red[1][k]);
        }
        part[(int64_t)c * gridDim.x + blockIdx.x] = make_double2(s, m);
    }
}

__global__ __launch_bounds__(kEvalBlock) void adjoint_kernel(
    int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, const double2 *__restrict__ yv,
    const int8_t *__restrict__ bt, OutageView ov, const double2 *__restrict__ V, const double *__restrict__ vm,
    int64_t ld, const double2 *__restrict__ w, const double2 *__restrict__ aI, double *__restrict__ g_vm,
    double *__restrict__ g_va) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    int32_t c = blockIdx.y;
    if (i >= n) return;
    const double2 *wc = w + (int64_t)c * n;
    double2 h = make_double2(0.0, 0.0);
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {  // Y^T w with Y = Y^T
        int32_t j = ci[q];
        if ((uint32_t)j < (uint32_t)n) h = cfma(yv[q], wc[j], h);
    }
    if (ov.outage) {
        int32_t k = ov.outage[c];
        if ((uint32_t)k < (uint32_t)ov.n_branch) {
            int32_t f = ov.from[k], t = ov.to[k];
            if ((i == f || i == t) && (uint32_t)f < (uint32_t)n && (uint32_t)t < (uint32_t)n)
                h = csub(h, outage_term(ov, k, i, wc[f], wc[t], f, t));
        }
    }
    int64_t o = (int64_t)c * n + i;
    double2 G = cadd(aI[o], cconj(h));
    double2 v = V[o];
    int8_t ty = bt[i];
    // conj(G) V = (G.x v.x + G.y v.y) + j (G.x v.y - G.y v.x)
    double gv = ty == kPQ ? (G.x * v.x + G.y * v.y) / vm[c * ld + i] : 0.0;
    double ga = ty != kSlack ? (G.y * v.x - G.x * v.y) : 0.0;
    g_vm[c * ld + i] = gv;
    g_va[c * ld + i] = ga;
}

// d loss / d(r, x, b) of every branch, from V and the adjoint seed w = a conj(V)
// of the forward kernel.  With d loss = Re sum_i w_i dI_i and dI = dY V, a branch
// (f, t) with y = 1/(r + jx) and charging b contributes
//   dI_f = dy (V_f - V_t) + j (db/2) V_f,  dI_t = dy (V_t - V_f) + j (db/2) V_t,
// so with D = (w_f - w_t)(V_f - V_t) and dy = -y^2 (dr + j dx):
//   d/dr = -Re(y^2 D),  d/dx = Im(y^2 D),  d/db = -Im(w_f V_f + w_t V_t) / 2.
// The outaged branch of a case is absent from its Y: gradient 0.
__global__ __launch_bounds__(kEvalBlock) void branch_grad_kernel(int32_t n, int32_t n_branch, OutageView ov,
                                                                  const double2 *__restrict__ V,
                                                                  const double2 *__restrict__ w, int64_t bld,
                                                                  double *__restrict__ g_r, double *__restrict__ g_x,
                                                                  double *__restrict__ g_b) {
    const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t c = blockIdx.y;
    if (e >= n_branch) return;
    const int32_t f = ov.from[e], t = ov.to[e];
    double gr = 0.0, gx = 0.0, gb = 0.0;
    const bool out = ov.outage && ov.outage[c] == e;
    if (!out && f != t && (uint32_t)f < (uint32_t)n && (uint32_t)t < (uint32_t)n) {
        const int64_t o = (int64_t)c * n;
        const double2 vf = V[o + f], vt = V[o + t], wf = w[o + f], wt = w[o + t];
        double2 y, ysh;
        branch_admittance(ov.r[e], ov.x[e], ov.b[e], y, ysh);
        const double2 D = cmul(csub(wf, wt), csub(vf, vt));
        const double2 y2D = cmul(cmul(y, y), D);
        gr = -y2D.x;
        gx = y2D.y;
        gb = -0.5 * (cmul(wf, vf).y + cmul(wt, vt).y);
    }
    const int64_t q = (int64_t)c * bld + e;
    g_r[q] = gr;
    g_x[q] = gx;
    g_b[q] = gb;
}

__global__ void finalize_kernel(int32_t B, int32_t nblk, const double2 *__restrict__ part,
                                const double *__restrict__ m_res, double *__restrict__ loss,
                                double *__restrict__ max_mis) {
    int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= B) return;
    double s = 0.0, m = 0.0;
    bool nan = false;
    for (int32_t k = 0; k < nblk; ++k) {
        double2 p = part[(int64_t)c * nblk + k];
        s += p.x;
        m = fmax(m, p.y);
        nan |= isnan(p.y);
    }
    double mm = *m_res;
    loss[c] = mm > 0.0 ? s / mm : 0.0;
    // a NaN residual makes the sum NaN; report it in max_mis too
    max_mis[c] = (nan || isnan(s)) ? __longlong_as_double(0x7ff8000000000000LL) : m;
}

}  // namespace dpf
