// DC power flow on the device: the linear approximation that the paper lists as
// a screening method (Sec. 3, direct methods) and that Algorithm 2 uses to
// initialise Newton-Raphson.  With |V| = 1, no losses and small angle
// differences, the active injections satisfy  L theta = P,  where L is the
// branch-susceptance Laplacian (weights 1/x) and the slack angle is fixed.
//
// L comes from an admittance matrix built with r = 0 and b = 0 (the "DC grid"):
// there Y = -j L, so L_ij = -Im(Y_ij).  One workgroup per case solves the
// grounded system by conjugate gradients with a Jacobi preconditioner; the
// search direction lives in LDS (8 B per bus), the other vectors in the
// workspace.  An N-1 outage removes the branch's 1/x (rank-1, on the fly).
#pragma once

#include "../../include/dpf.h"
#include "common.hpp"
#include "eval.hpp"

namespace dpf {

struct DcArgs {
    const int32_t *rp;
    const int32_t *ci;
    const double2 *yv;  // admittance matrix of the DC grid (r = 0, b = 0)
    const int8_t *bt;
    const double2 *s_spec;
    int64_t s_ld;
    OutageView ov;
    double *va;  // [B][ld] in: start (slack angle fixed), out: DC angles
    int64_t ld;
    double *r;   // [B][n] residual
    double *z;   // [B][n] preconditioned residual
    double *dg;  // [B][n] diagonal of L (after the outage)
    int32_t n;
    double tol;
    int32_t max_iter;
    int32_t *iters;    // [B] or null
    double *res_out;   // [B] relative residual ||r|| / ||P||, or null
};

template <int NT>
__device__ __forceinline__ void block_sum2(double &a, double &b, double (*red)[NT / kWave]) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int wv = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        red[0][wv] = a;
        red[1][wv] = b;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
#pragma unroll
    for (int k = 0; k < NT / kWave; ++k) {
        a += red[0][k];
        b += red[1][k];
    }
    a = uniform(a);
    b = uniform(b);
    __syncthreads();
}

// (L p)_i for a real vector p held in LDS; the outaged branch's block removed
__device__ __forceinline__ double dc_row(const DcArgs &a, int i, const double *p, int of, int ot, double oyi) {
    double acc = 0.0;
    for (int q = a.rp[i]; q < a.rp[i + 1]; ++q) {
        const int j = a.ci[q];
        if ((unsigned)j < (unsigned)a.n) acc += a.yv[q].y * p[j];
    }
    double v = -acc;  // L = -Im(Y)
    // outage: L loses (1/x)(e_f - e_t)(e_f - e_t)^T; Im(y) = -1/x for y = 1/(jx)
    if (i == of) v += oyi * (p[of] - p[ot]);
    else if (i == ot) v += oyi * (p[ot] - p[of]);
    return v;
}

template <int NT>
__global__ __launch_bounds__(NT) void dc_pcg_kernel(DcArgs a) {
    extern __shared__ double P[];
    __shared__ double red[2][NT / kWave];
    const int c = blockIdx.x;
    const int n = a.n;
    double *va = a.va + (int64_t)c * a.ld;
    double *r = a.r + (int64_t)c * n;
    double *z = a.z + (int64_t)c * n;
    double *dg = a.dg + (int64_t)c * n;
    const double2 *S = a.s_spec + (int64_t)c * a.s_ld;

    int of = -1, ot = -1;
    double oyi = 0.0;  // Im of the outaged branch's series admittance (= -1/x)
    if (a.ov.outage) {
        const int k = a.ov.outage[c];
        if (outage_index_bad(k, a.ov.n_branch)) {  // neither -1 nor a branch: va untouched
            if (threadIdx.x == 0) {
                if (a.iters) a.iters[c] = 0;
                if (a.res_out) a.res_out[c] = __longlong_as_double(0x7ff8000000000000LL);
            }
            return;
        }
        if ((unsigned)k < (unsigned)a.ov.n_branch) {
            const int f = a.ov.from[k], t = a.ov.to[k];
            if ((unsigned)f < (unsigned)n && (unsigned)t < (unsigned)n && f != t) {
                of = f;
                ot = t;
                double2 y, ysh;
                branch_admittance(a.ov.r[k], a.ov.x[k], a.ov.b[k], y, ysh);
                oyi = y.y;
            }
        }
    }

    // start: theta in LDS (slack entry fixed), diagonal, r = P - L theta, z = r / diag
    for (int i = threadIdx.x; i < n; i += NT) P[i] = va[i];
    __syncthreads();
    double bb = 0.0, rz = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) {
        double d = 0.0;
        for (int q = a.rp[i]; q < a.rp[i + 1]; ++q)
            if (a.ci[q] == i) d = -a.yv[q].y;
        if (i == of || i == ot) d += oyi;
        const bool free = a.bt[i] != kSlack;
        const double b = free ? S[i].x : 0.0;
        const double ri = free ? b - dc_row(a, i, P, of, ot, oyi) : 0.0;
        const double zi = free && d > 0.0 ? ri / d : 0.0;
        dg[i] = d;
        r[i] = ri;
        z[i] = zi;
        bb += b * b;
        rz += ri * zi;
    }
    block_sum2<NT>(bb, rz, red);  // ends with a barrier: every read of theta in P is done
    const double bnorm = sqrt(bb);
    // search direction p = z (the slack entry stays 0)
    for (int i = threadIdx.x; i < n; i += NT) P[i] = z[i];
    double rr = 0.0, dummy = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) rr += r[i] * r[i];
    block_sum2<NT>(rr, dummy, red);
    int it = 0;
    while (it < a.max_iter && !(sqrt(rr) <= a.tol * bnorm)) {
        // q = L p; alpha = rz / (p . q)
        double pq = 0.0, unused = 0.0;
        for (int i = threadIdx.x; i < n; i += NT) {
            const double qi = a.bt[i] != kSlack ? dc_row(a, i, P, of, ot, oyi) : 0.0;
            z[i] = qi;  // z holds q until the update below
            pq += P[i] * qi;
        }
        block_sum2<NT>(pq, unused, red);
        const double alpha = pq != 0.0 ? rz / pq : 0.0;
        double rz_new = 0.0, rr_new = 0.0;
        for (int i = threadIdx.x; i < n; i += NT) {
            if (a.bt[i] == kSlack) continue;
            va[i] += alpha * P[i];
            const double ri = r[i] - alpha * z[i];
            const double zi = dg[i] > 0.0 ? ri / dg[i] : 0.0;
            r[i] = ri;
            z[i] = zi;
            rz_new += ri * zi;
            rr_new += ri * ri;
        }
        block_sum2<NT>(rz_new, rr_new, red);
        const double beta = rz != 0.0 ? rz_new / rz : 0.0;
        rz = rz_new;
        rr = rr_new;
        for (int i = threadIdx.x; i < n; i += NT) P[i] = z[i] + beta * P[i];
        __syncthreads();
        ++it;
    }
    if (threadIdx.x == 0) {
        if (a.iters) a.iters[c] = it;
        if (a.res_out) a.res_out[c] = bnorm > 0.0 ? sqrt(rr) / bnorm : sqrt(rr);
    }
}

}  // namespace dpf
