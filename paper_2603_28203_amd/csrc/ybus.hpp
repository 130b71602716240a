// Bus admittance matrix assembly on the device (pi-model branches, Sec. 2.1).
//
// Pipeline (one thread per branch or per row; rows have a handful of entries):
//   1. validate branches, count incident branches per bus (integer atomics)
//   2. exclusive scan of (1 + degree)            -> slot offsets
//   3. scatter (neighbour, branch) slots per row  (slot 0 of each row = diagonal)
//   4. per row: order slots by branch, sum the diagonal in branch order, then
//      stable-order by column and count distinct columns
//   5. exclusive scan of the distinct counts      -> row_ptr
//   6. per row: emit merged entries; parallel branches are summed in branch order
// Products are not contracted into FMAs here, so every entry is the same
// correctly-rounded sequence as a plain sequential assembly.
#pragma once

#include "common.hpp"

namespace dpf {

__global__ void ybus_count_kernel(int32_t n_bus, int32_t n_branch, const int32_t *__restrict__ from,
                                  const int32_t *__restrict__ to, const double *__restrict__ r,
                                  const double *__restrict__ x, int32_t *__restrict__ deg,
                                  int32_t *__restrict__ err) {
    int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_branch) return;
    int32_t f = from[e], t = to[e];
    bool bad = f < 0 || f >= n_bus || t < 0 || t >= n_bus || f == t || (r[e] == 0.0 && x[e] == 0.0);
    if (bad) {
        atomicOr(err, 1);
        return;
    }
    atomicAdd(&deg[f], 1);
    atomicAdd(&deg[t], 1);
}

// Exclusive scan of in[i] + add for i < n into out[0..n]; one workgroup of
// 1024 threads, each scanning a contiguous chunk sequentially.
__global__ __launch_bounds__(1024) void scan_kernel(int32_t n, const int32_t *__restrict__ in, int32_t add,
                                                   int32_t *__restrict__ out) {
    __shared__ int32_t part[1024];
    int32_t tid = threadIdx.x;
    int32_t chunk = (n + 1023) / 1024;
    int32_t lo = tid * chunk;
    int32_t hi = min(n, lo + chunk);
    int32_t s = 0;
    for (int32_t i = lo; i < hi; ++i) s += in[i] + add;
    part[tid] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over the 1024 partial sums
    for (int32_t o = 1; o < 1024; o <<= 1) {
        int32_t v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int32_t run = tid > 0 ? part[tid - 1] : 0;
    for (int32_t i = lo; i < hi; ++i) {
        out[i] = run;
        run += in[i] + add;
    }
    if (tid == 1023) out[n] = part[1023];
}

// max over in[0..n) into *out (one workgroup of 1024 threads)
__global__ __launch_bounds__(1024) void imax_kernel(int32_t n, const int32_t *__restrict__ in, int32_t *__restrict__ out) {
    __shared__ int32_t part[1024 / kWave];
    int32_t m = 0;
    for (int32_t i = threadIdx.x; i < n; i += 1024) m = max(m, in[i]);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int k = 0; k < 1024 / kWave; ++k) t = max(t, part[k]);
        *out = t;
    }
}

__global__ void ybus_scatter_kernel(int32_t n_bus, int32_t n_branch, const int32_t *__restrict__ from,
                                    const int32_t *__restrict__ to, const int32_t *__restrict__ soff,
                                    int32_t *__restrict__ fill, int2 *__restrict__ slot) {
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n_bus) slot[soff[k]] = make_int2(k, -1);  // diagonal
    if (k >= n_branch) return;
    int32_t f = from[k], t = to[k];
    int32_t pf = atomicAdd(&fill[f], 1);
    int32_t pt = atomicAdd(&fill[t], 1);
    slot[soff[f] + 1 + pf] = make_int2(t, k);
    slot[soff[t] + 1 + pt] = make_int2(f, k);
}

__device__ __forceinline__ double2 series_admittance_rn(double r, double x) {
    double d = __dadd_rn(__dmul_rn(r, r), __dmul_rn(x, x));
    return make_double2(__ddiv_rn(r, d), __ddiv_rn(-x, d));
}

// Step 4: per row, insertion-sort slots by branch (diagonal first), sum the
// diagonal, then insertion-sort stably by column; count distinct columns.
__global__ void ybus_row_order_kernel(int32_t n_bus, const int32_t *__restrict__ soff, int2 *__restrict__ slot,
                                      const double *__restrict__ r, const double *__restrict__ x,
                                      const double *__restrict__ b, double2 *__restrict__ diag,
                                      int32_t *__restrict__ ucount) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_bus) return;
    int32_t lo = soff[i], hi = soff[i + 1];
    for (int32_t p = lo + 1; p < hi; ++p) {  // by branch id (diagonal slot has -1)
        int2 v = slot[p];
        int32_t q = p - 1;
        while (q >= lo && slot[q].y > v.y) {
            slot[q + 1] = slot[q];
            --q;
        }
        slot[q + 1] = v;
    }
    double2 acc = make_double2(0.0, 0.0);
    for (int32_t p = lo + 1; p < hi; ++p) {
        int32_t e = slot[p].y;
        double2 y = series_admittance_rn(r[e], x[e]);
        double2 yd = make_double2(y.x, __dadd_rn(y.y, __dmul_rn(b[e], 0.5)));
        acc.x = __dadd_rn(acc.x, yd.x);
        acc.y = __dadd_rn(acc.y, yd.y);
    }
    diag[i] = acc;
    for (int32_t p = lo + 1; p < hi; ++p) {  // stable by column
        int2 v = slot[p];
        int32_t q = p - 1;
        while (q >= lo && slot[q].x > v.x) {
            slot[q + 1] = slot[q];
            --q;
        }
        slot[q + 1] = v;
    }
    int32_t u = 0;
    for (int32_t p = lo; p < hi; ++p)
        if (p == lo || slot[p].x != slot[p - 1].x) ++u;
    ucount[i] = u;
}

__global__ void ybus_emit_kernel(int32_t n_bus, const int32_t *__restrict__ soff, const int2 *__restrict__ slot,
                                 const double *__restrict__ r, const double *__restrict__ x,
                                 const double2 *__restrict__ diag, const int32_t *__restrict__ row_ptr,
                                 int32_t nnz_cap, int32_t *__restrict__ col_idx, double2 *__restrict__ val) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_bus) return;
    int32_t lo = soff[i], hi = soff[i + 1];
    int32_t q = row_ptr[i];
    int32_t p = lo;
    while (p < hi) {
        int32_t c = slot[p].x;
        double2 acc = make_double2(0.0, 0.0);
        if (c == i) {
            acc = diag[i];
            while (p < hi && slot[p].x == c) ++p;
        } else {
            while (p < hi && slot[p].x == c) {
                double2 y = series_admittance_rn(r[slot[p].y], x[slot[p].y]);
                acc.x = __dadd_rn(acc.x, -y.x);
                acc.y = __dadd_rn(acc.y, -y.y);
                ++p;
            }
        }
        if (q < nnz_cap) {
            col_idx[q] = c;
            val[q] = acc;
        }
        ++q;
    }
}

}  // namespace dpf
