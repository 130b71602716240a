// Sliced-ELL copy of the admittance matrix for the solve kernels.
//
// A solve workgroup processes the rows of its sub-grid in waves of 64
// consecutive rows (row lo + 64*j + lane).  The matrix is re-laid out so that
// the neighbour entries of those 64 rows are stored column-major:
//     entry k of row (lo + 64 j + lane)  ->  start[g] + 64 k + lane,
// g = slice_off[s] + j.  A wave then loads 64 consecutive column indices and 64
// consecutive complex values per step instead of 64 scattered row segments,
// and every lane of the wave runs the same trip count (the slice width).
// Short rows are padded with (own column, 0): fma(0, x, acc) == acc, so the sums
// are bit-identical to the CSR order.  Entries whose column lies outside the
// sub-grid's bus range are dropped the same way, so the kernels may index the
// LDS exchange vector without a bounds check.
#pragma once

#include "common.hpp"

namespace dpf {

struct SellView {
    const int32_t *slice_off;  // [n_sub + 1] first slice of each sub-grid
    const int32_t *width;      // [n_slices]
    const int32_t *start;      // [n_slices + 1] first entry of each slice, in units of 64 entries
    const int32_t *col;        // [entries] LOCAL column (relative to the sub-grid)
    const double2 *val;        // [entries]
};

// slices per sub-grid: ceil(n_s / 64); clears the per-sub-grid bandwidth
// (thread 0 also clears the bad-grid flag and the two header words at `queue`,
// the second of which counts finished items for the tail handoff)
__global__ void sell_count_kernel(int32_t n_sub, const int32_t *__restrict__ sub_off, int32_t n_bus,
                                  int32_t *__restrict__ nslice, int32_t *__restrict__ bw, int32_t *__restrict__ bad,
                                  int32_t *__restrict__ queue) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0) {
        *bad = 0;
        queue[0] = 0;
        queue[1] = 0;
    }
    if (s >= n_sub) return;
    int32_t lo = sub_off ? sub_off[s] : 0;
    int32_t hi = sub_off ? sub_off[s + 1] : n_bus;
    nslice[s] = (hi - lo + kWave - 1) / kWave;
    bw[s] = 0;
}

__device__ __forceinline__ int32_t find_sub(int32_t g, int32_t n_sub, const int32_t *__restrict__ slice_off) {
    int32_t a = 0, b = n_sub - 1;  // largest s with slice_off[s] <= g
    while (a < b) {
        int32_t m = (a + b + 1) >> 1;
        if (slice_off[m] <= g) a = m;
        else b = m - 1;
    }
    return a;
}

// one wave per slice: width = longest row of the slice, clamped to the declared
// bound max_w (a longer row sets *bad, which every solve item then reports)
__global__ __launch_bounds__(kWave) void sell_width_kernel(int32_t n_sub, const int32_t *__restrict__ sub_off,
                                                           int32_t n_bus, const int32_t *__restrict__ slice_off,
                                                           const int32_t *__restrict__ rp, int32_t max_w,
                                                           int32_t *__restrict__ width, int32_t *__restrict__ bad) {
    int32_t g = blockIdx.x;
    int32_t s = find_sub(g, n_sub, slice_off);
    int32_t lo = sub_off ? sub_off[s] : 0;
    int32_t hi = sub_off ? sub_off[s + 1] : n_bus;
    int32_t r = lo + (g - slice_off[s]) * kWave + threadIdx.x;
    int len = r < hi ? rp[r + 1] - rp[r] : 0;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) len = max(len, __shfl_xor(len, o, kWave));
    if (threadIdx.x == 0) {
        if (len > max_w) {
            atomicOr(bad, 1);
            len = max_w;
        }
        width[g] = len;
    }
}

__global__ __launch_bounds__(kWave) void sell_fill_kernel(int32_t n_sub, const int32_t *__restrict__ sub_off,
                                                          int32_t n_bus, const int32_t *__restrict__ slice_off,
                                                          const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ ci,
                                                          const double2 *__restrict__ yv,
                                                          const int32_t *__restrict__ width,
                                                          const int32_t *__restrict__ start,
                                                          int32_t *__restrict__ col, double2 *__restrict__ val,
                                                          int32_t *__restrict__ bw) {
    int32_t g = blockIdx.x;
    int32_t s = find_sub(g, n_sub, slice_off);
    int32_t lo = sub_off ? sub_off[s] : 0;
    int32_t hi = sub_off ? sub_off[s + 1] : n_bus;
    int32_t r = lo + (g - slice_off[s]) * kWave + threadIdx.x;
    int32_t w = width[g];
    int32_t base = start[g] * kWave + threadIdx.x;
    int32_t q0 = r < hi ? rp[r] : 0;
    int32_t len = r < hi ? rp[r + 1] - q0 : 0;
    int32_t own = r < hi ? r - lo : 0;
    int32_t far = 0;  // largest |row - col| of the kept entries
    for (int32_t k = 0; k < w; ++k) {
        int32_t c = own;
        double2 v = make_double2(0.0, 0.0);
        if (k < len) {
            int32_t j = ci[q0 + k];
            if (j >= lo && j < hi) {
                c = j - lo;
                v = yv[q0 + k];
                far = max(far, abs(c - own));
            }
        }
        col[base + k * kWave] = c;
        val[base + k * kWave] = v;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) far = max(far, __shfl_xor(far, o, kWave));
    if (threadIdx.x == 0) atomicMax(&bw[s], far);
}

}  // namespace dpf
