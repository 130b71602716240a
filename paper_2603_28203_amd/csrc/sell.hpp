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

// width of slice g (rows [r0, hi) of its sub-grid, one per lane): the longest row
// of the slice, clamped to the declared bound max_w (a longer row sets *bad,
// which every solve item then reports); one wave, the result in every lane
__device__ __forceinline__ int32_t slice_width(int32_t r, int32_t hi, const int32_t *__restrict__ rp, int32_t max_w,
                                               int32_t *__restrict__ bad) {
    int len = r < hi ? rp[r + 1] - rp[r] : 0;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) len = max(len, __shfl_xor(len, o, kWave));
    if (len > max_w) {
        if ((threadIdx.x & (kWave - 1)) == 0) atomicOr(bad, 1);
        len = max_w;
    }
    return len;
}

// entries of slice g (w wide, first entry base - lane) for the row r of this lane
// in sub-grid [lo, hi); returns the wave's largest |row - col| of the kept entries
__device__ __forceinline__ int32_t slice_fill(int32_t r, int32_t lo, int32_t hi, int32_t w, int32_t base,
                                              const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                              const double2 *__restrict__ yv, int32_t *__restrict__ col,
                                              double2 *__restrict__ val) {
    int32_t q0 = r < hi ? rp[r] : 0;
    int32_t len = r < hi ? rp[r + 1] - q0 : 0;
    int32_t own = r < hi ? r - lo : 0;
    int32_t far = 0;
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
    return far;
}

// one wave per slice
__global__ __launch_bounds__(kWave) void sell_width_kernel(int32_t n_sub, const int32_t *__restrict__ sub_off,
                                                           int32_t n_bus, const int32_t *__restrict__ slice_off,
                                                           const int32_t *__restrict__ rp, int32_t max_w,
                                                           int32_t *__restrict__ width, int32_t *__restrict__ bad) {
    int32_t g = blockIdx.x;
    int32_t s = find_sub(g, n_sub, slice_off);
    int32_t lo = sub_off ? sub_off[s] : 0;
    int32_t hi = sub_off ? sub_off[s + 1] : n_bus;
    int32_t r = lo + (g - slice_off[s]) * kWave + threadIdx.x;
    const int32_t len = slice_width(r, hi, rp, max_w, bad);
    if (threadIdx.x == 0) width[g] = len;
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
    const int32_t far = slice_fill(r, lo, hi, width[g], start[g] * kWave + threadIdx.x, rp, ci, yv, col, val);
    if (threadIdx.x == 0) atomicMax(&bw[s], far);
}

// The whole build above (counts, the two scans, widths, entries) in one
// workgroup, for calls with at most kSellSmallSubs sub-grids and
// kSellSmallSlices slices: one launch instead of five for small grids, with the
// same layout (the same per-slice code).  Also clears the header words that
// sell_count_kernel clears.
constexpr int kSellSmallThreads = 1024;
constexpr int kSellSmallSubs = kSellSmallThreads;
constexpr int kSellSmallSlices = 64;

__global__ __launch_bounds__(kSellSmallThreads) void sell_small_kernel(
    int32_t n_sub, const int32_t *__restrict__ sub_off, int32_t n_bus, const int32_t *__restrict__ rp,
    const int32_t *__restrict__ ci, const double2 *__restrict__ yv, int32_t max_w, int32_t *__restrict__ nslice,
    int32_t *__restrict__ slice_off, int32_t *__restrict__ width, int32_t *__restrict__ start,
    int32_t *__restrict__ col, double2 *__restrict__ val, int32_t *__restrict__ bw, int32_t *__restrict__ bad,
    int32_t *__restrict__ queue) {
    __shared__ int32_t soff[kSellSmallSubs + 1];
    __shared__ int32_t wsh[kSellSmallSlices];       // widths
    __shared__ int32_t ssh[kSellSmallSlices + 1];   // first entries (units of 64)
    __shared__ int32_t part[kSellSmallThreads / kWave];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wv = tid / kWave;
    constexpr int kWaves = kSellSmallThreads / kWave;
    if (tid == 0) {
        *bad = 0;
        queue[0] = 0;
        queue[1] = 0;
    }
    // slices per sub-grid and their exclusive scan (one sub-grid per thread)
    int32_t ns = 0;
    if (tid < n_sub) {
        const int32_t lo = sub_off ? sub_off[tid] : 0;
        const int32_t hi = sub_off ? sub_off[tid + 1] : n_bus;
        ns = (hi - lo + kWave - 1) / kWave;
        nslice[tid] = ns;
        bw[tid] = 0;
    }
    int32_t incl = ns;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) part[wv] = incl;
    dev_stores_done();  // the cleared flag and bandwidths precede every atomic below
    __syncthreads();
    int32_t before = 0, total = 0;
    for (int k = 0; k < kWaves; ++k) {
        before += k < wv ? part[k] : 0;
        total += part[k];
    }
    if (tid < n_sub) {
        soff[tid] = before + incl - ns;
        slice_off[tid] = before + incl - ns;
    }
    if (tid == 0) {
        soff[n_sub] = total;
        slice_off[n_sub] = total;
    }
    __syncthreads();
    const int32_t n_slices = min(total, kSellSmallSlices);
    auto rows_of = [&](int32_t g, int32_t &s, int32_t &lo, int32_t &hi) {
        int32_t a = 0, b = n_sub - 1;  // largest s with soff[s] <= g
        while (a < b) {
            const int32_t m = (a + b + 1) >> 1;
            if (soff[m] <= g) a = m;
            else b = m - 1;
        }
        s = a;
        lo = sub_off ? sub_off[s] : 0;
        hi = sub_off ? sub_off[s + 1] : n_bus;
        return lo + (g - soff[s]) * kWave + lane;
    };
    // widths (one wave per slice), then their exclusive scan
    for (int32_t g = wv; g < n_slices; g += kWaves) {
        int32_t s, lo, hi;
        const int32_t r = rows_of(g, s, lo, hi);
        const int32_t len = slice_width(r, hi, rp, max_w, bad);
        if (lane == 0) {
            width[g] = len;
            wsh[g] = len;
        }
    }
    __syncthreads();
    if (tid == 0) {
        int32_t run = 0;
        for (int32_t g = 0; g < n_slices; ++g) {
            start[g] = run;
            ssh[g] = run;
            run += wsh[g];
        }
        start[n_slices] = run;
    }
    __syncthreads();
    // entries (one wave per slice)
    for (int32_t g = wv; g < n_slices; g += kWaves) {
        int32_t s, lo, hi;
        const int32_t r = rows_of(g, s, lo, hi);
        const int32_t far = slice_fill(r, lo, hi, wsh[g], ssh[g] * kWave + lane, rp, ci, yv, col, val);
        if (lane == 0) atomicMax(&bw[s], far);
    }
}

}  // namespace dpf
