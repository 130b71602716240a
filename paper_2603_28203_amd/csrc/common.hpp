// Device helpers shared by the libdpf kernels (gfx950, wave64, FP64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace dpf {

// status of an item handed over from a per-item solve kernel to the multi-workgroup
// path (internal: that path finishes the item and overwrites the status).  It lies
// outside the public per-case status codes of include/dpf.h (0..4), which the
// paths compare against it (checked at compile time in dpf.hip).
constexpr int kPaused = 256;

constexpr int kWave = 64;
constexpr int8_t kPQ = 0;
constexpr int8_t kPV = 1;
constexpr int8_t kSlack = 2;

// Complex numbers are double2 {re, im}; these are the few operations the
// power-flow kernels need, written out so the compiler can fuse them into FMAs.
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
// acc + a * b
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}

// acc + the products of one sliced-ELL row (entries base + q*kWave, q < w, w the
// same in every lane of the wave) with the exchange vector get(col), added in
// entry order as a plain loop adds them.  Entries go in groups of U whose loads
// are issued together, the last, partial group predicated instead of being left
// to a remainder loop: a row of up to U entries waits for the cache once and a
// longer one once per U entries (a loop unrolled by U with a remainder loop waits
// once per remainder entry).  Two forms, each the faster one where it is used:
//  - JOINT (kernels with few waves per CU and registers to spare): full groups
//    run unpredicated, and the gathers of a group are issued together (a missing
//    entry of the last group gathers the lane's own row `own`, always a valid
//    column, and adds nothing);
//  - otherwise (1024-thread kernels, where other waves hide the gathers and
//    registers are short): every group predicated, each gather in its own step.
template <int U, bool JOINT, typename Get>
__device__ __forceinline__ double2 sell_row(const double2 *__restrict__ val, const int32_t *__restrict__ col,
                                            int base, int w, int own, Get get, double2 acc) {
    auto group = [&](int q0, auto full) {
        constexpr bool FULL = decltype(full)::value;
        double2 v[U];
        int32_t cc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            v[u] = make_double2(0.0, 0.0);
            cc[u] = own;
            if (FULL || q0 + u < w) {
                v[u] = val[base + (q0 + u) * kWave];
                cc[u] = col[base + (q0 + u) * kWave];
            }
        }
        if constexpr (JOINT) {
            double2 x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) x[u] = get(cc[u]);
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (FULL || q0 + u < w) acc = cfma(v[u], x[u], acc);
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (FULL || q0 + u < w) acc = cfma(v[u], get(cc[u]), acc);
        }
    };
    int q0 = 0;
    if constexpr (JOINT)
        for (; q0 + U <= w; q0 += U) group(q0, std::true_type{});
    for (; q0 < w; q0 += U) group(q0, std::false_type{});
    return acc;
}

// Butterfly sum / max across the 64 lanes of a wave; every lane receives the
// result and the combination order is fixed, so results are reproducible.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}
// A value that every lane of the wave holds identically, moved to scalar
// registers: lets the compiler treat what depends on it as uniform.
__device__ __forceinline__ double uniform(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(unsigned)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// Device-scope (relaxed agent-scope atomic) store and load of a double: the store
// writes through to the device's coherence point and the load does not hit a
// possibly stale L1/L2 copy, so values handed between workgroups of one kernel
// on different XCDs need no cache-wide write-back or invalidation.  A thread
// makes its device-scope stores visible before signalling with
// dev_stores_done() followed by a device-scope atomic.
__device__ __forceinline__ void st_dev(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const double *p) {
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev2(double2 *p, double2 v) {
    st_dev(&p->x, v.x);
    st_dev(&p->y, v.y);
}
__device__ __forceinline__ double2 ld_dev2(const double2 *p) { return make_double2(ld_dev(&p->x), ld_dev(&p->y)); }
// The same device-scope access for 16 bytes in one instruction: a buffer
// load/store with the SC1 cache policy (the policy of the relaxed agent-scope
// loads and stores above) through a resource built from `base` and `bytes`,
// which MUST be the same in every lane of the wave (they are taken from the
// first active lane, so that the resource lives in scalar registers); DEV =
// false is an ordinary cached access.  The resource's range check makes an
// index at or past `bytes` read zero and drop a store.
constexpr int kCachePolicySC1 = 16;
constexpr int kBufferWord3 = 0x00020000;  // 32-bit data format, gfx9 family
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void *base, uint32_t bytes) {
    const unsigned long long b = (unsigned long long)base;
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b & 0xffffffffULL));
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    void *ub = (void *)(((unsigned long long)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(ub, 0, __builtin_amdgcn_readfirstlane((int)bytes), kBufferWord3);
}
// element idx (16 bytes each) through a resource made once (buffer_of) and kept in
// scalar registers; a loop around these stays free of lane-uniformity operations
template <bool DEV>
__device__ __forceinline__ double2 rsrc_ld2(__amdgpu_buffer_rsrc_t r, int idx) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)((uint32_t)idx * 16u), 0, DEV ? kCachePolicySC1 : 0);
    double2 out;
    __builtin_memcpy(&out, &v, sizeof(out));
    return out;
}
template <bool DEV>
__device__ __forceinline__ void rsrc_st2(__amdgpu_buffer_rsrc_t r, int idx, double2 x) {
    decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0)) v;
    __builtin_memcpy(&v, &x, sizeof(x));
    __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)((uint32_t)idx * 16u), 0, DEV ? kCachePolicySC1 : 0);
}
// this thread's stores have completed (and the compiler keeps every earlier
// memory access before this point)
__device__ __forceinline__ void dev_stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ int wave_isum(int v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Branch pi-model admittances of one branch: series y = 1/(r + jx) and the
// half charging j b/2.  Used by the N-1 rank-2 correction.
__device__ __forceinline__ void branch_admittance(double r, double x, double b, double2 &y, double2 &ysh) {
    double d = r * r + x * x;
    y = make_double2(r / d, -x / d);
    ysh = make_double2(0.0, 0.5 * b);
}

// ---------------------------------------------------------------- optimizer
// One optimizer update of a learnable coordinate x with gradient g and state
// m (first moment / momentum buffer), s (second moment); kind = DPF_OPT_*
// (0 Adam with bias corrections bc1 = 1 - b1^t, bc2 = 1 - b2^t; 1 SGD with
// momentum b1; 2 RMSprop with smoothing b2).
__device__ __forceinline__ double opt_update(int kind, double lr, double b1, double b2, double eps, double bc1,
                                             double bc2, double x, double g, double &m, double &s) {
    if (kind == 1) {
        m = b1 * m + g;
        return x - lr * m;
    }
    if (kind == 2) {
        s = b2 * s + (1.0 - b2) * (g * g);
        return x - lr * (g / (sqrt(s) + eps));
    }
    m = b1 * m + (1.0 - b1) * g;
    s = b2 * s + (1.0 - b2) * (g * g);
    return x - lr * (m / bc1) / (sqrt(s / bc2) + eps);
}

// ---------------------------------------------------------------- sin / cos
// The polynomial kernels and the Cody-Waite constants below follow fdlibm, whose
// notice is kept as its licence asks:
//   ====================================================
//   Copyright (C) 1993 by Sun Microsystems, Inc. All rights reserved.
//
//   Developed at SunPro, a Sun Microsystems, Inc. business.
//   Permission to use, copy, modify, and distribute this
//   software is freely granted, provided that this notice
//   is preserved.
//   ====================================================
//
// sincos for the voltage angles, after fdlibm (Sun Microsystems, 1993): a
// three-step Cody-Waite reduction by pi/2 (valid for |x| < 2^19 pi/2) and the
// fdlibm minimax polynomials on [-pi/4, pi/4] (error < 1 ulp).  Larger finite
// arguments are reduced exactly by the Payne-Hanek method (multiplication by a
// 192-bit window of the binary expansion of 2/pi), inline and without a call,
// so that the solve kernels keep their registers.

// 2/pi = 0.A2F9836E... in hexadecimal: 1280 bits, most significant first
// (computed with integer arithmetic from Machin's formula; checked by a test).
__constant__ const unsigned long long kTwoOverPiBits[20] = {
    0xA2F9836E4E441529ULL, 0xFC2757D1F534DDC0ULL, 0xDB6295993C439041ULL, 0xFE5163ABDEBBC561ULL,
    0xB7246E3A424DD2E0ULL, 0x06492EEA09D1921CULL, 0xFE1DEB1CB129A73EULL, 0xE88235F52EBB4484ULL,
    0xE99C7026B45F7E41ULL, 0x3991D639835339F4ULL, 0x9C845F8BBDF9283BULL, 0x1FF897FFDE05980FULL,
    0xEF2F118B5A0A6D1FULL, 0x6D367ECF27CB09B7ULL, 0x4F463F669E5FEA2DULL, 0x7527BAC7EBE5F17BULL,
    0x3D0739F78A5292EAULL, 0x6BFB5FB11F8D5D08ULL, 0x56033046FC7B6BABULL, 0xF0CFBC209AF4361DULL,
};

// 64 bits of 2/pi starting at bit z (bit 0 = weight 1/2)
__device__ __forceinline__ unsigned long long two_over_pi_bits(int z) {
    const int q = z >> 6, off = z & 63;
    const unsigned long long hi = kTwoOverPiBits[q];
    return off ? (hi << off) | (kTwoOverPiBits[q + 1] >> (64 - off)) : hi;
}

// bits [pos, pos + 64) of the 256-bit number p3:p2:p1:p0
__device__ __forceinline__ unsigned long long bits_at(unsigned long long p0, unsigned long long p1,
                                                      unsigned long long p2, unsigned long long p3, int pos) {
    const int q = pos >> 6, off = pos & 63;
    const unsigned long long w0 = q == 0 ? p0 : q == 1 ? p1 : q == 2 ? p2 : p3;
    const unsigned long long w1 = q == 0 ? p1 : q == 1 ? p2 : q == 2 ? p3 : 0ULL;
    return off ? (w0 >> off) | (w1 << (64 - off)) : w0;
}

// Payne-Hanek reduction of a finite x with |x| >= 2^19 pi/2: x = n pi/2 + (y0 + y1),
// |y0 + y1| <= pi/4, returns n mod 4.  |x| = m 2^E (m a 53-bit integer, E >= -33);
// bits of 2/pi of weight 2^-k with k <= E - 2 contribute multiples of 4 to
// x * 2/pi and are skipped, the next 192 bits give the quadrant and a fraction
// accurate to ~2^-137, far below the closest approach of a double to a multiple
// of pi/2.
__device__ __forceinline__ int reduce_payne_hanek(double x, double &y0, double &y1) {
    const unsigned long long bits = (unsigned long long)__double_as_longlong(x);
    const int E = (int)((bits >> 52) & 0x7ff) - 1075;
    const unsigned long long m = (bits & 0xFFFFFFFFFFFFFULL) | (1ULL << 52);
    const int k0 = E - 1 > 1 ? E - 1 : 1;  // first bit (1-based) of the window
    const unsigned long long W2 = two_over_pi_bits(k0 - 1), W1 = two_over_pi_bits(k0 + 63),
                             W0 = two_over_pi_bits(k0 + 127);
    // P = m * (W2:W1:W0), 245 bits; x 2/pi = P 2^(E - k0 - 191) (mod 4)
    const unsigned long long l0 = m * W0, h0 = __umul64hi(m, W0);
    const unsigned long long l1 = m * W1, h1 = __umul64hi(m, W1);
    const unsigned long long l2 = m * W2, h2 = __umul64hi(m, W2);
    const unsigned long long p0 = l0;
    const unsigned long long p1 = h0 + l1;
    const unsigned long long c1 = p1 < l1 ? 1ULL : 0ULL;
    const unsigned long long t2 = h1 + c1;  // h1 < 2^53: no carry out
    const unsigned long long p2 = t2 + l2;
    const unsigned long long p3 = h2 + (p2 < l2 ? 1ULL : 0ULL);
    const int sh = k0 + 191 - E;  // binary point of P, in [190, 225]
    int n = (int)(bits_at(p0, p1, p2, p3, sh) & 3ULL);
    unsigned long long fh = bits_at(p0, p1, p2, p3, sh - 64);   // fraction, top 64 bits
    const unsigned long long fl = bits_at(p0, p1, p2, p3, sh - 128);
    // centre the fraction on [-1/2, 1/2): a set top bit means fraction - 1 in two's complement
    if (fh >> 63) n += 1;
    // fraction as a double pair: the top word with its low 11 bits cleared is exact
    const long long fhs = (long long)fh;
    const double a = (double)(fhs & ~0x7FFLL) * 0x1p-64;
    const unsigned long long low = ((fh & 0x7FFULL) << 53) | (fl >> 11);
    const double b = (double)low * 0x1p-117;
    const double f = a + b, fe = b - (f - a);
    // times pi/2 in double-double
    const double pio2_hi = 1.57079632679489655800e+00, pio2_lo = 6.12323399573676603587e-17;
    const double rh = f * pio2_hi;
    const double rl = fma(f, pio2_hi, -rh) + (fe * pio2_hi + f * pio2_lo);
    double r0 = rh + rl;
    double r1 = rl - (r0 - rh);
    if (x < 0.0) {
        r0 = -r0;
        r1 = -r1;
        n = -n;
    }
    y0 = r0;
    y1 = r1;
    return n;
}

__device__ __forceinline__ double ksin(double x, double y) {
    const double S1 = -1.66666666666666324348e-01, S2 = 8.33333333332248946124e-03,
                 S3 = -1.98412698298579493134e-04, S4 = 2.75573137070700676789e-06,
                 S5 = -2.50507602534068634195e-08, S6 = 1.58969099521155010221e-10;
    double z = x * x, v = z * x;
    double r = S2 + z * (S3 + z * (S4 + z * (S5 + z * S6)));
    return x - ((z * (0.5 * y - v * r) - y) - v * S1);
}

__device__ __forceinline__ double kcos(double x, double y) {
    const double C1 = 4.16666666666666019037e-02, C2 = -1.38888888888741095749e-03,
                 C3 = 2.48015872894767294178e-05, C4 = -2.75573143513906633035e-07,
                 C5 = 2.08757232129817482790e-09, C6 = -1.13596475577881948265e-11;
    double z = x * x;
    double r = z * (C1 + z * (C2 + z * (C3 + z * (C4 + z * (C5 + z * C6)))));
    double ax = fabs(x);
    if (ax < 0.3) return 1.0 - (0.5 * z - (z * r - x * y));
    // qx = |x|/4 with the low mantissa word cleared (0.28125 above 0.78125),
    // so that 1 - qx is exact
    double qx = ax > 0.78125 ? 0.28125 : __hiloint2double(__double2hiint(ax) - 0x00200000, 0);
    double hz = 0.5 * z - qx, a = 1.0 - qx;
    return a - (hz - (z * r - x * y));
}

__device__ __forceinline__ void fast_sincos(double x, double &s, double &c) {
    const double invpio2 = 6.36619772367581382433e-01;
    const double p1 = 1.57079632673412561417e+00, p2 = 6.07710050630396597660e-11,
                 p2t = 2.02226624879595063154e-21, p3 = 2.02226624871116645580e-21,
                 p3t = 8.47842766036889956997e-32;
    double y0, y1;
    int n = 0;
    if (fabs(x) <= 0.785398163397448279) {
        y0 = x;
        y1 = 0.0;
    } else if (!(fabs(x) <= 823550.0)) {  // 2^19 pi/2, also catches NaN and Inf
        if (fabs(x) <= 1.79769313486231570815e+308) {
            n = reduce_payne_hanek(x, y0, y1);
        } else {
            s = c = x - x;  // NaN for NaN and +-Inf
            return;
        }
    } else {
        double fn = rint(x * invpio2);
        n = (int)fn;
        double r = x - fn * p1;  // exact: p1 has 33 significant bits, |fn| < 2^20
        // second and third steps (fdlibm's cancellation refinements), always taken
        double t = r;
        double w;
        w = fn * p2;
        r = t - w;
        w = fn * p2t - ((t - r) - w);
        y0 = r - w;
        t = r;
        w = fn * p3;
        r = t - w;
        w = fn * p3t - ((t - r) - w);
        y0 = r - w;
        y1 = (r - y0) - w;
    }
    double sn = ksin(y0, y1), cs = kcos(y0, y1);
    switch (n & 3) {
        case 0: s = sn; c = cs; break;
        case 1: s = cs; c = -sn; break;
        case 2: s = -sn; c = -cs; break;
        default: s = -cs; c = sn; break;
    }
}

}  // namespace dpf
