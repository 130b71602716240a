// Device helpers shared by the libdpf kernels (gfx950, wave64, FP64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpf {

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

// ---------------------------------------------------------------- sin / cos
// sincos for the voltage angles, after fdlibm (Sun Microsystems, 1993): a
// three-step Cody-Waite reduction by pi/2 (valid for |x| < 2^19 pi/2) and the
// fdlibm minimax polynomials on [-pi/4, pi/4] (error < 1 ulp).  It needs far
// fewer registers than a general-purpose routine; arguments outside the
// reduction range (and NaN/Inf) go to the HIP library routine, out of line.
__device__ __noinline__ void sincos_wide(double x, double *s, double *c) { ::sincos(x, s, c); }

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
    if (!(fabs(x) <= 823550.0)) {  // 2^19 * pi/2, also catches NaN and Inf
        sincos_wide(x, &s, &c);
        return;
    }
    const double invpio2 = 6.36619772367581382433e-01;
    const double p1 = 1.57079632673412561417e+00, p2 = 6.07710050630396597660e-11,
                 p2t = 2.02226624879595063154e-21, p3 = 2.02226624871116645580e-21,
                 p3t = 8.47842766036889956997e-32;
    double y0, y1;
    int n = 0;
    if (fabs(x) <= 0.785398163397448279) {
        y0 = x;
        y1 = 0.0;
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
