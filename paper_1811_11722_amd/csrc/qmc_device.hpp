// Device primitives for the gfx950 lattice kernels: exact integer helpers,
// error-free FP64 transformations and double-double reductions.
//
// All device code is compiled with -ffp-contract=off: every fused multiply-add
// below is written explicitly, so the rounding of each step is the one shown.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#else  // compiled at run time by hipRTC (specialised sector kernels)
using __hip_internal::int32_t;
using __hip_internal::int64_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
using __hip_internal::uint8_t;
#endif

namespace qmc {

constexpr int kBlock = 256;  // threads per workgroup (4 wave64)
constexpr int kWave = 64;

// ---------------------------------------------------------------- integers
// (a * b) mod n for a, b < n <= 2^31.  The quotient is estimated in FP64
// (error well below 1 because a*b/n < 2^31) and the remainder is formed in
// wrapping 64-bit arithmetic, then corrected by at most one n either way.
__device__ __forceinline__ uint32_t mulmod(uint32_t a, uint32_t b, uint32_t n, double inv_n) {
    const uint64_t p = (uint64_t)a * (uint64_t)b;
    const double qd = (double)a * (double)b * inv_n;
    const uint64_t q = (uint64_t)__builtin_floor(qd);
    int64_t r = (int64_t)(p - q * (uint64_t)n);
    if (r < 0) r += n;
    if (r >= (int64_t)n) r -= n;
    return (uint32_t)r;
}

// idx <- (idx + step) mod n for idx, step < n <= 2^31, with nms = n - step.
// When idx < nms, idx - nms wraps above 2^31 and the minimum is idx + step;
// otherwise idx + step >= n (no wrap since n <= 2^31) and idx - nms is the
// reduced value.
__device__ __forceinline__ uint32_t walk(uint32_t idx, uint32_t step, uint32_t nms) {
    const uint32_t a = idx + step;
    const uint32_t b = idx - nms;
    return a < b ? a : b;
}

// ------------------------------------------------------------ FP64 helpers
__device__ __forceinline__ double fract(double x) { return __builtin_amdgcn_fract(x); }

__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 1/b: hardware reciprocal estimate refined by two Newton steps.
__device__ __forceinline__ double recip(double b) {
    double r = __builtin_amdgcn_rcp(b);
    double e = fma_(-b, r, 1.0);
    r = fma_(r, e, r);
    e = fma_(-b, r, 1.0);
    return fma_(r, e, r);
}

// a / b via the refined reciprocal and one residual correction.
__device__ __forceinline__ double divide(double a, double b) {
    const double r = recip(b);
    const double q = a * r;
    const double res = fma_(-b, q, a);
    return fma_(res, r, q);
}

// ------------------------------------------------- FP64 exp and log
// gfx950 has no FP64 exponential or logarithm instruction.  These two are
// written for the sector integrand's U^a F^b = exp(a ln U + b ln F): finite
// arguments, no errno or special-case branches.

// exp(x), Cody & Waite argument reduction: k = rint(x / ln 2),
// r = x - k ln2_hi - k ln2_lo with ln2_hi holding 32 significant bits (so
// k * ln2_hi is exact for |k| < 2^21) and |r| <= ln2 / 2; exp(r) by its
// Taylor series to degree 13 (truncation < 5e-18 relative), scaled by 2^k
// with v_ldexp (overflow gives inf, underflow 0).
__device__ __forceinline__ double qexp(double x) {
    constexpr double kLog2e = 1.4426950408889634;
    constexpr double kLn2Hi = 6.93147180369123816490e-01;  // 0x3FE62E42FEE00000
    constexpr double kLn2Lo = 1.90821492927058770002e-10;  // ln 2 - kLn2Hi
    const double k = __builtin_rint(x * kLog2e);
    double r = fma_(-k, kLn2Hi, x);
    r = fma_(-k, kLn2Lo, r);
    // 1/i! for i = 13 .. 1, Horner from the top
    double p = 1.0 / 6227020800.0;  // 1/13!
    p = fma_(p, r, 1.0 / 479001600.0);
    p = fma_(p, r, 1.0 / 39916800.0);
    p = fma_(p, r, 1.0 / 3628800.0);
    p = fma_(p, r, 1.0 / 362880.0);
    p = fma_(p, r, 1.0 / 40320.0);
    p = fma_(p, r, 1.0 / 5040.0);
    p = fma_(p, r, 1.0 / 720.0);
    p = fma_(p, r, 1.0 / 120.0);
    p = fma_(p, r, 1.0 / 24.0);
    p = fma_(p, r, 1.0 / 6.0);
    p = fma_(p, r, 0.5);
    p = fma_(p, r, 1.0);
    p = fma_(p, r, 1.0);
    return __builtin_amdgcn_ldexp(p, (int)k);
}

// ln(x) for x > 0 (NaN for x <= 0 or NaN).  x = m 2^e with m in [1/2, 1);
// with y = m sqrt(2) in [0.707, 1.414), ln x = (e - 1/2) ln 2 + ln y and
// ln y = 2 atanh(s) = 2 sum_k s^(2k+1) / (2k+1), s = (y - 1)/(y + 1),
// |s| <= 0.1716; eleven terms leave a truncation below 1e-18 relative.  The
// absolute error is a few 1e-16, which is what exp(a ln x) needs.
__device__ __forceinline__ double qlog(double x) {
    constexpr double kSqrt2 = 1.4142135623730951;
    constexpr double kLn2Hi = 6.93147180369123816490e-01;
    constexpr double kLn2Lo = 1.90821492927058770002e-10;
    const double m = __builtin_amdgcn_frexp_mant(x);
    const double e = (double)__builtin_amdgcn_frexp_exp(x) - 0.5;
    const double y = m * kSqrt2;
    const double s = (y - 1.0) * recip(y + 1.0);
    const double s2 = s * s;
    double p = 1.0 / 21.0;
    p = fma_(p, s2, 1.0 / 19.0);
    p = fma_(p, s2, 1.0 / 17.0);
    p = fma_(p, s2, 1.0 / 15.0);
    p = fma_(p, s2, 1.0 / 13.0);
    p = fma_(p, s2, 1.0 / 11.0);
    p = fma_(p, s2, 1.0 / 9.0);
    p = fma_(p, s2, 1.0 / 7.0);
    p = fma_(p, s2, 1.0 / 5.0);
    p = fma_(p, s2, 1.0 / 3.0);
    const double ly = 2.0 * s * fma_(p, s2, 1.0);
    const double r = fma_(e, kLn2Hi, fma_(e, kLn2Lo, ly));
    return x > 0.0 ? r : __builtin_nan("");
}

// ------------------------------------------------- FP64 atan2 and sincos
// For the complex sector integrand (F - i delta)^p = |.|^p e^{i p arg}: the
// phase needs arg(F - i delta) = atan2(-delta, F) and the sine and cosine of
// p times it, a bounded argument.  Both are branch-free; their polynomials
// are Chebyshev fits (near-minimax) made for this library with multiprecision
// arithmetic, each below 3e-17 in its reduced range.

// atan2(y, x) for finite (x, y) not both zero.  With n = min(|x|, |y|) and
// d = max(|x|, |y|), t = n / d lies in [0, 1]; above tan(pi/8) it is replaced
// by (n - d) / (n + d) = tan(atan(t) - pi/4), so one division leaves
// |t| <= tan(pi/8), where atan(t) = t + t^3 P(t^2) with P of degree 10.  The
// octant and quadrant are restored with pi/4, pi/2 - a, pi - a and the sign
// of y.
__device__ __forceinline__ double qatan2(double y, double x) {
    constexpr double kTanPi8 = 0x1.a827999fcef32p-2;
    constexpr double kPi4 = 0x1.921fb54442d18p-1, kPi2 = 0x1.921fb54442d18p+0, kPi = 0x1.921fb54442d18p+1;
    const double ax = __builtin_fabs(x), ay = __builtin_fabs(y);
    const double n = __builtin_fmin(ax, ay), d = __builtin_fmax(ax, ay);
    const bool big = n > kTanPi8 * d;
    const double t = divide(big ? n - d : n, big ? n + d : d);
    const double s = t * t;
    double p = -0x1.3a31b1c0fd3b7p-6;
    p = fma_(p, s, 0x1.4162c02b1dda3p-5);
    p = fma_(p, s, -0x1.a0999c632b6edp-5);
    p = fma_(p, s, 0x1.dfe6497e96323p-5);
    p = fma_(p, s, -0x1.10fa77b1a6d57p-4);
    p = fma_(p, s, 0x1.3b1263064f6b9p-4);
    p = fma_(p, s, -0x1.745d0b28a7e37p-4);
    p = fma_(p, s, 0x1.c71c71853d7fap-4);
    p = fma_(p, s, -0x1.2492492436201p-3);
    p = fma_(p, s, 0x1.999999999934cp-3);
    p = fma_(p, s, -0x1.5555555555555p-2);
    double a = fma_(t * s, p, t);
    a = big ? a + kPi4 : a;
    a = ay > ax ? kPi2 - a : a;
    a = x < 0.0 ? kPi - a : a;
    return __builtin_copysign(a, y);
}

// sin and cos of x for |x| < 2^19 (the phase is |p| times an angle in
// [-pi, pi]).  x = k pi/2 + r with k = rint(2x/pi) and pi/2 in three parts
// (the first two with 33 significant bits, so k times them is exact for
// |k| < 2^20), |r| <= pi/4; sin r = r + r^3 S(r^2), cos r = 1 - r^2/2 +
// r^4 C(r^2) with S, C of degree 5; the quadrant k mod 4 swaps and negates.
__device__ __forceinline__ void qsincos(double x, double &sn, double &cs) {
    constexpr double k2Pi = 0x1.45f306dc9c883p-1;
    const double k = __builtin_rint(x * k2Pi);
    double r = fma_(-k, 0x1.921fb54400000p+0, x);
    r = fma_(-k, 0x1.0b4611a600000p-34, r);
    r = fma_(-k, 0x1.3198a2e037073p-69, r);
    const double r2 = r * r;
    double ps = 0x1.5e0b19f8b1451p-33;
    ps = fma_(ps, r2, -0x1.ae600b02b6262p-26);
    ps = fma_(ps, r2, 0x1.71de37968a100p-19);
    ps = fma_(ps, r2, -0x1.a01a019e83aaep-13);
    ps = fma_(ps, r2, 0x1.1111111110bb2p-7);
    ps = fma_(ps, r2, -0x1.5555555555555p-3);
    double pc = -0x1.907da367a37cbp-37;
    pc = fma_(pc, r2, 0x1.1eeb68e93b64cp-29);
    pc = fma_(pc, r2, -0x1.27e4fa17da09ep-22);
    pc = fma_(pc, r2, 0x1.a01a019f4eb01p-16);
    pc = fma_(pc, r2, -0x1.6c16c16c16967p-10);
    pc = fma_(pc, r2, 0x1.5555555555555p-5);
    const double sr = fma_(r * r2, ps, r);
    const double cr = fma_(r2 * r2, pc, fma_(-0.5, r2, 1.0));
    const int q = (int)k;
    const double ss = (q & 1) ? cr : sr, cc = (q & 1) ? sr : cr;
    sn = (q & 2) ? -ss : ss;
    cs = ((q + 1) & 2) ? -cc : cc;
}

// Knuth's TwoSum: s + e == a + b exactly.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    const double bp = s - a;
    e = (a - (s - bp)) + (b - bp);
}

// Dekker's Fast2Sum, valid for |a| >= |b| (or a == 0).
__device__ __forceinline__ void fast_two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    e = b - (s - a);
}

struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd dd_add(dd a, dd b) {
    double s, e;
    two_sum(a.hi, b.hi, s, e);
    e = e + (a.lo + b.lo);
    dd r;
    fast_two_sum(s, e, r.hi, r.lo);
    return r;
}

// add a plain double into a double-double accumulator
__device__ __forceinline__ void dd_accumulate(double &hi, double &lo, double v) {
    double s, e;
    two_sum(hi, v, s, e);
    hi = s;
    lo = lo + e;
}

// Butterfly reduction of a double-double across the 64 lanes of a wave.
// Every lane ends with the same total; the order of additions is fixed.
__device__ __forceinline__ dd wave_reduce(dd v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        dd o;
        o.hi = __shfl_xor(v.hi, off, kWave);
        o.lo = __shfl_xor(v.lo, off, kWave);
        v = dd_add(v, o);
    }
    return v;
}

// Uniform (wave-invariant) value as seen by the scalar unit.
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

template <class P>
__device__ __forceinline__ const P *uniform_ptr(const P *p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    // the builtin returns a signed int: widen through uint32_t so the low half
    // is not sign-extended into the high half
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<const P *>(lo | (hi << 32));
}

}  // namespace qmc
