// Device primitives for the gfx950 lattice kernels: exact integer helpers,
// error-free FP64 transformations and double-double reductions.
//
// All device code is compiled with -ffp-contract=off: every fused multiply-add
// below is written explicitly, so the rounding of each step is the one shown.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

}  // namespace qmc
