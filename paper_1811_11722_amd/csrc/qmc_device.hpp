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

// ln(x) for x > 0 (NaN for x <= 0, NaN or +inf).  x = m 2^e with m in
// [1/2, 1); the table splits [1/2, 1) into 256 intervals [c_j, c_j + 1/512)
// and holds ic_j = 1/c_j rounded and -ln(ic_j); with r = m ic_j - 1 (one
// FMA, |r| <= 1/256), ln x = e ln 2 - ln(ic_j) + ln(1 + r), and ln(1 + r)
// is its series to r^7 (truncation below 3e-20).  The absolute error is a
// few 1e-17 plus one rounding of the result, which is what exp(a ln x)
// needs; the table read is one 16-byte load from a 4 KB constant array that
// stays in the L1 cache.
struct QlogEntry {
    double ic, nl;
};
static __constant__ const QlogEntry kQlogTab[256] = {
    {0x1.0000000000000p+1, -0x1.62e42fefa39efp-1},
    {0x1.fe01fe01fe020p+0, -0x1.60e52f45788e4p-1},
    {0x1.fc07f01fc07f0p+0, -0x1.5ee82aa241920p-1},
    {0x1.fa11caa01fa12p+0, -0x1.5ced1e17c35c6p-1},
    {0x1.f81f81f81f820p+0, -0x1.5af405c3649e0p-1},
    {0x1.f6310aca0dbb5p+0, -0x1.58fcddce004c3p-1},
    {0x1.f44659e4a4271p+0, -0x1.5707a26bb8c66p-1},
    {0x1.f25f644230ab5p+0, -0x1.55144fdbcbd62p-1},
    {0x1.f07c1f07c1f08p+0, -0x1.5322e26867857p-1},
    {0x1.ee9c7f8458e02p+0, -0x1.513356667fc57p-1},
    {0x1.ecc07b301ecc0p+0, -0x1.4f45a835a4e19p-1},
    {0x1.eae807aba01ebp+0, -0x1.4d59d43fdaba2p-1},
    {0x1.e9131abf0b767p+0, -0x1.4b6fd6f970c1fp-1},
    {0x1.e741aa59750e4p+0, -0x1.4987ace0dabb0p-1},
    {0x1.e573ac901e574p+0, -0x1.47a1527e8a2d4p-1},
    {0x1.e3a9179dc1a73p+0, -0x1.45bcc464c893ap-1},
    {0x1.e1e1e1e1e1e1ep+0, -0x1.43d9ff2f923c5p-1},
    {0x1.e01e01e01e01ep+0, -0x1.41f8ff8471d61p-1},
    {0x1.de5d6e3f8868ap+0, -0x1.4019c2125ca93p-1},
    {0x1.dca01dca01dcap+0, -0x1.3e3c43918f76cp-1},
    {0x1.dae6076b981dbp+0, -0x1.3c6080c36bfb5p-1},
    {0x1.d92f2231e7f8ap+0, -0x1.3a86767257112p-1},
    {0x1.d77b654b82c34p+0, -0x1.38ae2171976e8p-1},
    {0x1.d5cac807572b2p+0, -0x1.36d77e9d34fd7p-1},
    {0x1.d41d41d41d41dp+0, -0x1.35028ad9d8c85p-1},
    {0x1.d272ca3fc5b1ap+0, -0x1.332f4314ad795p-1},
    {0x1.d0cb58f6ec074p+0, -0x1.315da4434068bp-1},
    {0x1.cf26e5c44bfc6p+0, -0x1.2f8dab6363379p-1},
    {0x1.cd85689039b0bp+0, -0x1.2dbf557b0df43p-1},
    {0x1.cbe6d9601cbe7p+0, -0x1.2bf29f9841c3bp-1},
    {0x1.ca4b3055ee191p+0, -0x1.2a2786d0ec107p-1},
    {0x1.c8b265afb8a42p+0, -0x1.285e0842ca384p-1},
    {0x1.c71c71c71c71cp+0, -0x1.269621134db92p-1},
    {0x1.c5894d10d4986p+0, -0x1.24cfce6f80d9bp-1},
    {0x1.c3f8f01c3f8f0p+0, -0x1.230b0d8bebc98p-1},
    {0x1.c26b5392ea01cp+0, -0x1.2147dba47a393p-1},
    {0x1.c0e070381c0e0p+0, -0x1.1f8635fc61658p-1},
    {0x1.bf583ee868d8bp+0, -0x1.1dc619de06944p-1},
    {0x1.bdd2b899406f7p+0, -0x1.1c07849ae6007p-1},
    {0x1.bc4fd65883e7bp+0, -0x1.1a4a738b7a33cp-1},
    {0x1.bacf914c1bad0p+0, -0x1.188ee40f23ca7p-1},
    {0x1.b951e2b18ff23p+0, -0x1.16d4d38c119fap-1},
    {0x1.b7d6c3dda338bp+0, -0x1.151c3f6f29612p-1},
    {0x1.b65e2e3beee05p+0, -0x1.1365252bf0865p-1},
    {0x1.b4e81b4e81b4fp+0, -0x1.11af823c75aa8p-1},
    {0x1.b37484ad806cep+0, -0x1.0ffb54213a476p-1},
    {0x1.b2036406c80d9p+0, -0x1.0e4898611cce1p-1},
    {0x1.b094b31d922a4p+0, -0x1.0c974c89431cep-1},
    {0x1.af286bca1af28p+0, -0x1.0ae76e2d054fap-1},
    {0x1.adbe87f94905ep+0, -0x1.0938fae5d8e9bp-1},
    {0x1.ac5701ac5701bp+0, -0x1.078bf0533c568p-1},
    {0x1.aaf1d2f87ebfdp+0, -0x1.05e04c1aa2c06p-1},
    {0x1.a98ef606a63bep+0, -0x1.04360be7603aep-1},
    {0x1.a82e65130e159p+0, -0x1.028d2d6a963f5p-1},
    {0x1.a6d01a6d01a6dp+0, -0x1.00e5ae5b207abp-1},
    {0x1.a574107688a4ap+0, -0x1.fe7f18eb03d3ep-2},
    {0x1.a41a41a41a41ap+0, -0x1.fb358af7a4884p-2},
    {0x1.a2c2a87c51ca0p+0, -0x1.f7eeae6b5761cp-2},
    {0x1.a16d3f97a4b02p+0, -0x1.f4aa7ee03192ep-2},
    {0x1.a01a01a01a01ap+0, -0x1.f168f7fb05c52p-2},
    {0x1.9ec8e951033d9p+0, -0x1.ee2a156b413e5p-2},
    {0x1.9d79f176b682dp+0, -0x1.eaedd2eac990cp-2},
    {0x1.9c2d14ee4a102p+0, -0x1.e7b42c3ddad74p-2},
    {0x1.9ae24ea5510dap+0, -0x1.e47d1d32e677dp-2},
    {0x1.999999999999ap+0, -0x1.e148a1a2726cfp-2},
    {0x1.9852f0d8ec0ffp+0, -0x1.de16b56ef90f0p-2},
    {0x1.970e4f80cb872p+0, -0x1.dae75484c9615p-2},
    {0x1.95cbb0be377aep+0, -0x1.d7ba7ad9e7da1p-2},
    {0x1.948b0fcd6e9e0p+0, -0x1.d490246defa6ap-2},
    {0x1.934c67f9b2ce6p+0, -0x1.d1684d49f46aep-2},
    {0x1.920fb49d0e229p+0, -0x1.ce42f18064744p-2},
    {0x1.90d4f120190d5p+0, -0x1.cb200d2ceb643p-2},
    {0x1.8f9c18f9c18fap+0, -0x1.c7ff9c74554cap-2},
    {0x1.8e6527af1373fp+0, -0x1.c4e19b84723c2p-2},
    {0x1.8d3018d3018d3p+0, -0x1.c1c60693fa39ep-2},
    {0x1.8bfce8062ff3ap+0, -0x1.beacd9e271ad1p-2},
    {0x1.8acb90f6bf3aap+0, -0x1.bb9611b80e2fcp-2},
    {0x1.899c0f601899cp+0, -0x1.b881aa659bc93p-2},
    {0x1.886e5f0abb04ap+0, -0x1.b56fa0446290ap-2},
    {0x1.87427bcc092b9p+0, -0x1.b25fefb60cb2ep-2},
    {0x1.8618618618618p+0, -0x1.af5295248cdcfp-2},
    {0x1.84f00c2780614p+0, -0x1.ac478d0205070p-2},
    {0x1.83c977ab2beddp+0, -0x1.a93ed3c8ad9e3p-2},
    {0x1.82a4a0182a4a0p+0, -0x1.a63865fabd0ecp-2},
    {0x1.8181818181818p+0, -0x1.a33440224fa79p-2},
    {0x1.8060180601806p+0, -0x1.a0325ed14fda4p-2},
    {0x1.7f405fd017f40p+0, -0x1.9d32bea15ed3ap-2},
    {0x1.7e225515a4f1dp+0, -0x1.9a355c33bd6bap-2},
    {0x1.7d05f417d05f4p+0, -0x1.973a3431356aep-2},
    {0x1.7beb3922e017cp+0, -0x1.9441434a0325ap-2},
    {0x1.7ad2208e0ecc3p+0, -0x1.914a8635bf689p-2},
    {0x1.79baa6bb6398bp+0, -0x1.8e55f9b349b82p-2},
    {0x1.78a4c8178a4c8p+0, -0x1.8b639a88b2df4p-2},
    {0x1.77908119ac60dp+0, -0x1.8873658327ccep-2},
    {0x1.767dce434a9b1p+0, -0x1.85855776dcbfbp-2},
    {0x1.756cac201756dp+0, -0x1.82996d3ef8bccp-2},
    {0x1.745d1745d1746p+0, -0x1.7fafa3bd8151cp-2},
    {0x1.734f0c541fe8dp+0, -0x1.7cc7f7db46a0ep-2},
    {0x1.724287f46debcp+0, -0x1.79e26687cfb3dp-2},
    {0x1.713786d9c7c09p+0, -0x1.76feecb947176p-2},
    {0x1.702e05c0b8170p+0, -0x1.741d876c67bb1p-2},
    {0x1.6f26016f26017p+0, -0x1.713e33a46a17cp-2},
    {0x1.6e1f76b4337c7p+0, -0x1.6e60ee6af1973p-2},
    {0x1.6d1a62681c861p+0, -0x1.6b85b4cffa3fdp-2},
    {0x1.6c16c16c16c17p+0, -0x1.68ac83e9c6a15p-2},
    {0x1.6b1490aa31a3dp+0, -0x1.65d558d4ce00bp-2},
    {0x1.6a13cd1537290p+0, -0x1.630030b3aac48p-2},
    {0x1.691473a88d0c0p+0, -0x1.602d08af091ecp-2},
    {0x1.6816816816817p+0, -0x1.5d5bddf595f31p-2},
    {0x1.6719f3601671ap+0, -0x1.5a8cadbbedfa1p-2},
    {0x1.661ec6a5122f9p+0, -0x1.57bf753c8d1fbp-2},
    {0x1.6524f853b4aa3p+0, -0x1.54f431b7be1a8p-2},
    {0x1.642c8590b2164p+0, -0x1.522ae0738a3d7p-2},
    {0x1.63356b88ac0dep+0, -0x1.4f637ebba9810p-2},
    {0x1.623fa77016240p+0, -0x1.4c9e09e172c3dp-2},
    {0x1.614b36831ae94p+0, -0x1.49da7f3bcc420p-2},
    {0x1.6058160581606p+0, -0x1.4718dc271c41cp-2},
    {0x1.5f66434292dfcp+0, -0x1.44591e0539f49p-2},
    {0x1.5e75bb8d015e7p+0, -0x1.419b423d5e8c6p-2},
    {0x1.5d867c3ece2a5p+0, -0x1.3edf463c1683ep-2},
    {0x1.5c9882b931057p+0, -0x1.3c25277333183p-2},
    {0x1.5babcc647fa91p+0, -0x1.396ce359bbf53p-2},
    {0x1.5ac056b015ac0p+0, -0x1.36b6776be1116p-2},
    {0x1.59d61f123ccaap+0, -0x1.3401e12aecba0p-2},
    {0x1.58ed2308158edp+0, -0x1.314f1e1d35ce3p-2},
    {0x1.5805601580560p+0, -0x1.2e9e2bce12286p-2},
    {0x1.571ed3c506b3ap+0, -0x1.2bef07cdc9355p-2},
    {0x1.56397ba7c52e2p+0, -0x1.2941afb186b7cp-2},
    {0x1.5555555555555p+0, -0x1.269621134db91p-2},
    {0x1.54725e6bb82fep+0, -0x1.23ec5991eba49p-2},
    {0x1.5390948f40febp+0, -0x1.214456d0eb8d5p-2},
    {0x1.52aff56a8054bp+0, -0x1.1e9e1678899f5p-2},
    {0x1.51d07eae2f815p+0, -0x1.1bf99635a6b95p-2},
    {0x1.50f22e111c4c5p+0, -0x1.1956d3b9bc2f9p-2},
    {0x1.5015015015015p+0, -0x1.16b5ccbacfb73p-2},
    {0x1.4f38f62dd4c9bp+0, -0x1.14167ef367784p-2},
    {0x1.4e5e0a72f0539p+0, -0x1.1178e8227e47ap-2},
    {0x1.4d843bedc2c4cp+0, -0x1.0edd060b78082p-2},
    {0x1.4cab88725af6ep+0, -0x1.0c42d676162e2p-2},
    {0x1.4bd3edda68fe1p+0, -0x1.09aa572e6c6d4p-2},
    {0x1.4afd6a052bf5bp+0, -0x1.07138604d5864p-2},
    {0x1.4a27fad76014ap+0, -0x1.047e60cde83b7p-2},
    {0x1.49539e3b2d067p+0, -0x1.01eae5626c691p-2},
    {0x1.4880522014880p+0, -0x1.feb2233ea07cbp-3},
    {0x1.47ae147ae147bp+0, -0x1.f991c6cb3b37ap-3},
    {0x1.46dce34596066p+0, -0x1.f474b134df228p-3},
    {0x1.460cbc7f5cf9ap+0, -0x1.ef5ade4dcffe5p-3},
    {0x1.453d9e2c776cap+0, -0x1.ea4449f04aaf5p-3},
    {0x1.446f86562d9fbp+0, -0x1.e530effe71013p-3},
    {0x1.43a2730abee4dp+0, -0x1.e020cc6235ab5p-3},
    {0x1.42d6625d51f87p+0, -0x1.db13db0d48941p-3},
    {0x1.420b5265e5951p+0, -0x1.d60a17f903514p-3},
    {0x1.4141414141414p+0, -0x1.d1037f2655e7bp-3},
    {0x1.40782d10e6566p+0, -0x1.cc000c9db3c52p-3},
    {0x1.3fb013fb013fbp+0, -0x1.c6ffbc6f00f71p-3},
    {0x1.3ee8f42a5af07p+0, -0x1.c2028ab17f9b5p-3},
    {0x1.3e22cbce4a902p+0, -0x1.bd087383bd8aap-3},
    {0x1.3d5d991aa75c6p+0, -0x1.b811730b823d4p-3},
    {0x1.3c995a47babe7p+0, -0x1.b31d8575bce3bp-3},
    {0x1.3bd60d9232955p+0, -0x1.ae2ca6f672bd8p-3},
    {0x1.3b13b13b13b14p+0, -0x1.a93ed3c8ad9e5p-3},
    {0x1.3a524387ac822p+0, -0x1.a454082e6ab03p-3},
    {0x1.3991c2c187f63p+0, -0x1.9f6c407089663p-3},
    {0x1.38d22d366088ep+0, -0x1.9a8778debaa3ap-3},
    {0x1.3813813813814p+0, -0x1.95a5adcf70182p-3},
    {0x1.3755bd1c945eep+0, -0x1.90c6db9fcbcdbp-3},
    {0x1.3698df3de0748p+0, -0x1.8beafeb38fe8fp-3},
    {0x1.35dce5f9f2af8p+0, -0x1.871213750e994p-3},
    {0x1.3521cfb2b78c1p+0, -0x1.823c16551a3c0p-3},
    {0x1.34679ace01346p+0, -0x1.7d6903caf5acdp-3},
    {0x1.33ae45b57bcb2p+0, -0x1.7898d85444c74p-3},
    {0x1.32f5ced6a1dfap+0, -0x1.73cb9074fd14dp-3},
    {0x1.323e34a2b10bfp+0, -0x1.6f0128b756ab9p-3},
    {0x1.3187758e9ebb6p+0, -0x1.6a399dabbd383p-3},
    {0x1.30d190130d190p+0, -0x1.6574ebe8c1339p-3},
    {0x1.301c82ac40260p+0, -0x1.60b3100b09474p-3},
    {0x1.2f684bda12f68p+0, -0x1.5bf406b543db0p-3},
    {0x1.2eb4ea1fed14bp+0, -0x1.5737cc9018cddp-3},
    {0x1.2e025c04b8097p+0, -0x1.527e5e4a1b58dp-3},
    {0x1.2d50a012d50a0p+0, -0x1.4dc7b897bc1c7p-3},
    {0x1.2c9fb4d812ca0p+0, -0x1.4913d8333b563p-3},
    {0x1.2bef98e5a3711p+0, -0x1.4462b9dc9b3dcp-3},
    {0x1.2b404ad012b40p+0, -0x1.3fb45a59928cap-3},
    {0x1.2a91c92f3c105p+0, -0x1.3b08b6757f2a7p-3},
    {0x1.29e4129e4129ep+0, -0x1.365fcb0159014p-3},
    {0x1.293725bb804a5p+0, -0x1.31b994d3a4f86p-3},
    {0x1.288b01288b013p+0, -0x1.2d1610c86813dp-3},
    {0x1.27dfa38a1ce4dp+0, -0x1.28753bc11aba2p-3},
    {0x1.27350b8812735p+0, -0x1.23d712a49c201p-3},
    {0x1.268b37cd60127p+0, -0x1.1f3b925f25d44p-3},
    {0x1.25e22708092f1p+0, -0x1.1aa2b7e23f729p-3},
    {0x1.2539d7e9177b2p+0, -0x1.160c8024b27b0p-3},
    {0x1.2492492492492p+0, -0x1.1178e8227e47ap-3},
    {0x1.23eb79717605bp+0, -0x1.0ce7ecdccc28bp-3},
    {0x1.23456789abcdfp+0, -0x1.08598b59e3a07p-3},
    {0x1.22a0122a0122ap+0, -0x1.03cdc0a51ec0dp-3},
    {0x1.21fb78121fb78p+0, -0x1.fe89139dbd565p-4},
    {0x1.21579804855e6p+0, -0x1.f57bc7d9005dbp-4},
    {0x1.20b470c67c0d9p+0, -0x1.ec739830a1126p-4},
    {0x1.2012012012012p+0, -0x1.e3707ee30487bp-4},
    {0x1.1f7047dc11f70p+0, -0x1.da7276384469ep-4},
    {0x1.1ecf43c7fb84cp+0, -0x1.d179788219362p-4},
    {0x1.1e2ef3b3fb874p+0, -0x1.c885801bc4b20p-4},
    {0x1.1d8f5672e4abdp+0, -0x1.bf968769fca18p-4},
    {0x1.1cf06ada2811dp+0, -0x1.b6ac88dad5b1dp-4},
    {0x1.1c522fc1ce059p+0, -0x1.adc77ee5aea8ep-4},
    {0x1.1bb4a4046ed29p+0, -0x1.a4e7640b1bc38p-4},
    {0x1.1b17c67f2bae3p+0, -0x1.9c0c32d4d254dp-4},
    {0x1.1a7b9611a7b96p+0, -0x1.9335e5d594988p-4},
    {0x1.19e0119e0119ep+0, -0x1.8a6477a91dc29p-4},
    {0x1.19453808ca29cp+0, -0x1.8197e2f40e3f0p-4},
    {0x1.18ab083902bdbp+0, -0x1.78d02263d82d7p-4},
    {0x1.1811811811812p+0, -0x1.700d30aeac0e8p-4},
    {0x1.1778a191bd684p+0, -0x1.674f089365a78p-4},
    {0x1.16e0689427379p+0, -0x1.5e95a4d9791cdp-4},
    {0x1.1648d50fc3201p+0, -0x1.55e10050e0382p-4},
    {0x1.15b1e5f75270dp+0, -0x1.4d3115d207eacp-4},
    {0x1.151b9a3fdd5c9p+0, -0x1.4485e03dbdfb0p-4},
    {0x1.1485f0e0acd3bp+0, -0x1.3bdf5a7d1ee5ep-4},
    {0x1.13f0e8d344724p+0, -0x1.333d7f8183f4ap-4},
    {0x1.135c81135c811p+0, -0x1.2aa04a44717a1p-4},
    {0x1.12c8b89edc0acp+0, -0x1.2207b5c7854a1p-4},
    {0x1.12358e75d3033p+0, -0x1.1973bd1465561p-4},
    {0x1.11a3019a74826p+0, -0x1.10e45b3cae829p-4},
    {0x1.1111111111111p+0, -0x1.08598b59e3a06p-4},
    {0x1.107fbbe011080p+0, -0x1.ffa6911ab9309p-5},
    {0x1.0fef010fef011p+0, -0x1.eea31c006b87cp-5},
    {0x1.0f5edfab325a2p+0, -0x1.dda8adc67ee59p-5},
    {0x1.0ecf56be69c90p+0, -0x1.ccb73cdddb2d0p-5},
    {0x1.0e40655826011p+0, -0x1.bbcebfc68f424p-5},
    {0x1.0db20a88f4696p+0, -0x1.aaef2d0fb1108p-5},
    {0x1.0d24456359e3ap+0, -0x1.9a187b573de81p-5},
    {0x1.0c9714fbcda3bp+0, -0x1.894aa149fb34bp-5},
    {0x1.0c0a7868b4171p+0, -0x1.788595a3577c8p-5},
    {0x1.0b7e6ec259dc8p+0, -0x1.67c94f2d4bb65p-5},
    {0x1.0af2f722eecb5p+0, -0x1.5715c4c03cee1p-5},
    {0x1.0a6810a6810a7p+0, -0x1.466aed42de3f9p-5},
    {0x1.09ddba6af8360p+0, -0x1.35c8bfaa13069p-5},
    {0x1.0953f39010954p+0, -0x1.252f32f8d1840p-5},
    {0x1.08cabb37565e2p+0, -0x1.149e3e4005a8dp-5},
    {0x1.0842108421084p+0, -0x1.0415d89e74440p-5},
    {0x1.07b9f29b8eae2p+0, -0x1.e72bf2813ce6ap-6},
    {0x1.073260a47f7c6p+0, -0x1.c63d2ec14aad7p-6},
    {0x1.06ab59c7912fbp+0, -0x1.a55f548c5c427p-6},
    {0x1.0624dd2f1a9fcp+0, -0x1.8492528c8cac5p-6},
    {0x1.059eea0727586p+0, -0x1.63d6178690bbep-6},
    {0x1.05197f7d73404p+0, -0x1.432a925980cbcp-6},
    {0x1.04949cc1664c5p+0, -0x1.228fb1fea2e0ap-6},
    {0x1.0410410410410p+0, -0x1.0205658935837p-6},
    {0x1.038c6b78247fcp+0, -0x1.c317384c75f0dp-7},
    {0x1.03091b51f5e1ap+0, -0x1.82448a388a283p-7},
    {0x1.02864fc7729e9p+0, -0x1.41929f968330cp-7},
    {0x1.0204081020408p+0, -0x1.010157588de69p-7},
    {0x1.0182436517a37p+0, -0x1.8121214586b02p-8},
    {0x1.0101010101010p+0, -0x1.0080559588b25p-8},
    {0x1.0080402010080p+0, -0x1.0040155d5881ep-9},
};

__device__ __forceinline__ double qlog(double x) {
    constexpr double kLn2Hi = 6.93147180369123816490e-01;
    constexpr double kLn2Lo = 1.90821492927058770002e-10;
    const double m = __builtin_amdgcn_frexp_mant(x);
    const double e = (double)__builtin_amdgcn_frexp_exp(x);
    // (m - 1/2) * 512 is exact; the clamp keeps inf and NaN inputs in bounds
    const int j = min(max((int)fma_(m, 512.0, -256.0), 0), 255);
    const QlogEntry t = kQlogTab[j];
    const double r = fma_(m, t.ic, -1.0);
    double q = -1.0 / 7.0;
    q = fma_(q, r, 1.0 / 6.0);
    q = fma_(q, r, -1.0 / 5.0);
    q = fma_(q, r, 1.0 / 4.0);
    q = fma_(q, r, -1.0 / 3.0);
    q = fma_(q, r, 0.5);
    const double lr = fma_(-r * r, q, r);
    const double res = fma_(e, kLn2Hi, t.nl + fma_(e, kLn2Lo, lr));
    return (x > 0.0 && x < __builtin_inf()) ? res : __builtin_nan("");
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
