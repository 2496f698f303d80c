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
// c in a scalar / vector register pair that the compiler cannot see through:
// a loop-invariant FP64 constant then stays in registers set up once (the
// empty asm has no side effects, so it is hoisted and merged) instead of
// being rebuilt as a literal before each use.
__device__ __forceinline__ double sreg_const(double c) {
    asm("" : "+s"(c));
    return c;
}
__device__ __forceinline__ double vreg_const(double c) {
    asm("" : "+v"(c));
    return c;
}

// 1/b: hardware reciprocal estimate refined by two Newton steps.
__device__ __forceinline__ double recip(double b) {
    double r = __builtin_amdgcn_rcp(b);
    double e = fma_(-b, r, 1.0);
    r = fma_(r, e, r);
    e = fma_(-b, r, 1.0);
    return fma_(r, e, r);
}

// r_k = 1 / b_k for T values from one reciprocal (v_rcp_f64 issues at a
// quarter of the FP64 rate): prefix products, the reciprocal of their total,
// then two multiplies back per value.  The caller guarantees that every
// product of the b_k is a normal number.
template <int T>
__device__ __forceinline__ void recip_tile(const double (&b)[T], double (&r)[T]) {
    double pre[T];
    pre[0] = b[0];
#pragma unroll
    for (int k = 1; k < T; ++k) pre[k] = pre[k - 1] * b[k];
    double inv = recip(pre[T - 1]);  // 1 / (b_0 ... b_{T-1})
#pragma unroll
    for (int k = T - 1; k > 0; --k) {
        r[k] = inv * pre[k - 1];
        inv *= b[k];  // 1 / (b_0 ... b_{k-1})
    }
    r[0] = inv;
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

// The tables of qlog and qexp in one 8 KB array (written by
// make_math_tables.py), so that one base address serves both: entries 2j and
// 2j + 1 (j < 256) are qlog's {ic_j, -ln ic_j}, entry 512 + j (j < 512) is
// qexp's 2^(j/512).  It stays in the L1 cache; each evaluation of qlog or
// qexp reads one entry.
static __constant__ const double kMathTab[1024] __attribute__((aligned(16))) = {
    // qlog: {1/(1/2 + (j + 1/2)/512), -ln of it}, j = 0..255
    0x1.ff007fc01ff00p+0, -0x1.61e46fda56466p-1,
    0x1.fd04794a10e6ap+0, -0x1.5fe66db228992p-1,
    0x1.fb0c610d5e939p+0, -0x1.5dea65985a350p-1,
    0x1.f9182b6813bafp+0, -0x1.5bf053a48690ep-1,
    0x1.f727cce5f530ap+0, -0x1.59f833f9d4290p-1,
    0x1.f53b3a3fa204ep+0, -0x1.580202c6c7353p-1,
    0x1.f3526859b8cecp+0, -0x1.560dbc45153c7p-1,
    0x1.f16d4c4401f17p+0, -0x1.541b5cb979809p-1,
    0x1.ef8bdb389ebadp+0, -0x1.522ae0738a3d8p-1,
    0x1.edae0a9b3d3a5p+0, -0x1.503c43cd8eb68p-1,
    0x1.ebd3cff850b0cp+0, -0x1.4e4f832c560ddp-1,
    0x1.e9fd21044e799p+0, -0x1.4c649aff0ee16p-1,
    0x1.e829f39aef509p+0, -0x1.4a7b87bf1fa82p-1,
    0x1.e65a3dbe74d6bp+0, -0x1.489445efffcccp-1,
    0x1.e48df596f3394p+0, -0x1.46aed21f117fcp-1,
    0x1.e2c511719ee16p+0, -0x1.44cb28e37c3eep-1,
    0x1.e0ff87c01e100p+0, -0x1.42e946de080c0p-1,
    0x1.df3d4f17de4dbp+0, -0x1.410928b8f950fp-1,
    0x1.dd7e5e316d94cp+0, -0x1.3f2acb27ed6c7p-1,
    0x1.dbc2abe7d71d4p+0, -0x1.3d4e2ae7b7e2bp-1,
    0x1.da0a2f3803b41p+0, -0x1.3b7344be40311p-1,
    0x1.d854df401d855p+0, -0x1.399a157a603e7p-1,
    0x1.d6a2b33ef7448p+0, -0x1.37c299f3c366ap-1,
    0x1.d4f3a293769cap+0, -0x1.35eccf0ac61d0p-1,
    0x1.d347a4bc01d34p+0, -0x1.3418b1a85622cp-1,
    0x1.d19eb155f08a4p+0, -0x1.32463ebdd34eap-1,
    0x1.cff8c01cff8c0p+0, -0x1.30757344f0e13p-1,
    0x1.ce55c8eac7900p+0, -0x1.2ea64c3f97654p-1,
    0x1.ccb5c3b636e3ap+0, -0x1.2cd8c6b7c716fp-1,
    0x1.cb18a8930de60p+0, -0x1.2b0cdfbf7ad03p-1,
    0x1.c97e6fb15e44dp+0, -0x1.294294708b773p-1,
    0x1.c7e7115d0ce95p+0, -0x1.2779e1ec93ecbp-1,
    0x1.c65285fd56843p+0, -0x1.25b2c55cd5762p-1,
    0x1.c4c0c61456a8ep+0, -0x1.23ed3bf21ca33p-1,
    0x1.c331ca3e91679p+0, -0x1.222942e4a6a9dp-1,
    0x1.c1a58b327f576p+0, -0x1.2066d7740737ep-1,
    0x1.c01c01c01c01cp+0, -0x1.1ea5f6e70eb83p-1,
    0x1.be9526d0769fap+0, -0x1.1ce69e8bb106bp-1,
    0x1.bd10f365451b6p+0, -0x1.1b28cbb6ec93ep-1,
    0x1.bb8f609879493p+0, -0x1.196c7bc4b1f3ap-1,
    0x1.ba10679bd8488p+0, -0x1.17b1ac17cbd5bp-1,
    0x1.b89401b89401cp+0, -0x1.15f85a19c765cp-1,
    0x1.b71a284ee6b34p+0, -0x1.1440833add112p-1,
    0x1.b5a2d4d5b081fp+0, -0x1.128a24f1d9affp-1,
    0x1.b42e00da17007p+0, -0x1.10d53cbc080f8p-1,
    0x1.b2bba5ff26a23p+0, -0x1.0f21c81d1adc3p-1,
    0x1.b14bbdfd760e6p+0, -0x1.0d6fc49f16e93p-1,
    0x1.afde42a2cb482p+0, -0x1.0bbf2fd23dd41p-1,
    0x1.ae732dd1c2a09p+0, -0x1.0a10074cf9019p-1,
    0x1.ad0a798177693p+0, -0x1.086248abc4f3bp-1,
    0x1.aba41fbd2e5b1p+0, -0x1.06b5f1911cf52p-1,
    0x1.aa401aa401aa4p+0, -0x1.050affa5671a5p-1,
    0x1.a8de64688ebabp+0, -0x1.03617096e0952p-1,
    0x1.a77ef750a56dap+0, -0x1.01b942198a5a1p-1,
    0x1.a621cdb4f8fdfp+0, -0x1.001271e716158p-1,
    0x1.a4c6e200d2637p+0, -0x1.fcd9fb7da6defp-2,
    0x1.a36e2eb1c432dp+0, -0x1.f991c6cb3b37ap-2,
    0x1.a217ae575ff2fp+0, -0x1.f64c414b926c5p-2,
    0x1.a0c35b92ecdf1p+0, -0x1.f309669e24cf9p-2,
    0x1.9f713117200d0p+0, -0x1.efc9326d16ab9p-2,
    0x1.9e2129a7d5f0ap+0, -0x1.ec8ba06d15ad8p-2,
    0x1.9cd34019cd340p+0, -0x1.e950ac5d36dc1p-2,
    0x1.9b876f5262dd1p+0, -0x1.e6185206d516fp-2,
    0x1.9a3db2474fb98p+0, -0x1.e2e28d3d701ccp-2,
    0x1.98f603fe670a0p+0, -0x1.dfaf59de8c15ep-2,
    0x1.97b05f8d56652p+0, -0x1.dc7eb3d1919ebp-2,
    0x1.966cc01966cc0p+0, -0x1.d9509707ae52fp-2,
    0x1.952b20d73ee97p+0, -0x1.d624ff7bb5d46p-2,
    0x1.93eb7d0aa6759p+0, -0x1.d2fbe932034c8p-2,
    0x1.92add0064ab74p+0, -0x1.cfd550385b659p-2,
    0x1.9172152b841ddp+0, -0x1.ccb130a5cebb0p-2,
    0x1.903847ea1cec1p+0, -0x1.c98f869a9cbbcp-2,
    0x1.8f0063c018f00p+0, -0x1.c6704e4016ff7p-2,
    0x1.8dca64397e408p+0, -0x1.c35383c8850b0p-2,
    0x1.8c9644f01efbcp+0, -0x1.c039236f08819p-2,
    0x1.8b64018b64019p+0, -0x1.bd21297781c30p-2,
    0x1.8a3395c018a34p+0, -0x1.ba0b922e74f23p-2,
    0x1.8904fd503744bp+0, -0x1.b6f859e8ef639p-2,
    0x1.87d8340ab6e97p+0, -0x1.b3e77d046d728p-2,
    0x1.86ad35cb59a84p+0, -0x1.b0d8f7e6c0b84p-2,
    0x1.8583fe7a7c018p+0, -0x1.adccc6fdf6a80p-2,
    0x1.845c8a0ce5129p+0, -0x1.aac2e6c03f895p-2,
    0x1.8336d48397a24p+0, -0x1.a7bb53abd5d21p-2,
    0x1.8212d9eba4018p+0, -0x1.a4b60a46e5dd2p-2,
    0x1.80f0965dfabcbp+0, -0x1.a1b3071f75fd9p-2,
    0x1.7fd005ff40180p+0, -0x1.9eb246cb4eea2p-2,
    0x1.7eb124ffa053bp+0, -0x1.9bb3c5e7e4814p-2,
    0x1.7d93ef9aa4b46p+0, -0x1.98b7811a3ee5cp-2,
    0x1.7c7862170949fp+0, -0x1.95bd750ee3ed3p-2,
    0x1.7b5e78c693733p+0, -0x1.92c59e79c0e55p-2,
    0x1.7a463005e918cp+0, -0x1.8fcffa1614aa0p-2,
    0x1.792f843c689c3p+0, -0x1.8cdc84a65a0bep-2,
    0x1.781a71dc01782p+0, -0x1.89eb3af432875p-2,
    0x1.7706f5610d8d0p+0, -0x1.86fc19d05148ep-2,
    0x1.75f50b522b17cp+0, -0x1.840f1e12667f1p-2,
    0x1.74e4b040174e5p+0, -0x1.812444990af64p-2,
    0x1.73d5e0c5899f7p+0, -0x1.7e3b8a49ac007p-2,
    0x1.72c899870f91fp+0, -0x1.7b54ec1077a48p-2,
    0x1.71bcd732e940ap+0, -0x1.787066e04915fp-2,
    0x1.70b29680e66fap+0, -0x1.758df7b29572cp-2,
    0x1.6fa9d43244380p+0, -0x1.72ad9b8758c60p-2,
    0x1.6ea28d118b474p+0, -0x1.6fcf4f65034fdp-2,
    0x1.6d9cbdf26eaefp+0, -0x1.6cf31058670ecp-2,
    0x1.6c9863b1ab429p+0, -0x1.6a18db74a58c4p-2,
    0x1.6b957b34e7803p+0, -0x1.6740add31de95p-2,
    0x1.6a94016a94017p+0, -0x1.646a84935b2a3p-2,
    0x1.6993f349cc726p+0, -0x1.61965cdb02c1ep-2,
    0x1.68954dd2390bap+0, -0x1.5ec433d5c35aep-2,
    0x1.67980e0bf08c7p+0, -0x1.5bf406b543db1p-2,
    0x1.669c31075ab40p+0, -0x1.5925d2b112a59p-2,
    0x1.65a1b3dd13357p+0, -0x1.565995069514cp-2,
    0x1.64a893adcd25fp+0, -0x1.538f4af8f72fcp-2,
    0x1.63b0cda236e1cp+0, -0x1.50c6f1d11b97bp-2,
    0x1.62ba5eeade65ep+0, -0x1.4e0086dd8baccp-2,
    0x1.61c544c0161c5p+0, -0x1.4b3c077267e9ap-2,
    0x1.60d17c61da198p+0, -0x1.487970e958771p-2,
    0x1.5fdf0317b5c6fp+0, -0x1.45b8c0a17df12p-2,
    0x1.5eedd630a9fb3p+0, -0x1.42f9f3ff62641p-2,
    0x1.5dfdf303137b6p+0, -0x1.403d086cea79bp-2,
    0x1.5d0f56ec91e57p+0, -0x1.3d81fb5946dbcp-2,
    0x1.5c21ff51ef005p+0, -0x1.3ac8ca38e5c5dp-2,
    0x1.5b35e99f06714p+0, -0x1.3811728564cb2p-2,
    0x1.5a4b1346add2bp+0, -0x1.355bf1bd82c8bp-2,
    0x1.596179c29d2cep+0, -0x1.32a84565120a9p-2,
    0x1.58791a9357ccep+0, -0x1.2ff66b04ea9d5p-2,
    0x1.5791f34015792p+0, -0x1.2d46602adccefp-2,
    0x1.56ac0156ac015p+0, -0x1.2a982269a3dbep-2,
    0x1.55c7426b79286p+0, -0x1.27ebaf58d8c9cp-2,
    0x1.54e3b4194ce66p+0, -0x1.25410494e56c8p-2,
    0x1.5401540154015p+0, -0x1.22981fbef797ap-2,
    0x1.53201fcb02fb1p+0, -0x1.1ff0fe7cf47a9p-2,
    0x1.5240152401524p+0, -0x1.1d4b9e796c245p-2,
    0x1.516131c015161p+0, -0x1.1aa7fd638d33ep-2,
    0x1.508373590ec9cp+0, -0x1.180618ef18adep-2,
    0x1.4fa6d7aeb597cp+0, -0x1.1565eed455fc2p-2,
    0x1.4ecb5c86b3d24p+0, -0x1.12c77cd00713cp-2,
    0x1.4df0ffac83c01p+0, -0x1.102ac0a35cc1bp-2,
    0x1.4d17bef15cb4ep+0, -0x1.0d8fb813eb1efp-2,
    0x1.4c3f982c20723p+0, -0x1.0af660eb9e278p-2,
    0x1.4b68893948d1cp+0, -0x1.085eb8f8ae799p-2,
    0x1.4a928ffad5b5cp+0, -0x1.05c8be0d9635ap-2,
    0x1.49bdaa583b401p+0, -0x1.03346e0106062p-2,
    0x1.48e9d63e504d1p+0, -0x1.00a1c6adda472p-2,
    0x1.4817119f3d325p+0, -0x1.fc218be620a5fp-3,
    0x1.47455a726abf2p+0, -0x1.f702d36777df0p-3,
    0x1.4674aeb4717e9p+0, -0x1.f1e75fadf9bdep-3,
    0x1.45a50c670938fp+0, -0x1.eccf2c8fe920bp-3,
    0x1.44d67190f8b43p+0, -0x1.e7ba35eb77e2ap-3,
    0x1.4408dc3e05b22p+0, -0x1.e2a877a6b2c0fp-3,
    0x1.433c4a7ee52b4p+0, -0x1.dd99edaf6d7e9p-3,
    0x1.4270ba692bc4dp+0, -0x1.d88e93fb2f451p-3,
    0x1.41a62a173e821p+0, -0x1.d38666871f467p-3,
    0x1.40dc97a843ae8p+0, -0x1.ce816157f1985p-3,
    0x1.4014014014014p+0, -0x1.c97f8079d44ecp-3,
    0x1.3f4c65072bf74p+0, -0x1.c480c0005cccfp-3,
    0x1.3e85c12a9d651p+0, -0x1.bf851c067555cp-3,
    0x1.3dc013dc013dcp+0, -0x1.ba8c90ae4ad19p-3,
    0x1.3cfb5b51698ebp+0, -0x1.b5971a213acd9p-3,
    0x1.3c3795c553afbp+0, -0x1.b0a4b48fc1b44p-3,
    0x1.3b74c1769aa5cp+0, -0x1.abb55c31693aep-3,
    0x1.3ab2dca869b81p+0, -0x1.a6c90d44b704cp-3,
    0x1.39f1e5a22f36ep+0, -0x1.a1dfc40f1b7f1p-3,
    0x1.3931daaf8f721p+0, -0x1.9cf97cdce0ec1p-3,
    0x1.3872ba2057e04p+0, -0x1.981634011aa74p-3,
    0x1.37b4824872744p+0, -0x1.9335e5d594985p-3,
    0x1.36f7317fd9212p+0, -0x1.8e588ebac2dc1p-3,
    0x1.363ac622898b1p+0, -0x1.897e2b17b19a6p-3,
    0x1.357f3e9078e5bp+0, -0x1.84a6b759f512dp-3,
    0x1.34c4992d87fd9p+0, -0x1.7fd22ff599d4cp-3,
    0x1.340ad461776d3p+0, -0x1.7b0091651528bp-3,
    0x1.3351ee97dbfc6p+0, -0x1.7631d82935a84p-3,
    0x1.3299e6401329ap+0, -0x1.716600c914055p-3,
    0x1.31e2b9cd37dc2p+0, -0x1.6c9d07d203fc4p-3,
    0x1.312c67b6173eep+0, -0x1.67d6e9d785770p-3,
    0x1.3076ee7525c2cp+0, -0x1.6313a37335d76p-3,
    0x1.2fc24c8874486p+0, -0x1.5e533144c1718p-3,
    0x1.2f0e8071a5703p+0, -0x1.59958ff1d52f4p-3,
    0x1.2e5b88b5e3104p+0, -0x1.54dabc26105d3p-3,
    0x1.2da963ddd3cfbp+0, -0x1.5022b292f6a45p-3,
    0x1.2cf8107590e67p+0, -0x1.4b6d6fefe22a5p-3,
    0x1.2c478d0c9c013p+0, -0x1.46baf0f9f5db8p-3,
    0x1.2b97d835d548ep+0, -0x1.420b32740fdd6p-3,
    0x1.2ae8f087718d0p+0, -0x1.3d5e3126bc281p-3,
    0x1.2a3ad49af0907p+0, -0x1.38b3e9e027477p-3,
    0x1.298d830d13780p+0, -0x1.340c59741142dp-3,
    0x1.28e0fa7dd35a3p+0, -0x1.2f677cbbc0a98p-3,
    0x1.2835399057efdp+0, -0x1.2ac55095f5c5bp-3,
    0x1.278a3eeaee650p+0, -0x1.2625d1e6ddf55p-3,
    0x1.26e009370049cp+0, -0x1.2188fd9807266p-3,
    0x1.263697210aa18p+0, -0x1.1ceed09853755p-3,
    0x1.258de75895121p+0, -0x1.185747dbecf34p-3,
    0x1.24e5f89029305p+0, -0x1.13c2605c398bfp-3,
    0x1.243ec97d49eaep+0, -0x1.0f301717cf0fbp-3,
    0x1.239858d86b11fp+0, -0x1.0aa06912675d5p-3,
    0x1.22f2a55ce8fc5p+0, -0x1.06135354d4b19p-3,
    0x1.224dadc900489p+0, -0x1.0188d2ecf613ep-3,
    0x1.21a970ddc5ba7p+0, -0x1.fa01c9db57ce7p-4,
    0x1.2105ed5f1e336p+0, -0x1.f0f70cdd992e4p-4,
    0x1.20632213b6c6dp+0, -0x1.e7f1691a32d3ap-4,
    0x1.1fc10dc4fce8bp+0, -0x1.def0d8d466dbbp-4,
    0x1.1f1faf3f16b64p+0, -0x1.d5f55659210e1p-4,
    0x1.1e7f0550db594p+0, -0x1.ccfedbfee13a8p-4,
    0x1.1ddf0ecbcb841p+0, -0x1.c40d6425a5cb4p-4,
    0x1.1d3fca840a074p+0, -0x1.bb20e936d6976p-4,
    0x1.1ca13750547fep+0, -0x1.b23965a52ff04p-4,
    0x1.1c035409fc1dfp+0, -0x1.a956d3ecade60p-4,
    0x1.1b661f8cde833p+0, -0x1.a0792e9277cadp-4,
    0x1.1ac998b75eb90p+0, -0x1.97a07024cbe6ep-4,
    0x1.1a2dbe6a5e3e4p+0, -0x1.8ecc933aeb6e2p-4,
    0x1.19928f89362b7p+0, -0x1.85fd927506a46p-4,
    0x1.18f80af9b06dcp+0, -0x1.7d33687c293c8p-4,
    0x1.185e2fa401186p+0, -0x1.746e100226edbp-4,
    0x1.17c4fc72bfcb9p+0, -0x1.6bad83c1883bap-4,
    0x1.172c7052e1316p+0, -0x1.62f1be7d7774ap-4,
    0x1.16948a33b08fap+0, -0x1.5a3abb01ade21p-4,
    0x1.15fd4906c96f1p+0, -0x1.5188742261311p-4,
    0x1.1566abc011567p+0, -0x1.48dae4bc3101dp-4,
    0x1.14d0b155b19aep+0, -0x1.403207b414b79p-4,
    0x1.143b58c01143bp+0, -0x1.378dd7f74970fp-4,
    0x1.13a6a0f9cf01ep+0, -0x1.2eee507b402ffp-4,
    0x1.131288ffbb3b6p+0, -0x1.26536c3d8c36cp-4,
    0x1.127f0fd0d2295p+0, -0x1.1dbd2643d1913p-4,
    0x1.11ec346e36092p+0, -0x1.152b799bb3cd0p-4,
    0x1.1159f5db29606p+0, -0x1.0c9e615ac4e19p-4,
    0x1.10c8531d0952ep+0, -0x1.0415d89e7444bp-4,
    0x1.10374b3b480aap+0, -0x1.f723b517fc51fp-5,
    0x1.0fa6dd3f67322p+0, -0x1.e624c4a0b5e15p-5,
    0x1.0f170834f27fap+0, -0x1.d52ed6405d87ap-5,
    0x1.0e87cb297a51ep+0, -0x1.c441e06f72a93p-5,
    0x1.0df9252c8e5e6p+0, -0x1.b35dd9b58baa8p-5,
    0x1.0d6b154fb86f9p+0, -0x1.a282b8a936174p-5,
    0x1.0cdd9aa677344p+0, -0x1.91b073efd7314p-5,
    0x1.0c50b446391f3p+0, -0x1.80e7023d8ccc8p-5,
    0x1.0bc4614657569p+0, -0x1.70265a550e77bp-5,
    0x1.0b38a0c010b39p+0, -0x1.5f6e73078efc3p-5,
    0x1.0aad71ce84d16p+0, -0x1.4ebf43349e26ap-5,
    0x1.0a22d38eaf2bfp+0, -0x1.3e18c1ca0ae99p-5,
    0x1.0998c51f624d5p+0, -0x1.2d7ae5c3c5bb7p-5,
    0x1.090f45a1430aap+0, -0x1.1ce5a62bc3540p-5,
    0x1.08865436c3cf7p+0, -0x1.0c58fa19dfaabp-5,
    0x1.07fdf0041ff7cp+0, -0x1.f7a9b16782855p-6,
    0x1.0776182f57386p+0, -0x1.d6b272597981fp-6,
    0x1.06eecbe029155p+0, -0x1.b5cc258b718e7p-6,
    0x1.06680a4010668p+0, -0x1.94f6b99a24473p-6,
    0x1.05e1d27a3ee9cp+0, -0x1.74321d3d006d2p-6,
    0x1.055c23bb98e2ap+0, -0x1.537e3f45f354ep-6,
    0x1.04d6fd32b0c7bp+0, -0x1.32db0ea132e10p-6,
    0x1.04525e0fc2fcbp+0, -0x1.12487a5507f68p-6,
    0x1.03ce4584b19a0p+0, -0x1.e38ce30333100p-7,
    0x1.034ab2c50040dp+0, -0x1.a2a9c6c17044dp-7,
    0x1.02c7a505cffbfp+0, -0x1.61e77e8b53f9fp-7,
    0x1.02451b7ddb2d2p+0, -0x1.2145e939ef1bcp-7,
    0x1.01c315657186bp+0, -0x1.c189cbb0e283fp-8,
    0x1.014191f674111p+0, -0x1.40c8a7478788dp-8,
    0x1.00c0906c513cfp+0, -0x1.809048289860ap-9,
    0x1.0040100401004p+0, -0x1.0020055655885p-10,
    // qexp: 2^(j/512), j = 0..511
    0x1.0000000000000p+0, 0x1.0058c86da1c0ap+0,
    0x1.00b1afa5abcbfp+0, 0x1.010ab5b2cbd11p+0,
    0x1.0163da9fb3335p+0, 0x1.01bd1e77170b4p+0,
    0x1.02168143b0281p+0, 0x1.027003103b10ep+0,
    0x1.02c9a3e778061p+0, 0x1.032363d42b027p+0,
    0x1.037d42e11bbccp+0, 0x1.03d7411915a8ap+0,
    0x1.04315e86e7f85p+0, 0x1.048b9b35659d8p+0,
    0x1.04e5f72f654b1p+0, 0x1.0540727fc1762p+0,
    0x1.059b0d3158574p+0, 0x1.05f5c74f0bec2p+0,
    0x1.0650a0e3c1f89p+0, 0x1.06ab99fa6407cp+0,
    0x1.0706b29ddf6dep+0, 0x1.0761ead925493p+0,
    0x1.07bd42b72a836p+0, 0x1.0818ba42e7d30p+0,
    0x1.0874518759bc8p+0, 0x1.08d0088f8093fp+0,
    0x1.092bdf66607e0p+0, 0x1.0987d61701716p+0,
    0x1.09e3ecac6f383p+0, 0x1.0a402331b9715p+0,
    0x1.0a9c79b1f3919p+0, 0x1.0af8f03834e52p+0,
    0x1.0b5586cf9890fp+0, 0x1.0bb23d833d93fp+0,
    0x1.0c0f145e46c85p+0, 0x1.0c6c0b6bdae53p+0,
    0x1.0cc922b7247f7p+0, 0x1.0d265a4b520bap+0,
    0x1.0d83b23395decp+0, 0x1.0de12a7b26300p+0,
    0x1.0e3ec32d3d1a2p+0, 0x1.0e9c7c55189c6p+0,
    0x1.0efa55fdfa9c5p+0, 0x1.0f58503328e6dp+0,
    0x1.0fb66affed31bp+0, 0x1.1014a66f951cep+0,
    0x1.1073028d7233ep+0, 0x1.10d17f64d9ef1p+0,
    0x1.11301d0125b51p+0, 0x1.118edb6db2dc1p+0,
    0x1.11edbab5e2ab6p+0, 0x1.124cbae51a5c8p+0,
    0x1.12abdc06c31ccp+0, 0x1.130b1e264a0e9p+0,
    0x1.136a814f204abp+0, 0x1.13ca058cbae1ep+0,
    0x1.1429aaea92de0p+0, 0x1.1489717425438p+0,
    0x1.14e95934f312ep+0, 0x1.154962388149ep+0,
    0x1.15a98c8a58e51p+0, 0x1.1609d83606e12p+0,
    0x1.166a45471c3c2p+0, 0x1.16cad3c92df73p+0,
    0x1.172b83c7d517bp+0, 0x1.178c554eaea89p+0,
    0x1.17ed48695bbc0p+0, 0x1.184e5d23816c9p+0,
    0x1.18af9388c8deap+0, 0x1.1910eba4df41fp+0,
    0x1.1972658375d2fp+0, 0x1.19d4013041dc2p+0,
    0x1.1a35beb6fcb75p+0, 0x1.1a979e2363cf8p+0,
    0x1.1af99f8138a1cp+0, 0x1.1b5bc2dc40bf0p+0,
    0x1.1bbe084045cd4p+0, 0x1.1c206fb91588fp+0,
    0x1.1c82f95281c6bp+0, 0x1.1ce5a51860746p+0,
    0x1.1d4873168b9aap+0, 0x1.1dab6358e15e8p+0,
    0x1.1e0e75eb44027p+0, 0x1.1e71aad999e82p+0,
    0x1.1ed5022fcd91dp+0, 0x1.1f387bf9cda38p+0,
    0x1.1f9c18438ce4dp+0, 0x1.1fffd7190241ep+0,
    0x1.2063b88628cd6p+0, 0x1.20c7bc96ffc18p+0,
    0x1.212be3578a819p+0, 0x1.21902cd3d09b9p+0,
    0x1.21f49917ddc96p+0, 0x1.2259282fc1f27p+0,
    0x1.22bdda27912d1p+0, 0x1.2322af0b63bffp+0,
    0x1.2387a6e756238p+0, 0x1.23ecc1c78903ap+0,
    0x1.2451ffb82140ap+0, 0x1.24b760c547f15p+0,
    0x1.251ce4fb2a63fp+0, 0x1.25828c65fa1ffp+0,
    0x1.25e85711ece75p+0, 0x1.264e450b3cb82p+0,
    0x1.26b4565e27cddp+0, 0x1.271a8b16f0a30p+0,
    0x1.2780e341ddf29p+0, 0x1.27e75eeb3ab98p+0,
    0x1.284dfe1f56381p+0, 0x1.28b4c0ea83f36p+0,
    0x1.291ba7591bb70p+0, 0x1.2982b17779965p+0,
    0x1.29e9df51fdee1p+0, 0x1.2a5130f50d65cp+0,
    0x1.2ab8a66d10f13p+0, 0x1.2b203fc675d1fp+0,
    0x1.2b87fd0dad990p+0, 0x1.2befde4f2e280p+0,
    0x1.2c57e39771b2fp+0, 0x1.2cc00cf2f6c18p+0,
    0x1.2d285a6e4030bp+0, 0x1.2d90cc15d5346p+0,
    0x1.2df961f641589p+0, 0x1.2e621c1c14833p+0,
    0x1.2ecafa93e2f56p+0, 0x1.2f33fd6a454d2p+0,
    0x1.2f9d24abd886bp+0, 0x1.300670653dfe4p+0,
    0x1.306fe0a31b715p+0, 0x1.30d975721b004p+0,
    0x1.31432edeeb2fdp+0, 0x1.31ad0cf63eeacp+0,
    0x1.32170fc4cd831p+0, 0x1.3281375752b40p+0,
    0x1.32eb83ba8ea32p+0, 0x1.3355f4fb45e20p+0,
    0x1.33c08b26416ffp+0, 0x1.342b46484ebb4p+0,
    0x1.3496266e3fa2dp+0, 0x1.35012ba4ea77dp+0,
    0x1.356c55f929ff1p+0, 0x1.35d7a577dd72bp+0,
    0x1.36431a2de883bp+0, 0x1.36aeb428335b4p+0,
    0x1.371a7373aa9cbp+0, 0x1.3786581d3f669p+0,
    0x1.37f26231e754ap+0, 0x1.385e91be9c811p+0,
    0x1.38cae6d05d866p+0, 0x1.393761742d808p+0,
    0x1.39a401b7140efp+0, 0x1.3a10c7a61d55bp+0,
    0x1.3a7db34e59ff7p+0, 0x1.3aeac4bcdf3eap+0,
    0x1.3b57fbfec6cf4p+0, 0x1.3bc559212ef89p+0,
    0x1.3c32dc313a8e5p+0, 0x1.3ca0853c10f28p+0,
    0x1.3d0e544ede173p+0, 0x1.3d7c4976d27fap+0,
    0x1.3dea64c123422p+0, 0x1.3e58a63b0a09bp+0,
    0x1.3ec70df1c5175p+0, 0x1.3f359bf29743fp+0,
    0x1.3fa4504ac801cp+0, 0x1.40132b07a35dfp+0,
    0x1.40822c367a024p+0, 0x1.40f153e4a136ap+0,
    0x1.4160a21f72e2ap+0, 0x1.41d016f44d8f5p+0,
    0x1.423fb2709468ap+0, 0x1.42af74a1af3f1p+0,
    0x1.431f5d950a897p+0, 0x1.438f6d5817663p+0,
    0x1.43ffa3f84b9d4p+0, 0x1.4470018321a1ap+0,
    0x1.44e086061892dp+0, 0x1.4551318eb43ecp+0,
    0x1.45c2042a7d232p+0, 0x1.4632fde7006f4p+0,
    0x1.46a41ed1d0057p+0, 0x1.471566f8827d0p+0,
    0x1.4786d668b3237p+0, 0x1.47f86d3001fe5p+0,
    0x1.486a2b5c13cd0p+0, 0x1.48dc10fa920a1p+0,
    0x1.494e1e192aed2p+0, 0x1.49c052c5916c4p+0,
    0x1.4a32af0d7d3dep+0, 0x1.4aa532feaada6p+0,
    0x1.4b17dea6db7d7p+0, 0x1.4b8ab213d5283p+0,
    0x1.4bfdad5362a27p+0, 0x1.4c70d073537cap+0,
    0x1.4ce41b817c114p+0, 0x1.4d578e8bb586bp+0,
    0x1.4dcb299fddd0dp+0, 0x1.4e3eeccbd7b2ap+0,
    0x1.4eb2d81d8abffp+0, 0x1.4f26eba2e35f0p+0,
    0x1.4f9b2769d2ca7p+0, 0x1.500f8b804f127p+0,
    0x1.508417f4531eep+0, 0x1.50f8ccd3deb0dp+0,
    0x1.516daa2cf6642p+0, 0x1.51e2b00da3b14p+0,
    0x1.5257de83f4eefp+0, 0x1.52cd359dfd53dp+0,
    0x1.5342b569d4f82p+0, 0x1.53b85df598d78p+0,
    0x1.542e2f4f6ad27p+0, 0x1.54a4298571b06p+0,
    0x1.551a4ca5d920fp+0, 0x1.559098bed1bdfp+0,
    0x1.56070dde910d2p+0, 0x1.567dac1351819p+0,
    0x1.56f4736b527dap+0, 0x1.576b63f4d854cp+0,
    0x1.57e27dbe2c4cfp+0, 0x1.5859c0d59ca07p+0,
    0x1.58d12d497c7fdp+0, 0x1.5948c32824135p+0,
    0x1.59c0827ff07ccp+0, 0x1.5a386b5f43d92p+0,
    0x1.5ab07dd485429p+0, 0x1.5b28b9ee20d1ep+0,
    0x1.5ba11fba87a03p+0, 0x1.5c19af482fc8fp+0,
    0x1.5c9268a5946b7p+0, 0x1.5d0b4be135accp+0,
    0x1.5d84590998b93p+0, 0x1.5dfd902d47c65p+0,
    0x1.5e76f15ad2148p+0, 0x1.5ef07ca0cbf0fp+0,
    0x1.5f6a320dceb71p+0, 0x1.5fe411b078d26p+0,
    0x1.605e1b976dc09p+0, 0x1.60d84fd15612ap+0,
    0x1.6152ae6cdf6f4p+0, 0x1.61cd3778bc944p+0,
    0x1.6247eb03a5585p+0, 0x1.62c2c91c56acdp+0,
    0x1.633dd1d1929fdp+0, 0x1.63b90532205d8p+0,
    0x1.6434634ccc320p+0, 0x1.64afec30678b7p+0,
    0x1.652b9febc8fb7p+0, 0x1.65a77e8dcc390p+0,
    0x1.6623882552225p+0, 0x1.669fbcc140be7p+0,
    0x1.671c1c70833f6p+0, 0x1.6798a7420a036p+0,
    0x1.68155d44ca973p+0, 0x1.68923e87bfb7ap+0,
    0x1.690f4b19e9538p+0, 0x1.698c830a4c8d4p+0,
    0x1.6a09e667f3bcdp+0, 0x1.6a877541ee718p+0,
    0x1.6b052fa75173ep+0, 0x1.6b8315a736c75p+0,
    0x1.6c012750bdabfp+0, 0x1.6c7f64b30aa09p+0,
    0x1.6cfdcddd47645p+0, 0x1.6d7c62dea2f8ap+0,
    0x1.6dfb23c651a2fp+0, 0x1.6e7a10a38cee8p+0,
    0x1.6ef9298593ae5p+0, 0x1.6f786e7ba9fefp+0,
    0x1.6ff7df9519484p+0, 0x1.70777ce1303f6p+0,
    0x1.70f7466f42e87p+0, 0x1.71773c4eaa988p+0,
    0x1.71f75e8ec5f74p+0, 0x1.7277ad3ef9011p+0,
    0x1.72f8286ead08ap+0, 0x1.7378d02d50b8fp+0,
    0x1.73f9a48a58174p+0, 0x1.747aa5953c849p+0,
    0x1.74fbd35d7cbfdp+0, 0x1.757d2df29ce7cp+0,
    0x1.75feb564267c9p+0, 0x1.768069c1a861dp+0,
    0x1.77024b1ab6e09p+0, 0x1.7784597eeba8fp+0,
    0x1.780694fde5d3fp+0, 0x1.7888fda749e5dp+0,
    0x1.790b938ac1cf6p+0, 0x1.798e56b7fcf03p+0,
    0x1.7a11473eb0187p+0, 0x1.7a94652e958aap+0,
    0x1.7b17b0976cfdbp+0, 0x1.7b9b2988fb9ecp+0,
    0x1.7c1ed0130c132p+0, 0x1.7ca2a4456e7a3p+0,
    0x1.7d26a62ff86f0p+0, 0x1.7daad5e2850acp+0,
    0x1.7e2f336cf4e62p+0, 0x1.7eb3bedf2e1b9p+0,
    0x1.7f3878491c491p+0, 0x1.7fbd5fbab091fp+0,
    0x1.80427543e1a12p+0, 0x1.80c7b8f4abaa9p+0,
    0x1.814d2add106d9p+0, 0x1.81d2cb0d1736ap+0,
    0x1.82589994cce13p+0, 0x1.82de968443d9ap+0,
    0x1.8364c1eb941f7p+0, 0x1.83eb1bdadb46dp+0,
    0x1.8471a4623c7adp+0, 0x1.84f85b91e07f1p+0,
    0x1.857f4179f5b21p+0, 0x1.8606562ab00ecp+0,
    0x1.868d99b4492edp+0, 0x1.87150c27004c2p+0,
    0x1.879cad931a436p+0, 0x1.88247e08e1957p+0,
    0x1.88ac7d98a6699p+0, 0x1.8934ac52be8f7p+0,
    0x1.89bd0a478580fp+0, 0x1.8a4597875c644p+0,
    0x1.8ace5422aa0dbp+0, 0x1.8b574029db01ep+0,
    0x1.8be05bad61778p+0, 0x1.8c69a6bdb5598p+0,
    0x1.8cf3216b5448cp+0, 0x1.8d7ccbc6c19e6p+0,
    0x1.8e06a5e0866d9p+0, 0x1.8e90afc931857p+0,
    0x1.8f1ae99157736p+0, 0x1.8fa553499284bp+0,
    0x1.902fed0282c8ap+0, 0x1.90bab6ccce12cp+0,
    0x1.9145b0b91ffc6p+0, 0x1.91d0dad829e70p+0,
    0x1.925c353aa2fe2p+0, 0x1.92e7bff148396p+0,
    0x1.93737b0cdc5e5p+0, 0x1.93ff669e2802bp+0,
    0x1.948b82b5f98e5p+0, 0x1.9517cf65253d1p+0,
    0x1.95a44cbc8520fp+0, 0x1.9630faccf9243p+0,
    0x1.96bdd9a7670b3p+0, 0x1.974ae95cba768p+0,
    0x1.97d829fde4e50p+0, 0x1.98659b9bddb5bp+0,
    0x1.98f33e47a22a2p+0, 0x1.9981121235681p+0,
    0x1.9a0f170ca07bap+0, 0x1.9a9d4d47f2598p+0,
    0x1.9b2bb4d53fe0dp+0, 0x1.9bba4dc5a3dd3p+0,
    0x1.9c49182a3f090p+0, 0x1.9cd81414380f2p+0,
    0x1.9d674194bb8d5p+0, 0x1.9df6a0bcfc15ep+0,
    0x1.9e86319e32323p+0, 0x1.9f15f4499c647p+0,
    0x1.9fa5e8d07f29ep+0, 0x1.a0360f4424fcbp+0,
    0x1.a0c667b5de565p+0, 0x1.a156f23701b15p+0,
    0x1.a1e7aed8eb8bbp+0, 0x1.a2789dacfe68cp+0,
    0x1.a309bec4a2d33p+0, 0x1.a39b1231475f7p+0,
    0x1.a42c980460ad8p+0, 0x1.a4be504f696b1p+0,
    0x1.a5503b23e255dp+0, 0x1.a5e25893523d4p+0,
    0x1.a674a8af46052p+0, 0x1.a7072b8950a73p+0,
    0x1.a799e1330b358p+0, 0x1.a82cc9be14dcap+0,
    0x1.a8bfe53c12e59p+0, 0x1.a95333beb0b7ep+0,
    0x1.a9e6b5579fdbfp+0, 0x1.aa7a6a1897fd2p+0,
    0x1.ab0e521356ebap+0, 0x1.aba26d59a09eep+0,
    0x1.ac36bbfd3f37ap+0, 0x1.accb3e100301ep+0,
    0x1.ad5ff3a3c2774p+0, 0x1.adf4dcca5a413p+0,
    0x1.ae89f995ad3adp+0, 0x1.af1f4a17a4735p+0,
    0x1.afb4ce622f2ffp+0, 0x1.b04a868742ee4p+0,
    0x1.b0e07298db666p+0, 0x1.b17692a8fa8cdp+0,
    0x1.b20ce6c9a8952p+0, 0x1.b2a36f0cf3f3ap+0,
    0x1.b33a2b84f15fbp+0, 0x1.b3d11c43bbd62p+0,
    0x1.b468415b749b1p+0, 0x1.b4ff9ade433c6p+0,
    0x1.b59728de5593ap+0, 0x1.b62eeb6ddfc87p+0,
    0x1.b6c6e29f1c52ap+0, 0x1.b75f0e844bfc6p+0,
    0x1.b7f76f2fb5e47p+0, 0x1.b89004b3a7804p+0,
    0x1.b928cf22749e4p+0, 0x1.b9c1ce8e77680p+0,
    0x1.ba5b030a1064ap+0, 0x1.baf46ca7a67a7p+0,
    0x1.bb8e0b79a6f1fp+0, 0x1.bc27df9285775p+0,
    0x1.bcc1e904bc1d2p+0, 0x1.bd5c27e2cb5e5p+0,
    0x1.bdf69c3f3a207p+0, 0x1.be91462c95b60p+0,
    0x1.bf2c25bd71e09p+0, 0x1.bfc73b0468d30p+0,
    0x1.c06286141b33dp+0, 0x1.c0fe06ff301f4p+0,
    0x1.c199bdd85529cp+0, 0x1.c235aab23e61ep+0,
    0x1.c2d1cd9fa652cp+0, 0x1.c36e26b34e065p+0,
    0x1.c40ab5fffd07ap+0, 0x1.c4a77b9881650p+0,
    0x1.c544778fafb22p+0, 0x1.c5e1a9f8630adp+0,
    0x1.c67f12e57d14bp+0, 0x1.c71cb269e601fp+0,
    0x1.c7ba88988c933p+0, 0x1.c8589584661a1p+0,
    0x1.c8f6d9406e7b5p+0, 0x1.c99553dfa8313p+0,
    0x1.ca3405751c4dbp+0, 0x1.cad2ee13da7cbp+0,
    0x1.cb720dcef9069p+0, 0x1.cc1164b994d23p+0,
    0x1.ccb0f2e6d1675p+0, 0x1.cd50b869d8f0fp+0,
    0x1.cdf0b555dc3fap+0, 0x1.ce90e9be12cb9p+0,
    0x1.cf3155b5bab74p+0, 0x1.cfd1f95018d17p+0,
    0x1.d072d4a07897cp+0, 0x1.d113e7ba2c38cp+0,
    0x1.d1b532b08c968p+0, 0x1.d256b596f948cp+0,
    0x1.d2f87080d89f2p+0, 0x1.d39a638197a3cp+0,
    0x1.d43c8eacaa1d6p+0, 0x1.d4def2158a91fp+0,
    0x1.d5818dcfba487p+0, 0x1.d62461eec14bep+0,
    0x1.d6c76e862e6d3p+0, 0x1.d76ab3a99745bp+0,
    0x1.d80e316c98398p+0, 0x1.d8b1e7e2d479dp+0,
    0x1.d955d71ff6075p+0, 0x1.d9f9ff37adb4ap+0,
    0x1.da9e603db3285p+0, 0x1.db42fa45c4dfdp+0,
    0x1.dbe7cd63a8315p+0, 0x1.dc8cd9ab294e4p+0,
    0x1.dd321f301b460p+0, 0x1.ddd79e065807dp+0,
    0x1.de7d5641c0658p+0, 0x1.df2347f63c159p+0,
    0x1.dfc97337b9b5fp+0, 0x1.e06fd81a2ece1p+0,
    0x1.e11676b197d17p+0, 0x1.e1bd4f11f8220p+0,
    0x1.e264614f5a129p+0, 0x1.e30bad7dcee90p+0,
    0x1.e3b333b16ee12p+0, 0x1.e45af3fe592e8p+0,
    0x1.e502ee78b3ff6p+0, 0x1.e5ab2334ac7eep+0,
    0x1.e653924676d76p+0, 0x1.e6fc3bc24e350p+0,
    0x1.e7a51fbc74c83p+0, 0x1.e84e3e4933c7ep+0,
    0x1.e8f7977cdb740p+0, 0x1.e9a12b6bc3181p+0,
    0x1.ea4afa2a490dap+0, 0x1.eaf503ccd2be5p+0,
    0x1.eb9f4867cca6ep+0, 0x1.ec49c80faa594p+0,
    0x1.ecf482d8e67f1p+0, 0x1.ed9f78d802dc2p+0,
    0x1.ee4aaa2188510p+0, 0x1.eef616ca06dd6p+0,
    0x1.efa1bee615a27p+0, 0x1.f04da28a52e59p+0,
    0x1.f0f9c1cb6412ap+0, 0x1.f1a61cbdf5be7p+0,
    0x1.f252b376bba97p+0, 0x1.f2ff860a70c22p+0,
    0x1.f3ac948dd7274p+0, 0x1.f459df15b82acp+0,
    0x1.f50765b6e4540p+0, 0x1.f5b5288633625p+0,
    0x1.f6632798844f8p+0, 0x1.f7116302bd526p+0,
    0x1.f7bfdad9cbe14p+0, 0x1.f86e8f32a4b45p+0,
    0x1.f91d802243c89p+0, 0x1.f9ccadbdac61dp+0,
    0x1.fa7c1819e90d8p+0, 0x1.fb2bbf4c0ba54p+0,
    0x1.fbdba3692d514p+0, 0x1.fc8bc4866e8adp+0,
    0x1.fd3c22b8f71f1p+0, 0x1.fdecbe15f6314p+0,
    0x1.fe9d96b2a23d9p+0, 0x1.ff4eaca4391b6p+0,
};

// exp(x): with k = rint(512 x / ln 2), x = k ln2 / 512 + r, |r| <= ln2 / 1024,
// and exp(x) = 2^(k >> 9) 2^((k & 511) / 512) exp(r).  The reduction is Cody
// and Waite's with ln2 / 512 split in two (the high part holds 32 significant
// bits, so k times it is exact for |k| < 2^21); the table holds 2^(j/512)
// rounded; exp(r) - 1 is its series to r^4 (truncation < 2e-18 relative).
// The result is t (1 + (exp(r) - 1)) scaled with v_ldexp (overflow gives
// inf, underflow 0): about one ulp.
__device__ __forceinline__ double qexp(double x) {
    constexpr double k512Log2e = 512.0 * 1.4426950408889634;
    constexpr double kLn2Hi = 6.93147180369123816490e-01 / 512.0;  // 0x3FE62E42FEE00000 / 2^9
    constexpr double kLn2Lo = 1.90821492927058770002e-10 / 512.0;  // (ln 2 - its high part) / 2^9
    const double k = __builtin_rint(x * k512Log2e);
    double r = fma_(-k, kLn2Hi, x);
    r = fma_(-k, kLn2Lo, r);
    const int ki = (int)k;
    const double t = kMathTab[512 + (ki & 511)];
    double p = fma_(1.0 / 24.0, r, 1.0 / 6.0);
    p = fma_(p, r, 0.5);
    p = fma_(p, r, 1.0);
    const double em1 = p * r;
    return __builtin_amdgcn_ldexp(fma_(t, em1, t), ki >> 9);
}

// ln(x) for x > 0 (NaN for x <= 0, NaN or +inf).  x = m 2^e with m in
// [1/2, 1); the table splits [1/2, 1) into 256 intervals of width 1/512 and
// holds, for each interval's midpoint c_j, ic_j = 1/c_j rounded and
// -ln(ic_j); with r = m ic_j - 1 (one FMA, |r| <= 1/512), ln x = e ln 2 -
// ln(ic_j) + ln(1 + r), and ln(1 + r) is its series to r^5 (truncation
// below 1e-17).  The absolute error is a few 1e-17 plus one rounding of the
// result, which is what exp(a ln x) needs; the table read is one 16-byte
// load.
__device__ __forceinline__ double qlog(double x) {
    constexpr double kLn2Hi = 6.93147180369123816490e-01;
    constexpr double kLn2Lo = 1.90821492927058770002e-10;
    const double m = __builtin_amdgcn_frexp_mant(x);
    const double e = (double)__builtin_amdgcn_frexp_exp(x);
    // j = floor((m - 1/2) 512) is the top 8 bits of m's fraction field, bits
    // 12..19 of its high word (one bit-field extract; any input, NaN and inf
    // included, gives a j in 0..255)
    const int j = (int)__builtin_amdgcn_ubfe((uint32_t)__double2hiint(m), 12, 8);
    const double ic = kMathTab[2 * j], nl = kMathTab[2 * j + 1];
    const double r = fma_(m, ic, -1.0);
    // ln(1 + r) = r - r^2 (1/2 - r/3 + r^2/4 - r^3/5)
    double q = -1.0 / 5.0;
    q = fma_(q, r, 1.0 / 4.0);
    q = fma_(q, r, -1.0 / 3.0);
    q = fma_(q, r, 0.5);
    const double lr = fma_(-r * r, q, r);
    const double res = fma_(e, kLn2Hi, nl + fma_(e, kLn2Lo, lr));
    // NaN unless x is positive and finite: only the high word is replaced
    // (0x7ff80000 there makes a quiet NaN whatever the low word holds)
    const bool ok = x > 0.0 && x < __builtin_inf();
    return __hiloint2double(ok ? __double2hiint(res) : 0x7ff80000, __double2loint(res));
}

// ------------------------------------------------- FP64 atan2 and sincos
// For the complex sector integrand (F - i delta)^p = |.|^p e^{i p arg}: the
// phase needs arg(F - i delta) = atan2(-delta, F) and the sine and cosine of
// p times it, a bounded argument.  Both are branch-free; their polynomials
// are Chebyshev interpolants (near-minimax) in 50-digit arithmetic, each
// below 3.2e-17 in its reduced range, written by make_math_tables.py --poly.

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
