// Learned control variate: a separable rank-R model on shifted Legendre
// polynomials,
//   g(z) = sum_r c_r prod_i h_{r,i}(z_i),  h_{r,i}(z) = sum_k W[r,i,k] P~_k(z),
// P~_k(z) = sqrt(2k+1) P_k(2z - 1) orthonormal on [0,1], so that
// int g = sum_r c_r prod_i W[r,i,0] exactly.  The estimate is
// int g + Qbar[f - g]: the residual f - g goes through the same periodising
// transform and lattice rule, so the estimator stays unbiased and the m
// shifts judge its error exactly as for f.
//
// Device code: the Legendre basis, the residual family whose FP64 model
// evaluation runs inside the lattice kernel, and the kernel that samples the
// training lattice.
#pragma once

#include "qmc_kernels.hpp"

namespace qmc {

// P_k(t), k < K, for t = 2z - 1 by Bonnet's recurrence
// (k+1) P_{k+1} = (2k+1) t P_k - k P_{k-1}.  The sqrt(2k+1) normalisation is
// folded into the model weights by the host.
template <int K, class F>
__device__ __forceinline__ void legendre_raw(F z, F (&p)[K]) {
    const F t = z + z - F(1);
    p[0] = F(1);
    if constexpr (K > 1) p[1] = t;
#pragma unroll
    for (int k = 1; k + 1 < K; ++k) {
        const F a = F(2 * k + 1) / F(k + 1), b = F(k) / F(k + 1);
        p[k + 1] = a * (t * p[k]) - b * p[k - 1];
    }
}

typedef double cv_d4 __attribute__((ext_vector_type(4)));

// One of four register values by lane group.  The values pass through an
// empty asm statement so the compiler keeps the selects on registers rather
// than turning them into an indexed load from a private array.
__device__ __forceinline__ double cv_pick4(double a, double b, double c, double d, bool s1, bool s2, bool s3) {
    asm volatile("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d));
    double t = a;
    t = s1 ? b : t;
    t = s2 ? c : t;
    t = s3 ? d : t;
    return t;
}

// Residual family.  For a real base integrand the parts are fhat and
// fhat - J g; for a complex one (Re fhat, Im fhat, Re fhat - J g_0,
// Im fhat - J g_1) with one model per component.  The transform constant is
// applied to the sums.
//
// g is evaluated for the wave's 64 points at once with FP64 matrix
// instructions.  For dimension i, H_i[r][pt] = sum_k W'[r,i,k] P_k(z_pt,i) is
// a (R x K) by (K x 64) product, done as 16 x 16 x 4 tiles by
// v_mfma_f64_16x16x4f64 (A = weights: lane l holds row l % 16, inner index
// l / 16; B = Legendre values: lane l holds column l % 16, inner index
// l / 16; output element e of lane l is row 4e + l / 16, column l % 16).
// The product over dimensions is taken elementwise on the output tiles and
// the sum over ranks by two cross-lane adds.  Each lane runs the Legendre
// recurrence of its own point once per dimension; the values reach the B
// layout (the 4 points a lane's columns stand for, one per 16-point block)
// through the wave's LDS rows.
//
// The weights sit in fragment order at word CvOff of the parameter blob,
// model after model (D * RB * KS * 64 words each): fragment
// ((i * RB + rb) * KS + ks) holds, for lane l,
// W[r = 16 rb + l % 16, i, k = 4 ks + l / 16] * sqrt(2k + 1), times c_r for
// i = 0, and 0 for r >= R or k >= K.
template <class Base, int R, int K, int CvOff>
struct FamCvResidual {
    static constexpr int NM = Base::NP;  // one model per component
    static constexpr int NP = 2 * NM;
    static constexpr bool kWaveUniform = true;  // the whole wave runs the matrix instructions
    static constexpr int RB = (R + 15) / 16, KS = (K + 3) / 4;

    // g of the lane's own point for the model whose fragments start at w
    template <int D>
    __device__ static double model(const double *__restrict__ w, const double *zw, uint32_t lane) {
        constexpr int NPK = 4 * KS, LP = NPK + 1;  // Legendre values per point, padded LDS row
        __shared__ double lvs[kBlock / kWave][kWave * LP];
        double *lw = lvs[threadIdx.x / kWave];
        const uint32_t grp = lane >> 4, col = lane & 15;
        const bool s1 = grp == 1, s2 = grp == 2, s3 = grp == 3;
        cv_d4 prod[RB][4];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) prod[rb][pb] = cv_d4{1.0, 1.0, 1.0, 1.0};
        double wa[RB][KS];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) wa[rb][ks] = w[(rb * KS + ks) * kWave];
        // the lane's own point's Legendre values of dimension i, through the
        // wave's LDS rows to the B layout (a wave's LDS accesses complete in
        // order)
        auto legendre_b = [&](int i, double (&bk)[4][KS]) {
            double pk[NPK];
            legendre_raw<NPK, double>(zw[lane * D + i], pk);
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int k = 0; k < NPK; ++k) lw[lane * LP + k] = pk[k];
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int pb = 0; pb < 4; ++pb)
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) bk[pb][ks] = lw[(16 * pb + col) * LP + 4 * ks + grp];
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        };
        double bk[4][KS];
        legendre_b(0, bk);
        // software-pipelined over the dimensions: dimension i's matrix
        // instructions are issued first, and the next dimension's Legendre
        // values (VALU and LDS work, independent of them) are formed while
        // they run
#pragma unroll 1
        for (int i = 0; i < D; ++i) {
            // weights of the next dimension, loaded while this one computes
            const int inext = i + 1 < D ? i + 1 : i;
            double wn[RB][KS];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) wn[rb][ks] = w[((inext * RB + rb) * KS + ks) * kWave];
            // RB x 4 independent accumulation chains, interleaved over ks
            cv_d4 acc[RB][4];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int pb = 0; pb < 4; ++pb) acc[rb][pb] = cv_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int pb = 0; pb < 4; ++pb)
                        acc[rb][pb] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[rb][ks], bk[pb][ks], acc[rb][pb], 0, 0, 0);
            if (i + 1 < D) legendre_b(i + 1, bk);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int pb = 0; pb < 4; ++pb) prod[rb][pb] *= acc[rb][pb];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) wa[rb][ks] = wn[rb][ks];
        }
        double s[4];
#pragma unroll
        for (int pb = 0; pb < 4; ++pb) {
            double t = 0.0;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) t += (prod[rb][pb][0] + prod[rb][pb][1]) + (prod[rb][pb][2] + prod[rb][pb][3]);
            t += __shfl_xor(t, 16);
            t += __shfl_xor(t, 32);
            s[pb] = t;
        }
        // the lane's own point is column l % 16 of block l / 16
        return cv_pick4(s[0], s[1], s[2], s[3], s1, s2, s3);
    }

    template <class Tr, int D, int T>
    __device__ static void eval(const double *__restrict__ p, const double (&x)[T][D], double (&v)[T][NP]) {
        static_assert(T == 1, "one shift per thread");
        double fb[1][NM];
        Base::template eval<Tr, D, 1>(p, x, fb);
        double z[1][D], jac[1];
        apply_transform<Tr, D, 1>(x, z, jac);
        const uint32_t lane = threadIdx.x & (kWave - 1);
        // the wave's z values go through LDS (each wave uses its own rows;
        // a wave's LDS accesses complete in order)
        __shared__ double zs[kBlock * D];
        double *zw = zs + (size_t)(threadIdx.x - lane) * D;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < D; ++i) zw[lane * D + i] = z[0][i];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int mi = 0; mi < NM; ++mi) {
            const double g = model<D>(p + CvOff + (size_t)mi * D * RB * KS * kWave + lane, zw, lane);
            v[0][mi] = fb[0][mi];
            v[0][NM + mi] = Tr::kJac ? fma_(-jac[0], g, fb[0][mi]) : fb[0][mi] - g;
        }
        __builtin_amdgcn_wave_barrier();
    }
};

struct CvSampleArgs {
    uint32_t n, d;
    double inv_n;
    const uint32_t *g;
    const double *shift;  // one shift, d values
    const double *params;
    float *z;             // (n, d) transformed coordinates
    float *sw;            // (n) Jacobian J: square root of the loss weight
    float *yw;            // (n) fhat = J f(z): the weighted target (component `part`)
    uint32_t part;        // 0 real part, 1 imaginary part of a complex integrand
    double tscale;        // the transform's constant (the functors leave it out of J and fhat)
};

// Points of the training lattice {j g / n + shift}, j < n: z(x), J(x) and
// fhat(x) for the model fit, which minimises sum_j (fhat_j - J_j g(z_j))^2.
template <class Fam, class Tr, int D>
__global__ __launch_bounds__(kBlock) void k_cv_sample(const CvSampleArgs a) {
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= a.n) return;
    double x[1][D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const uint32_t idx = mulmod(j, a.g[i], a.n, a.inv_n);
        x[0][i] = fract((double)idx * a.inv_n + a.shift[i]);
    }
    double v[1][Fam::NP], z[1][D], jac[1];
    Fam::template eval<Tr, D, 1>(a.params, x, v);
    apply_transform<Tr, D, 1>(x, z, jac);
#pragma unroll
    for (int i = 0; i < D; ++i) a.z[(size_t)j * D + i] = (float)z[0][i];
    a.sw[j] = (float)(jac[0] * a.tscale);
    a.yw[j] = (float)((Fam::NP == 1 || a.part == 0 ? v[0][0] : v[0][Fam::NP - 1]) * a.tscale);
}

}  // namespace qmc
