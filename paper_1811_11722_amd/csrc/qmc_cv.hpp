// Learned control variate: a separable rank-R model on shifted Legendre
// polynomials,
//   g(z) = sum_r c_r prod_i h_{r,i}(z_i),  h_{r,i}(z) = sum_k W[r,i,k] P~_k(z),
// P~_k(z) = sqrt(2k+1) P_k(2z - 1) orthonormal on [0,1], so that
// int g = sum_r c_r prod_i W[r,i,0] exactly.  The estimate is
// int g + Qbar[f - g]: the residual f - g goes through the same periodising
// transform and lattice rule, so the estimator stays unbiased and the m
// shifts judge its error exactly as for f.
//
// Device code: the Legendre basis, the FP64 model evaluation used inside the
// lattice kernel, and the kernel that samples the training lattice.
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

// g(z) in FP64 for one point.  ws holds W[r,i,k] * sqrt(2k+1) row-major
// (R, D, K); c holds c_r.  Both are wave-uniform (scalar loads).
template <int D, int R, int K>
__device__ __forceinline__ double cv_model(const double *__restrict__ c, const double *__restrict__ ws,
                                           const double (&z)[D]) {
    double prod[R];
#pragma unroll
    for (int r = 0; r < R; ++r) prod[r] = c[r];
    // one dimension at a time (a rolled loop keeps a single basis live)
#pragma unroll 1
    for (int i = 0; i < D; ++i) {
        double p[K];
        legendre_raw<K, double>(z[i], p);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double *w = ws + (r * D + i) * K;
            double h = w[K - 1] * p[K - 1];
#pragma unroll
            for (int k = K - 2; k >= 0; --k) h = fma_(w[k], p[k], h);
            prod[r] *= h;
        }
    }
    double g = prod[0];
#pragma unroll
    for (int r = 1; r < R; ++r) g += prod[r];
    return g;
}

// Residual family: part 0 is the base integrand fhat, part 1 is
// fhat - J g(z), both without the transform constant (applied to the sums).
// cv points at [c (R), ws (R*D*K)] inside the parameter blob at word CvOff.
template <class Base, int R, int K, int CvOff>
struct FamCvResidual {
    static constexpr int NP = 2;
    static_assert(Base::NP == 1, "control variate for real integrands");
    template <class Tr, int D, int T>
    __device__ static void eval(const double *__restrict__ p, const double (&x)[T][D], double (&v)[T][NP]) {
        double fb[T][1];
        Base::template eval<Tr, D, T>(p, x, fb);
        double z[T][D], jac[T];
        apply_transform<Tr, D, T>(x, z, jac);
        const double *cv = p + CvOff;
        asm volatile("" : "+s"(cv));  // weights are re-read per point, not held in registers
#pragma unroll
        for (int k = 0; k < T; ++k) {
            const double g = cv_model<D, R, K>(cv, cv + R, z[k]);
            v[k][0] = fb[k][0];
            v[k][1] = Tr::kJac ? fma_(-jac[k], g, fb[k][0]) : fb[k][0] - g;
        }
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
    float *yw;            // (n) fhat = J f(z): the weighted target
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
    double v[1][1], z[1][D], jac[1];
    Fam::template eval<Tr, D, 1>(a.params, x, v);
    apply_transform<Tr, D, 1>(x, z, jac);
#pragma unroll
    for (int i = 0; i < D; ++i) a.z[(size_t)j * D + i] = (float)z[0][i];
    a.sw[j] = (float)jac[0];
    a.yw[j] = (float)v[0][0];
}

}  // namespace qmc
