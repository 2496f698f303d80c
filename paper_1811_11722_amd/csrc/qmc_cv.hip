// Control-variate training and estimation (C ABI in qmc.h).
//
// Training fits the separable Legendre model of qmc_cv.hpp to samples of the
// integrand on an independent training lattice (one shift), minimising
//   L(W) = sum_j (yw_j - sw_j g(z_j))^2      (yw = fhat = J f, sw = J)
// by alternating least squares: with every factor but dimension i fixed the
// model is linear in W[., i, .], so each step solves the normal equations
//   (A^T A + lambda I) w = A^T y,  A_j = rho_j (x) phi_j,
// rho_j[r] = sw_j prod_{i' != i} h_{r,i'}(z_{j,i'}),  phi_j[k] = P~_k(z_{j,i}).
// A^T A has Kronecker structure: its (k, k') block is
//   sum_j phi_j[k] phi_j[k'] rho_j rho_j^T,
// a rank-N sum of R x R outer products, which k_cv_gram accumulates with
// BF16 MFMA (v_mfma_f32_32x32x16_bf16: 32 x 32 tiles, 16 points per
// instruction, FP32 accumulation).  The per-split tiles are added in a fixed
// order in FP64 and the (R K) x (R K) system is solved in FP64 by a Cholesky
// factorisation on the device.  Features and factors are FP32 during
// training; the trained model is evaluated in FP64 inside the estimator.
#include <cmath>
#include <cstring>

#include "qmc_cv.hpp"
#include "qmc_runtime.hpp"

namespace qmc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------- kernels
struct CvRhoArgs {
    uint32_t n, d, i;       // points, dimension, the dimension being solved
    const float *z, *sw;    // (n, d), (n)
    const float *ws;        // W * sqrt(2k+1), (R, d, K)
    float *rho;             // (n, R): sw prod_{i' != i} h_{r,i'}
    float *phi;             // (n, K): P~_k(z_i) (normalised)
};

template <int R, int K>
__global__ __launch_bounds__(kBlock) void k_cv_rho(const CvRhoArgs a) {
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= a.n) return;
    float prod[R];
    const float s = a.sw[j];
#pragma unroll
    for (int r = 0; r < R; ++r) prod[r] = s;
    for (uint32_t i = 0; i < a.d; ++i) {
        float p[K];
        legendre_raw<K, float>(a.z[(size_t)j * a.d + i], p);
        if (i == a.i) {
#pragma unroll
            for (int k = 0; k < K; ++k) a.phi[(size_t)j * K + k] = p[k] * sqrtf((float)(2 * k + 1));
            continue;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float *w = a.ws + ((size_t)r * a.d + i) * K;
            float h = w[K - 1] * p[K - 1];
#pragma unroll
            for (int k = K - 2; k >= 0; --k) h = __builtin_fmaf(w[k], p[k], h);
            prod[r] *= h;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) a.rho[(size_t)j * R + r] = prod[r];
}

// One wave job: `count` Gram blocks (k, k0 + q) for row block rb and column
// block cb of rho (type 0), or the right-hand side block rb (type 1).
struct CvJob {
    uint32_t type, k, k0, count, rb, cb, slot0, pad;
};
constexpr int kMaxJobCount = 4;

struct CvGramArgs {
    uint32_t n, R, K;
    uint32_t job0, njobs, nslots, splits;  // jobs job0 .. njobs-1 run
    float inv_scale;        // 1 / target scale
    const float *rho, *phi, *yw;
    const CvJob *jobs;
    float *partial;         // (splits, nslots, 32, 32)
};

__global__ __launch_bounds__(kBlock) void k_cv_gram(const CvGramArgs a) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t jid = a.job0 + blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (jid >= a.njobs) return;  // whole wave leaves together
    const CvJob job = a.jobs[jid];
    const uint32_t half = lane >> 5, col = lane & 31;
    const uint32_t ra = job.rb * 32 + col;  // rho column held as an A row
    const uint32_t rbcol = job.cb * 32 + col;
    const uint32_t j_begin = (uint32_t)((uint64_t)a.n * blockIdx.y / a.splits);
    const uint32_t j_end = (uint32_t)((uint64_t)a.n * (blockIdx.y + 1) / a.splits);
    f32x16 acc[kMaxJobCount];
#pragma unroll
    for (int q = 0; q < kMaxJobCount; ++q)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[q][e] = 0.0f;

    // Every feature a_j[(r, k)] = rho_j[r] phi_j[k] is rounded to BF16 once,
    // the same way in both operands, so the assembled matrix is exactly
    // sum_j a~_j a~_j^T (positive semi-definite up to FP32 accumulation).
    for (uint32_t base = j_begin; base < j_end; base += 16) {
        float rv[8], s[8];
        bf16x8 b, av;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t j = base + 8 * half + e;
            const bool ok = j < j_end;
            rv[e] = (ok && ra < a.R) ? a.rho[(size_t)j * a.R + ra] : 0.0f;
            if (job.type == 0) {
                s[e] = (ok && rbcol < a.R) ? a.rho[(size_t)j * a.R + rbcol] : 0.0f;
                const float pk = ok ? a.phi[(size_t)j * a.K + job.k] : 0.0f;
                av[e] = (__bf16)(rv[e] * pk);
            } else {
                const float ph = (ok && col < a.K) ? a.phi[(size_t)j * a.K + col] : 0.0f;
                b[e] = (__bf16)ph;
                s[e] = ok ? a.yw[j] * a.inv_scale : 0.0f;
            }
        }
        if (job.type == 0) {
#pragma unroll
            for (int q = 0; q < kMaxJobCount; ++q) {
                if ((uint32_t)q < job.count) {
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const uint32_t j = base + 8 * half + e;
                        const float pk2 = j < j_end ? a.phi[(size_t)j * a.K + job.k0 + q] : 0.0f;
                        b[e] = (__bf16)(s[e] * pk2);
                    }
                    acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b, acc[q], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) av[e] = (__bf16)(rv[e] * s[e]);
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b, acc[0], 0, 0, 0);
        }
    }
    // accumulator layout of the 32x32 tile: register e of lane l holds
    // row 8 (e / 4) + 4 (l / 32) + e % 4, column l % 32
    const uint32_t nq = job.type == 0 ? job.count : 1;
    for (uint32_t q = 0; q < nq; ++q) {
        float *out = a.partial + (((size_t)blockIdx.y * a.nslots + job.slot0 + q) << 10);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const uint32_t row = 8 * (e / 4) + 4 * half + (e % 4);
            out[row * 32 + col] = acc[q][e];
        }
    }
}

// sum the per-split tiles of slots first .. nslots-1 in split order, in FP64
__global__ __launch_bounds__(kBlock) void k_cv_reduce(const float *partial, uint32_t splits, uint32_t nslots,
                                                     uint32_t first, double *out) {
    const uint32_t t = (first << 10) + blockIdx.x * kBlock + threadIdx.x;
    const uint32_t total = nslots << 10;
    if (t >= total) return;
    double s = 0.0;
    for (uint32_t sp = 0; sp < splits; ++sp) s += (double)partial[(size_t)sp * total + t];
    out[t] = s;
}

// residual of the current fit of dimension i in FP32 arithmetic:
//   e_j = yw_j / scale - sum_{r,k} rho_j[r] phi_j[k] W[r,i,k]
// (the right-hand side of a refinement step is A^T e)
template <int R, int K>
__global__ __launch_bounds__(kBlock) void k_cv_resid(uint32_t n, uint32_t d, uint32_t i, const float *rho,
                                                    const float *phi, const float *yw, float inv_scale,
                                                    const double *w64, float *e) {
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    float ph[K];
#pragma unroll
    for (int k = 0; k < K; ++k) ph[k] = phi[(size_t)j * K + k];
    float g = 0.0f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double *w = w64 + ((size_t)r * d + i) * K;
        float h = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) h = __builtin_fmaf((float)w[k], ph[k], h);
        g = __builtin_fmaf(rho[(size_t)j * R + r], h, g);
    }
    e[j] = yw[j] * inv_scale - g;
}

struct CvSolveArgs {
    uint32_t R, K, d, i, nslots_pair_base, rhs_slot0, RB;
    double ridge;           // relative to the mean diagonal
    int refine;             // 1: reuse the factor in A and add the solution to W[., i, .]
    double *lam;            // absolute ridge of the current factorisation
    const double *tiles;    // (nslots, 32, 32)
    const uint32_t *pair_slot;  // (K, K): slot of the first (rb, cb) tile of pair (min, max)
    double *A;              // (F, F) scratch, F = R K
    double *w64;            // (R, d, K) model, normalised basis
    float *ws32;            // (R, d, K) model times sqrt(2k+1)
    int *status;            // 0 ok, 1 not positive definite
};

// One workgroup solves the normal equations of dimension i.
//
// Assembly: the lower triangle of A (F x F, F = R K, row-major in HBM) is
// gathered from the Gram tiles, plus the ridge lam = ridge * trace / F.
// Factorisation: blocked right-looking Cholesky, A = L L^T in place.  Each
// panel of kPanel columns is loaded into LDS and factorised there; the
// trailing lower triangle is then updated by A -= P P^T, each thread owning
// 4 x 4 blocks.  A non-positive pivot restarts the factorisation with a 100x
// larger ridge (at most three times).  Solves: blocked forward and backward
// substitution in LDS.  A refinement call (refine = 1) reuses the factor
// left in A, solves (A + lam I) delta = A^T e - lam w and adds delta to
// W[., i, .].
constexpr uint32_t kPanel = 8;
constexpr uint32_t kMaxF = 768;  // largest R K compiled: (64, 12)

__device__ void cv_load_rhs(const CvSolveArgs &a, uint32_t F, double *y, double lam) {
    for (uint32_t u = threadIdx.x; u < F; u += blockDim.x) {
        const uint32_t r = u / a.K, k = u - r * a.K;
        double v = a.tiles[((size_t)(a.rhs_slot0 + r / 32) << 10) + (r % 32) * 32 + k];
        if (a.refine) v -= lam * a.w64[((size_t)r * a.d + a.i) * a.K + k];
        y[u] = v;
    }
}

__global__ __launch_bounds__(1024) void k_cv_solve(const CvSolveArgs a) {
    const uint32_t F = a.R * a.K, tid = threadIdx.x, nt = blockDim.x;
    __shared__ double P[(kMaxF + 4) * kPanel];  // panel rows c0..F-1 (+4 rows of padding)
    __shared__ double y[kMaxF];                 // right-hand side / solution
    __shared__ double s_ridge;
    __shared__ int s_bad;
    double *A = a.A;

    if (!a.refine) {
        double ridge = a.ridge;
        for (int attempt = 0; attempt < 4; ++attempt, ridge *= 100.0) {
            // lower triangle of the normal matrix
            for (uint32_t u = tid / 32; u < F; u += nt / 32) {
                const uint32_t r = u / a.K, k = u - r * a.K;
                for (uint32_t v = tid % 32; v <= u; v += 32) {
                    const uint32_t rp = v / a.K, kp = v - rp * a.K;
                    double g;
                    if (k <= kp) {
                        const uint32_t slot = a.pair_slot[k * a.K + kp] + (r / 32) * a.RB + (rp / 32);
                        g = a.tiles[((size_t)slot << 10) + (r % 32) * 32 + (rp % 32)];
                    } else {
                        const uint32_t slot = a.pair_slot[kp * a.K + k] + (rp / 32) * a.RB + (r / 32);
                        g = a.tiles[((size_t)slot << 10) + (rp % 32) * 32 + (r % 32)];
                    }
                    A[(size_t)u * F + v] = g;
                }
            }
            __syncthreads();
            if (tid == 0) {
                double tr = 0.0;
                for (uint32_t u = 0; u < F; ++u) tr += A[(size_t)u * F + u];
                s_ridge = ridge * tr / F + 1e-300;
                s_bad = 0;
            }
            __syncthreads();
            for (uint32_t u = tid; u < F; u += nt) A[(size_t)u * F + u] += s_ridge;
            __syncthreads();

            for (uint32_t c0 = 0; c0 < F; c0 += kPanel) {
                const uint32_t nb = min(kPanel, F - c0), rows = F - c0;
                for (uint32_t t = tid; t < rows * kPanel; t += nt) {
                    const uint32_t r = t / kPanel, q = t % kPanel;
                    P[t] = (q < nb && q <= r) ? A[(size_t)(c0 + r) * F + c0 + q] : 0.0;
                }
                __syncthreads();
                for (uint32_t q = 0; q < nb; ++q) {
                    if (tid == 0) {
                        const double piv = P[q * kPanel + q];
                        if (!(piv > 0.0)) s_bad = 1;
                        P[q * kPanel + q] = piv > 0.0 ? sqrt(piv) : 1.0;
                    }
                    __syncthreads();
                    const double inv = 1.0 / P[q * kPanel + q];
                    for (uint32_t r = q + 1 + tid; r < rows; r += nt) P[r * kPanel + q] *= inv;
                    __syncthreads();
                    for (uint32_t r = q + 1 + tid; r < rows; r += nt) {
                        const double l = P[r * kPanel + q];
                        for (uint32_t q2 = q + 1; q2 < nb && q2 <= r; ++q2)
                            P[r * kPanel + q2] -= l * P[q2 * kPanel + q];
                    }
                    __syncthreads();
                }
                for (uint32_t t = tid; t < rows * kPanel; t += nt) {
                    const uint32_t r = t / kPanel, q = t % kPanel;
                    if (q < nb && q <= r) A[(size_t)(c0 + r) * F + c0 + q] = P[t];
                }
                // trailing update of rows / columns c1..F-1
                const uint32_t c1 = c0 + nb;
                if (c1 < F) {
                    const uint32_t M = F - c1, nbk = (M + 3) / 4;
                    for (uint32_t bu = tid / 32; bu < nbk; bu += nt / 32) {
                        for (uint32_t bv = tid % 32; bv <= bu; bv += 32) {
                            double acc[4][4] = {};
                            for (uint32_t q = 0; q < nb; ++q) {
                                double pu[4], pv[4];
#pragma unroll
                                for (int e = 0; e < 4; ++e) {
                                    pu[e] = P[(nb + 4 * bu + e) * kPanel + q];
                                    pv[e] = P[(nb + 4 * bv + e) * kPanel + q];
                                }
#pragma unroll
                                for (int e = 0; e < 4; ++e)
#pragma unroll
                                    for (int f = 0; f < 4; ++f) acc[e][f] = fma(pu[e], pv[f], acc[e][f]);
                            }
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const uint32_t u = c1 + 4 * bu + e;
#pragma unroll
                                for (int f = 0; f < 4; ++f) {
                                    const uint32_t v = c1 + 4 * bv + f;
                                    if (u < F && v <= u) A[(size_t)u * F + v] -= acc[e][f];
                                }
                            }
                        }
                    }
                }
                __syncthreads();
            }
            const int bad = s_bad;
            __syncthreads();
            if (!bad) break;
        }
        if (tid == 0) {
            *a.status = s_bad;
            *a.lam = s_ridge;
        }
        cv_load_rhs(a, F, y, 0.0);
    } else {
        cv_load_rhs(a, F, y, *a.lam);
    }
    __syncthreads();

    // forward substitution L z = y, one panel at a time
    for (uint32_t c0 = 0; c0 < F; c0 += kPanel) {
        const uint32_t nb = min(kPanel, F - c0);
        if (tid == 0) {
            for (uint32_t q = 0; q < nb; ++q) {
                double v = y[c0 + q];
                for (uint32_t q2 = 0; q2 < q; ++q2) v -= A[(size_t)(c0 + q) * F + c0 + q2] * y[c0 + q2];
                y[c0 + q] = v / A[(size_t)(c0 + q) * F + c0 + q];
            }
        }
        __syncthreads();
        for (uint32_t u = c0 + nb + tid; u < F; u += nt) {
            double v = y[u];
            for (uint32_t q = 0; q < nb; ++q) v -= A[(size_t)u * F + c0 + q] * y[c0 + q];
            y[u] = v;
        }
        __syncthreads();
    }
    // backward substitution L^T w = z, panels from the last; P holds the
    // per-column partial dot products (kPanel groups of nt / kPanel threads)
    const uint32_t per = nt / kPanel, grp = tid / per, lane = tid % per;
    for (uint32_t c0 = ((F - 1) / kPanel) * kPanel;; c0 -= kPanel) {
        const uint32_t nb = min(kPanel, F - c0), c1 = c0 + nb;
        double s = 0.0;
        if (grp < nb)
            for (uint32_t v = c1 + lane; v < F; v += per) s += A[(size_t)v * F + c0 + grp] * y[v];
        P[tid] = s;
        __syncthreads();
        for (uint32_t h = per / 2; h > 0; h >>= 1) {
            if (lane < h) P[tid] += P[tid + h];
            __syncthreads();
        }
        if (tid == 0) {
            for (uint32_t q = nb; q-- > 0;) {
                double v = y[c0 + q] - P[q * per];
                for (uint32_t q2 = q + 1; q2 < nb; ++q2) v -= A[(size_t)(c0 + q2) * F + c0 + q] * y[c0 + q2];
                y[c0 + q] = v / A[(size_t)(c0 + q) * F + c0 + q];
            }
        }
        __syncthreads();
        if (c0 == 0) break;
    }
    for (uint32_t u = tid; u < F; u += nt) {
        const uint32_t r = u / a.K, k = u - r * a.K;
        const size_t o = ((size_t)r * a.d + a.i) * a.K + k;
        const double w = a.refine ? a.w64[o] + y[u] : y[u];
        a.w64[o] = w;
        a.ws32[o] = (float)(w * sqrt(2.0 * k + 1.0));
    }
}

// Rescales the factors of each rank to equal norms across dimensions (the
// product, hence the model, is unchanged): keeps ALS well conditioned.
__global__ void k_cv_balance(uint32_t R, uint32_t d, uint32_t K, double *w64, float *ws32) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    double lg = 0.0;
    for (uint32_t i = 0; i < d; ++i) {
        double s = 0.0;
        for (uint32_t k = 0; k < K; ++k) s += w64[((size_t)r * d + i) * K + k] * w64[((size_t)r * d + i) * K + k];
        if (!(s > 0.0)) return;
        lg += 0.5 * log(s);
    }
    lg /= d;
    for (uint32_t i = 0; i < d; ++i) {
        double s = 0.0;
        for (uint32_t k = 0; k < K; ++k) s += w64[((size_t)r * d + i) * K + k] * w64[((size_t)r * d + i) * K + k];
        const double f = exp(lg - 0.5 * log(s));
        for (uint32_t k = 0; k < K; ++k) {
            const size_t o = ((size_t)r * d + i) * K + k;
            w64[o] *= f;
            ws32[o] = (float)(w64[o] * sqrt(2.0 * k + 1.0));
        }
    }
}

// training loss sum_j (yw_j / scale - sw_j g32(z_j))^2 and sum_j (yw_j / scale)^2,
// one pair of partial sums per block
template <int R, int K>
__global__ __launch_bounds__(kBlock) void k_cv_loss(uint32_t n, uint32_t d, const float *z, const float *sw,
                                                   const float *yw, float inv_scale, const float *ws,
                                                   double *partial) {
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    double e2 = 0.0, y2 = 0.0;
    if (j < n) {
        float prod[R];
#pragma unroll
        for (int r = 0; r < R; ++r) prod[r] = 1.0f;
        for (uint32_t i = 0; i < d; ++i) {
            float p[K];
            legendre_raw<K, float>(z[(size_t)j * d + i], p);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float *w = ws + ((size_t)r * d + i) * K;
                float h = w[K - 1] * p[K - 1];
#pragma unroll
                for (int k = K - 2; k >= 0; --k) h = __builtin_fmaf(w[k], p[k], h);
                prod[r] *= h;
            }
        }
        float g = 0.0f;
#pragma unroll
        for (int r = 0; r < R; ++r) g += prod[r];
        const double y = (double)yw[j] * inv_scale;
        const double e = y - (double)sw[j] * g;
        e2 = e * e;
        y2 = y * y;
    }
    __shared__ double se[kBlock], sy[kBlock];
    se[threadIdx.x] = e2;
    sy[threadIdx.x] = y2;
    __syncthreads();
    for (uint32_t h = kBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            se[threadIdx.x] += se[threadIdx.x + h];
            sy[threadIdx.x] += sy[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = se[0];
        partial[2 * blockIdx.x + 1] = sy[0];
    }
}

// mean |yw| for the target scale: per-block partial sums
__global__ __launch_bounds__(kBlock) void k_cv_absmean(uint32_t n, const float *yw, double *partial) {
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    __shared__ double s[kBlock];
    s[threadIdx.x] = j < n ? fabs((double)yw[j]) : 0.0;
    __syncthreads();
    for (uint32_t h = kBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

// ------------------------------------------------------------------- host
namespace {

using RhoFn = void (*)(const CvRhoArgs &, uint32_t, hipStream_t);
using LossFn = void (*)(uint32_t, uint32_t, const float *, const float *, const float *, float, const float *,
                        double *, uint32_t, hipStream_t);
using ResidFn = void (*)(uint32_t, uint32_t, uint32_t, const float *, const float *, const float *, float,
                         const double *, float *, uint32_t, hipStream_t);

template <int R, int K>
void launch_rho(const CvRhoArgs &a, uint32_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_cv_rho<R, K>), dim3(blocks), dim3(kBlock), 0, s, a);
}
template <int R, int K>
void launch_loss(uint32_t n, uint32_t d, const float *z, const float *sw, const float *yw, float is, const float *ws,
                 double *part, uint32_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_cv_loss<R, K>), dim3(blocks), dim3(kBlock), 0, s, n, d, z, sw, yw, is, ws, part);
}

template <int R, int K>
void launch_resid(uint32_t n, uint32_t d, uint32_t i, const float *rho, const float *phi, const float *yw, float is,
                  const double *w64, float *e, uint32_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_cv_resid<R, K>), dim3(blocks), dim3(kBlock), 0, s, n, d, i, rho, phi, yw, is, w64, e);
}

bool cv_fns(uint32_t R, uint32_t K, RhoFn &rho, LossFn &loss, ResidFn &resid) {
#define QMC_CV_CASE(RR, KK)                  \
    if (R == RR && K == KK) {                \
        rho = &launch_rho<RR, KK>;           \
        loss = &launch_loss<RR, KK>;         \
        resid = &launch_resid<RR, KK>;       \
        return true;                         \
    }
    QMC_CV_CASE(8, 4) QMC_CV_CASE(8, 8) QMC_CV_CASE(16, 8) QMC_CV_CASE(16, 12) QMC_CV_CASE(32, 8)
    QMC_CV_CASE(32, 12) QMC_CV_CASE(32, 16) QMC_CV_CASE(64, 12)
#undef QMC_CV_CASE
    return false;
}

// simple seeded generator for the initial factors (SplitMix64)
double splitmix_uniform(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53;
}

}  // namespace

}  // namespace qmc

using namespace qmc;

extern "C" {

qmc_status qmc_cv_train(qmc_plan_t p, qmc_family family, const void *params, uint32_t R, uint32_t K,
                        const qmc_cv_train_opts *opts, double *w_out, double *c_out, qmc_cv_train_report *rep) {
    if (!p || !w_out || !c_out) return fail(QMC_EINVAL, "null argument");
    if (family != QMC_F_SECTOR) return fail(QMC_EUNSUPPORTED, "control variates are built for QMC_F_SECTOR");
    RhoFn rho_fn;
    LossFn loss_fn;
    ResidFn resid_fn;
    if (!cv_fns(R, K, rho_fn, loss_fn, resid_fn))
        return fail(QMC_EUNSUPPORTED, "(R, K) = (%u, %u) not compiled; use (32,12), (64,12), (16,8), ...", R, K);
    if (p->d > 12) return fail(QMC_EUNSUPPORTED, "d > 12");
    const qmc_cv_train_opts o = opts ? *opts : qmc_cv_train_opts{12, 1e-5, 1e-4, 1};
    Packed pk;
    qmc_status st = pack_params((int)family, p->d, params, pk);
    if (st) return st;
    const uint32_t n = p->n, d = p->d, F = R * K, RB = (R + 31) / 32;
    hipError_t e;
    std::string err;
    if (pk.orders >= 2) return fail(QMC_EUNSUPPORTED, "control variates take the plain integrand (n_orders < 2)");
    if (pk.deform) return fail(QMC_EUNSUPPORTED, "control variates take undeformed sectors (deform_lambda = 0)");
    hipFunction_t sample = jit_sample_kernel(pk.blob, d, p->tr, pk.cplx, p->device, err);
    if (!sample) return fail(QMC_EUNSUPPORTED, "training sampler: %s", err.c_str());
    if ((st = plan_upload_params(p, pk))) return st;

    // jobs: Gram blocks (k, k0..k0+count) x (rb, cb), then the RHS blocks
    std::vector<CvJob> jobs;
    std::vector<uint32_t> pair_slot((size_t)K * K, 0);
    uint32_t slot = 0;
    for (uint32_t k = 0; k < K; ++k)
        for (uint32_t k0 = k; k0 < K; k0 += kMaxJobCount) {
            const uint32_t cnt = std::min<uint32_t>(kMaxJobCount, K - k0);
            for (uint32_t rb = 0; rb < RB; ++rb)
                for (uint32_t cb = 0; cb < RB; ++cb)
                    jobs.push_back(CvJob{0, k, k0, cnt, rb, cb, 0, 0});
        }
    // slots: pair (k, kp) occupies RB*RB consecutive slots (rb-major)
    for (uint32_t k = 0; k < K; ++k)
        for (uint32_t kp = k; kp < K; ++kp) {
            pair_slot[k * K + kp] = slot;
            slot += RB * RB;
        }
    for (CvJob &jb : jobs) jb.slot0 = pair_slot[jb.k * K + jb.k0] + jb.rb * RB + jb.cb;
    // a job's q-th pair (k, k0+q) must sit RB*RB slots after the previous one:
    // re-express slot0 + q as pair_slot[k, k0+q] by using stride RB*RB.
    const uint32_t rhs_slot0 = slot;
    for (uint32_t rb = 0; rb < RB; ++rb) jobs.push_back(CvJob{1, 0, 0, 1, rb, 0, rhs_slot0 + rb, 0});
    const uint32_t nslots = rhs_slot0 + RB;
    // the kernel writes job.slot0 + q; make q-steps land on the right pair by
    // splitting jobs so that each covers pairs at unit slot stride (RB == 1),
    // or one pair per job otherwise
    if (RB > 1) {
        std::vector<CvJob> split;
        for (const CvJob &jb : jobs) {
            if (jb.type != 0) {
                split.push_back(jb);
                continue;
            }
            for (uint32_t q = 0; q < jb.count; ++q)
                split.push_back(CvJob{0, jb.k, jb.k0 + q, 1, jb.rb, jb.cb,
                                      pair_slot[jb.k * K + jb.k0 + q] + jb.rb * RB + jb.cb, 0});
        }
        jobs.swap(split);
    }
    const uint32_t splits = std::max<uint32_t>(1, std::min<uint32_t>(256, n / 4096));
    const uint32_t rblocks = (n + kBlock - 1) / kBlock;

    DeviceScratch s;
    // 0 z, 1 sw, 2 yw, 3 rho, 4 phi, 5 ws32, 6 w64, 7 jobs, 8 partial, 9 tiles, 10 pair_slot, 11 A, 12 b,
    // 13 status, 14 loss partials, 15 absmean partials, 16 residual, 17 ridge
    if ((st = s.alloc((size_t)n * d * 4)) || (st = s.alloc((size_t)n * 4)) || (st = s.alloc((size_t)n * 4)) ||
        (st = s.alloc((size_t)n * R * 4)) || (st = s.alloc((size_t)n * K * 4)) ||
        (st = s.alloc((size_t)R * d * K * 4)) || (st = s.alloc((size_t)R * d * K * 8)) ||
        (st = s.alloc(jobs.size() * sizeof(CvJob))) || (st = s.alloc((size_t)splits * nslots * 4096)) ||
        (st = s.alloc((size_t)nslots * 8192)) || (st = s.alloc(pair_slot.size() * 4)) ||
        (st = s.alloc((size_t)F * F * 8)) || (st = s.alloc((size_t)F * 8)) || (st = s.alloc(8)) ||
        (st = s.alloc((size_t)rblocks * 16)) || (st = s.alloc((size_t)rblocks * 8)) ||
        (st = s.alloc((size_t)n * 4)) || (st = s.alloc(8)))
        return st;
    hipStream_t stream = p->stream;
    struct Events {
        hipEvent_t t0 = nullptr, t1 = nullptr;
        ~Events() {
            if (t0) (void)hipEventDestroy(t0);
            if (t1) (void)hipEventDestroy(t1);
        }
    } ev;
    (void)hipEventCreate(&ev.t0);
    (void)hipEventCreate(&ev.t1);
    (void)hipEventRecord(ev.t0, stream);

    // one model per component: the real part, then (complex integrands) the
    // imaginary part
    uint32_t sweeps_total = 0;
    double rel_worst = 0.0, scale0 = 0.0;
    for (uint32_t comp = 0; comp < pk.np; ++comp) {
    CvSampleArgs sa{};
    sa.n = n;
    sa.d = d;
    sa.inv_n = p->inv_n;
    sa.g = p->d_g;
    sa.shift = p->d_shifts;  // the plan's first shift
    sa.params = p->d_params;
    sa.z = (float *)s.ptr[0];
    sa.sw = (float *)s.ptr[1];
    sa.yw = (float *)s.ptr[2];
    sa.part = comp;
    if ((e = jit_launch_sample(sample, sa, rblocks, stream)) != hipSuccess) return hip_fail(e, "training sampler");
    hipLaunchKernelGGL(k_cv_absmean, dim3(rblocks), dim3(kBlock), 0, stream, n, (const float *)s.ptr[2],
                       (double *)s.ptr[15]);
    std::vector<double> part(2 * (size_t)rblocks);
    if ((e = hipMemcpyAsync(part.data(), s.ptr[15], rblocks * 8, hipMemcpyDeviceToHost, stream)) != hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess)
        return hip_fail(e, "training samples");
    double scale = 0.0;
    for (uint32_t b = 0; b < rblocks; ++b) scale += part[b];
    scale /= n;
    if (!(scale > 0.0) || !std::isfinite(scale)) return fail(QMC_ENONFINITE, "training targets are zero or not finite");

    // initial factors: near-constant with seeded perturbations (breaks the
    // symmetry between ranks)
    std::vector<double> w64((size_t)R * d * K, 0.0);
    std::vector<float> ws32(w64.size());
    uint64_t seed = o.seed ? o.seed : 1;
    const double base = std::pow(1.0 / R, 1.0 / d);
    for (uint32_t r = 0; r < R; ++r)
        for (uint32_t i = 0; i < d; ++i)
            for (uint32_t k = 0; k < K; ++k) {
                const double u = splitmix_uniform(seed) - 0.5;
                const double v = k == 0 ? base * (1.0 + 0.5 * u) : 0.1 * base * u / (k + 1);
                w64[((size_t)r * d + i) * K + k] = v;
            }
    for (size_t t = 0; t < w64.size(); ++t) ws32[t] = (float)(w64[t] * std::sqrt(2.0 * (t % K) + 1.0));
    if ((e = hipMemcpy(s.ptr[5], ws32.data(), ws32.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(s.ptr[6], w64.data(), w64.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(s.ptr[7], jobs.data(), jobs.size() * sizeof(CvJob), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(s.ptr[10], pair_slot.data(), pair_slot.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "training upload");

    CvRhoArgs ra{n, d, 0, (const float *)s.ptr[0], (const float *)s.ptr[1], (const float *)s.ptr[5],
                 (float *)s.ptr[3], (float *)s.ptr[4]};
    CvGramArgs ga{};
    ga.n = n;
    ga.R = R;
    ga.K = K;
    ga.job0 = 0;
    ga.njobs = (uint32_t)jobs.size();
    ga.nslots = nslots;
    ga.splits = splits;
    ga.inv_scale = (float)(1.0 / scale);
    ga.rho = ra.rho;
    ga.phi = ra.phi;
    ga.yw = (const float *)s.ptr[2];
    ga.jobs = (const CvJob *)s.ptr[7];
    ga.partial = (float *)s.ptr[8];
    CvSolveArgs so{};
    so.R = R;
    so.K = K;
    so.d = d;
    so.rhs_slot0 = rhs_slot0;
    so.RB = RB;
    so.ridge = o.ridge > 0 ? o.ridge : 1e-5;
    so.tiles = (const double *)s.ptr[9];
    so.pair_slot = (const uint32_t *)s.ptr[10];
    so.A = (double *)s.ptr[11];
    so.w64 = (double *)s.ptr[6];
    so.ws32 = (float *)s.ptr[5];
    so.status = (int *)s.ptr[13];
    so.lam = (double *)s.ptr[17];

    const uint32_t max_sweeps = o.max_sweeps ? o.max_sweeps : 12;
    double prev = INFINITY, rel = INFINITY, best = INFINITY;
    std::vector<double> w_best(w64.size());
    uint32_t sweeps = 0;
    const uint32_t gblocks = (ga.njobs + 3) / 4;
    const float inv_scale = (float)(1.0 / scale);
    uint32_t rhs_job0 = 0;
    while (jobs[rhs_job0].type == 0) ++rhs_job0;
    constexpr uint32_t kRefineSteps = 2;
    for (; sweeps < max_sweeps;) {
        for (uint32_t i = 0; i < d; ++i) {
            ra.i = i;
            rho_fn(ra, rblocks, stream);
            ga.job0 = 0;
            ga.yw = (const float *)s.ptr[2];
            ga.inv_scale = inv_scale;
            hipLaunchKernelGGL(k_cv_gram, dim3(gblocks, splits), dim3(kBlock), 0, stream, ga);
            hipLaunchKernelGGL(k_cv_reduce, dim3((nslots * 1024 + kBlock - 1) / kBlock), dim3(kBlock), 0, stream,
                               (const float *)ga.partial, splits, nslots, 0u, (double *)s.ptr[9]);
            so.i = i;
            so.refine = 0;
            hipLaunchKernelGGL(k_cv_solve, dim3(1), dim3(1024), 0, stream, so);
            // iterative refinement: the BF16 normal matrix only preconditions;
            // the right-hand side A^T e comes from the FP32 residual, so the
            // fixed point is the least-squares solution at FP32 accuracy
            ga.job0 = rhs_job0;
            ga.yw = (const float *)s.ptr[16];
            ga.inv_scale = 1.0f;
            so.refine = 1;
            for (uint32_t it = 0; it < kRefineSteps; ++it) {
                resid_fn(n, d, i, ra.rho, ra.phi, (const float *)s.ptr[2], inv_scale, so.w64, (float *)s.ptr[16],
                         rblocks, stream);
                hipLaunchKernelGGL(k_cv_gram, dim3((RB + 3) / 4, splits), dim3(kBlock), 0, stream, ga);
                hipLaunchKernelGGL(k_cv_reduce, dim3((RB * 1024 + kBlock - 1) / kBlock), dim3(kBlock), 0, stream,
                                   (const float *)ga.partial, splits, nslots, rhs_slot0, (double *)s.ptr[9]);
                hipLaunchKernelGGL(k_cv_solve, dim3(1), dim3(1024), 0, stream, so);
            }
        }
        ++sweeps;
        hipLaunchKernelGGL(k_cv_balance, dim3((R + 63) / 64), dim3(64), 0, stream, R, d, K, so.w64, so.ws32);
        loss_fn(n, d, ra.z, ra.sw, (const float *)s.ptr[2], inv_scale, so.ws32, (double *)s.ptr[14], rblocks,
                stream);
        int bad = 0;
        if ((e = hipMemcpyAsync(part.data(), s.ptr[14], (size_t)rblocks * 16, hipMemcpyDeviceToHost, stream)) !=
                hipSuccess ||
            (e = hipMemcpyAsync(&bad, s.ptr[13], 4, hipMemcpyDeviceToHost, stream)) != hipSuccess ||
            (e = hipStreamSynchronize(stream)) != hipSuccess)
            return hip_fail(e, "training loop");
        double se = 0.0, sy = 0.0;
        for (uint32_t b = 0; b < rblocks; ++b) {
            se += part[2 * b];
            sy += part[2 * b + 1];
        }
        rel = se / sy;
        if (!std::isfinite(rel)) {
            if (std::isfinite(best)) break;  // keep the best factors so far
            return fail(QMC_ENONFINITE, "training diverged");
        }
        if (rel < best) {  // the factors of the lowest loss are the result
            best = rel;
            if ((e = hipMemcpy(w_best.data(), s.ptr[6], w_best.size() * 8, hipMemcpyDeviceToHost)) != hipSuccess)
                return hip_fail(e, "training download");
        }
        if (prev - rel < o.tol * prev) break;
        prev = rel;
    }
    std::memcpy(w_out + (size_t)comp * R * d * K, w_best.data(), w_best.size() * 8);
    for (uint32_t r = 0; r < R; ++r) c_out[(size_t)comp * R + r] = scale;
    sweeps_total += sweeps;
    rel_worst = std::max(rel_worst, best);
    if (comp == 0) scale0 = scale;
    }  // components
    (void)hipEventRecord(ev.t1, stream);
    (void)hipStreamSynchronize(stream);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev.t0, ev.t1);
    if (rep) *rep = qmc_cv_train_report{sweeps_total, rel_worst, scale0, ms / 1e3};
    return QMC_OK;
}

qmc_status qmc_cv_integral(uint32_t R, uint32_t d, uint32_t K, const double *w, const double *c, double *out) {
    if (!w || !c || !out) return fail(QMC_EINVAL, "null argument");
    double s = 0.0;
    for (uint32_t r = 0; r < R; ++r) {
        double pr = c[r];
        for (uint32_t i = 0; i < d; ++i) pr *= w[((size_t)r * d + i) * K];
        s += pr;
    }
    *out = s;
    return QMC_OK;
}

qmc_status qmc_integrate_cv(qmc_plan_t p, qmc_family family, const void *params, uint32_t R, uint32_t K,
                            const double *w, const double *c, qmc_result *out, qmc_result *plain_out,
                            double *per_shift) {
    if (!p || !w || !c || !out) return fail(QMC_EINVAL, "null argument");
    if (family != QMC_F_SECTOR) return fail(QMC_EUNSUPPORTED, "control variates are built for QMC_F_SECTOR");
    RhoFn rf;
    LossFn lf;
    ResidFn ef;
    if (!cv_fns(R, K, rf, lf, ef)) return fail(QMC_EUNSUPPORTED, "(R, K) = (%u, %u) not compiled", R, K);
    if (p->d > 12) return fail(QMC_EUNSUPPORTED, "d > 12");
    Packed pk;
    qmc_status st = pack_params((int)family, p->d, params, pk);
    if (st) return st;
    if (pk.orders >= 2) return fail(QMC_EUNSUPPORTED, "control variates take the plain integrand (n_orders < 2)");
    if (pk.deform) return fail(QMC_EUNSUPPORTED, "control variates take undeformed sectors (deform_lambda = 0)");
    const uint32_t nm = pk.np, d = p->d;  // one model per component
    const size_t wsize = (size_t)R * d * K;
    for (uint32_t t = 0; t < nm * R; ++t)
        if (!std::isfinite(c[t])) return fail(QMC_EINVAL, "c not finite");
    for (size_t t = 0; t < nm * wsize; ++t)
        if (!std::isfinite(w[t])) return fail(QMC_EINVAL, "W not finite");
    // weights in the lane order of the FP64 matrix instructions (FamCvResidual):
    // per model, fragment ((i * RB + rb) * KS + ks), lane l ->
    // W[16 rb + l % 16, i, 4 ks + l / 16] * sqrt(2k + 1), times c_r in
    // dimension 0, zero outside R x K
    const size_t base = pk.blob.size();
    const uint32_t RB = (R + 15) / 16, KS = (K + 3) / 4;
    const size_t msize = (size_t)d * RB * KS * kWave;
    pk.blob.resize(base + nm * msize, 0.0);
    for (uint32_t mi = 0; mi < nm; ++mi)
        for (uint32_t i = 0; i < d; ++i)
            for (uint32_t rb = 0; rb < RB; ++rb)
                for (uint32_t ks = 0; ks < KS; ++ks)
                    for (uint32_t l = 0; l < kWave; ++l) {
                        const uint32_t r = 16 * rb + l % 16, k = 4 * ks + l / 16;
                        if (r >= R || k >= K) continue;
                        double v = w[mi * wsize + ((size_t)r * d + i) * K + k] * std::sqrt(2.0 * k + 1.0);
                        if (i == 0) v *= c[(size_t)mi * R + r];
                        pk.blob[base + mi * msize + (((size_t)i * RB + rb) * KS + ks) * kWave + l] = v;
                    }
    std::string err;
    hipFunction_t fn = jit_cv_kernel(pk.blob, base, d, p->tr, R, K, nm == 2, p->device, err);
    if (!fn) return fail(QMC_EUNSUPPORTED, "control-variate kernel: %s", err.c_str());
    Packed cv = pk;
    cv.np = 2 * nm;
    cv.key_family = -1;  // not in the kernel registry
    if ((st = plan_enqueue_fn(p, cv, fn, 1))) return st;
    qmc_result first;
    std::vector<double> q((size_t)cv.np * p->m);
    st = plan_collect(p, cv.np, &first, q.data());
    if (st && st != QMC_ENONFINITE) return st;
    // parts: real -> (f, f - g); complex -> (Re f, Im f, Re f - g_0, Im f - g_1)
    const double *res = p->h_out + out_res_offset(p->m);
    double ig[2] = {0.0, 0.0};
    for (uint32_t mi = 0; mi < nm; ++mi) qmc_cv_integral(R, d, K, w + mi * wsize, c + (size_t)mi * R, &ig[mi]);
    qmc_result plain, cvr;
    if (nm == 1) {
        plain = qmc_result{res[0], 0.0, res[2], 0.0, 0, 0};
        cvr = qmc_result{ig[0] + res[1], 0.0, res[3], 0.0, 0, 1};
    } else {
        plain = qmc_result{res[0], res[1], res[2], res[3], 1, 0};
        cvr = qmc_result{ig[0] + res[4], ig[1] + res[5], res[6], res[7], 1, 1};
    }
    if (plain_out) *plain_out = plain;
    if (per_shift) std::memcpy(per_shift, q.data(), q.size() * 8);
    if (st == QMC_ENONFINITE) {
        *out = qmc_result{NAN, NAN, NAN, NAN, (int32_t)(nm == 2), 0};
        return st;
    }
    const double e_cv = std::hypot(cvr.err_re, cvr.err_im), e_plain = std::hypot(plain.err_re, plain.err_im);
    *out = e_cv < e_plain ? cvr : plain;
    return QMC_OK;
}

}  // extern "C"
