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
#include <type_traits>

#include "qmc_cv.hpp"
#include "qmc_runtime.hpp"

namespace qmc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------- kernels
// Design-matrix factors of dimension i in FP64:
//   rho_j[r] = sw_j prod_{i' != i} h_{r,i'}(z_{j,i'}),  phi_j[k] = P~_k(z_{j,i}).
struct CvRhoArgs {
    uint32_t n, d, i;       // points, dimension, the dimension being solved
    const float *z, *sw;    // (n, d), (n)
    const double *ws;       // W * sqrt(2k+1), (R, d, K)
    double *rho;            // (n, R)
    double *phi;            // (n, K) (normalised)
};

template <int R, int K>
__global__ __launch_bounds__(kBlock) void k_cv_rho(const CvRhoArgs a) {
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= a.n) return;
    double prod[R];
    const double s = a.sw[j];
#pragma unroll
    for (int r = 0; r < R; ++r) prod[r] = s;
    for (uint32_t i = 0; i < a.d; ++i) {
        double p[K];
        legendre_raw<K, double>((double)a.z[(size_t)j * a.d + i], p);
        if (i == a.i) {
#pragma unroll
            for (int k = 0; k < K; ++k) a.phi[(size_t)j * K + k] = p[k] * sqrt((double)(2 * k + 1));
            continue;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double *w = a.ws + ((size_t)r * a.d + i) * K;
            double h = w[K - 1] * p[K - 1];
#pragma unroll
            for (int k = K - 2; k >= 0; --k) h = fma(w[k], p[k], h);
            prod[r] *= h;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) a.rho[(size_t)j * R + r] = prod[r];
}

// ----------------------------------------------------------- Gram (SYRK)
// A~^T A~ for the BF16 design matrix a~_j[u'] = bf16(fl32(rho_j[r]) fl32(phi_j[k]))
// with the columns in the order u' = k R + r (a block of 32 consecutive
// columns is one k when R >= 32).  The lower triangle of the NB x NB grid of
// 32 x 32 tiles (NB = R K / 32) is split into tasks (grid.y).  A task gives
// each of its 4 waves one region of tiles: rows [r0, r0 + NR) x columns
// [c0, c0 + NC) of the block grid, the lower part only for a diagonal region
// (then the rows lie inside the columns).  The region shapes are fixed per
// task type at compile time (at most 11 tiles, 176 accumulator registers per
// lane, so two workgroups fit on a CU); the bases come with the task.  A
// workgroup runs one task over one contiguous range of points (grid.x), 64
// points per round:
//   1. the round's rho, phi go to LDS as FP32 (the next round's are loaded
//      into registers meanwhile),
//   2. wave w builds the BF16 fragments of points 16 w .. 16 w + 15 for the
//      task's blocks [blo, bhi) into LDS (v_mfma_f32_32x32x16_bf16 operand
//      layout: lane l holds column 32 b + l % 32 of points 8 (l / 32) .. +7;
//      the same fragment serves as A or B),
//   3. every wave accumulates its tiles over the 4 steps of 16 points.
// The tiles' FP32 sums go to partial[split][slot], slot = bu (bu + 1) / 2 + bv
// for the tile (bu >= bv).
struct CvSyrkTask {
    uint32_t type, blo, bhi;
    uint32_t r0[4], c0[4];
};

struct CvSyrkArgs {
    uint32_t n, splits, nslots;
    const double *rho, *phi;
    const CvSyrkTask *tasks;
    float *partial;  // (splits, nslots, 32, 32)
};

constexpr int kSyrkPts = 64;  // points per round (4 steps of 16)
constexpr int kSyrkMaxTiles = 11;

// region shapes (NR rows, NC columns, lower part only) of the 4 waves
template <int NR0, int NC0, bool D0, int NR1, int NC1, bool D1, int NR2, int NC2, bool D2, int NR3, int NC3, bool D3>
struct SyrkShapes {
    static constexpr int NR[4] = {NR0, NR1, NR2, NR3}, NC[4] = {NC0, NC1, NC2, NC3};
    static constexpr bool DG[4] = {D0, D1, D2, D3};
};
// triangles of 1, 2, 4, 6, 8 blocks in one task
using ShapeTri1 = SyrkShapes<1, 1, true, 0, 0, false, 0, 0, false, 0, 0, false>;
using ShapeTri2 = SyrkShapes<1, 1, true, 1, 1, true, 1, 1, false, 0, 0, false>;
using ShapeTri4 = SyrkShapes<2, 2, true, 2, 2, true, 1, 2, false, 1, 2, false>;
using ShapeTri6 = SyrkShapes<3, 3, true, 3, 3, true, 2, 3, false, 1, 3, false>;
using ShapeTri8 = SyrkShapes<4, 4, true, 4, 4, true, 2, 4, false, 2, 4, false>;
// half of a triangle of 12 blocks (two tasks cover it)
using ShapeHalf12 = SyrkShapes<4, 4, true, 2, 6, true, 3, 3, false, 3, 3, false>;
// rectangles: 8 x 4 and 6 x 6 blocks
using ShapeRect8x4 = SyrkShapes<2, 4, false, 2, 4, false, 2, 4, false, 2, 4, false>;
using ShapeRect6x6 = SyrkShapes<3, 3, false, 3, 3, false, 3, 3, false, 3, 3, false>;

template <class S, int W>
constexpr int syrk_tiles() {
    int t = 0;
    for (int i = 0; i < S::NR[W]; ++i)
        for (int j = 0; j < S::NC[W]; ++j)
            if (!S::DG[W] || j <= i + (S::NC[W] - S::NR[W])) ++t;
    return t;
}

// One step of 16 points for wave W: load the region's column fragments
// (rows of a diagonal region are among them), accumulate its tiles.  In a
// diagonal region, row i is block r0 + i = c0 + (NC - NR) + i.
template <class S, int W>
__device__ __forceinline__ void syrk_step(const bf16x8 *fr, uint32_t lane, uint32_t r0, uint32_t c0,
                                          f32x16 (&acc)[kSyrkMaxTiles]) {
    constexpr int NR = S::NR[W], NC = S::NC[W];
    static_assert(syrk_tiles<S, W>() <= kSyrkMaxTiles, "too many tiles for one wave");
    if constexpr (NR > 0) {
        bf16x8 fb[NC];
#pragma unroll
        for (int j = 0; j < NC; ++j) fb[j] = fr[(c0 + j) * (4 * kWave) + lane];
        int t = 0;
        if constexpr (S::DG[W]) {
#pragma unroll
            for (int i = 0; i < NR; ++i)
#pragma unroll
                for (int j = 0; j <= i + (NC - NR); ++j, ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fb[i + (NC - NR)], fb[j], acc[t], 0, 0, 0);
        } else {
            bf16x8 fa[NR];
#pragma unroll
            for (int i = 0; i < NR; ++i) fa[i] = fr[(r0 + i) * (4 * kWave) + lane];
#pragma unroll
            for (int i = 0; i < NR; ++i)
#pragma unroll
                for (int j = 0; j < NC; ++j, ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[t], 0, 0, 0);
        }
    }
}

template <class S, int W>
__device__ __forceinline__ void syrk_store(uint32_t lane, uint32_t r0, uint32_t c0,
                                           const f32x16 (&acc)[kSyrkMaxTiles], float *out) {
    constexpr int NR = S::NR[W], NC = S::NC[W];
    const uint32_t half = lane >> 5, col = lane & 31;
    int t = 0;
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            if (S::DG[W] && j > i + (NC - NR)) continue;
            const uint32_t bu = S::DG[W] ? c0 + (NC - NR) + i : r0 + i, bv = c0 + j;
            float *o = out + (((size_t)bu * (bu + 1) / 2 + bv) << 10);
#pragma unroll
            for (int e = 0; e < 16; ++e) o[(8 * (e / 4) + 4 * half + (e % 4)) * 32 + col] = acc[t][e];
            ++t;
        }
}

template <int R, int K, class S>
__device__ __forceinline__ void syrk_task(const CvSyrkArgs &a, const CvSyrkTask &task, float *srho, float *sphi,
                                          bf16x8 *frag) {
    constexpr int NV = (kSyrkPts * (R + K) + kBlock - 1) / kBlock;  // staged values per thread
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const uint32_t j_begin = (uint32_t)((uint64_t)a.n * blockIdx.x / a.splits);
    const uint32_t j_end = (uint32_t)((uint64_t)a.n * (blockIdx.x + 1) / a.splits);
    // the wave's bases straight from memory (indexing a private copy by the
    // wave number would put it in scratch)
    const uint32_t r0 = a.tasks[blockIdx.y].r0[wave], c0 = a.tasks[blockIdx.y].c0[wave];

    f32x16 acc[kSyrkMaxTiles];
#pragma unroll
    for (int t = 0; t < kSyrkMaxTiles; ++t)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[t][e] = 0.0f;

    // value v of a round: v < 64 R -> rho[p][r], else phi[p][k]
    double nxt[NV];
    auto load_round = [&](uint32_t base) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const uint32_t v = tid + q * kBlock;
            double x = 0.0;
            if (v < (uint32_t)(kSyrkPts * R)) {
                if (base + v / R < j_end) x = a.rho[(size_t)base * R + v];
            } else if (v < (uint32_t)(kSyrkPts * (R + K))) {
                const uint32_t w = v - kSyrkPts * R;
                if (base + w / K < j_end) x = a.phi[(size_t)base * K + w];
            }
            nxt[q] = x;
        }
    };
    if (j_begin < j_end) load_round(j_begin);
    for (uint32_t base = j_begin; base < j_end; base += kSyrkPts) {
        __syncthreads();  // the previous round's fragments are consumed
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const uint32_t v = tid + q * kBlock;
            if (v < (uint32_t)(kSyrkPts * R)) srho[v] = (float)nxt[q];
            else if (v < (uint32_t)(kSyrkPts * (R + K))) sphi[v - kSyrkPts * R] = (float)nxt[q];
        }
        if (base + kSyrkPts < j_end) load_round(base + kSyrkPts);
        __syncthreads();
        {
            const uint32_t half = lane >> 5, c = lane & 31;
            for (uint32_t b = task.blo; b < task.bhi; ++b) {
                const uint32_t u = 32 * b + c, k = u / R, r = u - k * R;
                bf16x8 f;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint32_t p = 16 * wave + 8 * half + e;
                    f[e] = (__bf16)(srho[p * R + r] * sphi[p * K + k]);
                }
                frag[(b * 4 + wave) * kWave + lane] = f;
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bf16x8 *fr = frag + s * kWave;
            switch (wave) {
            case 0: syrk_step<S, 0>(fr, lane, r0, c0, acc); break;
            case 1: syrk_step<S, 1>(fr, lane, r0, c0, acc); break;
            case 2: syrk_step<S, 2>(fr, lane, r0, c0, acc); break;
            default: syrk_step<S, 3>(fr, lane, r0, c0, acc); break;
            }
        }
    }
    float *out = a.partial + (size_t)blockIdx.x * a.nslots * 1024;
    switch (wave) {
    case 0: syrk_store<S, 0>(lane, r0, c0, acc, out); break;
    case 1: syrk_store<S, 1>(lane, r0, c0, acc, out); break;
    case 2: syrk_store<S, 2>(lane, r0, c0, acc, out); break;
    default: syrk_store<S, 3>(lane, r0, c0, acc, out); break;
    }
}

// S0: shapes of task type 0, S1 of type 1 (void: none); NB blocks of fragments in LDS
template <int R, int K, class S0, class S1>
__global__ __launch_bounds__(kBlock, 2) void k_cv_syrk(const CvSyrkArgs a) {
    constexpr int NB = R * K / 32;
    __shared__ float srho[kSyrkPts * R], sphi[kSyrkPts * K];
    __shared__ bf16x8 frag[NB * 4 * kWave];
    const CvSyrkTask task = a.tasks[blockIdx.y];
    if (task.type == 0) {
        syrk_task<R, K, S0>(a, task, srho, sphi, frag);
    } else if constexpr (!std::is_same<S1, void>::value) {
        syrk_task<R, K, S1>(a, task, srho, sphi, frag);
    }
}

// Sum the per-split tiles in split order, in FP64, into the lower triangle
// of the normal matrix A0 (F x F row-major, rows and columns u = r K + k):
// row u = blockIdx.y, column v = blockIdx.x * kBlock + thread.  Column u of
// A0 is column u' = k R + r of the tiles.
__global__ __launch_bounds__(kBlock) void k_cv_gather(const float *partial, uint32_t splits, uint32_t nslots,
                                                     uint32_t R, uint32_t K, double *A0) {
    // one wave per entry (u, v), v <= u: lanes take splits lane, lane + 64,
    // ... in order, then a fixed butterfly over the lanes
    const uint32_t F = R * K, lane = threadIdx.x & (kWave - 1);
    const uint64_t e = (uint64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (e >= (uint64_t)F * (F + 1) / 2) return;
    uint32_t u = (uint32_t)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
    while ((uint64_t)u * (u + 1) / 2 > e) --u;
    while ((uint64_t)(u + 1) * (u + 2) / 2 <= e) ++u;
    const uint32_t v = (uint32_t)(e - (uint64_t)u * (u + 1) / 2);
    const uint32_t r = u / K, k = u - r * K, rp = v / K, kp = v - rp * K;
    uint32_t a = k * R + r, b = kp * R + rp;
    if (a < b) {
        const uint32_t t = a;
        a = b;
        b = t;
    }
    const uint32_t ba = a / 32, bb = b / 32;
    const size_t o = (((size_t)ba * (ba + 1) / 2 + bb) << 10) + (a % 32) * 32 + b % 32;
    double s = 0.0;
    for (uint32_t sp = lane; sp < splits; sp += kWave) s += (double)partial[(size_t)sp * nslots * 1024 + o];
#pragma unroll
    for (int w = kWave / 2; w > 0; w >>= 1) s += __shfl_xor(s, w);
    if (lane == 0) A0[(size_t)u * F + v] = s;
}

// Right-hand side partial sums of the FP64 design matrix:
//   part[split][u] = sum_{j in split} (rho_j[r] phi_j[k]) y_j,  u = r K + k,
// y_j = yd_j, or yf_j * y_scale when yd is null; FP64, points in order (one
// thread per column; a block of 32 points is staged in LDS).
// R <= 64, K <= 16, R K <= 3 kBlock.
constexpr uint32_t kRhsStage = 32;
__global__ __launch_bounds__(kBlock) void k_cv_rhs(uint32_t n, uint32_t R, uint32_t K, uint32_t splits,
                                                  const double *rho, const double *phi, const float *yf,
                                                  double y_scale, const double *yd, double *part) {
    const uint32_t F = R * K, tid = threadIdx.x;
    const uint32_t j0 = (uint32_t)((uint64_t)n * blockIdx.x / splits);
    const uint32_t j1 = (uint32_t)((uint64_t)n * (blockIdx.x + 1) / splits);
    __shared__ double srho[kRhsStage * 64], sphi[kRhsStage * 16], sy[kRhsStage];
    double acc[3] = {0.0, 0.0, 0.0};
    uint32_t ru[3], ku[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const uint32_t u = tid + q * kBlock;
        ru[q] = u < F ? u / K : 0;
        ku[q] = u < F ? u % K : 0;
    }
    for (uint32_t base = j0; base < j1; base += kRhsStage) {
        const uint32_t cnt = min(kRhsStage, j1 - base);
        __syncthreads();
        for (uint32_t t = tid; t < cnt * R; t += kBlock) srho[t] = rho[(size_t)base * R + t];
        for (uint32_t t = tid; t < cnt * K; t += kBlock) sphi[t] = phi[(size_t)base * K + t];
        if (tid < cnt) sy[tid] = yd ? yd[base + tid] : (double)yf[base + tid] * y_scale;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (tid + q * kBlock < F) {
                double s = acc[q];
                for (uint32_t p = 0; p < cnt; ++p) s = fma(srho[p * R + ru[q]] * sphi[p * K + ku[q]], sy[p], s);
                acc[q] = s;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
        if (tid + q * kBlock < F) part[(size_t)blockIdx.x * F + tid + q * kBlock] = acc[q];
}

// b[u] = sum over splits of the right-hand side partials: one wave per
// column, lanes take splits lane, lane + 64, ... in order, then a fixed
// butterfly over the lanes
__global__ __launch_bounds__(kBlock) void k_cv_rhs_reduce(const double *part, uint32_t splits, uint32_t F, double *b) {
    const uint32_t u = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    if (u >= F) return;
    double s = 0.0;
    for (uint32_t sp = lane; sp < splits; sp += kWave) s += part[(size_t)sp * F + u];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) b[u] = s;
}

// residual of the current fit of dimension i in FP64:
//   e_j = yw_j / scale - sum_{r,k} rho_j[r] phi_j[k] W[r,i,k]
// (the right-hand side of a refinement step is A^T e)
template <int R, int K>
__global__ __launch_bounds__(kBlock) void k_cv_resid(uint32_t n, uint32_t d, uint32_t i, const double *rho,
                                                    const double *phi, const float *yw, double inv_scale,
                                                    const double *w64, double *e) {
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    double ph[K];
#pragma unroll
    for (int k = 0; k < K; ++k) ph[k] = phi[(size_t)j * K + k];
    double g = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double *w = w64 + ((size_t)r * d + i) * K;
        double h = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) h = fma(w[k], ph[k], h);
        g = fma(rho[(size_t)j * R + r], h, g);
    }
    e[j] = (double)yw[j] * inv_scale - g;
}

struct CvSolveArgs {
    uint32_t R, K, d, i;
    double ridge;           // relative to the mean diagonal
    int refine;             // 1: reuse the factor in A and add the solution to W[., i, .]
    double *lam;            // absolute ridge of the current factorisation
    const double *A0;       // (F, F) assembled normal matrix, lower triangle
    const double *b;        // (F) right-hand side
    double *A;              // (F, F) factor, F = R K
    double *w64;            // (R, d, K) model, normalised basis
    double *ws;             // (R, d, K) model times sqrt(2k+1)
    int *status;            // number of ridge escalations, or -1: not positive definite
};

// One workgroup solves the normal equations of dimension i.
//
// Assembly: the lower triangle of A0 is copied to A plus the ridge
// lam = ridge * trace / F.  Factorisation: blocked right-looking Cholesky,
// A = L L^T in place.  Each panel of kPanel columns is loaded into LDS and
// factorised there; the trailing lower triangle is then updated by
// A -= P P^T, each thread owning 4 x 4 blocks.  A non-positive pivot
// restarts the factorisation with a 100x larger ridge (at most three
// times).  Solves: blocked forward and backward substitution in LDS.  A
// refinement call (refine = 1) reuses the factor left in A, solves
// (A + lam I) delta = b - lam w (b = A^T e of the current residual e) and
// adds delta to W[., i, .].
constexpr uint32_t kPanel = 8;
constexpr uint32_t kMaxF = 768;  // largest R K compiled: (64, 12)

__device__ void cv_load_rhs(const CvSolveArgs &a, uint32_t F, double *y, double lam) {
    for (uint32_t u = threadIdx.x; u < F; u += blockDim.x) {
        const uint32_t r = u / a.K, k = u - r * a.K;
        double v = a.b[u];
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
        int attempt = 0;
        for (; attempt < 4; ++attempt, ridge *= 100.0) {
            // lower triangle of the normal matrix
            for (uint32_t u = tid / 32; u < F; u += nt / 32)
                for (uint32_t v = tid % 32; v <= u; v += 32) A[(size_t)u * F + v] = a.A0[(size_t)u * F + v];
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
                // the panel is factorised by wave 0 alone (its lanes take
                // rows lane, lane + 64, ...), ordered by wave-level fences
                // instead of workgroup barriers
                if (tid < kWave) {
                    for (uint32_t q = 0; q < nb; ++q) {
                        const double piv = P[q * kPanel + q];
                        const double dq = piv > 0.0 ? sqrt(piv) : 1.0;
                        if (tid == 0) {
                            if (!(piv > 0.0)) s_bad = 1;
                            P[q * kPanel + q] = dq;
                        }
                        const double inv = 1.0 / dq;
                        for (uint32_t r = q + 1 + tid; r < rows; r += kWave) P[r * kPanel + q] *= inv;
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                        for (uint32_t r = q + 1 + tid; r < rows; r += kWave) {
                            const double l = P[r * kPanel + q];
                            for (uint32_t q2 = q + 1; q2 < nb && q2 <= r; ++q2)
                                P[r * kPanel + q2] -= l * P[q2 * kPanel + q];
                        }
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    }
                }
                __syncthreads();
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
            *a.status = s_bad ? -1 : attempt;
            *a.lam = s_ridge;
        }
        cv_load_rhs(a, F, y, 0.0);
    } else {
        cv_load_rhs(a, F, y, *a.lam);
    }
    __syncthreads();

    // forward substitution L z = y, one panel at a time: the panel's
    // diagonal block goes to LDS, one thread solves it, then every thread
    // updates its rows below
    __shared__ double D[kPanel * kPanel];
    for (uint32_t c0 = 0; c0 < F; c0 += kPanel) {
        const uint32_t nb = min(kPanel, F - c0);
        if (tid < nb * nb) D[tid] = A[(size_t)(c0 + tid / nb) * F + c0 + tid % nb];
        __syncthreads();
        if (tid == 0) {
            for (uint32_t q = 0; q < nb; ++q) {
                double v = y[c0 + q];
                for (uint32_t q2 = 0; q2 < q; ++q2) v -= D[q * nb + q2] * y[c0 + q2];
                y[c0 + q] = v / D[q * nb + q];
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
    // backward substitution L^T w = z by columns of L^T, panels from the
    // last: solve the panel's diagonal block, then every thread removes the
    // panel's unknowns from its rows above, z[r] -= sum_q L[c0 + q][r] w[c0 + q]
    for (uint32_t c0 = ((F - 1) / kPanel) * kPanel;; c0 -= kPanel) {
        const uint32_t nb = min(kPanel, F - c0);
        if (tid < nb * nb) D[tid] = A[(size_t)(c0 + tid / nb) * F + c0 + tid % nb];
        __syncthreads();
        if (tid == 0) {
            for (uint32_t q = nb; q-- > 0;) {
                double v = y[c0 + q];
                for (uint32_t q2 = q + 1; q2 < nb; ++q2) v -= D[q2 * nb + q] * y[c0 + q2];
                y[c0 + q] = v / D[q * nb + q];
            }
        }
        __syncthreads();
        for (uint32_t r = tid; r < c0; r += nt) {
            double v = y[r];
            for (uint32_t q = 0; q < nb; ++q) v -= A[(size_t)(c0 + q) * F + r] * y[c0 + q];
            y[r] = v;
        }
        __syncthreads();
        if (c0 == 0) break;
    }
    for (uint32_t u = tid; u < F; u += nt) {
        const uint32_t r = u / a.K, k = u - r * a.K;
        const size_t o = ((size_t)r * a.d + a.i) * a.K + k;
        const double w = a.refine ? a.w64[o] + y[u] : y[u];
        a.w64[o] = w;
        a.ws[o] = w * sqrt(2.0 * k + 1.0);
    }
}

// Rescales the factors of each rank to equal norms across dimensions (the
// product, hence the model, is unchanged): keeps ALS well conditioned.
__global__ void k_cv_balance(uint32_t R, uint32_t d, uint32_t K, double *w64, double *ws) {
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
            ws[o] = w64[o] * sqrt(2.0 * k + 1.0);
        }
    }
}

// training loss sum_j (yw_j / scale - sw_j g(z_j))^2 and sum_j (yw_j / scale)^2
// (FP64), one pair of partial sums per block
template <int R, int K>
__global__ __launch_bounds__(kBlock) void k_cv_loss(uint32_t n, uint32_t d, const float *z, const float *sw,
                                                   const float *yw, double inv_scale, const double *ws,
                                                   double *partial) {
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    double e2 = 0.0, y2 = 0.0;
    if (j < n) {
        double prod[R];
#pragma unroll
        for (int r = 0; r < R; ++r) prod[r] = 1.0;
        for (uint32_t i = 0; i < d; ++i) {
            double p[K];
            legendre_raw<K, double>((double)z[(size_t)j * d + i], p);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double *w = ws + ((size_t)r * d + i) * K;
                double h = w[K - 1] * p[K - 1];
#pragma unroll
                for (int k = K - 2; k >= 0; --k) h = fma(w[k], p[k], h);
                prod[r] *= h;
            }
        }
        double g = 0.0;
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
using LossFn = void (*)(uint32_t, uint32_t, const float *, const float *, const float *, double, const double *,
                        double *, uint32_t, hipStream_t);
using ResidFn = void (*)(uint32_t, uint32_t, uint32_t, const double *, const double *, const float *, double,
                         const double *, double *, uint32_t, hipStream_t);
using SyrkFn = void (*)(const CvSyrkArgs &, dim3, hipStream_t);

template <int R, int K>
void launch_rho(const CvRhoArgs &a, uint32_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_cv_rho<R, K>), dim3(blocks), dim3(kBlock), 0, s, a);
}
template <int R, int K>
void launch_loss(uint32_t n, uint32_t d, const float *z, const float *sw, const float *yw, double is, const double *ws,
                 double *part, uint32_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_cv_loss<R, K>), dim3(blocks), dim3(kBlock), 0, s, n, d, z, sw, yw, is, ws, part);
}
template <int R, int K>
void launch_resid(uint32_t n, uint32_t d, uint32_t i, const double *rho, const double *phi, const float *yw,
                  double is, const double *w64, double *e, uint32_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_cv_resid<R, K>), dim3(blocks), dim3(kBlock), 0, s, n, d, i, rho, phi, yw, is, w64, e);
}
template <int R, int K, class S0, class S1>
void launch_syrk(const CvSyrkArgs &a, dim3 grid, hipStream_t s) {
    hipLaunchKernelGGL((k_cv_syrk<R, K, S0, S1>), grid, dim3(kBlock), 0, s, a);
}

struct CvFns {
    RhoFn rho;
    LossFn loss;
    ResidFn resid;
    SyrkFn syrk;
};

// (R, K) pairs compiled, with the Gram kernel's task shapes (see
// syrk_tasks for how they cover the triangle)
bool cv_fns(uint32_t R, uint32_t K, CvFns &f) {
#define QMC_CV_CASE(RR, KK, S0, S1)              \
    if (R == RR && K == KK) {                    \
        f.rho = &launch_rho<RR, KK>;             \
        f.loss = &launch_loss<RR, KK>;           \
        f.resid = &launch_resid<RR, KK>;         \
        f.syrk = &launch_syrk<RR, KK, S0, S1>;   \
        return true;                             \
    }
    QMC_CV_CASE(8, 4, ShapeTri1, void) QMC_CV_CASE(8, 8, ShapeTri2, void) QMC_CV_CASE(16, 8, ShapeTri4, void)
    QMC_CV_CASE(16, 12, ShapeTri6, void) QMC_CV_CASE(32, 8, ShapeTri8, void)
    QMC_CV_CASE(32, 12, ShapeHalf12, void) QMC_CV_CASE(32, 16, ShapeTri8, ShapeRect8x4)
    QMC_CV_CASE(64, 12, ShapeHalf12, ShapeRect6x6)
#undef QMC_CV_CASE
    return false;
}

// Tasks covering the lower triangle of NB x NB tiles once, with the shapes
// cv_fns names: NB <= 8 one triangle; NB = 12 two halves; NB = 16 two
// triangles of 8 and the 8 x 8 block below them as two 8 x 4 rectangles;
// NB = 24 two 12-triangles (two halves each) and the 12 x 12 block below as
// four 6 x 6 rectangles.  Fragments are built for blocks [blo, bhi).
std::vector<CvSyrkTask> syrk_tasks(uint32_t NB) {
    std::vector<CvSyrkTask> out;
    auto tri = [&](uint32_t o, const uint32_t (&r)[4], const uint32_t (&c)[4], uint32_t n) {
        CvSyrkTask t{0, o, o + n, {o + r[0], o + r[1], o + r[2], o + r[3]}, {o + c[0], o + c[1], o + c[2], o + c[3]}};
        out.push_back(t);
    };
    switch (NB) {
    case 1: tri(0, {0, 0, 0, 0}, {0, 0, 0, 0}, 1); break;
    case 2: tri(0, {0, 1, 1, 0}, {0, 1, 0, 0}, 2); break;
    case 4: tri(0, {0, 2, 2, 3}, {0, 2, 0, 0}, 4); break;
    case 6: tri(0, {0, 3, 3, 5}, {0, 3, 0, 0}, 6); break;
    case 8: tri(0, {0, 4, 4, 6}, {0, 4, 0, 0}, 8); break;
    case 16:
        for (uint32_t o : {0u, 8u}) tri(o, {0, 4, 4, 6}, {0, 4, 0, 0}, 8);
        for (uint32_t c : {0u, 4u}) out.push_back(CvSyrkTask{1, 0, 16, {8, 10, 12, 14}, {c, c, c, c}});
        break;
    case 12:
    case 24:
        for (uint32_t o = 0; o < NB; o += 12) {
            // half A: rows 0..5 (lower), rows 6..8 x columns 0..5; half B:
            // rows 6..11 (lower), rows 9..11 x columns 0..5 (diagonal
            // regions name their first column block)
            tri(o, {0, 0, 6, 6}, {0, 0, 0, 3}, 9);
            tri(o, {6, 6, 9, 9}, {6, 6, 0, 3}, 12);
        }
        if (NB == 24)
            for (uint32_t a = 0; a < 2; ++a)
                for (uint32_t b = 0; b < 2; ++b) {
                    const uint32_t r = 12 + 6 * a, c = 6 * b;
                    out.push_back(CvSyrkTask{1, c, r + 6, {r, r, r + 3, r + 3}, {c, c + 3, c, c + 3}});
                }
        break;
    default: break;
    }
    return out;
}

// simple seeded generator for the initial factors (SplitMix64)
double splitmix_uniform(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53;
}

uint32_t rhs_splits(uint32_t n) { return std::max<uint32_t>(1, std::min<uint32_t>(1024, (n + 255) / 256)); }

// Device buffers of one training problem (n samples, d dimensions, rank R,
// K Legendre degrees) and the launches of one alternating-least-squares
// step.  Everything is freed with the object.
struct CvTrainer {
    uint32_t n = 0, d = 0, R = 0, K = 0, F = 0, NB = 0;
    uint32_t splits = 1, rsplits = 1, rblocks = 1, nslots = 0, ntasks = 0;
    CvFns fn{};
    DeviceScratch s;
    float *z = nullptr, *sw = nullptr, *yw = nullptr, *partial = nullptr;
    double *rho = nullptr, *phi = nullptr, *rpart = nullptr, *resid = nullptr, *ws = nullptr;
    double *w64 = nullptr, *A0 = nullptr, *A = nullptr, *b = nullptr, *lam = nullptr;
    double *loss_part = nullptr, *abs_part = nullptr;
    int *status = nullptr;
    CvSyrkTask *tasks = nullptr;

    // samples: allocate z, sw, yw too; features: rho, phi and the Gram's
    // and right-hand side's partial sums
    qmc_status init(uint32_t n_, uint32_t d_, uint32_t R_, uint32_t K_, bool samples, bool features) {
        n = n_;
        d = d_;
        R = R_;
        K = K_;
        F = R * K;
        NB = F / 32;
        if (!cv_fns(R, K, fn))
            return fail(QMC_EUNSUPPORTED, "(R, K) = (%u, %u) not compiled; use (32,12), (64,12), (16,8), ...", R, K);
        const std::vector<CvSyrkTask> tk = syrk_tasks(NB);
        if (tk.empty()) return fail(QMC_EUNSUPPORTED, "no Gram task layout for %u blocks", NB);
        ntasks = (uint32_t)tk.size();
        nslots = NB * (NB + 1) / 2;
        // two workgroups per CU in flight: about 512 workgroups in all, each
        // with at least one round of points
        splits = std::max<uint32_t>(1, std::min<uint32_t>(512 / ntasks, (n + kSyrkPts - 1) / kSyrkPts));
        rsplits = rhs_splits(n);
        rblocks = (n + kBlock - 1) / kBlock;
        qmc_status st;
        auto take = [&](size_t bytes, auto *&ptr) -> qmc_status {
            qmc_status r = s.alloc(bytes);
            if (!r) ptr = reinterpret_cast<std::remove_reference_t<decltype(ptr)>>(s.ptr.back());
            return r;
        };
        if ((samples && ((st = take((size_t)n * d * 4, z)) || (st = take((size_t)n * 4, sw)) ||
                         (st = take((size_t)n * 4, yw)))) ||
            (features && ((st = take((size_t)n * R * 8, rho)) || (st = take((size_t)n * K * 8, phi)) ||
                          (st = take((size_t)splits * nslots * 4096, partial)) ||
                          (st = take((size_t)rsplits * F * 8, rpart)) || (st = take((size_t)n * 8, resid)))) ||
            (st = take((size_t)R * d * K * 8, ws)) || (st = take((size_t)R * d * K * 8, w64)) ||
            (st = take(tk.size() * sizeof(CvSyrkTask), tasks)) || (st = take((size_t)F * F * 8, A0)) ||
            (st = take((size_t)F * F * 8, A)) || (st = take((size_t)F * 8, b)) || (st = take(8, lam)) ||
            (st = take(8, status)) || (st = take((size_t)rblocks * 16, loss_part)) ||
            (st = take((size_t)rblocks * 8, abs_part)))
            return st;
        hipError_t e = hipMemcpy(tasks, tk.data(), tk.size() * sizeof(CvSyrkTask), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "training setup");
        return QMC_OK;
    }

    // factors in the orthonormal basis (R, d, K), and a copy with the
    // sqrt(2k+1) normalisation folded in
    qmc_status set_weights(const double *w) {
        std::vector<double> wsh((size_t)R * d * K);
        for (size_t t = 0; t < wsh.size(); ++t) wsh[t] = w[t] * std::sqrt(2.0 * (t % K) + 1.0);
        hipError_t e;
        if ((e = hipMemcpy(w64, w, wsh.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(ws, wsh.data(), wsh.size() * 8, hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "training weights");
        return QMC_OK;
    }

    void features(uint32_t i, hipStream_t st) {
        const CvRhoArgs ra{n, d, i, z, sw, ws, rho, phi};
        fn.rho(ra, rblocks, st);
    }

    // A0 = sum_j a~_j a~_j^T (BF16 MFMA, FP32 accumulation per split, FP64 over splits)
    void gram(hipStream_t st) {
        const CvSyrkArgs ga{n, splits, nslots, rho, phi, tasks, partial};
        fn.syrk(ga, dim3(splits, ntasks), st);
        const uint64_t entries = (uint64_t)F * (F + 1) / 2, per = kBlock / kWave;
        hipLaunchKernelGGL(k_cv_gather, dim3((uint32_t)((entries + per - 1) / per)), dim3(kBlock), 0, st,
                           (const float *)partial, splits, nslots, R, K, A0);
    }

    // b = sum_j rho_j phi_j^T y_j, y = yd, or yf * y_scale when yd is null
    void rhs(const float *yf, double y_scale, const double *yd, hipStream_t st) {
        hipLaunchKernelGGL(k_cv_rhs, dim3(rsplits), dim3(kBlock), 0, st, n, R, K, rsplits, (const double *)rho,
                           (const double *)phi, yf, y_scale, yd, rpart);
        hipLaunchKernelGGL(k_cv_rhs_reduce, dim3((F + kBlock / kWave - 1) / (kBlock / kWave)), dim3(kBlock), 0, st,
                           (const double *)rpart, rsplits, F, b);
    }

    void solve(uint32_t dd, uint32_t i, double ridge, int refine, hipStream_t st) {
        CvSolveArgs so{};
        so.R = R;
        so.K = K;
        so.d = dd;
        so.i = i;
        so.ridge = ridge;
        so.refine = refine;
        so.lam = lam;
        so.A0 = A0;
        so.b = b;
        so.A = A;
        so.w64 = w64;
        so.ws = ws;
        so.status = status;
        hipLaunchKernelGGL(k_cv_solve, dim3(1), dim3(1024), 0, st, so);
    }

    // One alternating-least-squares step for dimension i: FP64 features,
    // the BF16 normal matrix, the FP64 solve, then `refine` refinements
    // against the FP64 residual e = y - A w, whose right-hand side
    // A^T e - lam w comes from the FP64 design matrix: the BF16 matrix only
    // preconditions, so the fixed point is the FP64 least-squares solution.
    void step(uint32_t i, double inv_scale, double ridge, uint32_t refine, hipStream_t st) {
        features(i, st);
        gram(st);
        rhs(yw, inv_scale, nullptr, st);
        solve(d, i, ridge, 0, st);
        for (uint32_t it = 0; it < refine; ++it) {
            fn.resid(n, d, i, rho, phi, yw, inv_scale, w64, resid, rblocks, st);
            rhs(nullptr, 1.0, resid, st);
            solve(d, i, ridge, 1, st);
        }
    }
};

constexpr uint32_t kRefineSteps = 4;

qmc_status check_step_sizes(uint32_t n, uint32_t d, uint32_t R, uint32_t K, uint32_t i) {
    if (n == 0) return fail(QMC_EINVAL, "n must be >= 1");
    if (n > (1u << 26)) return fail(QMC_EUNSUPPORTED, "n > 2^26 training samples");
    if (d == 0) return fail(QMC_EINVAL, "d must be >= 1");
    if (d > 12) return fail(QMC_EUNSUPPORTED, "d > 12");
    if (i >= d) return fail(QMC_EINVAL, "dimension %u >= d = %u", i, d);
    CvFns f;
    if (!cv_fns(R, K, f)) return fail(QMC_EUNSUPPORTED, "(R, K) = (%u, %u) not compiled", R, K);
    return QMC_OK;
}

}  // namespace

}  // namespace qmc

using namespace qmc;

extern "C" {

qmc_status qmc_cv_train(qmc_plan_t p, qmc_family family, const void *params, uint32_t R, uint32_t K,
                        const qmc_cv_train_opts *opts, double *w_out, double *c_out, qmc_cv_train_report *rep) {
    if (!p || !w_out || !c_out) return fail(QMC_EINVAL, "null argument");
    if (family != QMC_F_SECTOR) return fail(QMC_EUNSUPPORTED, "control variates are built for QMC_F_SECTOR");
    CvFns fns;
    if (!cv_fns(R, K, fns))
        return fail(QMC_EUNSUPPORTED, "(R, K) = (%u, %u) not compiled; use (32,12), (64,12), (16,8), ...", R, K);
    if (p->d > 12) return fail(QMC_EUNSUPPORTED, "d > 12");
    const qmc_cv_train_opts o = opts ? *opts : qmc_cv_train_opts{12, 1e-5, 1e-4, 1, 0};
    if (o.refine > 8) return fail(QMC_EINVAL, "refine > 8");
    const uint32_t refine = o.refine ? o.refine : kRefineSteps;
    Packed pk;
    qmc_status st = pack_params((int)family, p->d, params, pk);
    if (st) return st;
    const uint32_t n = p->n, d = p->d;
    hipError_t e;
    std::string err;
    if (pk.orders >= 2) return fail(QMC_EUNSUPPORTED, "control variates take the plain integrand (n_orders < 2)");
    if (pk.deform) return fail(QMC_EUNSUPPORTED, "control variates take undeformed sectors (deform_lambda = 0)");
    hipFunction_t sample = jit_sample_kernel(pk.blob, d, p->tr, pk.cplx, p->device, err);
    if (!sample) return fail(QMC_EUNSUPPORTED, "training sampler: %s", err.c_str());
    if ((st = plan_upload_params(p, pk))) return st;

    CvTrainer t;
    if ((st = t.init(n, d, R, K, true, true))) return st;
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
    std::vector<double> part(2 * (size_t)t.rblocks);
    for (uint32_t comp = 0; comp < pk.np; ++comp) {
        CvSampleArgs sa{};
        sa.n = n;
        sa.d = d;
        sa.inv_n = p->inv_n;
        sa.g = p->d_g;
        sa.shift = p->d_shifts;  // the plan's first shift
        sa.params = p->d_params;
        sa.z = t.z;
        sa.sw = t.sw;
        sa.yw = t.yw;
        sa.part = comp;
        sa.tscale = transform_scale(p->tr, d);
        if ((e = jit_launch_sample(sample, sa, t.rblocks, stream)) != hipSuccess)
            return hip_fail(e, "training sampler");
        hipLaunchKernelGGL(k_cv_absmean, dim3(t.rblocks), dim3(kBlock), 0, stream, n, (const float *)t.yw,
                           t.abs_part);
        if ((e = hipMemcpyAsync(part.data(), t.abs_part, t.rblocks * 8, hipMemcpyDeviceToHost, stream)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(stream)) != hipSuccess)
            return hip_fail(e, "training samples");
        double scale = 0.0;
        for (uint32_t b = 0; b < t.rblocks; ++b) scale += part[b];
        scale /= n;
        if (!(scale > 0.0) || !std::isfinite(scale))
            return fail(QMC_ENONFINITE, "training targets are zero or not finite");

        // initial factors: near-constant with seeded perturbations (breaks the
        // symmetry between ranks)
        std::vector<double> w64((size_t)R * d * K, 0.0);
        uint64_t seed = o.seed ? o.seed : 1;
        const double base = std::pow(1.0 / R, 1.0 / d);
        for (uint32_t r = 0; r < R; ++r)
            for (uint32_t i = 0; i < d; ++i)
                for (uint32_t k = 0; k < K; ++k) {
                    const double u = splitmix_uniform(seed) - 0.5;
                    const double v = k == 0 ? base * (1.0 + 0.5 * u) : 0.1 * base * u / (k + 1);
                    w64[((size_t)r * d + i) * K + k] = v;
                }
        if ((st = t.set_weights(w64.data()))) return st;

        const uint32_t max_sweeps = o.max_sweeps ? o.max_sweeps : 12;
        const double ridge = o.ridge > 0 ? o.ridge : 1e-5;
        double prev = INFINITY, rel = INFINITY, best = INFINITY;
        std::vector<double> w_best(w64.size());
        uint32_t sweeps = 0;
        const double inv_scale = 1.0 / scale;
        for (; sweeps < max_sweeps;) {
            for (uint32_t i = 0; i < d; ++i) t.step(i, inv_scale, ridge, refine, stream);
            ++sweeps;
            hipLaunchKernelGGL(k_cv_balance, dim3((R + 63) / 64), dim3(64), 0, stream, R, d, K, t.w64, t.ws);
            t.fn.loss(n, d, t.z, t.sw, t.yw, inv_scale, t.ws, t.loss_part, t.rblocks, stream);
            if ((e = hipMemcpyAsync(part.data(), t.loss_part, (size_t)t.rblocks * 16, hipMemcpyDeviceToHost,
                                    stream)) != hipSuccess ||
                (e = hipStreamSynchronize(stream)) != hipSuccess)
                return hip_fail(e, "training loop");
            double se = 0.0, sy = 0.0;
            for (uint32_t b = 0; b < t.rblocks; ++b) {
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
                if ((e = hipMemcpy(w_best.data(), t.w64, w_best.size() * 8, hipMemcpyDeviceToHost)) != hipSuccess)
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

qmc_status qmc_cv_samples(qmc_plan_t p, qmc_family family, const void *params, uint32_t part, float *z_out,
                          float *sw_out, float *yw_out) {
    if (!p || !z_out || !sw_out || !yw_out) return fail(QMC_EINVAL, "null argument");
    if (family != QMC_F_SECTOR) return fail(QMC_EUNSUPPORTED, "control variates are built for QMC_F_SECTOR");
    if (p->d > 12) return fail(QMC_EUNSUPPORTED, "d > 12");
    Packed pk;
    qmc_status st = pack_params((int)family, p->d, params, pk);
    if (st) return st;
    if (pk.orders >= 2 || pk.deform)
        return fail(QMC_EUNSUPPORTED, "control variates take the plain, undeformed integrand");
    if (part >= pk.np) return fail(QMC_EINVAL, "part %u of a %s integrand", part, pk.cplx ? "complex" : "real");
    std::string err;
    hipFunction_t sample = jit_sample_kernel(pk.blob, p->d, p->tr, pk.cplx, p->device, err);
    if (!sample) return fail(QMC_EUNSUPPORTED, "training sampler: %s", err.c_str());
    if ((st = plan_upload_params(p, pk))) return st;
    const uint32_t n = p->n, d = p->d, blocks = (n + kBlock - 1) / kBlock;
    DeviceScratch s;
    if ((st = s.alloc((size_t)n * d * 4)) || (st = s.alloc((size_t)n * 4)) || (st = s.alloc((size_t)n * 4)))
        return st;
    CvSampleArgs sa{};
    sa.n = n;
    sa.d = d;
    sa.inv_n = p->inv_n;
    sa.g = p->d_g;
    sa.shift = p->d_shifts;
    sa.params = p->d_params;
    sa.z = (float *)s.ptr[0];
    sa.sw = (float *)s.ptr[1];
    sa.yw = (float *)s.ptr[2];
    sa.part = part;
    sa.tscale = transform_scale(p->tr, d);
    hipError_t e = jit_launch_sample(sample, sa, blocks, p->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(z_out, s.ptr[0], (size_t)n * d * 4, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(sw_out, s.ptr[1], (size_t)n * 4, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(yw_out, s.ptr[2], (size_t)n * 4, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "training samples");
    return QMC_OK;
}

qmc_status qmc_cv_features(uint32_t n, uint32_t d, uint32_t R, uint32_t K, uint32_t i, const float *z,
                           const float *sw, const double *w, double *rho_out, double *phi_out) {
    if (!z || !sw || !w || !rho_out || !phi_out) return fail(QMC_EINVAL, "null argument");
    qmc_status st = check_step_sizes(n, d, R, K, i);
    if (st) return st;
    for (size_t t = 0; t < (size_t)R * d * K; ++t)
        if (!std::isfinite(w[t])) return fail(QMC_EINVAL, "W not finite");
    CvTrainer t;
    if ((st = t.init(n, d, R, K, true, true)) || (st = t.set_weights(w))) return st;
    hipError_t e;
    if ((e = hipMemcpy(t.z, z, (size_t)n * d * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(t.sw, sw, (size_t)n * 4, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "features upload");
    t.features(i, nullptr);
    if ((e = hipMemcpy(rho_out, t.rho, (size_t)n * R * 8, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(phi_out, t.phi, (size_t)n * K * 8, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "features download");
    return QMC_OK;
}

qmc_status qmc_cv_normal(uint32_t n, uint32_t R, uint32_t K, const double *rho, const double *phi, const double *y,
                         double *gram_out, double *rhs_out, uint32_t *acc_len_out) {
    if (!rho || !phi || !y || !gram_out || !rhs_out) return fail(QMC_EINVAL, "null argument");
    qmc_status st = check_step_sizes(n, 1, R, K, 0);
    if (st) return st;
    CvTrainer t;
    if ((st = t.init(n, 1, R, K, false, true))) return st;
    hipError_t e;
    if ((e = hipMemcpy(t.rho, rho, (size_t)n * R * 8, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(t.phi, phi, (size_t)n * K * 8, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(t.resid, y, (size_t)n * 8, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "normal-equation upload");
    t.gram(nullptr);
    t.rhs(nullptr, 1.0, t.resid, nullptr);
    const uint32_t F = t.F;
    std::vector<double> A((size_t)F * F);
    if ((e = hipMemcpy(A.data(), t.A0, A.size() * 8, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(rhs_out, t.b, (size_t)F * 8, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "normal-equation download");
    for (uint32_t u = 0; u < F; ++u)
        for (uint32_t v = 0; v <= u; ++v) gram_out[(size_t)u * F + v] = gram_out[(size_t)v * F + u] = A[(size_t)u * F + v];
    if (acc_len_out) {
        acc_len_out[0] = (n + t.splits - 1) / t.splits;
        acc_len_out[1] = (n + t.rsplits - 1) / t.rsplits;
    }
    return QMC_OK;
}

qmc_status qmc_cv_solve(uint32_t R, uint32_t K, const double *gram, const double *rhs, double ridge,
                        double *lam_out, double *x_out, int32_t *escalations) {
    if (!gram || !rhs || !x_out) return fail(QMC_EINVAL, "null argument");
    if (!(ridge > 0.0) || !std::isfinite(ridge)) return fail(QMC_EINVAL, "ridge must be positive and finite");
    qmc_status st = check_step_sizes(1, 1, R, K, 0);
    if (st) return st;
    const uint32_t F = R * K;
    for (size_t t = 0; t < (size_t)F * F; ++t)
        if (!std::isfinite(gram[t])) return fail(QMC_EINVAL, "matrix not finite");
    for (uint32_t u = 0; u < F; ++u)
        if (!std::isfinite(rhs[u])) return fail(QMC_EINVAL, "right-hand side not finite");
    CvTrainer t;
    if ((st = t.init(1, 1, R, K, false, false))) return st;
    hipError_t e;
    if ((e = hipMemcpy(t.A0, gram, (size_t)F * F * 8, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(t.b, rhs, (size_t)F * 8, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "solve upload");
    t.solve(1, 0, ridge, 0, nullptr);
    int32_t esc = 0;
    double lam = 0.0;
    if ((e = hipMemcpy(x_out, t.w64, (size_t)F * 8, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(&esc, t.status, 4, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(&lam, t.lam, 8, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "solve download");
    if (lam_out) *lam_out = lam;
    if (escalations) *escalations = esc;
    if (esc < 0) return fail(QMC_ENONFINITE, "matrix not positive definite after raising the ridge 10^6-fold");
    return QMC_OK;
}

qmc_status qmc_cv_als_step(uint32_t n, uint32_t d, uint32_t R, uint32_t K, uint32_t i, const float *z,
                           const float *sw, const float *yw, double scale, const double *w_in, double ridge,
                           uint32_t refine, double *w_out, double *lam_out) {
    if (!z || !sw || !yw || !w_in || !w_out) return fail(QMC_EINVAL, "null argument");
    qmc_status st = check_step_sizes(n, d, R, K, i);
    if (st) return st;
    if (!(scale > 0.0) || !std::isfinite(scale)) return fail(QMC_EINVAL, "scale must be positive and finite");
    if (!(ridge > 0.0) || !std::isfinite(ridge)) return fail(QMC_EINVAL, "ridge must be positive and finite");
    if (refine > 8) return fail(QMC_EINVAL, "refine > 8");
    for (size_t t = 0; t < (size_t)R * d * K; ++t)
        if (!std::isfinite(w_in[t])) return fail(QMC_EINVAL, "W not finite");
    CvTrainer t;
    if ((st = t.init(n, d, R, K, true, true)) || (st = t.set_weights(w_in))) return st;
    hipError_t e;
    if ((e = hipMemcpy(t.z, z, (size_t)n * d * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(t.sw, sw, (size_t)n * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(t.yw, yw, (size_t)n * 4, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "step upload");
    t.step(i, 1.0 / scale, ridge, refine, nullptr);
    int32_t esc = 0;
    double lam = 0.0;
    if ((e = hipMemcpy(w_out, t.w64, (size_t)R * d * K * 8, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(&esc, t.status, 4, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(&lam, t.lam, 8, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "step download");
    if (lam_out) *lam_out = lam;
    if (esc < 0) return fail(QMC_ENONFINITE, "normal matrix not positive definite after raising the ridge");
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
    CvFns fns;
    if (!cv_fns(R, K, fns)) return fail(QMC_EUNSUPPORTED, "(R, K) = (%u, %u) not compiled", R, K);
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
