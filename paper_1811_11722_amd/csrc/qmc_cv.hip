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
// a rank-N sum of R x R outer products, which k_cv_syrk2 / k_cv_syrk
// accumulate with BF16 MFMA (v_mfma_f32_32x32x16_bf16: 32 x 32 tiles, 16
// points per instruction, FP32 accumulation).  The per-split tiles are added
// in a fixed order in FP64, factorised in FP64 by a blocked Cholesky over
// many workgroups (k_cv_chol_*), which also forms the explicit inverse.  That
// inverse preconditions passes against the FP64 design matrix (k_cv_pass,
// FP64 MFMA; k_cv_gemv and k_cv_subst apply the correction), so each step
// converges to the FP64 ridge solution.  The trained model is evaluated in
// FP64 inside the estimator.
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
//   rho_j[r] = sw_j prod_{i' != i} h_{r,i'}(z_{j,i'}),  phi_j[k] = P~_k(z_{j,i}),
// h_{r,i'}(z) = sum_k ws[r, i', k] P_k(z) on v_mfma_f64_16x16x4f64: A = the
// Legendre values (lane l: point l % 16, degree 4 s + l / 16), B = the
// weights.  Up to 32 ranks a wave takes 64 points at a time, each lane runs
// the recurrence of one point and the values reach the A layout through
// LDS (four 16-point blocks); 64 ranks take 16 points at a time, each lane
// running the recurrence of its A-operand point, with the weight fragments
// staged in LDS once per workgroup.  The coordinates of a point are all
// loaded before the first is used.  The product over
// dimensions is taken elementwise on the output tiles (element v of lane l:
// point 4 v + l / 16, rank 16 t + l % 16), which are also the layout of the
// 128-byte rows of rho the lanes store.
struct CvRhoArgs {
    uint32_t n, d, i;       // points, dimension, the dimension being solved
    const float *z, *sw;    // (n, d), (n)
    const double *ws;       // W * sqrt(2k+1), (R, d, K)
    double *rho;            // (n, R)
    double *phi;            // (n, K) (normalised)
};

constexpr uint32_t kCvMaxD = 12;

template <int R, int K>
__global__ __launch_bounds__(kBlock) void k_cv_rho(const CvRhoArgs a) {
    constexpr int RT = (R + 15) / 16, KS = (K + 3) / 4, NP = 4 * KS;
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const uint32_t li = lane & 15, lg = lane >> 4;
    if constexpr (R <= 32) {
        // 64 points per wave at a time: lane l runs the recurrence of point
        // p0 + l only, and the values reach the operand layout through the
        // wave's own LDS rows (a wave's LDS accesses complete in order);
        // the weight fragments come from memory, one dimension ahead
        constexpr uint32_t LP = NP + 1;  // padded row of a point's values
        __shared__ double lv[4][kWave * LP];
        double *lw = lv[wave];
        auto weights = [&](uint32_t i, double (&wb)[RT][KS]) {
#pragma unroll
            for (int t = 0; t < RT; ++t)
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    const uint32_t r = 16 * t + li, k = 4 * s + lg;
                    wb[t][s] = (r < (uint32_t)R && k < (uint32_t)K)
                                   ? a.ws[((size_t)r * a.d + i) * K + k] : 0.0;
                }
        };
        for (uint32_t p0 = (blockIdx.x * 4 + wave) * 64; p0 < a.n; p0 += gridDim.x * 256) {
            const uint32_t pm = p0 + lane, pc = pm < a.n ? pm : a.n - 1;
            float zr[kCvMaxD];
#pragma unroll
            for (uint32_t i = 0; i < kCvMaxD; ++i) zr[i] = a.z[(size_t)pc * a.d + (i < a.d ? i : a.d - 1)];
            cv_d4 prod[4][RT];
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int t = 0; t < RT; ++t) prod[c][t] = cv_d4{1.0, 1.0, 1.0, 1.0};
            double wb[RT][KS];
            weights(a.i == 0 ? (a.d > 1 ? 1 : 0) : 0, wb);
#pragma unroll 1
            for (uint32_t i = 0; i < a.d; ++i) {
                double pk[NP];
                legendre_raw<NP, double>(pm < a.n ? (double)zr[i] : 0.5, pk);
                if (i == a.i) {
                    if (pm < a.n) {
#pragma unroll
                        for (int k = 0; k < K; ++k) a.phi[(size_t)pm * K + k] = pk[k] * sqrt((double)(2 * k + 1));
                    }
                    continue;
                }
                // the next dimension's weights while this one is computed
                uint32_t in = i + 1 == a.i ? i + 2 : i + 1;
                in = in < a.d ? in : i;
                double wn[RT][KS];
                weights(in, wn);
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int k = 0; k < NP; ++k) lw[lane * LP + k] = pk[k];
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    double fa[KS];
#pragma unroll
                    for (int s = 0; s < KS; ++s) fa[s] = lw[(16 * c + li) * LP + 4 * s + lg];
#pragma unroll
                    for (int t = 0; t < RT; ++t) {
                        cv_d4 h = cv_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                        for (int s = 0; s < KS; ++s) h = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s], wb[t][s], h, 0, 0, 0);
                        prod[c][t] *= h;
                    }
                    // one 16-point block at a time: fewer registers live
                    __builtin_amdgcn_sched_barrier(0);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int t = 0; t < RT; ++t)
#pragma unroll
                    for (int s = 0; s < KS; ++s) wb[t][s] = wn[t][s];
            }
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const uint32_t p = p0 + 16 * c + 4 * v + lg;
                    if (p < a.n) {
                        const double sw = a.sw[p];
#pragma unroll
                        for (int t = 0; t < RT; ++t) {
                            const uint32_t r = 16 * t + li;
                            if (r < (uint32_t)R) a.rho[(size_t)p * R + r] = sw * prod[c][t][v];
                        }
                    }
                }
        }
    } else {
        __shared__ double wf[kCvMaxD * RT * KS * kWave];  // ((i RT + t) KS + s) 64 + lane
        for (uint32_t f = tid; f < a.d * RT * KS * kWave; f += kBlock) {
            const uint32_t fl = f % kWave, idx = f / kWave, s = idx % KS, t = (idx / KS) % RT, i = idx / (KS * RT);
            const uint32_t r = 16 * t + fl % 16, k = 4 * s + fl / 16;
            wf[f] = (r < (uint32_t)R && k < (uint32_t)K) ? a.ws[((size_t)r * a.d + i) * K + k] : 0.0;
        }
        __syncthreads();
        const bool s1 = lg == 1, s2 = lg == 2, s3 = lg == 3;
        for (uint32_t p0 = (blockIdx.x * 4 + wave) * 16; p0 < a.n; p0 += gridDim.x * 64) {
            cv_d4 prod[RT];
#pragma unroll
            for (int t = 0; t < RT; ++t) prod[t] = cv_d4{1.0, 1.0, 1.0, 1.0};
            const uint32_t pa = p0 + li;  // this lane's point in the A operand
            // the point's coordinates, all loaded before any is used (branch-free:
            // index clamped, so that the chunk waits on memory once)
            const uint32_t pc = pa < a.n ? pa : a.n - 1;
            float zr[kCvMaxD];
#pragma unroll
            for (uint32_t i = 0; i < kCvMaxD; ++i) zr[i] = a.z[(size_t)pc * a.d + (i < a.d ? i : a.d - 1)];
#pragma unroll
            for (uint32_t i = 0; i < kCvMaxD; ++i) {
                if (i >= a.d) break;
                const double zz = pa < a.n ? (double)zr[i] : 0.5;
                double pk[4 * KS];
                legendre_raw<4 * KS, double>(zz, pk);
                double fa[KS];
#pragma unroll
                for (int s = 0; s < KS; ++s) fa[s] = cv_pick4(pk[4 * s], pk[4 * s + 1], pk[4 * s + 2], pk[4 * s + 3], s1, s2, s3);
                if (i == a.i) {
#pragma unroll
                    for (int s = 0; s < KS; ++s) {
                        const uint32_t k = 4 * s + lg;
                        if (pa < a.n && k < (uint32_t)K) a.phi[(size_t)pa * K + k] = fa[s] * sqrt((double)(2 * k + 1));
                    }
                    continue;
                }
#pragma unroll
                for (int t = 0; t < RT; ++t) {
                    cv_d4 h = cv_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int s = 0; s < KS; ++s)
                        h = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s], wf[((i * RT + t) * KS + s) * kWave + lane], h, 0, 0, 0);
                    prod[t] *= h;
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint32_t p = p0 + 4 * v + lg;
                if (p < a.n) {
                    const double sw = a.sw[p];
#pragma unroll
                    for (int t = 0; t < RT; ++t) {
                        const uint32_t r = 16 * t + li;
                        if (r < (uint32_t)R) a.rho[(size_t)p * R + r] = sw * prod[t][v];
                    }
                }
            }
        }
    }
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
    uint32_t n, splits, nslots, ntasks;
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

// The same accumulation with two tasks per workgroup of 8 waves (waves 0-3
// take task 2 y, waves 4-7 task 2 y + 1), so that each round's rho and phi
// are read and turned into fragments once for both: for the triangle of 12
// blocks (its two halves) the features are read once in all.  All NB
// blocks' fragments are built (wave w: 16-point group w % 4, blocks
// w / 4, w / 4 + 2, ...).  One workgroup per CU.
template <int R, int K, class S0, class S1>
__global__ __launch_bounds__(2 * kBlock, 1) void k_cv_syrk2(const CvSyrkArgs a) {
    constexpr int NB = R * K / 32;
    constexpr uint32_t nt = 2 * kBlock;
    constexpr int NV = (kSyrkPts * (R + K) + nt - 1) / nt;  // staged values per thread
    __shared__ float srho[kSyrkPts * R], sphi[kSyrkPts * K];
    __shared__ bf16x8 frag[NB * 4 * kWave];
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave, w4 = wave & 3;
    const uint32_t ti = 2 * blockIdx.y + (wave >> 2);
    const bool active = ti < a.ntasks;
    const uint32_t type = active ? a.tasks[ti].type : 0;
    // the wave's bases straight from memory (indexing a private copy by the
    // wave number would put it in scratch)
    const uint32_t r0 = active ? a.tasks[ti].r0[w4] : 0, c0 = active ? a.tasks[ti].c0[w4] : 0;
    const uint32_t j_begin = (uint32_t)((uint64_t)a.n * blockIdx.x / a.splits);
    const uint32_t j_end = (uint32_t)((uint64_t)a.n * (blockIdx.x + 1) / a.splits);

    f32x16 acc[kSyrkMaxTiles];
#pragma unroll
    for (int t = 0; t < kSyrkMaxTiles; ++t)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[t][e] = 0.0f;

    double nxt[NV];
    auto load_round = [&](uint32_t base) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const uint32_t v = tid + q * nt;
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
            const uint32_t v = tid + q * nt;
            if (v < (uint32_t)(kSyrkPts * R)) srho[v] = (float)nxt[q];
            else if (v < (uint32_t)(kSyrkPts * (R + K))) sphi[v - kSyrkPts * R] = (float)nxt[q];
        }
        if (base + kSyrkPts < j_end) load_round(base + kSyrkPts);
        __syncthreads();
        {
            const uint32_t half = lane >> 5, c = lane & 31;
            for (uint32_t b = wave >> 2; b < (uint32_t)NB; b += 2) {
                const uint32_t u = 32 * b + c, k = u / R, r = u - k * R;
                bf16x8 f;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint32_t p = 16 * w4 + 8 * half + e;
                    f[e] = (__bf16)(srho[p * R + r] * sphi[p * K + k]);
                }
                frag[(b * 4 + w4) * kWave + lane] = f;
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const bf16x8 *fr = frag + s * kWave;
                if (type == 0) {
                    switch (w4) {
                    case 0: syrk_step<S0, 0>(fr, lane, r0, c0, acc); break;
                    case 1: syrk_step<S0, 1>(fr, lane, r0, c0, acc); break;
                    case 2: syrk_step<S0, 2>(fr, lane, r0, c0, acc); break;
                    default: syrk_step<S0, 3>(fr, lane, r0, c0, acc); break;
                    }
                } else if constexpr (!std::is_same<S1, void>::value) {
                    switch (w4) {
                    case 0: syrk_step<S1, 0>(fr, lane, r0, c0, acc); break;
                    case 1: syrk_step<S1, 1>(fr, lane, r0, c0, acc); break;
                    case 2: syrk_step<S1, 2>(fr, lane, r0, c0, acc); break;
                    default: syrk_step<S1, 3>(fr, lane, r0, c0, acc); break;
                    }
                }
            }
        }
    }
    if (!active) return;
    float *out = a.partial + (size_t)blockIdx.x * a.nslots * 1024;
    if (type == 0) {
        switch (w4) {
        case 0: syrk_store<S0, 0>(lane, r0, c0, acc, out); break;
        case 1: syrk_store<S0, 1>(lane, r0, c0, acc, out); break;
        case 2: syrk_store<S0, 2>(lane, r0, c0, acc, out); break;
        default: syrk_store<S0, 3>(lane, r0, c0, acc, out); break;
        }
    } else if constexpr (!std::is_same<S1, void>::value) {
        switch (w4) {
        case 0: syrk_store<S1, 0>(lane, r0, c0, acc, out); break;
        case 1: syrk_store<S1, 1>(lane, r0, c0, acc, out); break;
        case 2: syrk_store<S1, 2>(lane, r0, c0, acc, out); break;
        default: syrk_store<S1, 3>(lane, r0, c0, acc, out); break;
        }
    }
}

// Sum the per-split tiles in split order, in FP64, into the lower triangle
// of the normal matrix A0 (F x F row-major, rows and columns u = r K + k):
// one thread per tile element (consecutive threads read consecutive
// elements of each split), adding the splits in order.  Tile element
// (i, j) of slot bu (bu + 1) / 2 + bv is columns u' = 32 bu + i, 32 bv + j
// in the order u' = k R + r; the upper part of a diagonal tile is skipped.
__global__ __launch_bounds__(kBlock) void k_cv_gather(const float *partial, uint32_t splits, uint32_t nslots,
                                                     uint32_t R, uint32_t K, double *A0) {
    const uint32_t F = R * K, g = blockIdx.x * kBlock + threadIdx.x;
    if (g >= nslots * 1024) return;
    const uint32_t slot = g >> 10, i = (g >> 5) & 31, j = g & 31;
    uint32_t bu = (uint32_t)((sqrt(8.0 * (double)slot + 1.0) - 1.0) * 0.5);
    while (bu * (bu + 1) / 2 > slot) --bu;
    while ((bu + 1) * (bu + 2) / 2 <= slot) ++bu;
    const uint32_t bv = slot - bu * (bu + 1) / 2;
    const uint32_t a = 32 * bu + i, b = 32 * bv + j;
    if (b > a) return;
    const size_t stride = (size_t)nslots * 1024;
    double s = 0.0;
#pragma unroll 16
    for (uint32_t sp = 0; sp < splits; ++sp) s += (double)partial[sp * stride + g];
    const uint32_t ka = a / R, ra = a - ka * R, kb = b / R, rb = b - kb * R;
    const uint32_t u = ra * K + ka, v = rb * K + kb;
    if (u >= v) A0[(size_t)u * F + v] = s;
    else A0[(size_t)v * F + u] = s;
}

// One pass over the training set for the right-hand side of dimension i:
//   part[split][u] = sum_{j in split} rho_j[r] phi_j[k] e_j,  u = r K + k,
//   e_j = yf_j y_scale - sum_{r,k} rho_j[r] phi_j[k] w[r, i, k]   (training), or
//   e_j = yd_j                                                 (NORMAL);
// FP64 throughout, on
// v_mfma_f64_16x16x4f64 (A[i][k] and B[k][j] at lane i (or j) + 16 k;
// output element v of lane l at row 4 v + l / 16, column l % 16).  A wave
// takes 16 points at a time:
//   1. H = Phi W^T (16 points x 16 ranks per tile; A: lane l holds
//      phi[point l % 16][4 s + l / 16], B: the weights, kept in registers),
//      so lane l holds H at point 4 v + l / 16 and rank 16 t + l % 16;
//   2. rho is read in that layout (128-byte rows), and the 16 lanes of a
//      point add rho H (row16_sum): e of the point;
//   3. the right-hand side tile accumulates (rho e)^T Phi, 4 points per
//      instruction: A = rho e as held, B = phi[point 4 g + l / 16][l % 16]
//      (0 for Legendre indices >= K).
// Waves take 16-point chunks in turn over the workgroup's range (all the
// loads of a chunk first, so that it waits on memory once); their tiles
// are added in wave order.  Entry R K of a split's partials is its sum of
// e_j^2 (the objective of the current factor).  A set *flag (a converged
// solve) makes the kernel return at once.
// Sum over the 16 lanes of a row (every lane gets it) with DPP moves: xor 1
// and xor 2 within quads, then the half-row and row mirrors, which pair each
// quad with its partner quad as the xor-4 and xor-8 butterfly does (the
// partner's quad sums are uniform), so the result equals that butterfly's bit
// for bit; cross-lane moves at VALU latency instead of LDS permutes.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row16_sum(double v) {
    v += dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x141>(v);  // row_half_mirror
    v += dpp_d<0x140>(v);  // row_mirror
    return v;
}

struct CvPassArgs {
    uint32_t n, d, i, splits;
    const double *rho, *phi;  // (n, R), (n, K)
    const float *yf;          // targets (float) times y_scale, or
    double y_scale;
    const double *yd;         // targets (double), if not null
    const double *w;          // (R, d, K) model in the normalised basis, or null
    const int *flag;          // nullable
    double *part;             // (splits, R K + 1)
};

template <int R, int K, bool NORMAL>
__global__ __launch_bounds__(kBlock) void k_cv_pass(const CvPassArgs a) {
    constexpr int RT = (R + 15) / 16, KS = (K + 3) / 4;
    static_assert(K <= 16 && RT <= 4, "one B tile of Legendre indices, at most 4 rank tiles");
    if (a.flag && *a.flag) return;
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const uint32_t li = lane & 15, lg = lane >> 4;
    const uint32_t j0 = (uint32_t)((uint64_t)a.n * blockIdx.x / a.splits);
    const uint32_t j1 = (uint32_t)((uint64_t)a.n * (blockIdx.x + 1) / a.splits);
    double wb[RT][KS];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const uint32_t r = 16 * t + li, k = 4 * s + lg;
            wb[t][s] = (!NORMAL && r < (uint32_t)R && k < (uint32_t)K) ? a.w[((size_t)r * a.d + a.i) * K + k] : 0.0;
        }
    cv_d4 acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t] = cv_d4{0.0, 0.0, 0.0, 0.0};
    double e2 = 0.0;  // lanes l < 16 add e^2 of points 4 v + l / 16 ... one lane per point
    // Every operand of a 16-point chunk is loaded first, branch-free (indices
    // clamped into the range, values outside it zeroed afterwards), so that
    // a chunk waits on memory once.
    const uint32_t rl = li < (uint32_t)R ? li : 0;  // rank lane, clamped (R = 8)
    const uint32_t kl = li < (uint32_t)K ? li : 0;           // Legendre lane, clamped
    for (uint32_t p0 = j0 + 16 * wave; p0 < j1; p0 += 64) {
        double rh[RT][4], y[4], fa[KS], fb[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const uint32_t p = p0 + 4 * v + lg, pc = p < j1 ? p : j1 - 1;
#pragma unroll
            for (int t = 0; t < RT; ++t) rh[t][v] = a.rho[(size_t)pc * R + (16 * t + rl)];
            y[v] = NORMAL ? a.yd[pc] : (double)a.yf[pc] * a.y_scale;
            fb[v] = a.phi[(size_t)pc * K + kl];
        }
        {
            const uint32_t p = p0 + li, pc = p < j1 ? p : j1 - 1;
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const uint32_t k = 4 * s + lg;
                fa[s] = a.phi[(size_t)pc * K + (k < (uint32_t)K ? k : 0)];
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const bool in = p0 + 4 * v + lg < j1;
#pragma unroll
            for (int t = 0; t < RT; ++t) rh[t][v] = (in && 16 * t + li < (uint32_t)R) ? rh[t][v] : 0.0;
            y[v] = in ? y[v] : 0.0;
            fb[v] = (in && li < (uint32_t)K) ? fb[v] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < KS; ++s) fa[s] = (p0 + li < j1 && 4 * s + lg < (uint32_t)K) ? fa[s] : 0.0;
        double e[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) e[v] = y[v];
        if (!NORMAL) {
            double dot[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                cv_d4 h = cv_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < KS; ++s) h = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s], wb[t][s], h, 0, 0, 0);
#pragma unroll
                for (int v = 0; v < 4; ++v) dot[v] = fma(rh[t][v], h[v], dot[v]);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) e[v] -= row16_sum(dot[v]);
        }
        if (li == 0) {
#pragma unroll
            for (int v = 0; v < 4; ++v) e2 = fma(e[v], e[v], e2);
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
#pragma unroll
            for (int t = 0; t < RT; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(rh[t][g] * e[g], fb[g], acc[t], 0, 0, 0);
        }
    }
    // tiles of the 4 waves, added in wave order; element v of lane l is
    // rank 16 t + 4 v + l / 16, Legendre index l % 16
    __shared__ double red[4][RT * 256];
    __shared__ double se2[4][4];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wave][t * 256 + (4 * v + lg) * 16 + li] = acc[t][v];
    if (li == 0) se2[wave][lg] = e2;
    __syncthreads();
    constexpr uint32_t FP = R * K + 1;
    for (uint32_t u = tid; u < (uint32_t)(R * K); u += kBlock) {
        const uint32_t r = u / K, k = u - r * K, o = (r / 16) * 256 + (r % 16) * 16 + k;
        a.part[(size_t)blockIdx.x * FP + u] = ((red[0][o] + red[1][o]) + red[2][o]) + red[3][o];
    }
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < 4; ++w)
            for (int g = 0; g < 4; ++g) s += se2[w][g];
        a.part[(size_t)blockIdx.x * FP + R * K] = s;
    }
}

// b[u] = sum over splits of the partials: one wave per column, lanes take
// splits lane, lane + 64, ... in order, then a fixed butterfly over the lanes
// (F counts the extra entry of the pass: R K + 1 columns)
__global__ __launch_bounds__(kBlock) void k_cv_rhs_reduce(const double *part, uint32_t splits, uint32_t F,
                                                         const int *flag, double *b) {
    if (flag && *flag) return;
    const uint32_t u = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    if (u >= F) return;
    double s = 0.0;
    for (uint32_t sp = lane; sp < splits; sp += kWave) s += part[(size_t)sp * F + u];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) b[u] = s;
}

// ------------------------------------------------------------ the solve
// Escalation path of the factorisation (the main path is k_cv_chol_diag0 /
// k_cv_chol_step below; this kernel runs only when that one met a
// non-positive pivot).
// (A0 + lam I) = L L^T by a blocked right-looking Cholesky in one workgroup
// of 512 threads, panels of B columns (B = 32, or 16 when F > 512 so that
// the panel fits in LDS):
//   1. the diagonal block and the rows below are staged in LDS (coalesced
//      reads); wave 0 factorises the block in registers (lane r holds row
//      r; each column is scaled, then the lanes below take the rank-1
//      update with the column's entries broadcast by readlane);
//   2. wave 0 also forms W = L_pp^-1 (lane c: column c by forward
//      substitution), and the rows below become X = A_panel W^T, a matrix
//      product on FP64 MFMA; the panel goes back to A;
//   3. the trailing lower triangle takes A -= P P^T in 16 x 16 tiles on
//      FP64 MFMA; the panel sits in LDS transposed (column q of the panel
//      contiguous), so consecutive lanes read consecutive rows.
// lam = ridge * trace / F (trace summed in index order); a non-positive
// pivot restarts with a 100x larger ridge (at most three times).  The
// factor overwrites A (lower triangle), rdiag receives 1 / L_uu, *status the
// number of escalations (-1: failed), *lam the ridge, and *flag is cleared
// for the solves that follow.  With first > 0 the kernel starts at that
// attempt (ridge * 100^first) and returns at once unless *status < 0.
struct CvFactorArgs {
    uint32_t F;
    double ridge;           // relative to the mean diagonal
    const double *A0;       // (F, F) assembled normal matrix, lower triangle
    double *A;              // (F, F) factor
    double *rdiag;          // (F) reciprocals of the factor's diagonal
    double *lam;
    int *status;
    int *flag;
    uint32_t first;
};

constexpr uint32_t kMaxF = 768;  // largest R K compiled: (64, 12)
// 512 threads leave 256 registers per lane for the unrolled panel solve
constexpr uint32_t kFactorThreads = 512;

__device__ __forceinline__ double readlane_d(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

template <int B>
__global__ __launch_bounds__(kFactorThreads) void k_cv_factor(const CvFactorArgs a) {
    // panel rows per LDS column: F - B at most, plus 2 so that the columns
    // start in different banks (and stay 16-byte aligned)
    constexpr uint32_t LD = (B == 32 ? 512u : kMaxF) - B + 2;
    constexpr uint32_t nt = kFactorThreads;
    const uint32_t F = a.F, tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    __shared__ __align__(16) double PT[B * LD];  // panel, PT[q * LD + row]
    constexpr uint32_t DP = B + 1;               // padded row of the diagonal block
    __shared__ double D[B * DP];                 // the diagonal block's factor
    __shared__ double Wl[B * DP];                // its inverse, W = L_pp^-1
    __shared__ double sdiag[kMaxF];              // the diagonal, for the trace in index order
    __shared__ double s_ridge;
    __shared__ int s_bad;
    if (a.first > 0 && *a.status >= 0) return;
    double *A = a.A;
    double ridge = a.ridge;
    int attempt = 0;
    for (; attempt < (int)a.first; ++attempt) ridge *= 100.0;
    for (; attempt < 4; ++attempt, ridge *= 100.0) {
        for (uint32_t u = tid / 32; u < F; u += nt / 32)
            for (uint32_t v = tid % 32; v <= u; v += 32) {
                const double x = a.A0[(size_t)u * F + v];
                A[(size_t)u * F + v] = x;
                if (u == v) sdiag[u] = x;
            }
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (uint32_t u = 0; u < F; ++u) t += sdiag[u];
            s_ridge = ridge * t / F + 1e-300;
            s_bad = 0;
        }
        __syncthreads();
        for (uint32_t u = tid; u < F; u += nt) A[(size_t)u * F + u] += s_ridge;
        __syncthreads();

        for (uint32_t c0 = 0; c0 < F; c0 += B) {
            const uint32_t c1 = c0 + B, M = F - c1;
            // 1. the diagonal block (to D) and the rows below (to PT) go to
            // LDS, then wave 0 factorises the block
            for (uint32_t t = tid; t < B * B; t += nt) {
                const uint32_t r = t / B, q = t - r * B;
                D[r * DP + q] = q <= r ? A[(size_t)(c0 + r) * F + c0 + q] : 0.0;
            }
            for (uint32_t t = tid; t < M * B; t += nt) {
                const uint32_t r = t / B, q = t - r * B;
                PT[q * LD + r] = A[(size_t)(c1 + r) * F + c0 + q];
            }
            __syncthreads();
            if (wave == 0) {
                // lane r holds row r of the block; entries right of the
                // diagonal are never read, so the updates need no masks
                double row[B];
#pragma unroll
                for (int c = 0; c < B; ++c) row[c] = lane < (uint32_t)B ? D[lane * DP + c] : 0.0;
                bool bad = false;
#pragma unroll
                for (int q = 0; q < B; ++q) {
                    const double piv = readlane_d(row[q], q);
                    bad = bad || !(piv > 0.0);
                    const double dq = piv > 0.0 ? sqrt(piv) : 1.0, rq = 1.0 / dq;
                    row[q] = lane == (uint32_t)q ? dq : row[q] * rq;
#pragma unroll
                    for (int c = q + 1; c < B; ++c) row[c] = fma(-row[q], readlane_d(row[q], c), row[c]);
                }
                if (bad && lane == 0) s_bad = 1;
                if (lane < (uint32_t)B) {
#pragma unroll
                    for (int c = 0; c < B; ++c) D[lane * DP + c] = (uint32_t)c <= lane ? row[c] : 0.0;
                    a.rdiag[c0 + lane] = 1.0 / D[lane * DP + lane];
                }
                // lane c: column c of W = L_pp^-1 by forward substitution,
                // W[r][c] = (delta_rc - sum_{s < r} L[r][s] W[s][c]) / L[r][r]
                // (entries above the diagonal come out 0); L from LDS
                double wcol[B];
#pragma unroll
                for (int r = 0; r < B; ++r) {
                    double v = lane == (uint32_t)r ? 1.0 : 0.0;
#pragma unroll
                    for (int q = 0; q < r; ++q) v = fma(-D[r * DP + q], wcol[q], v);
                    wcol[r] = v / D[r * DP + r];
                }
                if (lane < (uint32_t)B) {
#pragma unroll
                    for (int c = 0; c < B; ++c) Wl[c * DP + lane] = wcol[c];
                }
            }
            __syncthreads();
            // 2. the panel below: X = A_panel W^T on v_mfma_f64_16x16x4f64
            // (A: lane l holds panel row 16 ti + l % 16, column 4 s + l / 16;
            // B: W[16 tj + l % 16][4 s + l / 16]); a wave owns all the column
            // tiles of its rows, so it overwrites them in place after reading
            {
                const uint32_t li = lane & 15, lg = lane >> 4;
                for (uint32_t ti = wave; ti < M / 16; ti += nt / kWave) {
                    cv_d4 acc[B / 16];
#pragma unroll
                    for (int tj = 0; tj < B / 16; ++tj) acc[tj] = cv_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int s = 0; s < B / 4; ++s) {
                        const double av = PT[(4 * s + lg) * LD + 16 * ti + li];
#pragma unroll
                        for (int tj = 0; tj < B / 16; ++tj)
                            acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Wl[(16 * tj + li) * DP + 4 * s + lg],
                                                                          acc[tj], 0, 0, 0);
                    }
#pragma unroll
                    for (int tj = 0; tj < B / 16; ++tj)
#pragma unroll
                        for (int v = 0; v < 4; ++v) PT[(16 * tj + li) * LD + 16 * ti + 4 * v + lg] = acc[tj][v];
                }
            }
            __syncthreads();
            for (uint32_t t = tid; t < B * B; t += nt) {
                const uint32_t r = t / B, q = t - r * B;
                if (q <= r) A[(size_t)(c0 + r) * F + c0 + q] = D[r * DP + q];
            }
            for (uint32_t t = tid; t < M * B; t += nt) {
                const uint32_t r = t / B, q = t - r * B;
                A[(size_t)(c1 + r) * F + c0 + q] = PT[q * LD + r];
            }
            // 3. trailing update of rows / columns c1 .. F - 1 on
            // v_mfma_f64_16x16x4f64, 16 x 16 tiles of the lower triangle, two
            // per wave at a time (independent chains): A = 16 rows of the
            // panel (lane l: row 16 ti + l % 16, column 4 s + l / 16), B = the
            // same for tj; output element v of lane l is row 4 v + l / 16,
            // column l % 16.  A tile's old values are loaded before its
            // products.
            {
                const uint32_t li = lane & 15, lg = lane >> 4, nb16 = M / 16, ntl = nb16 * (nb16 + 1) / 2;
                auto tile_of = [](uint32_t tI, uint32_t &ti, uint32_t &tj) {
                    ti = (uint32_t)((sqrt(8.0 * (double)tI + 1.0) - 1.0) * 0.5);
                    while (ti * (ti + 1) / 2 > tI) --ti;
                    while ((ti + 1) * (ti + 2) / 2 <= tI) ++ti;
                    tj = tI - ti * (ti + 1) / 2;
                };
                for (uint32_t t0 = wave; t0 < ntl; t0 += 2 * (nt / kWave)) {
                    const uint32_t t1 = t0 + nt / kWave;
                    const bool two = t1 < ntl;
                    uint32_t ti0, tj0, ti1 = 0, tj1 = 0;
                    tile_of(t0, ti0, tj0);
                    if (two) tile_of(t1, ti1, tj1);
                    const uint32_t col0 = c1 + 16 * tj0 + li, col1 = c1 + 16 * tj1 + li;
                    double old0[4], old1[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const uint32_t u0 = c1 + 16 * ti0 + 4 * v + lg, u1 = c1 + 16 * ti1 + 4 * v + lg;
                        old0[v] = col0 <= u0 ? A[(size_t)u0 * F + col0] : 0.0;
                        old1[v] = (two && col1 <= u1) ? A[(size_t)u1 * F + col1] : 0.0;
                    }
                    cv_d4 acc0 = cv_d4{0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
#pragma unroll
                    for (int s = 0; s < B / 4; ++s) {
                        const double *pq = PT + (4 * s + lg) * LD;
                        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(pq[16 * ti0 + li], pq[16 * tj0 + li], acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(pq[16 * ti1 + li], pq[16 * tj1 + li], acc1, 0, 0, 0);
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const uint32_t u0 = c1 + 16 * ti0 + 4 * v + lg, u1 = c1 + 16 * ti1 + 4 * v + lg;
                        if (col0 <= u0) A[(size_t)u0 * F + col0] = old0[v] - acc0[v];
                        if (two && col1 <= u1) A[(size_t)u1 * F + col1] = old1[v] - acc1[v];
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
        *a.flag = 0;
    }
}

// The factorisation on many workgroups: a blocked right-looking Cholesky
// with 32 x 32 blocks and one launch per panel.
//   k_cv_chol_diag0: lam (as above), then block (0, 0) of A0 + lam I;
//   k_cv_chol_step(p), p = 0 .. NB - 2: one workgroup per block (I, J) of
//     the trailing lower triangle, p < J <= I < NB.  It forms the panel
//     rows L_Ip = A_Ip W_p^T and L_Jp = A_Jp W_p^T (W_p = L_pp^-1, FP64
//     MFMA; every workgroup that needs a panel block recomputes it, the
//     diagonal one (I, I) stores it in the factor), then takes
//     A_IJ -= L_Ip L_Jp^T into the working copy Aw (A0 + lam I for p = 0).
//     The workgroup of block (p + 1, p + 1) then factorises that block.
//     Further workgroups, one per block (I, J) with I > p >= J, carry the
//     same panel through the block forward substitution L M = I for the
//     inverse M = L^-1: block row p of M is M_pJ = W_p R_pJ (R = I minus
//     the updates so far, R_pp = I), and the rows below take
//     R_IJ -= L_Ip M_pJ; the workgroups of row I = p + 1 store M_p.;
//   k_cv_chol_last: block row NB - 1 of M;
//   k_cv_chol_inverse: (A0 + lam I)^-1 = M^T M, both triangles, for the
//     corrections (k_cv_subst multiplies by it).
// A diagonal block is factorised by one wave: lanes r < 32 hold row r,
// lanes 32 + c hold row c of the identity; every column q is scaled by
// 1 / sqrt(pivot) (hardware reciprocal square root and two Newton steps)
// and the lanes take the rank-1 update with the column's entries broadcast
// through LDS (the entry of the next pivot's row by readlane, which is
// quicker).  The same operations on the identity rows are column-wise
// forward substitution, so lanes 32 + c end with column c of W = L_pp^-1
// at no extra latency.  The factor goes to A (lower triangle), 1 / L_uu to
// rdiag, W_p to Wd; a non-positive pivot sets *status = -1 and the launches
// left return at once, so that the escalation kernel above takes over.
struct CvCholArgs {
    uint32_t F;
    double ridge;       // relative to the mean diagonal
    const double *A0;   // (F, F) normal matrix, lower triangle
    double *Aw;         // (F, F) working copy of the trailing blocks
    double *A;          // (F, F) factor L, lower triangle
    double *Wd;         // (F / 32, 32, 32) W_p, row-major
    double *rdiag;      // (F) 1 / L_uu
    double *lam;
    int *status;
    int *flag;
    double *Rm;         // (F, F) the substitution's right-hand sides R, blocks below the diagonal
    double *Mi;         // (F, F) M = L^-1, lower triangle
    double *Ai;         // (F, F) (A0 + lam I)^-1, both triangles
};

constexpr uint32_t kCholB = 32;
constexpr uint32_t kCholDP = kCholB + 1;  // padded LDS row

// Factorises the block held in D (LDS, row-major, rows padded to kCholDP;
// only the lower triangle is used) on the calling wave (every lane of one
// wave calls it; D is overwritten with L_pp).  cb: 32 x 64 doubles of LDS
// for the broadcasts.  c0 = first row of the block, slot = its index p.
__device__ void chol_diag_block(double *D, double *cb, uint32_t c0, uint32_t slot, const CvCholArgs &a,
                                uint32_t lane) {
    constexpr int B = kCholB;
    const uint32_t r = lane & (B - 1);
    const bool fac = lane < (uint32_t)B;
    double x[B];
#pragma unroll
    for (int c = 0; c < B; ++c) x[c] = fac ? D[r * kCholDP + c] : (c == (int)r ? 1.0 : 0.0);
    bool bad = false;
    double rinv = 0.0;
#pragma unroll
    for (int q = 0; q < B; ++q) {
        const double piv = readlane_d(x[q], q);
        bad = bad || !(piv > 0.0);
        const double pv = piv > 0.0 ? piv : 1.0;
        double rq = __builtin_amdgcn_rsq(pv);
        rq = fma(0.5 * rq, fma(-(pv * rq), rq, 1.0), rq);
        rq = fma(0.5 * rq, fma(-(pv * rq), rq, 1.0), rq);
        const bool own = lane == (uint32_t)q;
        rinv = own ? rq : rinv;
        x[q] = own ? pv * rq : x[q] * rq;
        cb[q * kWave + lane] = x[q];  // unconditional: a branch here lets the updates sink
        if (q + 1 < B) x[q + 1] = fma(-x[q], readlane_d(x[q], q + 1), x[q + 1]);
#pragma unroll
        for (int c = q + 2; c < B; ++c) x[c] = fma(-x[q], cb[q * kWave + c], x[c]);
        // one column at a time: reads hoisted across columns would take
        // hundreds of registers
        __builtin_amdgcn_sched_barrier(0);
    }
    // W_p: lane 32 + c holds column c, x[q] = W[q][c]
    double *W = a.Wd + (size_t)slot * B * B;
    if (!fac) {
#pragma unroll
        for (int q = 0; q < B; ++q) W[q * B + r] = x[q];
    } else {
#pragma unroll
        for (int c = 0; c < B; ++c) D[r * kCholDP + c] = x[c];
        a.rdiag[c0 + r] = rinv;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (uint32_t t = lane; t < (uint32_t)(B * B); t += kWave) {
        const uint32_t u = t / B, v = t - u * B;
        if (v <= u) a.A[(size_t)(c0 + u) * a.F + c0 + v] = D[u * kCholDP + v];
    }
    if (bad && lane == 0) *a.status = -1;
}

__global__ __launch_bounds__(kWave) void k_cv_chol_diag0(const CvCholArgs a) {
    __shared__ double sdiag[kMaxF];
    __shared__ double D[kCholB * kCholDP], cb[kCholB * kWave];
    const uint32_t F = a.F, lane = threadIdx.x;
    for (uint32_t u = lane; u < F; u += kWave) sdiag[u] = a.A0[(size_t)u * F + u];
    __syncthreads();
    double lam = 0.0;
    if (lane == 0) {
        // in index order (F is a multiple of 32), 8 reads in flight
        double t = 0.0;
        for (uint32_t u = 0; u < F; u += 8) {
            double v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = sdiag[u + k];
#pragma unroll
            for (int k = 0; k < 8; ++k) t += v[k];
        }
        lam = a.ridge * t / F + 1e-300;
        *a.lam = lam;
        *a.status = 0;
        *a.flag = 0;
    }
    lam = readlane_d(lam, 0);
    for (uint32_t t = lane; t < kCholB * kCholB; t += kWave) {
        const uint32_t u = t / kCholB, v = t - u * kCholB;
        D[u * kCholDP + v] = v <= u ? a.A0[(size_t)u * F + v] + (u == v ? lam : 0.0) : 0.0;
    }
    __syncthreads();
    chol_diag_block(D, cb, 0, 0, a, lane);
}

// Block (I, J), I > p >= J, of the inverse's substitution in step p (see
// above): wave w takes the 16 x 16 tiles (w >> 1, w & 1) of L_Ip, M_pJ and
// R_IJ.
__device__ void chol_inverse_tile(const CvCholArgs &a, uint32_t p, uint32_t I, uint32_t J, double *LI, double *LM,
                                  uint32_t tid) {
    constexpr uint32_t B = kCholB, DP = kCholDP;
    const uint32_t F = a.F, lane = tid & (kWave - 1), wave = tid / kWave;
    const uint32_t li = lane & 15, lg = lane >> 4, h = wave >> 1, j2 = wave & 1;
    const double *src = p == 0 ? a.A0 : a.Aw;
    const double *W = a.Wd + (size_t)p * B * B;
    const uint32_t c0 = B * p;
    double old[4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
        old[v] = p == J ? 0.0 : a.Rm[(size_t)(B * I + 16 * h + 4 * v + lg) * F + B * J + 16 * j2 + li];
    double ai[B / 4], wl[B / 4], wa[B / 4], rr[B / 4];
#pragma unroll
    for (int s = 0; s < (int)B / 4; ++s) {
        const uint32_t k = 4 * s + lg;
        ai[s] = src[(size_t)(B * I + 16 * h + li) * F + c0 + k];
        wl[s] = W[(16 * j2 + li) * B + k];
        wa[s] = W[(16 * h + li) * B + k];
        rr[s] = p == J ? (k == 16 * j2 + li ? 1.0 : 0.0) : a.Rm[(size_t)(c0 + k) * F + B * J + 16 * j2 + li];
    }
    cv_d4 xl = cv_d4{0.0, 0.0, 0.0, 0.0}, xm = xl;
#pragma unroll
    for (int s = 0; s < (int)B / 4; ++s) {
        xl = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[s], wl[s], xl, 0, 0, 0);  // L_Ip = A_Ip W_p^T
        xm = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[s], rr[s], xm, 0, 0, 0);  // M_pJ = W_p R_pJ
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        LI[(16 * h + 4 * v + lg) * DP + 16 * j2 + li] = xl[v];
        LM[(16 * h + 4 * v + lg) * DP + 16 * j2 + li] = xm[v];
    }
    __syncthreads();
    cv_d4 acc = cv_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < (int)B / 4; ++s)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(LI[(16 * h + li) * DP + 4 * s + lg],
                                                  LM[(4 * s + lg) * DP + 16 * j2 + li], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v)
        a.Rm[(size_t)(B * I + 16 * h + 4 * v + lg) * F + B * J + 16 * j2 + li] = old[v] - acc[v];
    if (I == p + 1) {
        for (uint32_t e = tid; e < B * B; e += 256) {
            const uint32_t u = e / B, v = e - u * B;
            a.Mi[(size_t)(c0 + u) * F + B * J + v] = LM[u * DP + v];
        }
    }
}

__global__ __launch_bounds__(256) void k_cv_chol_step(const CvCholArgs a, uint32_t p) {
    if (*a.status < 0) return;
    constexpr uint32_t B = kCholB, DP = kCholDP;
    __shared__ double LI[B * DP], LJ[B * DP], D[B * DP], cb[B * kWave];
    const uint32_t F = a.F, tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const uint32_t li = lane & 15, lg = lane >> 4;
    const uint32_t NB = F / B, m = NB - 1 - p, ntrail = m * (m + 1) / 2;
    if (blockIdx.x >= ntrail) {
        const uint32_t t = blockIdx.x - ntrail;
        chol_inverse_tile(a, p, p + 1 + t / (p + 1), t % (p + 1), LI, LJ, tid);
        return;
    }
    // block t -> (ti, tj), tj <= ti, of the trailing triangle
    const uint32_t t = blockIdx.x;
    uint32_t ti = (uint32_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (ti * (ti + 1) / 2 > t) --ti;
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    const uint32_t tj = t - ti * (ti + 1) / 2;
    const uint32_t I = p + 1 + ti, J = p + 1 + tj;
    const bool diag = I == J, next = diag && I == p + 1;
    const double *src = p == 0 ? a.A0 : a.Aw;
    const double lam = p == 0 ? *a.lam : 0.0;
    const uint32_t c0 = B * p;

    // wave w: 16 x 16 tile (w >> 1, w & 1) of L_Ip and of L_Jp, and tile
    // (hI, hJ) = (w >> 1, w & 1) of the update (none above the diagonal)
    const uint32_t h = wave >> 1, j2 = wave & 1;
    const bool upd = !(diag && h < j2);
    double old[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const uint32_t u = B * I + 16 * h + 4 * v + lg, c = B * J + 16 * j2 + li;
        old[v] = (upd && c <= u) ? src[(size_t)u * F + c] + (u == c ? lam : 0.0) : 0.0;
    }
    double ai[B / 4], aj[B / 4], w[B / 4];
    const double *W = a.Wd + (size_t)p * B * B;
#pragma unroll
    for (int s = 0; s < (int)B / 4; ++s) {
        ai[s] = src[(size_t)(B * I + 16 * h + li) * F + c0 + 4 * s + lg];
        aj[s] = src[(size_t)(B * J + 16 * h + li) * F + c0 + 4 * s + lg];
        w[s] = W[(16 * j2 + li) * B + 4 * s + lg];
    }
    cv_d4 xi = cv_d4{0.0, 0.0, 0.0, 0.0}, xj = xi;
#pragma unroll
    for (int s = 0; s < (int)B / 4; ++s) {
        xi = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[s], w[s], xi, 0, 0, 0);
        xj = __builtin_amdgcn_mfma_f64_16x16x4f64(aj[s], w[s], xj, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        LI[(16 * h + 4 * v + lg) * DP + 16 * j2 + li] = xi[v];
        LJ[(16 * h + 4 * v + lg) * DP + 16 * j2 + li] = xj[v];
    }
    __syncthreads();
    cv_d4 acc = cv_d4{0.0, 0.0, 0.0, 0.0};
    if (upd) {
#pragma unroll
        for (int s = 0; s < (int)B / 4; ++s)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(LI[(16 * h + li) * DP + 4 * s + lg],
                                                      LJ[(16 * j2 + li) * DP + 4 * s + lg], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const uint32_t ru = 16 * h + 4 * v + lg, cu = 16 * j2 + li;
        const double nv = old[v] - acc[v];
        if (next) D[ru * DP + cu] = upd ? nv : 0.0;
        else if (upd && (!diag || cu <= ru)) a.Aw[(size_t)(B * I + ru) * F + B * J + cu] = nv;
    }
    if (diag) {
        // the panel block L_Ip into the factor
        for (uint32_t e = tid; e < B * B; e += 256) {
            const uint32_t u = e / B, v = e - u * B;
            a.A[(size_t)(B * I + u) * F + c0 + v] = LI[u * DP + v];
        }
    }
    if (next) {
        __syncthreads();
        if (wave == 0) chol_diag_block(D, cb, B * I, I, a, lane);
    }
}

// Block row NB - 1 of M: M_pJ = W_p R_pJ (p = NB - 1), one workgroup per J.
__global__ __launch_bounds__(256) void k_cv_chol_last(const CvCholArgs a) {
    if (*a.status < 0) return;
    constexpr uint32_t B = kCholB;
    const uint32_t F = a.F, NB = F / B, p = NB - 1, J = blockIdx.x, tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1), wave = tid / kWave, li = lane & 15, lg = lane >> 4;
    const uint32_t h = wave >> 1, j2 = wave & 1, c0 = B * p;
    const double *W = a.Wd + (size_t)p * B * B;
    double wa[B / 4], rr[B / 4];
#pragma unroll
    for (int s = 0; s < (int)B / 4; ++s) {
        const uint32_t k = 4 * s + lg;
        wa[s] = W[(16 * h + li) * B + k];
        rr[s] = p == J ? (k == 16 * j2 + li ? 1.0 : 0.0) : a.Rm[(size_t)(c0 + k) * F + B * J + 16 * j2 + li];
    }
    cv_d4 xm = cv_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < (int)B / 4; ++s) xm = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[s], rr[s], xm, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) a.Mi[(size_t)(c0 + 16 * h + 4 * v + lg) * F + B * J + 16 * j2 + li] = xm[v];
}

// (A0 + lam I)^-1 = M^T M: block (I, J), J <= I, is sum_{K >= I} M_KI^T M_KJ
// (FP64 MFMA, wave w: tile (w >> 1, w & 1)); written to both triangles.
__global__ __launch_bounds__(256) void k_cv_chol_inverse(const CvCholArgs a) {
    if (*a.status < 0) return;
    constexpr uint32_t B = kCholB;
    const uint32_t F = a.F, NB = F / B, t = blockIdx.x, tid = threadIdx.x;
    uint32_t I = (uint32_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > t) --I;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const uint32_t J = t - I * (I + 1) / 2;
    const uint32_t lane = tid & (kWave - 1), wave = tid / kWave, li = lane & 15, lg = lane >> 4;
    const uint32_t h = wave >> 1, j2 = wave & 1;
    const double *M = a.Mi;
    cv_d4 acc = cv_d4{0.0, 0.0, 0.0, 0.0};
    for (uint32_t K = I; K < NB; ++K) {
        double x[B / 4], y[B / 4];
#pragma unroll
        for (int s = 0; s < (int)B / 4; ++s) {
            const size_t row = (size_t)(B * K + 4 * s + lg) * F;
            x[s] = M[row + B * I + 16 * h + li];
            y[s] = M[row + B * J + 16 * j2 + li];
        }
#pragma unroll
        for (int s = 0; s < (int)B / 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x[s], y[s], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const uint32_t u = B * I + 16 * h + 4 * v + lg, c = B * J + 16 * j2 + li;
        a.Ai[(size_t)u * F + c] = acc[v];
        if (I != J) a.Ai[(size_t)c * F + u] = acc[v];
    }
}

// One correction of dimension i's factor from the right-hand side b of the
// current residual (k_cv_pass): solves L L^T delta = b - lam w and adds
// delta to w[., i, .] (and its sqrt(2k+1)-scaled copy ws), in one
// workgroup.  After the many-workgroup factorisation (*status = 0) delta is
// the product with the explicit inverse, which k_cv_gemv has left in dl.
// After an escalation the factor is solved by substitution, blocks of B
// unknowns:
//   forward:  the block's unknowns by wave 0 (lane r holds row r of the
//             diagonal block, staged through LDS), then every row below
//             takes the block's contribution (32 lanes per row);
//   backward: the block's rows first take the contribution of the unknowns
//             below (32 row groups by 32 columns, added in group order),
//             then wave 0 solves with the transposed diagonal block.
// The step's objective J = sum e^2 + lam ||w||^2 (entry F of b holds
// sum e^2) falls by delta . g under the correction, g = b - lam w; with
// delta . g <= tol J, *flag is set: the passes and solves left in this step
// return at once (tol = 0 never stops early).  A set flag on entry does the
// same.
struct CvSubstArgs {
    uint32_t F, R, K, d, i;
    double tol;
    const double *Ai;       // (F, F) inverse, both triangles (when *status = 0)
    double *dl;             // (F) the inverse times the right-hand side
    const int *status;
    const double *A;        // factor (lower triangle)
    const double *rdiag;    // (F) 1 / L_uu
    const double *b;        // (F + 1) right-hand side of the residual, sum e^2
    const double *lam;
    double *w64, *ws;       // (R, d, K)
    int *flag;
};

// dl = (A0 + lam I)^-1 (b - lam w[., i, .]) after the many-workgroup
// factorisation: workgroup t takes rows 16 t .. 16 t + 15 (wave w four of
// them, lane c the columns c, c + 64, ..., c + 64 (NC - 1); a fixed
// butterfly per row).  Returns at once after an escalation (*status != 0)
// or once the step has converged (*flag).
template <int NC>
__global__ __launch_bounds__(kBlock) void k_cv_gemv(const CvSubstArgs a) {
    if (*a.flag || *a.status != 0) return;
    const uint32_t F = a.F, tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    __shared__ double g[kMaxF];
    const double lam = *a.lam;
    for (uint32_t u = tid; u < F; u += kBlock) {
        const uint32_t r = u / a.K, k = u - r * a.K;
        g[u] = a.b[u] - lam * a.w64[((size_t)r * a.d + a.i) * a.K + k];
    }
    __syncthreads();
    double gk[NC];
#pragma unroll
    for (int m = 0; m < NC; ++m) gk[m] = lane + kWave * m < F ? g[lane + kWave * m] : 0.0;
    const uint32_t u0 = 16 * blockIdx.x + 4 * wave;  // F is a multiple of 16
    double x[4][NC];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            const uint32_t c = lane + kWave * m;
            x[q][m] = a.Ai[(size_t)(u0 + q) * F + (c < F ? c : 0)];
        }
    double sq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        sq[q] = 0.0;
#pragma unroll
        for (int m = 0; m < NC; ++m) sq[q] = fma(x[q][m], gk[m], sq[q]);
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1)
#pragma unroll
        for (int q = 0; q < 4; ++q) sq[q] += __shfl_xor(sq[q], o);
    if (lane < 4) a.dl[u0 + lane] = lane == 0 ? sq[0] : lane == 1 ? sq[1] : lane == 2 ? sq[2] : sq[3];
}

template <int B>
__global__ __launch_bounds__(1024) void k_cv_subst(const CvSubstArgs a) {
    if (*a.flag) return;
    const uint32_t F = a.F, tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    constexpr uint32_t nt = 1024;
    __shared__ double y[kMaxF], gs[kMaxF];
    __shared__ double D[B * (B + 1)];  // the diagonal block, rows padded against bank conflicts
    __shared__ double red[32][33];
    __shared__ double s_n[2][16];
    const double lam = *a.lam;
    for (uint32_t u = tid; u < F; u += nt) {
        const uint32_t r = u / a.K, k = u - r * a.K;
        y[u] = gs[u] = a.b[u] - lam * a.w64[((size_t)r * a.d + a.i) * a.K + k];
    }
    const double *A = a.A;
    if (*a.status == 0) {
        for (uint32_t u = tid; u < F; u += nt) y[u] = a.dl[u];
        __syncthreads();
    } else {
    // forward substitution L z = y
    for (uint32_t c0 = 0; c0 < F; c0 += B) {
        if (tid < B * B) D[(tid / B) * (B + 1) + tid % B] = tid % B <= tid / B ? A[(size_t)(c0 + tid / B) * F + c0 + tid % B] : 0.0;
        __syncthreads();
        if (wave == 0) {
            double row[B];
#pragma unroll
            for (int c = 0; c < B; ++c) row[c] = lane < (uint32_t)B ? D[lane * (B + 1) + c] : 0.0;
            double v = lane < (uint32_t)B ? y[c0 + lane] : 0.0;
            const double rd = lane < (uint32_t)B ? a.rdiag[c0 + lane] : 0.0;
#pragma unroll
            for (int q = 0; q < B; ++q) {
                const double xq = readlane_d(v, q) * readlane_d(rd, q);
                if (lane == (uint32_t)q) v = xq;
                else if (lane > (uint32_t)q) v = fma(-row[q], xq, v);
            }
            if (lane < (uint32_t)B) y[c0 + lane] = v;
        }
        __syncthreads();
        // rows below: y_u -= sum_{q < B} L[u][c0 + q] z_{c0 + q}, one thread
        // per row (F <= 1024), its B entries read as 16-byte pairs
        for (uint32_t u = c0 + B + tid; u < F; u += nt) {
            const double2 *lr = reinterpret_cast<const double2 *>(A + (size_t)u * F + c0);
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int q = 0; q < B / 2; ++q) {
                const double2 l = lr[q];
                s0 = fma(l.x, y[c0 + 2 * q], s0);
                s1 = fma(l.y, y[c0 + 2 * q + 1], s1);
            }
            y[u] -= s0 + s1;
        }
        __syncthreads();
    }
    // backward substitution L^T x = z
    for (uint32_t c0 = F - B;; c0 -= B) {
        // the block's rows: z_{c0 + j} -= sum_{c >= c0 + B} L[c][c0 + j] x_c
        {
            // 32 row groups by 32 columns; every row of the group is read in
            // one batch
            const uint32_t j = tid & 31, g = tid / 32;
            double s = 0.0;
            if (j < (uint32_t)B) {
#pragma unroll
                for (uint32_t it = 0; it < kMaxF / 32; ++it) {
                    const uint32_t c = c0 + B + g + 32 * it;
                    if (c < F) s = fma(A[(size_t)c * F + c0 + j], y[c], s);
                }
            }
            red[g][j] = s;
        }
        if (tid < B * B) D[(tid / B) * (B + 1) + tid % B] = tid % B <= tid / B ? A[(size_t)(c0 + tid / B) * F + c0 + tid % B] : 0.0;
        __syncthreads();
        if (wave == 0) {
            double col[B];  // lane r: column r of the block, col[s] = L[c0 + s][c0 + r]
#pragma unroll
            for (int s = 0; s < B; ++s) col[s] = lane < (uint32_t)B ? D[s * (B + 1) + lane] : 0.0;
            double v = 0.0;
            if (lane < (uint32_t)B) {
                double t = 0.0;
                for (int g = 0; g < 32; ++g) t += red[g][lane];
                v = y[c0 + lane] - t;
            }
            const double rd = lane < (uint32_t)B ? a.rdiag[c0 + lane] : 0.0;
#pragma unroll
            for (int q = B - 1; q >= 0; --q) {
                const double xq = readlane_d(v, q) * readlane_d(rd, q);
                if (lane == (uint32_t)q) v = xq;
                else if (lane < (uint32_t)q) v = fma(-col[q], xq, v);
            }
            if (lane < (uint32_t)B) y[c0 + lane] = v;
        }
        __syncthreads();
        if (c0 == 0) break;
    }
    }  // substitution
    // w += delta, and the convergence test
    double dn = 0.0, wn = 0.0;
    for (uint32_t u = tid; u < F; u += nt) {
        const uint32_t r = u / a.K, k = u - r * a.K;
        const size_t o = ((size_t)r * a.d + a.i) * a.K + k;
        const double w0 = a.w64[o], w = w0 + y[u];
        a.w64[o] = w;
        a.ws[o] = w * sqrt(2.0 * k + 1.0);
        dn = fma(y[u], gs[u], dn);
        wn = fma(w0, w0, wn);
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        dn += __shfl_xor(dn, o);
        wn += __shfl_xor(wn, o);
    }
    if (lane == 0) {
        s_n[0][wave] = dn;
        s_n[1][wave] = wn;
    }
    __syncthreads();
    if (tid == 0) {
        double d2 = 0.0, w2 = 0.0;
        for (int w = 0; w < 16; ++w) {
            d2 += s_n[0][w];
            w2 += s_n[1][w];
        }
        if (d2 <= a.tol * (a.b[F] + lam * w2)) *a.flag = 1;
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
using PassFn = void (*)(const CvPassArgs &, uint32_t, hipStream_t);
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
void launch_pass(const CvPassArgs &a, uint32_t blocks, hipStream_t s) {
    // targets yd alone (normal equations), or yf and the model w (training)
    if (a.yd) hipLaunchKernelGGL((k_cv_pass<R, K, true>), dim3(blocks), dim3(kBlock), 0, s, a);
    else if (a.yf && a.w) hipLaunchKernelGGL((k_cv_pass<R, K, false>), dim3(blocks), dim3(kBlock), 0, s, a);
}
// one task per workgroup of 4 waves when the triangle is one task, two
// per workgroup of 8 waves otherwise (grid.y = tasks / 2)
template <int R, int K, class S0, class S1>
void launch_syrk(const CvSyrkArgs &a, dim3 grid, hipStream_t s) {
    if (a.ntasks == 1) hipLaunchKernelGGL((k_cv_syrk<R, K, S0, S1>), grid, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_cv_syrk2<R, K, S0, S1>), grid, dim3(2 * kBlock), 0, s, a);
}

struct CvFns {
    RhoFn rho;
    LossFn loss;
    PassFn pass;
    SyrkFn syrk;
};

// (R, K) pairs compiled, with the Gram kernel's task shapes (see
// syrk_tasks for how they cover the triangle)
bool cv_fns(uint32_t R, uint32_t K, CvFns &f) {
#define QMC_CV_CASE(RR, KK, S0, S1)              \
    if (R == RR && K == KK) {                    \
        f.rho = &launch_rho<RR, KK>;             \
        f.loss = &launch_loss<RR, KK>;           \
        f.pass = &launch_pass<RR, KK>;           \
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

// workgroups of a right-hand side pass: about 8 per CU, at least 256 points each
uint32_t rhs_splits(uint32_t n) { return std::max<uint32_t>(1, std::min<uint32_t>(1024, (n + 255) / 256)); }

// a correction whose objective decrease is below this fraction of the
// step's objective ends the step's passes
constexpr double kSolveTol = 1e-7;

// Device buffers of one training problem (n samples, d dimensions, rank R,
// K Legendre degrees) and the launches of one alternating-least-squares
// step.  Everything is freed with the object.
struct CvTrainer {
    uint32_t n = 0, d = 0, R = 0, K = 0, F = 0, NB = 0;
    uint32_t splits = 1, rsplits = 1, rblocks = 1, nslots = 0, ntasks = 0, gy = 1;
    CvFns fn{};
    DeviceScratch s;
    float *z = nullptr, *sw = nullptr, *yw = nullptr, *partial = nullptr;
    double *rho = nullptr, *phi = nullptr, *rpart = nullptr, *ydev = nullptr, *ws = nullptr;
    double *w64 = nullptr, *A0 = nullptr, *A = nullptr, *Aw = nullptr, *Wd = nullptr, *rdiag = nullptr;
    double *Rm = nullptr, *Mi = nullptr, *Ai = nullptr, *dl = nullptr;
    double *b = nullptr, *lam = nullptr;
    double *loss_part = nullptr, *abs_part = nullptr;
    int *status = nullptr, *flag = nullptr;
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
        // about 512 workgroups of 4 waves (one task each, two per CU) or 256
        // of 8 waves (two tasks each, one per CU) in all, each with at least
        // one round of points
        gy = ntasks == 1 ? 1 : (ntasks + 1) / 2;
        splits = std::max<uint32_t>(1, std::min<uint32_t>((ntasks == 1 ? 512 : 256) / gy,
                                                          (n + kSyrkPts - 1) / kSyrkPts));
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
                          (st = take((size_t)rsplits * (F + 1) * 8, rpart)) || (st = take((size_t)n * 8, ydev)))) ||
            (st = take((size_t)R * d * K * 8, ws)) || (st = take((size_t)R * d * K * 8, w64)) ||
            (st = take(tk.size() * sizeof(CvSyrkTask), tasks)) || (st = take((size_t)F * F * 8, A0)) ||
            (st = take((size_t)F * F * 8, A)) || (st = take((size_t)F * F * 8, Aw)) ||
            (st = take((size_t)F * F * 8, Rm)) || (st = take((size_t)F * F * 8, Mi)) ||
            (st = take((size_t)F * F * 8, Ai)) || (st = take((size_t)F * 8, dl)) ||
            (st = take((size_t)F * kCholB * 8, Wd)) || (st = take((size_t)F * 8, rdiag)) ||
            (st = take((size_t)(F + 1) * 8, b)) ||
            (st = take(8, lam)) ||
            (st = take(8, status)) || (st = take(8, flag)) || (st = take((size_t)rblocks * 16, loss_part)) ||
            (st = take((size_t)rblocks * 8, abs_part)))
            return st;
        hipError_t e = hipMemcpy(tasks, tk.data(), tk.size() * sizeof(CvSyrkTask), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(w64, 0, (size_t)R * d * K * 8);
        if (e == hipSuccess) e = hipMemset(ws, 0, (size_t)R * d * K * 8);
        if (e == hipSuccess) e = hipMemset(flag, 0, 8);
        if (e == hipSuccess) e = hipMemset(b, 0, (size_t)(F + 1) * 8);
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
        fn.rho(ra, std::min<uint32_t>(rblocks, 1024), st);
    }

    // A0 = sum_j a~_j a~_j^T (BF16 MFMA, FP32 accumulation per split, FP64 over splits)
    void gram(hipStream_t st) {
        const CvSyrkArgs ga{n, splits, nslots, ntasks, rho, phi, tasks, partial};
        fn.syrk(ga, dim3(splits, gy), st);
        hipLaunchKernelGGL(k_cv_gather, dim3(nslots * 1024 / kBlock), dim3(kBlock), 0, st, (const float *)partial,
                           splits, nslots, R, K, A0);
    }

    // b = sum_j rho_j phi_j^T e_j with e = yf * y_scale - A w (use_w: the
    // current factor of dimension i, yd null) or e = yd (the normal
    // equations' own right-hand side: use_w false, yd set)
    void rhs(uint32_t i, bool use_w, const float *yf, double y_scale, const double *yd, const int *fl,
             hipStream_t st) {
        const CvPassArgs pa{n, d, i, rsplits, rho, phi, yf, y_scale, yd, use_w ? w64 : nullptr, fl, rpart};
        fn.pass(pa, rsplits, st);
        hipLaunchKernelGGL(k_cv_rhs_reduce, dim3((F + 1 + kBlock / kWave - 1) / (kBlock / kWave)), dim3(kBlock), 0,
                           st, (const double *)rpart, rsplits, F + 1, fl, b);
    }

    // L L^T = A0 + lam I (one launch per panel of 32 columns, then the
    // escalation kernel, which returns at once unless a pivot failed);
    // clears the convergence flag
    void factor(double ridge, hipStream_t st) {
        const CvCholArgs ca{F, ridge, A0, Aw, A, Wd, rdiag, lam, status, flag, Rm, Mi, Ai};
        hipLaunchKernelGGL(k_cv_chol_diag0, dim3(1), dim3(kWave), 0, st, ca);
        for (uint32_t p = 0; p + 1 < NB; ++p) {
            const uint32_t m = NB - 1 - p;
            hipLaunchKernelGGL(k_cv_chol_step, dim3(m * (m + 1) / 2 + m * (p + 1)), dim3(256), 0, st, ca, p);
        }
        hipLaunchKernelGGL(k_cv_chol_last, dim3(NB), dim3(256), 0, st, ca);
        hipLaunchKernelGGL(k_cv_chol_inverse, dim3(NB * (NB + 1) / 2), dim3(256), 0, st, ca);
        const CvFactorArgs fa{F, ridge, A0, A, rdiag, lam, status, flag, 1};
        if (F <= 512) hipLaunchKernelGGL(k_cv_factor<32>, dim3(1), dim3(kFactorThreads), 0, st, fa);
        else hipLaunchKernelGGL(k_cv_factor<16>, dim3(1), dim3(kFactorThreads), 0, st, fa);
    }

    // w[., i, .] += (L L^T)^-1 (b - lam w[., i, .]); tol as in k_cv_subst
    void subst(uint32_t dd, uint32_t i, double tol, hipStream_t st) {
        const CvSubstArgs sa{F, R, K, dd, i, tol, Ai, dl, status, A, rdiag, b, lam, w64, ws, flag};
        const dim3 gg(F / 16), gb(kBlock);
        switch ((F + kWave - 1) / kWave) {  // columns per lane
            case 1: hipLaunchKernelGGL(k_cv_gemv<1>, gg, gb, 0, st, sa); break;
            case 2: hipLaunchKernelGGL(k_cv_gemv<2>, gg, gb, 0, st, sa); break;
            case 3: hipLaunchKernelGGL(k_cv_gemv<3>, gg, gb, 0, st, sa); break;
            case 4: hipLaunchKernelGGL(k_cv_gemv<4>, gg, gb, 0, st, sa); break;
            case 6: hipLaunchKernelGGL(k_cv_gemv<6>, gg, gb, 0, st, sa); break;
            case 8: hipLaunchKernelGGL(k_cv_gemv<8>, gg, gb, 0, st, sa); break;
            default: hipLaunchKernelGGL(k_cv_gemv<12>, gg, gb, 0, st, sa); break;
        }
        if (F <= 512) hipLaunchKernelGGL(k_cv_subst<32>, dim3(1), dim3(1024), 0, st, sa);
        else hipLaunchKernelGGL(k_cv_subst<16>, dim3(1), dim3(1024), 0, st, sa);
    }

    // One alternating-least-squares step for dimension i: FP64 features,
    // the BF16 normal matrix and its FP64 factorisation, then up to `passes`
    // corrections starting from the current factor: each pass forms the
    // FP64 residual e = y - A w and its right-hand side A^T e - lam w from
    // the FP64 design matrix and solves with the factor.  The BF16 matrix
    // only preconditions, so the fixed point is the FP64 ridge solution;
    // the passes stop once a correction would lower the step's objective
    // by less than tol of it (tol = 0: all passes run).
    void step(uint32_t i, double inv_scale, double ridge, uint32_t passes, double tol, hipStream_t st) {
        features(i, st);
        gram(st);
        factor(ridge, st);
        for (uint32_t it = 0; it < passes; ++it) {
            rhs(i, true, yw, inv_scale, nullptr, flag, st);
            subst(d, i, tol, st);
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
            for (uint32_t i = 0; i < d; ++i) t.step(i, inv_scale, ridge, refine + 1, kSolveTol, stream);
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
        (e = hipMemcpy(t.ydev, y, (size_t)n * 8, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "normal-equation upload");
    t.gram(nullptr);
    t.rhs(0, false, nullptr, 1.0, t.ydev, nullptr, nullptr);
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
    t.factor(ridge, nullptr);
    t.subst(1, 0, 0.0, nullptr);
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
    t.step(i, 1.0 / scale, ridge, refine + 1, 0.0, nullptr);
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
