// Lattice kernels for gfx950.
//
// k_lattice evaluates eq. (2) of arXiv:1811.11722: for a tile of T shifts it
// sums fhat({j g / n + Delta_k}) over the lattice points j = 0..n-1 (the
// paper's j - 1).  Thread t of the x-grid (S threads in total) visits
// j = t, t + S, t + 2S, ...; its indices idx_i = (j g_i) mod n start from
// one exact 64-bit product and then advance by the precomputed
// (S g_i) mod n with a single conditional wrap, so the lattice is walked
// exactly in 32-bit integers.  idx_i / n is shared by the T shifts of the
// tile.  Sums are compensated: a plain FP64 partial over a chunk of points is
// folded into a (hi, lo) pair with TwoSum, the wave reduces the pairs with a
// double-double butterfly, LDS joins the 4 waves, and one pair per block
// and shift goes to HBM.  k_finalize then adds the block pairs in a fixed
// order and forms Q_k, the mean and the error of eq. (3), so results are
// bitwise reproducible for a fixed launch shape.
#pragma once

#include "qmc_integrands.hpp"

namespace qmc {

struct LatticeArgs {
    uint32_t n;             // lattice size, 2 <= n <= 2^31
    uint32_t d;             // dimension (== template D)
    uint32_t m;             // shifts per instance
    uint32_t tiles;         // shift tiles per instance = ceil(m / T)
    double inv_n;           // 1.0 / n
    const uint32_t *g;      // generating vectors, instance stride g_stride
    const uint32_t *gstep;  // (S * g_i) mod n, same layout as g
    const double *shifts;   // shifts (m, d) row-major, instance stride shift_stride
    const double *params;   // parameter blobs, instance stride param_stride (words)
    uint32_t g_stride, shift_stride, param_stride;
    uint32_t np;            // 1 real, 2 complex
    double2 *partials;      // (inst, m, np, gridDim.x) of (hi, lo)
};

constexpr int kChunk = 8;  // points per plain-FP64 partial before the TwoSum fold

template <class Fam, class Tr, int D, int T>
__global__ __launch_bounds__(kBlock) void k_lattice(const LatticeArgs a) {
    constexpr int NP = Fam::NP;
    const uint32_t inst = blockIdx.y / a.tiles;
    const uint32_t k0 = (blockIdx.y - inst * a.tiles) * T;
    const uint32_t *__restrict__ g = a.g + (size_t)inst * a.g_stride;
    const uint32_t *__restrict__ gs = a.gstep + (size_t)inst * a.g_stride;
    const double *__restrict__ sh = a.shifts + (size_t)inst * a.shift_stride;
    const double *__restrict__ prm = a.params + (size_t)inst * a.param_stride;
    const uint32_t n = a.n;
    const uint32_t S = gridDim.x * kBlock;
    const uint32_t t0 = blockIdx.x * kBlock + threadIdx.x;

    double hi[T][NP], lo[T][NP];
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
        for (int p = 0; p < NP; ++p) hi[k][p] = lo[k][p] = 0.0;

    if (t0 < n) {
        // shifts of this tile; rows past m repeat the last shift (discarded)
        double dl[T][D];
#pragma unroll
        for (int k = 0; k < T; ++k) {
            const uint32_t row = min(k0 + (uint32_t)k, a.m - 1u);
#pragma unroll
            for (int i = 0; i < D; ++i) dl[k][i] = sh[row * D + i];
        }
        uint32_t idx[D], step[D], nms[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            idx[i] = mulmod(t0, g[i], n, a.inv_n);
            step[i] = gs[i];
            nms[i] = n - gs[i];
        }
        uint32_t j = t0;
#pragma unroll 1
        while (j < n) {
            double s[T][NP];
#pragma unroll
            for (int k = 0; k < T; ++k)
#pragma unroll
                for (int p = 0; p < NP; ++p) s[k][p] = 0.0;
#pragma unroll 1
            for (int c = 0; c < kChunk && j < n; ++c) {
                double y[D];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    y[i] = (double)idx[i] * a.inv_n;
                    idx[i] = walk(idx[i], step[i], nms[i]);
                }
                double x[T][D];
#pragma unroll
                for (int k = 0; k < T; ++k)
#pragma unroll
                    for (int i = 0; i < D; ++i) x[k][i] = fract(y[i] + dl[k][i]);
                double v[T][NP];
                Fam::template eval<Tr, D, T>(prm, x, v);
#pragma unroll
                for (int k = 0; k < T; ++k)
#pragma unroll
                    for (int p = 0; p < NP; ++p) s[k][p] += v[k][p];
                j += S;
            }
#pragma unroll
            for (int k = 0; k < T; ++k)
#pragma unroll
                for (int p = 0; p < NP; ++p) dd_accumulate(hi[k][p], lo[k][p], s[k][p]);
        }
    }

    // block reduction: wave butterfly, then the 4 waves in order via LDS
    __shared__ dd red[kBlock / kWave][T * NP];
    const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            dd r = wave_reduce(dd{hi[k][p], lo[k][p]});
            if (lane == 0) red[wave][k * NP + p] = r;
        }
    __syncthreads();
    if (threadIdx.x < (uint32_t)(T * NP)) {
        const uint32_t k = threadIdx.x / NP, p = threadIdx.x - k * NP;
        dd r = red[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < kBlock / kWave; ++w) r = dd_add(r, red[w][threadIdx.x]);
        if (k0 + k < a.m) {
            const size_t o = (((size_t)inst * a.m + k0 + k) * a.np + p) * gridDim.x + blockIdx.x;
            a.partials[o] = make_double2(r.hi, r.lo);
        }
    }
}

struct FinalizeArgs {
    const double2 *partials;  // (inst, m, np, nblk)
    uint32_t nblk, m, np;
    double n;                 // lattice size as a double
    double scale;             // transform constant applied to every Q_k
    double sub;               // subtracted from each sum before scaling (0, or n for P2)
    double *q;                // (inst, m, np): Q_k
    double *res;              // (inst, 4): mean_re, mean_im, err_re, err_im
};

constexpr uint32_t kMaxRows = 4096;  // m * np per instance

struct DumpArgs {
    uint32_t n, d;
    double inv_n;
    const uint32_t *g, *gstep;
    uint64_t j_lo, j_hi;       // indices j in [j_lo, j_hi) are written
    uint32_t *idx_out;         // (j_hi - j_lo, d)
    unsigned long long *sums;  // (d, 2): sum idx, sum idx^2 (mod 2^64), zeroed by the host
};

}  // namespace qmc
