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
    const double *shifts;   // shifts (m, d) row-major, padded to whole shift tiles by
                            // repeating the last row; instance stride shift_stride
    const double *params;   // parameter blobs, instance stride param_stride (words)
    uint32_t g_stride, shift_stride, param_stride;
    uint32_t np;            // 1 real, 2 complex
    double2 *partials;      // (inst, m, np, gridDim.x) of (hi, lo)
    uint32_t jend;          // points j < jend are summed; 0 means all n (only
                            // the P2 search, whose sum is symmetric in j and
                            // n - j, sets n/2 + 1)
};

constexpr int kChunk = 8;  // points per plain-FP64 partial before the TwoSum fold

// Adds fhat over the lattice points j = j, j + S, j + 2S, ... < j1 of one
// thread into (hi, lo) for the T shifts starting at row pointer dls (T rows
// of D doubles; shift tables are padded to whole tiles).  gs holds
// (S g_i) mod n.  With Reload the shifts are re-read through the scalar
// cache at every point instead of being held in registers across the loop
// (the persistent kernel, whose tile loop would otherwise keep them in
// vector registers).
// A family that sets kWaveUniform = true (one that runs matrix instructions
// across the wave) is walked with a wave-uniform trip count: lanes past the
// end of the range keep evaluating valid lattice points and their values are
// discarded.  Lanes of a wave hold consecutive j, so lane 0 decides.
template <class F>
__device__ constexpr auto wave_uniform_walk(int) -> decltype(F::kWaveUniform, bool()) {
    return F::kWaveUniform;
}
template <class F>
__device__ constexpr bool wave_uniform_walk(long) {
    return false;
}
// A family that sets kShiftsInVgprs = true has the T x D shift values of
// its tile copied into vector registers before the point loop.  Held as
// scalars they compete with the integrand's coefficients for the 106 scalar
// registers, and the compiler spills them into vector lanes, paying a
// v_readlane per value and point; the run-time specialised sector functors
// have vector registers to spare and ask for this (for tiles of up to 24
// values).
template <class F>
__device__ constexpr auto shifts_in_vgprs(int) -> decltype(F::kShiftsInVgprs, bool()) {
    return F::kShiftsInVgprs;
}
template <class F>
__device__ constexpr bool shifts_in_vgprs(long) {
    return false;
}

template <class Fam, class Tr, int D, int T, bool Reload = false>
__device__ __forceinline__ void walk_points(uint32_t j, uint32_t j1, uint32_t S, uint32_t n, double inv_n,
                                            const uint32_t *__restrict__ g, const uint32_t *__restrict__ gs,
                                            const double *__restrict__ dls, const double *__restrict__ prm,
                                            double (&hi)[T][Fam::NP], double (&lo)[T][Fam::NP]) {
    constexpr int NP = Fam::NP;
    constexpr bool kUniform = wave_uniform_walk<Fam>(0);
    auto more = [&]() {
        if constexpr (kUniform)
            return (uint32_t)__builtin_amdgcn_readfirstlane(j) < j1;
        else
            return j < j1;
    };
    if (!more()) return;
    uint32_t idx[D], step[D], nms[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        idx[i] = mulmod(j, g[i], n, inv_n);
        step[i] = gs[i];
        nms[i] = n - gs[i];
    }
    // (bounded: 24 doubles are 48 VGPRs; larger tiles keep the scalar copies)
    constexpr bool kVgprShifts = !Reload && shifts_in_vgprs<Fam>(0) && T * D <= 24;
    double dlv[T * D];
    if constexpr (kVgprShifts) {
#pragma unroll
        for (int q = 0; q < T * D; ++q) {
            dlv[q] = dls[q];
            asm volatile("" : "+v"(dlv[q]));  // a vector register from here on
        }
    }
#pragma unroll 1
    while (more()) {
        double s[T][NP];
#pragma unroll
        for (int k = 0; k < T; ++k)
#pragma unroll
            for (int p = 0; p < NP; ++p) s[k][p] = 0.0;
#pragma unroll 1
        for (int c = 0; c < kChunk && more(); ++c) {
            double y[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                y[i] = (double)idx[i] * inv_n;
                idx[i] = walk(idx[i], step[i], nms[i]);
            }
            const double *dl = dls;
            if constexpr (Reload) {
                dl = uniform_ptr(dls);
                asm volatile("" : "+s"(dl));  // keep the shift loads inside the loop
            }
            double x[T][D];
#pragma unroll
            for (int k = 0; k < T; ++k)
#pragma unroll
                for (int i = 0; i < D; ++i) x[k][i] = fract(y[i] + (kVgprShifts ? dlv[k * D + i] : dl[k * D + i]));
            double v[T][NP];
            Fam::template eval<Tr, D, T>(prm, x, v);
            const bool ok = !kUniform || j < j1;
#pragma unroll
            for (int k = 0; k < T; ++k)
#pragma unroll
                for (int p = 0; p < NP; ++p) s[k][p] += ok ? v[k][p] : 0.0;
            j += S;
        }
#pragma unroll
        for (int k = 0; k < T; ++k)
#pragma unroll
            for (int p = 0; p < NP; ++p) dd_accumulate(hi[k][p], lo[k][p], s[k][p]);
    }
}

// Block-wide double-double sum of every thread's (hi, lo)[k][p]: the wave
// butterfly, then the 4 waves in order.  Thread r < T*NP returns row r.
template <int T, int NP>
__device__ __forceinline__ dd block_reduce(const double (&hi)[T][NP], const double (&lo)[T][NP],
                                           dd (&red)[kBlock / kWave][T * NP]) {
    const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            dd r = wave_reduce(dd{hi[k][p], lo[k][p]});
            if (lane == 0) red[wave][k * NP + p] = r;
        }
    __syncthreads();
    dd r{0.0, 0.0};
    if (threadIdx.x < (uint32_t)(T * NP)) {
        r = red[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < kBlock / kWave; ++w) r = dd_add(r, red[w][threadIdx.x]);
    }
    return r;
}

template <class Fam, class Tr, int D, int T>
__device__ __forceinline__ void lattice_body(const LatticeArgs &a) {
    constexpr int NP = Fam::NP;
    const uint32_t inst = blockIdx.y / a.tiles;
    const uint32_t k0 = (blockIdx.y - inst * a.tiles) * T;
    const uint32_t *__restrict__ g = a.g + (size_t)inst * a.g_stride;
    const uint32_t *__restrict__ gs = a.gstep + (size_t)inst * a.g_stride;
    const double *__restrict__ sh = a.shifts + (size_t)inst * a.shift_stride;
    const double *__restrict__ prm = a.params + (size_t)inst * a.param_stride;

    double hi[T][NP], lo[T][NP];
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
        for (int p = 0; p < NP; ++p) hi[k][p] = lo[k][p] = 0.0;
    const uint32_t j1 = a.jend ? a.jend : a.n;
    walk_points<Fam, Tr, D, T>(blockIdx.x * kBlock + threadIdx.x, j1, gridDim.x * kBlock, a.n, a.inv_n, g, gs,
                               sh + (size_t)k0 * D, prm, hi, lo);

    __shared__ dd red[kBlock / kWave][T * NP];
    const dd r = block_reduce<T, NP>(hi, lo, red);
    if (threadIdx.x < (uint32_t)(T * NP)) {
        const uint32_t k = threadIdx.x / NP, p = threadIdx.x - k * NP;
        if (k0 + k < a.m) {
            const size_t o = (((size_t)inst * a.m + k0 + k) * a.np + p) * gridDim.x + blockIdx.x;
            a.partials[o] = make_double2(r.hi, r.lo);
        }
    }
}

template <class Fam, class Tr, int D, int T>
__global__ __launch_bounds__(kBlock) void k_lattice(const LatticeArgs a) {
    lattice_body<Fam, Tr, D, T>(a);
}

// The same kernel held to at least two waves per SIMD (at most 256 VGPRs):
// for families whose matrix instructions need another wave to hide their
// latency.
template <class Fam, class Tr, int D, int T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_lattice_w2(const LatticeArgs a) {
    lattice_body<Fam, Tr, D, T>(a);
}

// ------------------------------------------------------- batched estimates
// Many plans (sectors) of different d, n, m in one persistent launch.  The
// work is a list of tiles (plan, shift tile, range of tile_points lattice
// points) ordered longest first; each workgroup takes the next tile from an
// atomic counter until the list is exhausted and writes one (hi, lo) pair per
// shift of the tile to that tile's slot.  k_finalize_batch then adds each
// plan's slots in a fixed order, so results do not depend on which
// workgroup ran which tile.
struct BatchSector {
    uint32_t n, d, m, jtiles;  // jtiles = ceil(n / tile_points)
    double inv_n;
    double scale;              // transform constant
    uint32_t g_off, shift_off, param_off, slot_base;
    uint32_t q_off, pad;
};

struct BatchTile {
    uint32_t sector, k0, jt, pad;
};

struct BatchArgs {
    const BatchSector *sectors;
    const BatchTile *tiles;
    uint32_t ntiles;
    uint32_t tile_points;  // multiple of kBlock
    const uint32_t *g;     // concatenated generating vectors
    const uint32_t *gstep; // (kBlock g_i) mod n, same layout
    const double *shifts;  // concatenated (m, d) tables, each padded to whole tiles
    const double *params;  // concatenated parameter blobs
    uint32_t *counter;     // next tile of this list; zeroed before the launch
    double2 *partials;     // (slot, T * np)
};

template <class Fam, class Tr, int D, int T>
__device__ __forceinline__ void batch_tile(const BatchArgs &a, const BatchTile &tl, const BatchSector &sc,
                                           dd (&red)[kBlock / kWave][T * Fam::NP]) {
    constexpr int NP = Fam::NP;
    double hi[T][NP], lo[T][NP];
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
        for (int p = 0; p < NP; ++p) hi[k][p] = lo[k][p] = 0.0;
    const uint32_t j0 = tl.jt * a.tile_points;
    const uint32_t j1 = min(sc.n, j0 + a.tile_points);
    walk_points<Fam, Tr, D, T, true>(j0 + threadIdx.x, j1, kBlock, sc.n, sc.inv_n, a.g + sc.g_off, a.gstep + sc.g_off,
                               a.shifts + sc.shift_off + (size_t)tl.k0 * D, a.params + sc.param_off, hi, lo);
    const dd r = block_reduce<T, NP>(hi, lo, red);
    if (threadIdx.x < (uint32_t)(T * NP)) {
        const size_t slot = (size_t)sc.slot_base + (size_t)(tl.k0 / T) * sc.jtiles + tl.jt;
        a.partials[slot * (T * NP) + threadIdx.x] = make_double2(r.hi, r.lo);
    }
}

// One persistent kernel per dimension: the tiles of the plans with d = D
// are a contiguous run of the list (tiles, ntiles) with their own counter.
template <class Fam, class Tr, int D, int T>
__global__ __launch_bounds__(kBlock) void k_batch(const BatchArgs a) {
    __shared__ uint32_t s_tile;
    __shared__ dd red[kBlock / kWave][T * Fam::NP];
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(a.counter, 1u);
        __syncthreads();
        const uint32_t t = uniform(s_tile);
        if (t >= a.ntiles) break;
        const BatchTile tl = a.tiles[t];
        const BatchSector sc = a.sectors[tl.sector];
        batch_tile<Fam, Tr, D, T>(a, tl, sc, red);
        __syncthreads();
    }
}

// The same work list with one workgroup per tile, workgroup t running tile
// t: workgroups are dispatched in index order, so tiles start in list order
// (longest first) and the hardware dispatcher balances the load.  Without
// the tile loop (and the counter broadcast through LDS) the kernel keeps
// 30-40 fewer registers live than k_batch and runs at the occupancy of
// k_lattice.
template <class Fam, class Tr, int D, int T>
__global__ __launch_bounds__(kBlock) void k_batch_flat(const BatchArgs a) {
    __shared__ dd red[kBlock / kWave][T * Fam::NP];
    const BatchTile tl = a.tiles[blockIdx.x];  // the grid has exactly ntiles workgroups
    const BatchSector sc = a.sectors[tl.sector];
    batch_tile<Fam, Tr, D, T>(a, tl, sc, red);
}

struct FinalizeBatchArgs {
    const BatchSector *sectors;
    const double2 *partials;
    uint32_t T, np;
    double *q;    // per sector at q_off: (m, np)
    double *res;  // (sector, 4)
};

struct FinalizeArgs {
    const double2 *partials;  // (inst, m, np, nblk)
    uint32_t nblk, m, np;
    double n;                 // lattice size as a double
    double scale;             // transform constant applied to every Q_k
    double sub;               // subtracted from each sum before scaling (0, or n for P2)
    double *q;                // (inst, m, np): Q_k
    double *res;              // (inst, 4 ceil(np / 2)): per pair of parts (mean a, mean b, err a, err b)
};

constexpr uint32_t kMaxRows = 4096;  // m * np per instance
constexpr uint32_t kMaxParts = 10;   // parts per shift (k_finalize, result buffers): 4 complex orders + crossings

struct DumpArgs {
    uint32_t n, d;
    double inv_n;
    const uint32_t *g, *gstep;
    uint64_t j_lo, j_hi;       // indices j in [j_lo, j_hi) are written
    uint32_t *idx_out;         // (j_hi - j_lo, d)
    unsigned long long *sums;  // (d, 2): sum idx, sum idx^2 (mod 2^64), zeroed by the host
};

}  // namespace qmc
