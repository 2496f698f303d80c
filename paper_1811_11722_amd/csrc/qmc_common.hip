// Kernel registry storage and the non-templated helper kernels.
#include "qmc_registry.hpp"

namespace qmc {

// Threads of a finalize block: 16 waves, so that m = 32 rows take two
// rounds of loads (each row's partials are a dependent read per wave).
constexpr uint32_t kFinalizeThreads = 1024;

// One block per instance.  Wave w adds block pairs of (k, p) rows in a fixed
// strided order and reduces them with the butterfly (the same order whatever
// the number of waves); thread 0 forms the mean and the two-pass error of
// eq. (3) for each part.
__global__ __launch_bounds__(kFinalizeThreads) void k_finalize(const FinalizeArgs a) {
    __shared__ double qs[kMaxRows];
    const uint32_t inst = blockIdx.x;
    const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const uint32_t rows = a.m * a.np;
    for (uint32_t r = wave; r < rows; r += kFinalizeThreads / kWave) {
        const double2 *src = a.partials + ((size_t)inst * rows + r) * a.nblk;
        dd acc{0.0, 0.0};
        for (uint32_t b = lane; b < a.nblk; b += kWave) acc = dd_add(acc, dd{src[b].x, src[b].y});
        acc = wave_reduce(acc);
        if (lane == 0) {
            const double q = (((acc.hi - a.sub) + acc.lo) * a.scale) / a.n;
            qs[r] = q;
            a.q[(size_t)inst * rows + r] = q;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // results per pair of parts: (mean a, mean b, err a, err b)
        const uint32_t rs = 4 * ((a.np + 1) / 2);
        double out[2 * kMaxParts] = {};
        for (uint32_t p = 0; p < a.np; ++p) {
            dd s{0.0, 0.0};
            for (uint32_t k = 0; k < a.m; ++k) dd_accumulate(s.hi, s.lo, qs[k * a.np + p]);
            const double mean = (s.hi + s.lo) / (double)a.m;
            dd v{0.0, 0.0};
            for (uint32_t k = 0; k < a.m; ++k) {
                const double t = qs[k * a.np + p] - mean;
                dd_accumulate(v.hi, v.lo, t * t);
            }
            out[4 * (p / 2) + p % 2] = mean;
            out[4 * (p / 2) + 2 + p % 2] = sqrt((v.hi + v.lo) / ((double)a.m * (double)(a.m - 1)));
        }
        for (uint32_t t = 0; t < rs; ++t) a.res[(size_t)inst * rs + t] = out[t];
    }
}

// The lattice kernel's index walk, with the integrand replaced by writes of
// the indices and per-dimension sums (integer atomics; exact and
// order-independent).
template <int D>
__global__ __launch_bounds__(kBlock) void k_dump(const DumpArgs a) {
    const uint32_t n = a.n;
    const uint32_t S = gridDim.x * kBlock;
    const uint32_t t0 = blockIdx.x * kBlock + threadIdx.x;
    unsigned long long s1[D], s2[D];
#pragma unroll
    for (int i = 0; i < D; ++i) s1[i] = s2[i] = 0ull;
    if (t0 < n) {
        uint32_t idx[D], step[D], nms[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            idx[i] = mulmod(t0, a.g[i], n, a.inv_n);
            step[i] = a.gstep[i];
            nms[i] = n - a.gstep[i];
        }
        for (uint32_t j = t0; j < n; j += S) {
            const bool wr = j >= a.j_lo && j < a.j_hi;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                if (wr) a.idx_out[(size_t)(j - a.j_lo) * D + i] = idx[i];
                s1[i] += idx[i];
                s2[i] += (unsigned long long)idx[i] * idx[i];
                idx[i] = walk(idx[i], step[i], nms[i]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
        atomicAdd(&a.sums[2 * i], s1[i]);
        atomicAdd(&a.sums[2 * i + 1], s2[i]);
    }
}


std::map<KernelKey, LatticeLaunch> &lattice_registry() {
    static std::map<KernelKey, LatticeLaunch> reg;
    return reg;
}

// device math on an array: fn 0 = qlog, 1 = qexp
__global__ __launch_bounds__(kBlock) void k_math(int fn, uint64_t count, const double *x, double *y) {
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= count) return;
    if (fn == 0) y[i] = qlog(x[i]);
    else if (fn == 1) y[i] = qexp(x[i]);
    else if (fn == 2) y[i] = qatan2(x[2 * i], x[2 * i + 1]);
    else qsincos(x[i], y[2 * i], y[2 * i + 1]);
}

hipError_t launch_math(int fn, uint64_t count, const double *x, double *y, hipStream_t s) {
    const uint64_t blocks = (count + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_math, dim3((uint32_t)blocks), dim3(kBlock), 0, s, fn, count, x, y);
    return hipGetLastError();
}

// Clears a small counter array (used inside captured graphs, where a memset
// node is avoided).
__global__ void k_zero_u32(uint32_t *p, uint32_t count) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

hipError_t launch_zero_u32(uint32_t *p, uint32_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u32, dim3((count + 63) / 64), dim3(64), 0, s, p, count);
    return hipGetLastError();
}

// One block per plan of a batch: adds the plan's tile slots of every
// (shift, part) row in slot order, then forms Q_k, the mean and the error.
__global__ __launch_bounds__(kFinalizeThreads) void k_finalize_batch(const FinalizeBatchArgs a) {
    __shared__ double qs[kMaxRows];
    const BatchSector sc = a.sectors[blockIdx.x];
    const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const uint32_t rows = sc.m * a.np, width = a.T * a.np;
    for (uint32_t r = wave; r < rows; r += kFinalizeThreads / kWave) {
        const uint32_t k = r / a.np, p = r - k * a.np;
        const uint32_t kt = k / a.T, col = (k - kt * a.T) * a.np + p;
        const double2 *src = a.partials + ((size_t)sc.slot_base + (size_t)kt * sc.jtiles) * width + col;
        dd acc{0.0, 0.0};
        for (uint32_t b = lane; b < sc.jtiles; b += kWave) acc = dd_add(acc, dd{src[(size_t)b * width].x, src[(size_t)b * width].y});
        acc = wave_reduce(acc);
        if (lane == 0) {
            const double q = ((acc.hi + acc.lo) * sc.scale) / (double)sc.n;
            qs[r] = q;
            a.q[sc.q_off + r] = q;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // results per pair of parts: (mean a, mean b, err a, err b)
        const uint32_t rs = 4 * ((a.np + 1) / 2);
        double out[2 * kMaxParts] = {};
        for (uint32_t p = 0; p < a.np; ++p) {
            dd s{0.0, 0.0};
            for (uint32_t k = 0; k < sc.m; ++k) dd_accumulate(s.hi, s.lo, qs[k * a.np + p]);
            const double mean = (s.hi + s.lo) / (double)sc.m;
            dd v{0.0, 0.0};
            for (uint32_t k = 0; k < sc.m; ++k) {
                const double t = qs[k * a.np + p] - mean;
                dd_accumulate(v.hi, v.lo, t * t);
            }
            out[p] = mean;
            out[2 + p] = sqrt((v.hi + v.lo) / ((double)sc.m * (double)(sc.m - 1)));
        }
        for (int t = 0; t < 4; ++t) a.res[(size_t)blockIdx.x * 4 + t] = out[t];
    }
}

hipError_t launch_finalize_batch(const FinalizeBatchArgs &a, uint32_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_batch, dim3(count), dim3(kFinalizeThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeArgs &a, uint32_t ninst, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(ninst), dim3(kFinalizeThreads), 0, s, a);
    return hipGetLastError();
}

template <int D>
static hipError_t launch_dump_d(const DumpArgs &a, uint32_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_dump<D>), dim3(blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_dump(const DumpArgs &a, uint32_t blocks, hipStream_t s) {
    switch (a.d) {
    case 1: return launch_dump_d<1>(a, blocks, s);
    case 2: return launch_dump_d<2>(a, blocks, s);
    case 3: return launch_dump_d<3>(a, blocks, s);
    case 4: return launch_dump_d<4>(a, blocks, s);
    case 5: return launch_dump_d<5>(a, blocks, s);
    case 6: return launch_dump_d<6>(a, blocks, s);
    case 7: return launch_dump_d<7>(a, blocks, s);
    case 8: return launch_dump_d<8>(a, blocks, s);
    case 9: return launch_dump_d<9>(a, blocks, s);
    case 10: return launch_dump_d<10>(a, blocks, s);
    case 11: return launch_dump_d<11>(a, blocks, s);
    case 12: return launch_dump_d<12>(a, blocks, s);
    case 13: return launch_dump_d<13>(a, blocks, s);
    case 14: return launch_dump_d<14>(a, blocks, s);
    case 15: return launch_dump_d<15>(a, blocks, s);
    case 16: return launch_dump_d<16>(a, blocks, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace qmc
