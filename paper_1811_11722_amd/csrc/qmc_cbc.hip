// Component-by-component construction of a rank-1 generating vector for the
// weighted Korobov space of smoothness 2 (the P2 criterion of the Korobov
// search, with product weights).  For component s every admissible candidate
// c needs
//   S(c) = sum_{j<n} p_j (1 + w_s B2({j c / n})),   w_s = 2 pi^2 gamma_s,
// with p_j the product over the components already chosen.  B2(1 - x) =
// B2(x), so the point n - j contributes what j does (p_j inherits the
// symmetry from the chosen components), and only j <= n/2 is summed:
// S(c) = 2 sum_{j <= n/2} - term(0) - [n even] term(n/2).  One thread owns
// one candidate and walks its index j c mod n exactly (u32 add and
// conditional subtract); the p_j are staged through LDS in tiles that every
// thread of the block reads in the same order (broadcast reads), and the
// point range is split over grid.y so that small candidate sets still fill
// the chip.  Partial sums are double-double; a second kernel folds them in
// a fixed order, restores the full sum and forms e^2(c) = (S(c) - n) / n.
// The argmin runs on the host, then p_j (j <= n/2) is multiplied by the
// chosen factor.
#include <algorithm>
#include <cmath>

#include "qmc_registry.hpp"
#include "qmc_runtime.hpp"

namespace qmc {

namespace {

constexpr uint32_t kCbcTile = 2048;  // doubles of p_j per LDS tile (16 KB)

struct CbcArgs {
    uint32_t n;
    uint32_t jend;    // points j < jend are summed (n/2 + 1)
    uint32_t ncand;
    uint32_t jchunk;  // points per grid.y slice
    double inv_n;
    double w;         // 2 pi^2 gamma_s
    const double *prod;
    const uint32_t *cand;
    double2 *partial;  // [gridDim.y][ncand]
};

__global__ __launch_bounds__(kBlock) void k_cbc_eval(const CbcArgs a) {
    __shared__ double tile[kCbcTile];
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    const bool live = t < a.ncand;
    const uint32_t c = live ? a.cand[t] : 1u;
    const uint32_t j0 = blockIdx.y * a.jchunk;
    const uint32_t j1 = min(a.jend, j0 + a.jchunk);
    dd acc{0.0, 0.0};
    for (uint32_t base = j0; base < j1; base += kCbcTile) {
        const uint32_t cnt = min(kCbcTile, j1 - base);
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) tile[i] = a.prod[base + i];
        __syncthreads();
        uint32_t idx = (uint32_t)(((uint64_t)base * c) % a.n);
        // 1 + w B2(x) = w x (x - 1) + (1 + w / 6): two FMAs per point
        const double w6 = 1.0 + a.w / 6.0;
        auto pair = [&](uint32_t i, double &s) {
            const double x = (double)idx * a.inv_n;
            s = fma_(tile[i], fma_(x, fma_(a.w, x, -a.w), w6), s);
            idx += c;
            idx = idx >= a.n ? idx - a.n : idx;
        };
        // groups of 8 points into one plain sum, then the double-double fold
        // (written as a loop over whole groups: a fold guarded inside the
        // point loop was if-converted and ran at every unrolled step)
        uint32_t i = 0;
        for (; i + 8 <= cnt; i += 8) {
            double s = 0.0;
#pragma unroll
            for (uint32_t u = 0; u < 8; ++u) pair(i + u, s);
            dd_accumulate(acc.hi, acc.lo, s);
        }
        double s = 0.0;
        for (; i < cnt; ++i) pair(i, s);
        dd_accumulate(acc.hi, acc.lo, s);
    }
    if (live) a.partial[(size_t)blockIdx.y * a.ncand + t] = make_double2(acc.hi, acc.lo);
}

// e2[t] = (S - n) / n with S = 2 (sum over slices) - term(0) - [n even]
// term(n/2), slices folded in order; the two terms are formed as k_cbc_eval
// forms them (x = idx / n through inv_n)
__global__ __launch_bounds__(kBlock) void k_cbc_reduce(const double2 *partial, uint32_t slices, uint32_t ncand,
                                                       uint32_t n, double inv_n, double w, const double *prod,
                                                       double *e2) {
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= ncand) return;
    dd acc{0.0, 0.0};
    for (uint32_t y = 0; y < slices; ++y) {
        const double2 v = partial[(size_t)y * ncand + t];
        acc = dd_add(acc, dd{v.x, v.y});
    }
    acc = dd{2.0 * acc.hi, 2.0 * acc.lo};
    const double w6 = 1.0 + w / 6.0;
    acc = dd_add(acc, dd{-(prod[0] * w6), 0.0});
    if ((n & 1u) == 0) {  // j = n/2 is its own mirror; c is odd, so idx = n/2
        const double x = (double)(n / 2) * inv_n;
        acc = dd_add(acc, dd{-(prod[n / 2] * fma_(x, fma_(w, x, -w), w6)), 0.0});
    }
    e2[t] = ((acc.hi - (double)n) + acc.lo) / (double)n;
}

// p_j *= 1 + w B2({j z / n}) for j < jend
__global__ __launch_bounds__(kBlock) void k_cbc_update(double *prod, uint32_t n, uint32_t jend, double inv_n,
                                                       uint32_t z, double w) {
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= jend) return;
    const uint32_t idx = (uint32_t)(((uint64_t)j * z) % n);
    const double x = (double)idx * inv_n;
    prod[j] = prod[j] * fma_(w, fma_(x, x - 1.0, 1.0 / 6.0), 1.0);
}

__global__ __launch_bounds__(kBlock) void k_fill(double *p, uint32_t count, double v) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < count) p[i] = v;
}

uint64_t gcd_u64(uint64_t a, uint64_t b) {
    while (b) {
        const uint64_t r = a % b;
        a = b;
        b = r;
    }
    return a;
}

}  // namespace
}  // namespace qmc

using namespace qmc;

extern "C" qmc_status qmc_cbc_search(uint64_t n, uint32_t d, const double *gamma, const uint64_t *cand,
                                     uint32_t ncand, uint64_t *z_out, double *e2_out) {
    if (!z_out || !e2_out) return fail(QMC_EINVAL, "null output");
    if (d == 0) return fail(QMC_EINVAL, "d must be >= 1");
    if (d > kMaxDim) return fail(QMC_EUNSUPPORTED, "d > %u", kMaxDim);
    if (n < 2) return fail(QMC_EINVAL, "n must be >= 2");
    if (n > (1ull << 31)) return fail(QMC_EUNSUPPORTED, "n > 2^31");
    std::vector<double> gam(d, 1.0);
    if (gamma)
        for (uint32_t i = 0; i < d; ++i) {
            if (!(gamma[i] >= 0.0) || !std::isfinite(gamma[i])) return fail(QMC_EINVAL, "gamma_%u not finite or < 0", i);
            gam[i] = gamma[i];
        }
    std::vector<uint32_t> cs;
    if (cand) {
        if (ncand == 0) return fail(QMC_EINVAL, "ncand must be >= 1");
        for (uint32_t t = 0; t < ncand; ++t) {
            if (cand[t] == 0 || cand[t] >= n || gcd_u64(cand[t], n) != 1)
                return fail(QMC_EINVAL, "candidate %u is not a unit mod n", t);
            cs.push_back((uint32_t)cand[t]);
        }
        std::sort(cs.begin(), cs.end());
        cs.erase(std::unique(cs.begin(), cs.end()), cs.end());
    } else {
        // every unit up to n/2: bound the work before enumerating them
        if ((double)(n / 2) * (double)n > 17592186044416.0)
            return fail(QMC_EUNSUPPORTED, "n/2 candidates x n = %.3g > 2^44: pass a candidate subset",
                        (double)(n / 2) * (double)n);
        for (uint64_t c = 1; c <= n / 2; ++c)
            if (gcd_u64(c, n) == 1) cs.push_back((uint32_t)c);
        if (cs.empty()) cs.push_back(1u);
    }
    // keep the cost of one component within a few seconds
    if ((double)cs.size() * (double)n > 17592186044416.0)
        return fail(QMC_EUNSUPPORTED, "candidates x n = %.3g > 2^44: pass a candidate subset", (double)cs.size() * (double)n);
    const uint32_t nc = (uint32_t)cs.size();
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    const uint32_t bx = (nc + kBlock - 1) / kBlock;
    const uint32_t want = 8u * (uint32_t)device_cu_count(dev);
    const uint32_t jend = (uint32_t)(n / 2 + 1);  // j <= n/2 (mirror symmetry j <-> n - j)
    const uint32_t max_slices = std::max<uint32_t>(1, jend / kCbcTile);
    const uint32_t slices = std::min(max_slices, std::max(1u, (want + bx - 1) / bx));
    DeviceScratch s;
    qmc_status st;
    if ((st = s.alloc((size_t)jend * 8)) || (st = s.alloc((size_t)nc * 4)) ||
        (st = s.alloc((size_t)slices * nc * sizeof(double2))) || (st = s.alloc((size_t)nc * 8)) ||
        (st = s.alloc(4)))
        return st;
    double *prod = (double *)s.ptr[0];
    uint32_t *dcand = (uint32_t *)s.ptr[1];
    double2 *partial = (double2 *)s.ptr[2];
    double *e2 = (double *)s.ptr[3];
    uint32_t *one = (uint32_t *)s.ptr[4];
    const uint32_t one_h = 1u;
    if ((e = hipMemcpy(dcand, cs.data(), (size_t)nc * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(one, &one_h, 4, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "cbc upload");
    const uint32_t nb = (jend + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_fill, dim3(nb), dim3(kBlock), 0, nullptr, prod, jend, 1.0);
    const double inv_n = 1.0 / (double)n;
    const double two_pi2 = 2.0 * 3.141592653589793 * 3.141592653589793;
    std::vector<double> h(nc);
    for (uint32_t comp = 0; comp < d; ++comp) {
        const double w = two_pi2 * gam[comp];
        // z_1 = 1: in one dimension every unit gives the same point set
        const bool first = comp == 0;
        const uint32_t cnt = first ? 1u : nc;
        const uint32_t cbx = first ? 1u : bx;
        const uint32_t csl = first ? std::min(max_slices, want) : slices;
        const uint32_t cch = (jend + csl - 1) / csl;
        CbcArgs a{(uint32_t)n, jend, cnt, cch, inv_n, w, prod, first ? one : dcand, partial};
        hipLaunchKernelGGL(k_cbc_eval, dim3(cbx, csl), dim3(kBlock), 0, nullptr, a);
        hipLaunchKernelGGL(k_cbc_reduce, dim3((cnt + kBlock - 1) / kBlock), dim3(kBlock), 0, nullptr,
                           (const double2 *)partial, csl, cnt, (uint32_t)n, inv_n, w, (const double *)prod, e2);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "launch CBC kernels");
        if ((e = hipMemcpy(h.data(), e2, (size_t)cnt * 8, hipMemcpyDeviceToHost)) != hipSuccess)
            return hip_fail(e, "cbc download");
        // lattice symmetries make exact ties common (in two dimensions c and
        // c^-1 mod n give the same error) and rounding would choose among
        // them: values within 1e-13 (1 + e^2) of the minimum are ties, and
        // ties go to the smallest c (candidates ascend)
        double vmin = h[0];
        for (uint32_t t = 1; t < cnt; ++t) vmin = std::min(vmin, h[t]);
        if (!std::isfinite(vmin)) return fail(QMC_ENONFINITE, "CBC error not finite");
        const double tau = 1e-13 * (1.0 + std::fabs(vmin));
        uint32_t best = 0;
        while (!(h[best] <= vmin + tau)) ++best;
        const uint32_t z = first ? 1u : cs[best];
        z_out[comp] = z;
        e2_out[comp] = h[best];
        hipLaunchKernelGGL(k_cbc_update, dim3(nb), dim3(kBlock), 0, nullptr, prod, (uint32_t)n, jend, inv_n, z, w);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "launch CBC update");
    }
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "cbc synchronize");
    return QMC_OK;
}
