// One estimate of eqs. (2)-(3) without any device allocation
// (qmc_integrate_static in qmc.h).
//
// The rule's device copies (g, the thread-stride steps, the padded shift
// table), the integrand's parameter blob, the per-block partial sums and the
// result buffer all live in one file-scope device array, `scratch`, of
// kScratchBytes.  Its address on each device is taken once with
// hipGetSymbolAddress (the array's name is only a host-side stand-in) and
// kept per device.  Every call on a device shares that device's array, so
// calls that overlap on one device race; nothing in it has to start at zero
// (the lattice kernel writes every partial it produces, the finalize kernel
// every result).
#include "qmc_runtime.hpp"

#include <cstring>
#include <mutex>

namespace qmc {

constexpr size_t kScratchBytes = size_t(1) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr uint32_t kStaticMaxM = 64;
constexpr size_t kStaticMaxBlob = 8192;  // doubles

// byte offsets of the regions (each 256-byte aligned)
constexpr size_t kOffG = 0;
constexpr size_t kOffGstep = 256;
constexpr size_t kOffShifts = 512;                                    // <= 64 rows x 16 x 8 B
constexpr size_t kOffOut = kOffShifts + (size_t)kStaticMaxM * kMaxDim * 8;
constexpr size_t kOutBytes = ((kMaxParts * kStaticMaxM + 2 * kMaxParts) * 8 + 255) / 256 * 256;
constexpr size_t kOffBlob = kOffOut + kOutBytes;
constexpr size_t kOffPartials = kOffBlob + kStaticMaxBlob * 8;
static_assert(kOffPartials % 256 == 0, "aligned regions");
static_assert(kOffPartials < kScratchBytes, "scratch too small");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_lock;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// address of the current device's array, looked up once per device
qmc_status scratch_for(int dev, unsigned char *&ptr) {
    if (dev < 0 || dev >= kMaxDevices) return fail(QMC_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_lock);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    ptr = g_scratch_ptr[dev];
    return QMC_OK;
}

}  // namespace
}  // namespace qmc

using namespace qmc;

extern "C" qmc_status qmc_integrate_static(uint32_t d, uint64_t n, const uint64_t *g, uint32_t m,
                                           const double *shifts, qmc_transform t, qmc_family family,
                                           const void *params, void *stream, qmc_result *out, double *per_shift) {
    if (!out) return fail(QMC_EINVAL, "out is NULL");
    qmc_status st = validate_rule(d, n, g, m, shifts, t);
    if (st) return st;
    if (m > kStaticMaxM) return fail(QMC_EUNSUPPORTED, "m = %u > %u shifts in the static scratch", m, kStaticMaxM);
    Packed pk;
    if ((st = pack_params((int)family, d, params, pk))) return st;
    if (pk.orders >= 2 || pk.deform)
        return fail(QMC_EUNSUPPORTED, "expansion orders and contour deformation need the specialised kernels");
    if (pk.blob.size() > kStaticMaxBlob)
        return fail(QMC_EUNSUPPORTED, "parameter blob of %zu doubles > %zu in the static scratch", pk.blob.size(),
                    kStaticMaxBlob);
    if ((size_t)m * pk.np > kMaxRows) return fail(QMC_EUNSUPPORTED, "m * parts > %u", kMaxRows);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    unsigned char *base = nullptr;
    if ((st = scratch_for(dev, base))) return st;

    // precompiled kernels only: a specialised sector kernel needs a code
    // object loaded, which allocates
    uint32_t T = 0;
    LatticeLaunch fn = find_kernel(pk.key_family, t, d, default_tile(pk.key_family), T);
    if (!fn) return fail(QMC_EUNSUPPORTED, "no kernel for family %d, transform %d/%d, d = %u", pk.key_family, t.kind,
                         t.alpha, d);
    const uint32_t nn = (uint32_t)n, tiles = (m + T - 1) / T;
    uint32_t bx = grid_x(nn, tiles, dev, 8);
    const size_t part_cap = (kScratchBytes - kOffPartials) / sizeof(double2);
    while (bx > 1 && (size_t)m * pk.np * bx > part_cap) bx /= 2;
    if ((size_t)m * pk.np * bx > part_cap) return fail(QMC_EUNSUPPORTED, "partials beyond the static scratch");

    uint32_t g32[kMaxDim], gs[kMaxDim];
    for (uint32_t i = 0; i < d; ++i) g32[i] = (uint32_t)(g[i] % n);
    gstep_for(g32, d, nn, (uint64_t)bx * kBlock, gs);
    const uint32_t rows = padded_rows(m);
    const std::vector<double> sh = padded_shifts(std::vector<double>(shifts, shifts + (size_t)m * d), m, d, rows, t);

    hipStream_t s = (hipStream_t)stream;
    uint32_t *d_g = reinterpret_cast<uint32_t *>(base + kOffG);
    uint32_t *d_gs = reinterpret_cast<uint32_t *>(base + kOffGstep);
    double *d_sh = reinterpret_cast<double *>(base + kOffShifts);
    double *d_out = reinterpret_cast<double *>(base + kOffOut);
    double *d_blob = reinterpret_cast<double *>(base + kOffBlob);
    double2 *d_part = reinterpret_cast<double2 *>(base + kOffPartials);
    if ((e = hipMemcpyAsync(d_g, g32, d * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(d_gs, gs, d * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(d_sh, sh.data(), sh.size() * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(d_blob, pk.blob.data(), pk.blob.size() * 8, hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "static upload");

    LatticeArgs a{};
    a.n = nn;
    a.d = d;
    a.m = m;
    a.tiles = tiles;
    a.inv_n = 1.0 / (double)n;
    a.g = d_g;
    a.gstep = d_gs;
    a.shifts = d_sh;
    a.params = d_blob;
    a.g_stride = a.shift_stride = a.param_stride = 0;
    a.np = pk.np;
    a.partials = d_part;
    if ((e = fn(a, dim3(bx, tiles), s)) != hipSuccess) return hip_fail(e, "launch lattice kernel");
    FinalizeArgs f{};
    f.partials = d_part;
    f.nblk = bx;
    f.m = m;
    f.np = pk.np;
    f.n = (double)n;
    f.scale = transform_scale(t, d);
    f.sub = 0.0;
    f.q = d_out;
    f.res = d_out + out_res_offset(m);
    if ((e = launch_finalize(f, 1, s)) != hipSuccess) return hip_fail(e, "launch finalize kernel");
    double h[kMaxParts * kStaticMaxM + 2 * kMaxParts];
    if ((e = hipMemcpyAsync(h, d_out, out_doubles(m) * 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "static results");
    const size_t nq = (size_t)m * pk.np;
    bool finite = true;
    for (size_t i = 0; i < nq; ++i) finite = finite && std::isfinite(h[i]);
    if (per_shift) std::memcpy(per_shift, h, nq * sizeof(double));
    const double *res = h + out_res_offset(m);
    out->is_complex = pk.np >= 2;
    out->used_cv = 0;
    out->contour_crossed = 0.0;
    if (!finite) {
        out->mean_re = out->mean_im = out->err_re = out->err_im = NAN;
        return fail(QMC_ENONFINITE, "a per-shift sum is not finite");
    }
    out->mean_re = res[0];
    out->mean_im = pk.np >= 2 ? res[1] : 0.0;
    out->err_re = res[2];
    out->err_im = pk.np >= 2 ? res[3] : 0.0;
    return QMC_OK;
}
