// Host runtime and C ABI of the lattice estimator (declarations in qmc.h).
//
// A plan holds the rule of eq. (2) of arXiv:1811.11722 -- d, n, g, m, the m
// shifts and the periodising transform -- resident in device memory.  Each
// qmc_integrate call packs the integrand parameters into a blob (uploaded
// only when it changed), launches the lattice kernel and the finalize kernel
// on the plan's stream and copies back the m per-shift values and the
// (mean, error) of eqs. (2)-(3): one small host->device copy at most and
// one device->host copy per estimate.
#include "qmc_runtime.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>

namespace qmc {

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

qmc_status fail(qmc_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

qmc_status hip_fail(hipError_t e, const char *what) {
    return fail(QMC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int device_cu_count(int dev) {
    static std::map<int, int> cache;
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0)
        cu = 256;
    cache[dev] = cu;
    return cu;
}

// ------------------------------------------------------- parameter packing
static inline double bits(uint64_t v) {
    double d;
    std::memcpy(&d, &v, sizeof d);
    return d;
}

static bool finite_all(const double *p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// factor-list code of one monomial: count in bits 0..3, then 5 bits per factor
static qmc_status monomial_code(const uint8_t *e, uint32_t d, uint64_t &code) {
    uint64_t c = 0;
    uint32_t cnt = 0;
    for (uint32_t i = 0; i < d; ++i) {
        if (e[i] > 2) return fail(QMC_EINVAL, "exponent %u > 2 in variable %u", (unsigned)e[i], i);
        for (uint32_t r = 0; r < e[i]; ++r) {
            if (cnt >= 12) return fail(QMC_EUNSUPPORTED, "monomial of total degree > 12");
            c |= (uint64_t)i << (4 + 5 * cnt);
            ++cnt;
        }
    }
    code = c | cnt;
    return QMC_OK;
}

qmc_status pack_params(int family, uint32_t d, const void *params, Packed &pk) {
    const uint32_t D = d;
    pk.blob.clear();
    pk.np = 1;
    pk.key_family = family;
    switch (family) {
    case QMC_F_CONST: {
        if (!params) return fail(QMC_EINVAL, "QMC_F_CONST needs qmc_const_params");
        const auto *p = static_cast<const qmc_const_params *>(params);
        if (!std::isfinite(p->c)) return fail(QMC_EINVAL, "constant is not finite");
        pk.blob = {p->c};
        break;
    }
    case QMC_F_P2KERNEL:
        pk.blob = {0.0};
        break;
    case QMC_F_TRIG: {
        if (!params) return fail(QMC_EINVAL, "QMC_F_TRIG needs qmc_trig_params");
        const auto *p = static_cast<const qmc_trig_params *>(params);
        if (p->n_terms > 4096) return fail(QMC_EUNSUPPORTED, "more than 4096 trigonometric terms");
        if (p->n_terms && (!p->h || !p->c || !p->phi)) return fail(QMC_EINVAL, "null trig arrays");
        if (!std::isfinite(p->c0)) return fail(QMC_EINVAL, "c0 is not finite");
        pk.blob.push_back(bits(p->n_terms));
        pk.blob.push_back(p->c0);
        for (uint32_t t = 0; t < p->n_terms; ++t) {
            if (!std::isfinite(p->c[t]) || !std::isfinite(p->phi[t]))
                return fail(QMC_EINVAL, "trig coefficient %u is not finite", t);
            pk.blob.push_back(p->c[t]);
            pk.blob.push_back(p->phi[t] / (2.0 * M_PI));
            for (uint32_t i = 0; i < D; ++i) pk.blob.push_back((double)p->h[(size_t)t * d + i]);
        }
        break;
    }
    case QMC_F_GENZ_PRODUCT_PEAK:
    case QMC_F_GENZ_OSCILLATORY:
    case QMC_F_GENZ_GAUSSIAN:
    case QMC_F_GENZ_CONTINUOUS:
    case QMC_F_GENZ_CORNER_PEAK: {
        if (!params) return fail(QMC_EINVAL, "Genz family needs qmc_genz_params");
        const auto *p = static_cast<const qmc_genz_params *>(params);
        if (!p->a || !p->u) return fail(QMC_EINVAL, "null Genz arrays");
        if (!finite_all(p->a, d) || !finite_all(p->u, d)) return fail(QMC_EINVAL, "Genz parameter not finite");
        if (family == QMC_F_GENZ_PRODUCT_PEAK) {
            for (uint32_t i = 0; i < d; ++i)
                if (p->a[i] == 0.0) return fail(QMC_EINVAL, "product peak needs a_i != 0");
            for (uint32_t i = 0; i < D; ++i) pk.blob.push_back(1.0 / (p->a[i] * p->a[i]));
            for (uint32_t i = 0; i < D; ++i) pk.blob.push_back(p->u[i]);
            for (uint32_t i = 0; i < D; ++i) pk.blob.push_back(0.5 - p->u[i]);
            // tile flag: one reciprocal may serve a thread's shifts if every
            // denominator prod_i q_i, a^-2 <= q_i <= a^-2 + max(u^2, (1-u)^2),
            // lies within 2^-62 .. 2^62 (products of up to 16 of them then stay
            // within 2^-1000 .. 2^1000)
            double lg_lo = 0.0, lg_hi = 0.0;
            for (uint32_t i = 0; i < d; ++i) {
                const double a2 = 1.0 / (p->a[i] * p->a[i]);
                const double s2 = std::max(p->u[i] * p->u[i], (1.0 - p->u[i]) * (1.0 - p->u[i]));
                lg_lo += std::log2(a2);
                lg_hi += std::log2(a2 + s2);
            }
            pk.blob.push_back(std::isfinite(lg_lo) && std::isfinite(lg_hi) && lg_lo >= -62.0 && lg_hi <= 62.0 ? 1.0
                                                                                                                : 0.0);
        } else if (family == QMC_F_GENZ_OSCILLATORY) {
            for (uint32_t i = 0; i < D; ++i) pk.blob.push_back(p->a[i]);
            pk.blob.push_back(2.0 * M_PI * p->u[0]);
        } else if (family == QMC_F_GENZ_GAUSSIAN) {
            for (uint32_t i = 0; i < D; ++i) pk.blob.push_back(p->a[i] * p->a[i]);
            for (uint32_t i = 0; i < D; ++i) pk.blob.push_back(p->u[i]);
        } else if (family == QMC_F_GENZ_CONTINUOUS) {
            for (uint32_t i = 0; i < D; ++i) pk.blob.push_back(p->a[i]);
            for (uint32_t i = 0; i < D; ++i) pk.blob.push_back(p->u[i]);
        } else {
            for (uint32_t i = 0; i < D; ++i) pk.blob.push_back(p->a[i]);
        }
        break;
    }
    case QMC_F_SECTOR: {
        if (!params) return fail(QMC_EINVAL, "QMC_F_SECTOR needs qmc_sector_params");
        const auto *p = static_cast<const qmc_sector_params *>(params);
        if (p->n_u == 0 || p->n_f == 0) return fail(QMC_EINVAL, "n_u and n_f must be >= 1");
        if (p->n_u > 4096 || p->n_f > 4096) return fail(QMC_EUNSUPPORTED, "more than 4096 monomials");
        if (!p->coef_u || !p->exp_u || !p->coef_f || !p->exp_f || !p->nu)
            return fail(QMC_EINVAL, "null sector arrays");
        if (!finite_all(p->coef_u, p->n_u) || !finite_all(p->coef_f, p->n_f))
            return fail(QMC_EINVAL, "polynomial coefficient not finite");
        if (!std::isfinite(p->pow_u) || !std::isfinite(p->pow_f)) return fail(QMC_EINVAL, "power not finite");
        const bool cplx = p->is_complex != 0;
        if (cplx && (!std::isfinite(p->delta_im))) return fail(QMC_EINVAL, "delta_im not finite");
        // the phase pow_f * arg(F - i delta) must stay inside the exact range
        // of the device sine and cosine (|x| < 2^19)
        if (cplx && std::fabs(p->pow_f) > 1.0e5) return fail(QMC_EUNSUPPORTED, "|pow_f| > 1e5 for a complex sector");
        uint64_t nucode = 0;
        for (uint32_t i = 0; i < d; ++i) {
            if (p->nu[i] > 2) return fail(QMC_EINVAL, "nu_%u = %u > 2", i, (unsigned)p->nu[i]);
            nucode |= (uint64_t)p->nu[i] << (2 * i);
        }
        qmc_status st = QMC_OK;
        uint32_t flags = (cplx ? 1u : 0u) | (p->pow_u == -2.0 ? 2u : 0u);
        pk.blob = {bits(p->n_u), bits(p->n_f), bits(flags), p->pow_u, p->pow_f, cplx ? p->delta_im : 0.0,
                   bits(nucode)};
        // terms are stored in the order the specialised code reads them (the
        // polynomial is the same sum in any order)
        std::vector<uint64_t> cu(p->n_u), cf(p->n_f);
        for (uint32_t t = 0; t < p->n_u; ++t)
            if ((st = monomial_code(p->exp_u + (size_t)t * d, d, cu[t]))) return st;
        for (uint32_t t = 0; t < p->n_f; ++t)
            if ((st = monomial_code(p->exp_f + (size_t)t * d, d, cf[t]))) return st;
        const std::vector<uint32_t> ou = horner_term_order(cu, d), of = horner_term_order(cf, d);
        for (uint32_t t : ou) pk.blob.push_back(p->coef_u[t]);
        for (uint32_t t : ou) pk.blob.push_back(bits(cu[t]));
        for (uint32_t t : of) pk.blob.push_back(p->coef_f[t]);
        for (uint32_t t : of) pk.blob.push_back(bits(cf[t]));
        if (cplx) {
            pk.np = 2;
            pk.key_family = kFamSectorComplex;
            pk.cplx = true;
        }
        if (p->n_orders >= 2) {
            if (p->n_orders > kSectorMaxOrders)
                return fail(QMC_EUNSUPPORTED, "n_orders = %u > %u", p->n_orders, kSectorMaxOrders);
            if (!std::isfinite(p->eps_u) || !std::isfinite(p->eps_f)) return fail(QMC_EINVAL, "eps not finite");
            flags |= kSectorOrders;
            pk.blob[2] = bits(flags);
            pk.blob.push_back(p->eps_u);
            pk.blob.push_back(p->eps_f);
            pk.blob.push_back(bits(p->n_orders));
            pk.orders = p->n_orders;
            pk.np *= p->n_orders;
        }
        if (p->deform_lambda != 0.0) {
            if (!std::isfinite(p->deform_lambda)) return fail(QMC_EINVAL, "deform_lambda not finite");
            if (std::fabs(p->pow_f) > 1.0e5 || std::fabs(p->pow_u) > 1.0e5)
                return fail(QMC_EUNSUPPORTED, "|pow_u| or |pow_f| > 1e5 for a deformed sector");
            flags |= kSectorComplex | kSectorDeform;
            pk.blob[2] = bits(flags);
            pk.blob.push_back(p->deform_lambda);
            pk.deform = true;
            pk.cplx = true;
            pk.key_family = kFamSectorComplex;
            // Re, Im per order, then the count of points on the wrong side
            pk.np = 2 * (p->n_orders >= 2 ? p->n_orders : 1u) + 1;
            pk.crossing = true;
        }
        break;
    }
    default:
        return fail(QMC_EINVAL, "unknown family %d", family);
    }
    return QMC_OK;
}

double transform_scale(const qmc_transform &t, uint32_t d) {
    if (t.kind == QMC_T_SIDI) {
        // 1 / T_m per dimension, T_m = int_0^1 sin^m(pi x) dx
        const int m = t.alpha, p = m / 2;
        double tm;
        if (m % 2 == 0) {
            tm = 1.0;  // binom(2p, p) / 4^p
            for (int k = 1; k <= p; ++k) tm *= (double)(p + k) / (4.0 * k);
        } else {
            double p1 = 0.0, b = 1.0;  // sum_k binom(p, k) (-1)^k / (2k + 1)
            for (int k = 0; k <= p; ++k) {
                p1 += ((k & 1) ? -b : b) / (2 * k + 1);
                b = b * (p - k) / (k + 1);
            }
            tm = 2.0 * p1 / 3.141592653589793;
        }
        return std::pow(1.0 / tm, (double)d);
    }
    if (t.kind != QMC_T_KOROBOV) return 1.0;
    double c = 1.0;  // (2a+1)! / (a!)^2
    for (int k = t.alpha + 1; k <= 2 * t.alpha + 1; ++k) c *= k;
    for (int k = 2; k <= t.alpha; ++k) c /= k;
    return std::pow(c, (double)d);
}

// ------------------------------------------------------------ kernel choice
static const int kTChoices[] = {8, 4, 2, 1};

LatticeLaunch find_kernel(int key_family, const qmc_transform &t, uint32_t d, uint32_t want_T,
                          uint32_t &T_out) {
    auto &reg = lattice_registry();
    const int alpha = (t.kind == QMC_T_KOROBOV || t.kind == QMC_T_SIDI) ? t.alpha : 0;
    if (want_T) {
        auto it = reg.find(KernelKey{key_family, t.kind, alpha, (int)d, (int)want_T});
        if (it != reg.end()) {
            T_out = want_T;
            return it->second;
        }
    }
    for (int T : kTChoices) {
        auto it = reg.find(KernelKey{key_family, t.kind, alpha, (int)d, T});
        if (it != reg.end()) {
            T_out = (uint32_t)T;
            return it->second;
        }
    }
    return nullptr;
}

uint32_t default_tile(int key_family) {
    switch (key_family) {
    case QMC_F_GENZ_PRODUCT_PEAK: return 4;
    case QMC_F_SECTOR: return 2;
    case kFamSectorComplex: return 1;
    case QMC_F_P2KERNEL: return 1;
    default: return 4;
    }
}

// Workgroups along the points: about blocks_per_cu (default 8) per CU over
// all shift tiles, and at most one per kBlock x kMinPointsPerThread points.
// Below that floor a thread would walk one or two points and the launch
// would be all block reductions and partials (one instance of n = 131071,
// m = 16: 17.4 us -> 13.2 us per kernel with the floor).
constexpr uint64_t kMinPointsPerThread = 4;

uint32_t grid_x(uint32_t n, uint32_t tiles_total, int dev, uint32_t blocks_per_cu) {
    const uint64_t target = (uint64_t)device_cu_count(dev) * (blocks_per_cu ? blocks_per_cu : 8);
    uint64_t bx = std::max<uint64_t>(1, target / std::max<uint32_t>(1, tiles_total));
    const uint64_t cap = (n + kBlock * kMinPointsPerThread - 1) / (kBlock * kMinPointsPerThread);
    bx = std::min(bx, cap);
    return (uint32_t)std::max<uint64_t>(bx, 1);
}

void gstep_for(const uint32_t *g, uint32_t d, uint32_t n, uint64_t S, uint32_t *out) {
    const uint64_t s = S % n;
    for (uint32_t i = 0; i < d; ++i) out[i] = (uint32_t)((s * (uint64_t)g[i]) % n);
}

// shift tables on the device hold whole tiles of up to kMaxTile rows; rows
// past m repeat the last shift (their sums are never read)
uint32_t padded_rows(uint32_t m) { return (m + kMaxTile - 1) / kMaxTile * kMaxTile; }

// The baker's transform reads its points moved by 1/2 (TrBaker): the device
// table holds {Delta + 1/2} for it, so the move costs nothing per point.
std::vector<double> padded_shifts(const std::vector<double> &sh, uint32_t m, uint32_t d, uint32_t rows,
                                  const qmc_transform &tr) {
    const bool half = tr.kind == QMC_T_BAKER;
    std::vector<double> out((size_t)rows * d);
    for (uint32_t r = 0; r < rows; ++r)
        for (uint32_t i = 0; i < d; ++i) {
            const double v = sh[(size_t)std::min(r, m - 1) * d + i];
            out[(size_t)r * d + i] = !half ? v : (v < 0.5 ? v + 0.5 : v - 0.5);
        }
    return out;
}

// --------------------------------------------------------------- plan ops
qmc_status plan_upload_params(qmc_plan_s *p, const Packed &pk) {
    if (pk.blob.size() > p->params_cap) {
        if (p->d_params) hipFree(p->d_params);
        p->d_params = nullptr;
        p->params_cap = 0;
        hipError_t e = hipMalloc(&p->d_params, pk.blob.size() * sizeof(double));
        if (e != hipSuccess) return fail(QMC_ENOMEM, "hipMalloc params: %s", hipGetErrorString(e));
        p->params_cap = pk.blob.size();
        p->last_blob.clear();
    }
    if (pk.blob != p->last_blob) {
        hipError_t e = hipMemcpyAsync(p->d_params, pk.blob.data(), pk.blob.size() * sizeof(double),
                                      hipMemcpyHostToDevice, p->stream);
        if (e != hipSuccess) return hip_fail(e, "upload params");
        e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return hip_fail(e, "upload params");
        p->last_blob = pk.blob;
    }
    return QMC_OK;
}

qmc_status ensure_buffer(void **ptr, size_t &cap, size_t bytes, const char *what) {
    if (bytes <= cap) return QMC_OK;
    if (*ptr) hipFree(*ptr);
    *ptr = nullptr;
    cap = 0;
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) return fail(QMC_ENOMEM, "hipMalloc %s (%zu bytes): %s", what, bytes, hipGetErrorString(e));
    cap = bytes;
    return QMC_OK;
}

qmc_status plan_set_gstep(qmc_plan_s *p, uint32_t S) {
    if (S == p->cur_S) return QMC_OK;
    std::vector<uint32_t> gs(p->d);
    gstep_for(p->g.data(), p->d, p->n, S, gs.data());
    hipError_t e = hipMemcpyAsync(p->d_gstep, gs.data(), p->d * sizeof(uint32_t), hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) return hip_fail(e, "upload gstep");
    e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "upload gstep");
    p->cur_S = S;
    return QMC_OK;
}

// Enqueue the lattice kernel (a registry launcher or a specialised module
// function) and the finalize kernel of one estimate.
static qmc_status plan_launch(qmc_plan_s *p, const Packed &pk, LatticeLaunch fn, hipFunction_t jfn, uint32_t T,
                              uint32_t bpc) {
    if (p->m * pk.np > kMaxRows) return fail(QMC_EUNSUPPORTED, "m * parts > %u", kMaxRows);
    qmc_status st = plan_upload_params(p, pk);
    if (st) return st;
    const uint32_t tiles = (p->m + T - 1) / T;
    const uint32_t bx = grid_x(p->n, tiles, p->device, bpc);
    if ((st = plan_set_gstep(p, bx * kBlock))) return st;
    const size_t pbytes = (size_t)p->m * pk.np * bx * sizeof(double2);
    if ((st = ensure_buffer((void **)&p->d_partials, p->partials_cap, pbytes, "partials"))) return st;

    LatticeArgs a{};
    a.n = p->n;
    a.d = p->d;
    a.m = p->m;
    a.tiles = tiles;
    a.inv_n = p->inv_n;
    a.g = p->d_g;
    a.gstep = p->d_gstep;
    a.shifts = p->d_shifts;
    a.params = p->d_params;
    a.g_stride = a.shift_stride = a.param_stride = 0;
    a.np = pk.np;
    a.partials = p->d_partials;
    if (p->timing) hipEventRecord(p->ev0, p->stream);
    hipError_t e = jfn ? jit_launch(jfn, a, dim3(bx, tiles), p->stream) : fn(a, dim3(bx, tiles), p->stream);
    if (e != hipSuccess) return hip_fail(e, "launch lattice kernel");
    if (p->timing) hipEventRecord(p->ev1, p->stream);

    FinalizeArgs f{};
    f.partials = p->d_partials;
    f.nblk = bx;
    f.m = p->m;
    f.np = pk.np;
    f.n = (double)p->n;
    f.scale = transform_scale(p->tr, p->d);
    f.sub = 0.0;
    f.q = p->d_out;
    f.res = p->d_out + out_res_offset(p->m);
    e = launch_finalize(f, 1, p->stream);
    if (e != hipSuccess) return hip_fail(e, "launch finalize kernel");
    p->last_T = T;
    p->last_bx = bx;
    p->last_jit = jfn != nullptr;
    return QMC_OK;
}

qmc_status plan_enqueue_fn(qmc_plan_s *p, const Packed &pk, hipFunction_t jfn, uint32_t T) {
    return plan_launch(p, pk, nullptr, jfn, T, p->launch.blocks_per_cu);
}

qmc_status plan_enqueue(qmc_plan_s *p, const Packed &pk, uint32_t want_T, uint32_t bpc) {
    uint32_t T = 0;
    LatticeLaunch fn = nullptr;
    hipFunction_t jfn = nullptr;
    const bool sector = pk.key_family == QMC_F_SECTOR || pk.key_family == kFamSectorComplex;
    if (sector && p->jit_mode != 0) {
        // four shifts per thread for real sectors of up to eight dimensions
        // (measured at n = 2^24 - 3, m = 32: 2.19, 2.43, 2.36 ms against
        // 2.29, 2.50, 2.44 ms with two at d = 6, 7, 8; at d = 9 four run
        // 27 % slower) and for real expansion orders up to six (three
        // orders: 2.45 against 2.60 ms at d = 6, 8 % slower at d = 8), two
        // for the others; a deformed point carries the Jacobian's triangle,
        // so one
        const bool wide = !pk.cplx && p->d <= (pk.orders < 2 ? 8u : 6u);
        T = want_T ? want_T : (pk.deform ? 1u : wide ? 4u : 2u);
        std::string err;
        jfn = jit_kernel(pk.blob, p->d, p->tr, T, pk.cplx, p->device, err);
        if (!jfn && (p->jit_mode == 2 || pk.orders >= 2 || pk.deform))
            return fail(QMC_EUNSUPPORTED, "specialised sector kernel: %s", err.c_str());
    }
    if (!jfn && pk.orders >= 2) return fail(QMC_EUNSUPPORTED, "expansion orders need the specialised kernel (jit mode 1 or 2)");
    if (!jfn && pk.deform) return fail(QMC_EUNSUPPORTED, "contour deformation needs the specialised kernel (jit mode 1 or 2)");
    if (!jfn) {
        fn = find_kernel(pk.key_family, p->tr, p->d, want_T ? want_T : default_tile(pk.key_family), T);
        if (!fn)
            return fail(QMC_EUNSUPPORTED, "no kernel for family %d, transform %d/%d, d = %u", pk.key_family,
                        p->tr.kind, p->tr.alpha, p->d);
    } else if (bpc == 0) {
        // the specialised sector kernels hold few enough registers for four
        // waves per SIMD; 16 workgroups per CU fill whole residency rounds
        bpc = 16;
    }
    return plan_launch(p, pk, fn, jfn, T, bpc);
}

qmc_status plan_collect(qmc_plan_s *p, uint32_t np, qmc_result *out, double *per_shift, bool crossing) {
    hipError_t e = hipMemcpyAsync(p->h_out, p->d_out, out_doubles(p->m) * sizeof(double), hipMemcpyDeviceToHost,
                                  p->stream);
    if (e != hipSuccess) return hip_fail(e, "copy results");
    e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "synchronize");
    if (p->timing) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->ev0, p->ev1) == hipSuccess) {
            p->kernel_ms += ms;
            p->kernel_launches += 1;
        }
    }
    return plan_results(p, np, out, per_shift, crossing);
}

// The result of an estimate whose output is in the plan's pinned mirror.
qmc_status plan_results(qmc_plan_s *p, uint32_t np, qmc_result *out, double *per_shift, bool crossing) {
    // with a crossing count the last of the np parts is the count, not a
    // value: it is left out of per_shift and of the finiteness check
    const uint32_t nv = crossing ? np - 1 : np;
    const double *q = p->h_out, *res = p->h_out + out_res_offset(p->m);
    bool finite = true;
    for (uint32_t k = 0; k < p->m; ++k)
        for (uint32_t j = 0; j < nv; ++j) {
            const double v = q[(size_t)k * np + j];
            finite = finite && std::isfinite(v);
            if (per_shift) per_shift[(size_t)k * nv + j] = v;
        }
    double crossed = 0.0;
    if (crossing) {
        // finalize scaled every part by the transform's constant and 1/n
        long double s = 0.0L;
        for (uint32_t k = 0; k < p->m; ++k) s += q[(size_t)k * np + nv];
        crossed = (double)(s / ((long double)p->m * transform_scale(p->tr, p->d)));
    }
    out->is_complex = nv >= 2;
    out->used_cv = 0;
    out->contour_crossed = crossed;
    if (!finite) {
        out->mean_re = out->mean_im = out->err_re = out->err_im = NAN;
        return fail(QMC_ENONFINITE, "a per-shift sum is not finite");
    }
    out->mean_re = res[0];
    out->mean_im = nv >= 2 ? res[1] : 0.0;
    out->err_re = res[2];
    out->err_im = nv >= 2 ? res[3] : 0.0;
    if (crossed > 0.0)
        return fail(QMC_ECONTOUR, "the deformed contour has Im(F - i delta) > 0 at a fraction %.3g of the points",
                    crossed);
    return QMC_OK;
}

// The conditions of a rule (eq. (2)) every entry point that takes one
// checks before any device call; t.alpha is cleared for transforms
// without a parameter.
qmc_status validate_rule(uint32_t d, uint64_t n, const uint64_t *g, uint32_t m, const double *shifts,
                         qmc_transform &t) {
    if (d == 0) return fail(QMC_EINVAL, "d must be >= 1");
    if (d > kMaxDim) return fail(QMC_EUNSUPPORTED, "d = %u > %u", d, kMaxDim);
    if (n < 2) return fail(QMC_EINVAL, "n must be >= 2");
    if (n > (1ull << 31)) return fail(QMC_EUNSUPPORTED, "n > 2^31");
    if (!g) return fail(QMC_EINVAL, "g is NULL");
    for (uint32_t i = 0; i < d; ++i)
        if (g[i] % n == 0) return fail(QMC_EINVAL, "g_%u mod n == 0", i);
    if (m < 2) return fail(QMC_EINVAL, "m must be >= 2 (eq. (3) divides by m - 1)");
    if (m > kMaxRows) return fail(QMC_EUNSUPPORTED, "m > %u", kMaxRows);
    if (!shifts) return fail(QMC_EINVAL, "shifts is NULL");
    for (size_t i = 0; i < (size_t)m * d; ++i)
        if (!(shifts[i] >= 0.0 && shifts[i] < 1.0)) return fail(QMC_EINVAL, "shift %zu outside [0,1)", i);
    if (t.kind != QMC_T_NONE && t.kind != QMC_T_KOROBOV && t.kind != QMC_T_BAKER && t.kind != QMC_T_SIDI)
        return fail(QMC_EINVAL, "unknown transform %d", t.kind);
    if (t.kind == QMC_T_KOROBOV && t.alpha < 1) return fail(QMC_EINVAL, "Korobov weight must be >= 1");
    if (t.kind == QMC_T_KOROBOV && t.alpha > 6) return fail(QMC_EUNSUPPORTED, "Korobov weight > 6");
    if (t.kind == QMC_T_SIDI && t.alpha < 1) return fail(QMC_EINVAL, "Sidi order must be >= 1");
    if (t.kind == QMC_T_SIDI && t.alpha > 6) return fail(QMC_EUNSUPPORTED, "Sidi order > 6");
    if (t.kind != QMC_T_KOROBOV && t.kind != QMC_T_SIDI) t.alpha = 0;
    return QMC_OK;
}

}  // namespace qmc

using namespace qmc;

// ==================================================================== C ABI
extern "C" {

const char *qmc_status_string(int32_t status) {
    // an int, not the enum: any value a caller passes is defined behaviour
    switch (status) {
    case QMC_OK: return "ok";
    case QMC_EINVAL: return "invalid argument";
    case QMC_EUNSUPPORTED: return "unsupported";
    case QMC_ENOMEM: return "out of memory";
    case QMC_EDEVICE: return "device error";
    case QMC_ENONFINITE: return "non-finite result";
    case QMC_ECONTOUR: return "deformed contour crosses the cut";
    }
    return "unknown status";
}

const char *qmc_last_error(void) { return g_last_error.c_str(); }

qmc_status qmc_plan_create(uint32_t d, uint64_t n, const uint64_t *g, uint32_t m, const double *shifts,
                           qmc_transform t, qmc_plan_t *out) {
    if (!out) return fail(QMC_EINVAL, "out is NULL");
    qmc_status vs = validate_rule(d, n, g, m, shifts, t);
    if (vs) return vs;

    auto *p = new (std::nothrow) qmc_plan_s();
    if (!p) return fail(QMC_ENOMEM, "host allocation");
    p->d = d;
    p->n = (uint32_t)n;
    p->m = m;
    p->inv_n = 1.0 / (double)n;
    p->tr = t;
    p->g.resize(d);
    for (uint32_t i = 0; i < d; ++i) p->g[i] = (uint32_t)(g[i] % n);
    p->shifts.assign(shifts, shifts + (size_t)m * d);
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipGetDevice");
    }
    qmc_status st = QMC_OK;
    size_t cap = 0;
    if ((st = ensure_buffer((void **)&p->d_g, cap, d * sizeof(uint32_t), "g")) ||
        (cap = 0, st = ensure_buffer((void **)&p->d_gstep, cap, d * sizeof(uint32_t), "gstep")) ||
        (cap = 0, st = ensure_buffer((void **)&p->d_shifts, cap, (size_t)padded_rows(m) * d * sizeof(double),
                                     "shifts")) ||
        (cap = 0, st = ensure_buffer((void **)&p->d_out, cap, out_doubles(m) * sizeof(double), "out"))) {
        qmc_plan_destroy(p);
        return st;
    }
    e = hipHostMalloc((void **)&p->h_out, out_doubles(m) * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        qmc_plan_destroy(p);
        return fail(QMC_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    if ((e = hipMemcpy(p->d_g, p->g.data(), d * sizeof(uint32_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->d_shifts, padded_shifts(p->shifts, m, d, padded_rows(m), p->tr).data(),
                       (size_t)padded_rows(m) * d * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipEventCreate(&p->ev0)) != hipSuccess || (e = hipEventCreate(&p->ev1)) != hipSuccess) {
        qmc_plan_destroy(p);
        return hip_fail(e, "plan setup");
    }
    *out = p;
    return QMC_OK;
}

void qmc_plan_destroy(qmc_plan_t p) {
    if (!p) return;
    if (p->stream) hipStreamSynchronize(p->stream);
    else hipDeviceSynchronize();
    if (p->d_g) hipFree(p->d_g);
    if (p->d_gstep) hipFree(p->d_gstep);
    if (p->d_shifts) hipFree(p->d_shifts);
    if (p->d_params) hipFree(p->d_params);
    if (p->d_partials) hipFree(p->d_partials);
    if (p->d_out) hipFree(p->d_out);
    if (p->h_out) hipHostFree(p->h_out);
    if (p->ev0) hipEventDestroy(p->ev0);
    if (p->ev1) hipEventDestroy(p->ev1);
    plan_release_extra(p);
    delete p;
}

qmc_status qmc_plan_set_stream(qmc_plan_t p, void *stream) {
    if (!p) return fail(QMC_EINVAL, "plan is NULL");
    p->stream = (hipStream_t)stream;
    return QMC_OK;
}

qmc_status qmc_plan_set_launch(qmc_plan_t p, const qmc_launch *cfg) {
    if (!p) return fail(QMC_EINVAL, "plan is NULL");
    if (!cfg) {
        p->launch = qmc_launch{0, 0};
        return QMC_OK;
    }
    const uint32_t T = cfg->shift_tile;
    if (T != 0 && T != 1 && T != 2 && T != 4 && T != 8) return fail(QMC_EINVAL, "shift_tile must be 1, 2, 4 or 8");
    if (cfg->blocks_per_cu > 1024) return fail(QMC_EINVAL, "blocks_per_cu > 1024");
    p->launch = *cfg;
    return QMC_OK;
}

qmc_status qmc_plan_set_jit(qmc_plan_t p, int32_t mode) {
    if (!p) return fail(QMC_EINVAL, "plan is NULL");
    if (mode < 0 || mode > 2) return fail(QMC_EINVAL, "jit mode must be 0, 1 or 2");
    p->jit_mode = mode;
    return QMC_OK;
}

qmc_status qmc_plan_get_launch(qmc_plan_t p, qmc_launch *cfg, int32_t *used_jit) {
    if (!p || !cfg) return fail(QMC_EINVAL, "null argument");
    cfg->shift_tile = p->last_T;
    cfg->blocks_per_cu = p->last_bx;
    if (used_jit) *used_jit = p->last_jit ? 1 : 0;
    return QMC_OK;
}

qmc_status qmc_plan_set_timing(qmc_plan_t p, int32_t enable) {
    if (!p) return fail(QMC_EINVAL, "plan is NULL");
    p->timing = enable != 0;
    return QMC_OK;
}

qmc_status qmc_plan_kernel_time(qmc_plan_t p, double *total_ms, uint64_t *launches, int32_t reset) {
    if (!p) return fail(QMC_EINVAL, "plan is NULL");
    if (total_ms) *total_ms = p->kernel_ms;
    if (launches) *launches = p->kernel_launches;
    if (reset) {
        p->kernel_ms = 0.0;
        p->kernel_launches = 0;
    }
    return QMC_OK;
}

qmc_status qmc_integrate(qmc_plan_t p, qmc_family family, const void *params, qmc_result *out,
                         double *per_shift) {
    if (!p) return fail(QMC_EINVAL, "plan is NULL");
    if (!out) return fail(QMC_EINVAL, "out is NULL");
    Packed pk;
    qmc_status st = pack_params((int)family, p->d, params, pk);
    if (st) return st;
    if (pk.orders >= 2) return fail(QMC_EINVAL, "n_orders >= 2: use qmc_integrate_orders");
    qmc_launch L = p->launch;
    if (L.shift_tile == 0 && L.blocks_per_cu == 0) {
        const bool sector = pk.key_family == QMC_F_SECTOR || pk.key_family == kFamSectorComplex;
        qmc_launch tuned;
        if (tune_lookup(p, pk, sector && p->jit_mode != 0, tuned)) L = tuned;
    }
    if ((st = plan_enqueue(p, pk, L.shift_tile, L.blocks_per_cu))) return st;
    return plan_collect(p, pk.np, out, per_shift, pk.crossing);
}

qmc_status qmc_integrate_orders(qmc_plan_t p, qmc_family family, const void *params, qmc_result *out,
                                double *per_shift) {
    if (!p) return fail(QMC_EINVAL, "plan is NULL");
    if (!out) return fail(QMC_EINVAL, "out is NULL");
    if (family != QMC_F_SECTOR) return fail(QMC_EUNSUPPORTED, "expansion orders are built for QMC_F_SECTOR");
    Packed pk;
    qmc_status st = pack_params((int)family, p->d, params, pk);
    if (st) return st;
    const uint32_t no = pk.orders >= 2 ? pk.orders : 1u;
    if ((st = plan_enqueue(p, pk, p->launch.shift_tile, p->launch.blocks_per_cu))) return st;
    qmc_result first;
    st = plan_collect(p, pk.np, &first, per_shift, pk.crossing);
    if (st && st != QMC_ENONFINITE && st != QMC_ECONTOUR) return st;
    const double *res = p->h_out + out_res_offset(p->m);
    for (uint32_t k = 0; k < no; ++k) {
        if (pk.cplx) {  // parts (2k, 2k+1) = (Re, Im) of order k form pair k
            out[k] = qmc_result{res[4 * k], res[4 * k + 1], res[4 * k + 2], res[4 * k + 3], 1, 0, 0.0};
        } else {        // part k = order k, pairs of orders share a result block
            const uint32_t b = 4 * (k / 2), o = k % 2;
            out[k] = qmc_result{res[b + o], 0.0, res[b + 2 + o], 0.0, 0, 0, 0.0};
        }
        if (st == QMC_ENONFINITE) out[k] = qmc_result{NAN, NAN, NAN, NAN, pk.cplx ? 1 : 0, 0, 0.0};
        out[k].contour_crossed = first.contour_crossed;
    }
    return st;
}

qmc_status qmc_integrate_sum(qmc_plan_t p, uint32_t count, const qmc_sector_params *const *params, qmc_result *out,
                             double *per_shift) {
    if (!p) return fail(QMC_EINVAL, "plan is NULL");
    if (!params || !out) return fail(QMC_EINVAL, "null argument");
    if (count == 0) return fail(QMC_EINVAL, "count must be >= 1");
    if (count > kMaxSumSectors) return fail(QMC_EUNSUPPORTED, "more than %u sectors in one sum", kMaxSumSectors);
    Packed sum;
    std::vector<size_t> offs;
    for (uint32_t i = 0; i < count; ++i) {
        if (!params[i]) return fail(QMC_EINVAL, "params[%u] is NULL", i);
        Packed pk;
        qmc_status st = pack_params(QMC_F_SECTOR, p->d, params[i], pk);
        if (st) return st;
        if (pk.orders >= 2 || pk.deform)
            return fail(QMC_EUNSUPPORTED, "sums take plain sectors (n_orders < 2, deform_lambda = 0)");
        if (i == 0) {
            sum.np = pk.np;
            sum.cplx = pk.cplx;
            sum.key_family = pk.key_family;
        } else if (pk.cplx != sum.cplx) {
            return fail(QMC_EINVAL, "mixed real and complex sectors");
        }
        offs.push_back(sum.blob.size());
        sum.blob.insert(sum.blob.end(), pk.blob.begin(), pk.blob.end());
    }
    const uint32_t T = p->launch.shift_tile ? p->launch.shift_tile : 2u;
    std::string err;
    hipFunction_t jfn = jit_sum_kernel(sum.blob, offs, p->d, p->tr, T, sum.cplx, p->device, err);
    if (!jfn) return fail(QMC_EUNSUPPORTED, "specialised sum kernel: %s", err.c_str());
    qmc_status st = plan_launch(p, sum, nullptr, jfn, T, p->launch.blocks_per_cu ? p->launch.blocks_per_cu : 16);
    if (st) return st;
    return plan_collect(p, sum.np, out, per_shift);
}

qmc_status qmc_deform_check(qmc_plan_t p, const qmc_sector_params *params, double *fraction, double *per_shift) {
    if (!p) return fail(QMC_EINVAL, "plan is NULL");
    if (!fraction || !params) return fail(QMC_EINVAL, "null argument");
    if (params->deform_lambda == 0.0) return fail(QMC_EINVAL, "deform_lambda is 0");
    Packed pk;
    qmc_status st = pack_params(QMC_F_SECTOR, p->d, params, pk);
    if (st) return st;
    // the check functor: one real part, 1 where Im(F(z) - i delta) > 0
    uint64_t flags;
    std::memcpy(&flags, &pk.blob[2], sizeof flags);
    pk.blob[2] = bits(flags | kSectorDeformCheck);
    pk.np = 1;
    pk.cplx = false;
    pk.crossing = false;
    pk.orders = 0;
    if ((st = plan_enqueue(p, pk, p->launch.shift_tile, p->launch.blocks_per_cu))) return st;
    qmc_result r;
    st = plan_collect(p, 1, &r, per_shift);
    if (st) return st;
    // finalize multiplies every sum by the transform's constant
    const double scale = transform_scale(p->tr, p->d);
    *fraction = r.mean_re / scale;
    if (per_shift)
        for (uint32_t k = 0; k < p->m; ++k) per_shift[k] /= scale;
    return QMC_OK;
}

qmc_status qmc_deform_select(qmc_plan_t p, const qmc_sector_params *params, double lam_max, double shrink,
                             uint32_t count, double *lam_out, qmc_result *out) {
    if (!p) return fail(QMC_EINVAL, "plan is NULL");
    if (!params || !lam_out || !out) return fail(QMC_EINVAL, "null argument");
    if (!(lam_max > 0.0) || !std::isfinite(lam_max)) return fail(QMC_EINVAL, "lam_max must be positive and finite");
    if (!(shrink > 0.0 && shrink < 1.0)) return fail(QMC_EINVAL, "shrink must lie in (0, 1)");
    if (count == 0 || count > 64) return fail(QMC_EINVAL, "count must be 1..64");
    if (params->n_orders >= 2) return fail(QMC_EINVAL, "select lambda on the plain integrand (n_orders < 2)");
    qmc_sector_params q = *params;
    bool found = false;
    double best_err = 0.0;
    double lam = lam_max;
    for (uint32_t i = 0; i < count; ++i, lam *= shrink) {
        q.deform_lambda = lam;
        double frac;
        qmc_status st = qmc_deform_check(p, &q, &frac, nullptr);
        if (st) return st;
        if (frac > 0.0) continue;
        qmc_result r;
        st = qmc_integrate(p, QMC_F_SECTOR, &q, &r, nullptr);
        if (st == QMC_ENONFINITE || st == QMC_ECONTOUR) continue;
        if (st) return st;
        const double err = std::hypot(r.err_re, r.err_im);
        if (!found || err < best_err) {
            found = true;
            best_err = err;
            *lam_out = lam;
            *out = r;
        }
    }
    if (!found) return fail(QMC_EUNSUPPORTED, "every lambda of the ladder crosses the -i0 side or is not finite");
    return QMC_OK;
}

qmc_status qmc_math_eval(int32_t fn, uint64_t count, const double *x, double *y) {
    if (fn < 0 || fn > 3) return fail(QMC_EINVAL, "fn must be 0 (log), 1 (exp), 2 (atan2) or 3 (sincos)");
    if (count && (!x || !y)) return fail(QMC_EINVAL, "null array");
    if (count > (1ull << 28)) return fail(QMC_EINVAL, "count > 2^28");
    if (count == 0) return QMC_OK;
    const size_t nx = fn == 2 ? 2 * count : count, ny = fn == 3 ? 2 * count : count;
    DeviceScratch s;
    qmc_status st;
    if ((st = s.alloc(nx * 8)) || (st = s.alloc(ny * 8))) return st;
    hipError_t e = hipMemcpy(s.ptr[0], x, nx * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_math(fn, count, (const double *)s.ptr[0], (double *)s.ptr[1], nullptr);
    if (e == hipSuccess) e = hipMemcpy(y, s.ptr[1], ny * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "math eval");
    return QMC_OK;
}

qmc_status qmc_korobov_vector(uint64_t n, uint32_t d, uint64_t a, uint64_t *g) {
    if (!g) return fail(QMC_EINVAL, "g is NULL");
    if (n < 2 || d == 0) return fail(QMC_EINVAL, "need n >= 2 and d >= 1");
    if (n > (1ull << 32)) return fail(QMC_EUNSUPPORTED, "n > 2^32");
    uint64_t v = 1 % n;
    a %= n;
    for (uint32_t i = 0; i < d; ++i) {
        g[i] = v;
        v = (v * a) % n;
    }
    return QMC_OK;
}

qmc_status qmc_lattice_dump(qmc_plan_t p, uint64_t j_lo, uint64_t count, uint32_t *idx_out, uint64_t *sums_out) {
    if (!p) return fail(QMC_EINVAL, "plan is NULL");
    if (count && !idx_out) return fail(QMC_EINVAL, "idx_out is NULL");
    if (count > (1ull << 24)) return fail(QMC_EINVAL, "count > 2^24");
    if (j_lo + count > p->n) return fail(QMC_EINVAL, "j range beyond n");
    // same grid as the lattice kernel's default launch for a real family
    const uint32_t T = p->launch.shift_tile ? p->launch.shift_tile : 1;
    const uint32_t tiles = (p->m + T - 1) / T;
    const uint32_t bx = grid_x(p->n, tiles, p->device, p->launch.blocks_per_cu);
    qmc_status st = plan_set_gstep(p, bx * kBlock);
    if (st) return st;
    uint32_t *d_idx = nullptr;
    unsigned long long *d_sums = nullptr;
    hipError_t e;
    if ((e = hipMalloc(&d_sums, 2 * p->d * sizeof(unsigned long long))) != hipSuccess)
        return fail(QMC_ENOMEM, "hipMalloc sums");
    if (count && (e = hipMalloc(&d_idx, count * p->d * sizeof(uint32_t))) != hipSuccess) {
        hipFree(d_sums);
        return fail(QMC_ENOMEM, "hipMalloc idx");
    }
    e = hipMemsetAsync(d_sums, 0, 2 * p->d * sizeof(unsigned long long), p->stream);
    DumpArgs a{};
    a.n = p->n;
    a.d = p->d;
    a.inv_n = p->inv_n;
    a.g = p->d_g;
    a.gstep = p->d_gstep;
    a.j_lo = j_lo;
    a.j_hi = j_lo + count;
    a.idx_out = d_idx;
    a.sums = d_sums;
    if (e == hipSuccess) e = launch_dump(a, bx, p->stream);
    if (e == hipSuccess && count)
        e = hipMemcpyAsync(idx_out, d_idx, count * p->d * sizeof(uint32_t), hipMemcpyDeviceToHost, p->stream);
    std::vector<unsigned long long> sums(2 * p->d);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sums.data(), d_sums, 2 * p->d * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    hipFree(d_sums);
    if (d_idx) hipFree(d_idx);
    if (e != hipSuccess) return hip_fail(e, "lattice dump");
    if (sums_out)
        for (uint32_t i = 0; i < 2 * p->d; ++i) sums_out[i] = sums[i];
    return QMC_OK;
}

qmc_status qmc_korobov_search(uint64_t n, uint32_t d, const uint64_t *cand, uint32_t ncand, uint64_t *a_best,
                              double *p2_best, double *p2_all) {
    if (!cand || !a_best || !p2_best) return fail(QMC_EINVAL, "null argument");
    if (ncand == 0) return fail(QMC_EINVAL, "ncand must be >= 1");
    if (ncand > 4096) return fail(QMC_EUNSUPPORTED, "ncand > 4096");
    if (d == 0) return fail(QMC_EINVAL, "d must be >= 1");
    if (d > kMaxDim) return fail(QMC_EUNSUPPORTED, "d > %u", kMaxDim);
    if (n < 2) return fail(QMC_EINVAL, "n must be >= 2");
    if (n > (1ull << 31)) return fail(QMC_EUNSUPPORTED, "n > 2^31");
    for (uint32_t c = 0; c < ncand; ++c)
        if (cand[c] % n == 0) return fail(QMC_EINVAL, "candidate %u is 0 mod n", c);
    const qmc_transform tr{QMC_T_NONE, 0};
    uint32_t T = 0;
    LatticeLaunch fn = find_kernel(QMC_F_P2KERNEL, tr, d, 1, T);
    if (!fn || T != 1) return fail(QMC_EUNSUPPORTED, "no P2 kernel for d = %u", d);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    const uint32_t bx = grid_x((uint32_t)n, ncand, dev, 8);
    std::vector<uint32_t> g((size_t)ncand * d), gs((size_t)ncand * d);
    for (uint32_t c = 0; c < ncand; ++c) {
        uint64_t v = 1 % n;
        for (uint32_t i = 0; i < d; ++i) {
            g[(size_t)c * d + i] = (uint32_t)v;
            v = (v * (cand[c] % n)) % n;
        }
        gstep_for(&g[(size_t)c * d], d, (uint32_t)n, (uint64_t)bx * kBlock, &gs[(size_t)c * d]);
    }
    DeviceScratch s;
    std::vector<double> zero(d, 0.0), blob(1, 0.0);
    qmc_status st;
    if ((st = s.alloc(g.size() * 4)) || (st = s.alloc(gs.size() * 4)) || (st = s.alloc(d * 8)) ||
        (st = s.alloc(8)) || (st = s.alloc((size_t)ncand * bx * sizeof(double2))) ||
        (st = s.alloc((size_t)ncand * 8)) || (st = s.alloc((size_t)ncand * 32)))
        return st;
    hipStream_t stream = nullptr;
    if ((e = hipMemcpy(s.ptr[0], g.data(), g.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(s.ptr[1], gs.data(), gs.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(s.ptr[2], zero.data(), d * 8, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(s.ptr[3], blob.data(), 8, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "search upload");
    LatticeArgs a{};
    a.n = (uint32_t)n;
    a.d = d;
    a.m = 1;
    a.tiles = 1;
    a.inv_n = 1.0 / (double)n;
    a.g = (const uint32_t *)s.ptr[0];
    a.gstep = (const uint32_t *)s.ptr[1];
    a.shifts = (const double *)s.ptr[2];
    a.params = (const double *)s.ptr[3];
    a.g_stride = d;
    a.shift_stride = 0;
    a.param_stride = 0;
    a.np = 1;
    a.partials = (double2 *)s.ptr[4];
    // The point n - j is the mirror 1 - x of the point j and B2(1 - x) =
    // B2(x), so the sum S over all points is 2 sum_{j <= n/2} - term(0) -
    // [n even] term(n/2), term(0) = (1 + pi^2/3)^d.  For even n and odd
    // candidates every g_i is odd and the point n/2 is (1/2, ..., 1/2) for
    // all of them; an even candidate puts 0 in some coordinates there, and
    // then all n points are summed.  Both terms are formed as the kernel
    // forms them (q(0) is exactly the constant; x = (n/2) / n through 1/n),
    // multiplied up in order.
    bool half = true;
    if ((n & 1) == 0)
        for (uint32_t c = 0; c < ncand; ++c) half = half && (cand[c] % n) % 2 == 1;
    double t0 = 0.0;
    if (half) {
        const double c2 = 2.0 * 9.869604401089358, c0 = 1.0 + 9.869604401089358 / 3.0;
        double th = 1.0;
        if ((n & 1) == 0) {
            const double x = (double)(n / 2) * (1.0 / (double)n);
            const double q = std::fma(std::fma(c2, x, -c2), x, c0);
            th = q;
            for (uint32_t i = 1; i < d; ++i) th *= q;
        }
        t0 = c0;
        for (uint32_t i = 1; i < d; ++i) t0 *= c0;
        if ((n & 1) == 0) t0 += th;  // both self-mirrored terms
    }
    a.jend = half ? (uint32_t)(n / 2 + 1) : 0;
    if ((e = fn(a, dim3(bx, ncand), stream)) != hipSuccess) return hip_fail(e, "launch P2 kernel");
    FinalizeArgs f{};
    f.partials = a.partials;
    f.nblk = bx;
    f.m = 1;
    f.np = 1;
    f.n = (double)n;
    // q = (S - n) / n = ((sum - (n + t0) / 2) 2) / n, t0 the self-mirrored terms
    f.scale = half ? 2.0 : 1.0;
    f.sub = half ? ((double)n + t0) / 2.0 : (double)n;
    f.q = (double *)s.ptr[5];
    f.res = (double *)s.ptr[6];
    if ((e = launch_finalize(f, ncand, stream)) != hipSuccess) return hip_fail(e, "launch finalize");
    std::vector<double> p2(ncand);
    if ((e = hipMemcpy(p2.data(), s.ptr[5], ncand * 8, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "search download");
    uint64_t best_a = 0;
    double best = INFINITY;
    for (uint32_t c = 0; c < ncand; ++c) {
        if (p2_all) p2_all[c] = p2[c];
        if (p2[c] < best || (p2[c] == best && cand[c] < best_a)) {
            best = p2[c];
            best_a = cand[c];
        }
    }
    if (!std::isfinite(best)) return fail(QMC_ENONFINITE, "P2 not finite");
    *a_best = best_a;
    *p2_best = best;
    return QMC_OK;
}

}  // extern "C"
