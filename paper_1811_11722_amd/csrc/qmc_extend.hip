// Embedded (extensible) rank-1 lattices in base 2.
//
// With n = 2^k and a generating vector g taken mod 2^K (K >= k), the lattice
// of 2n points contains the lattice of n points: its even points j = 2j' are
// {j' g / n}, and its odd points are {j' g / n + g / (2n)}, the n-point
// lattice again with every shift moved by g / (2n) (g read mod 2n).  A ladder
// n, 2n, 4n, ... therefore evaluates each point once: every rung integrates
// one n-point lattice with moved shifts and averages its per-shift sums with
// the previous rung's.  This module holds the two host-side pieces: the
// search for a Korobov parameter that is good on every rung, and the merge
// of two half-lattice estimates into eq. (2)-(3)'s mean and error.
#include <cmath>
#include <vector>

#include "qmc_runtime.hpp"

using namespace qmc;

extern "C" qmc_status qmc_korobov_search_extensible(uint32_t kmin, uint32_t kmax, uint32_t d, const uint64_t *cand,
                                                    uint32_t ncand, uint64_t *a_best, double *score,
                                                    double *p2_levels) {
    if (!cand || !a_best || !score) return fail(QMC_EINVAL, "null argument");
    if (kmin < 1 || kmin > kmax) return fail(QMC_EINVAL, "need 1 <= kmin <= kmax");
    if (kmax > 31) return fail(QMC_EUNSUPPORTED, "kmax > 31");
    if (ncand == 0) return fail(QMC_EINVAL, "ncand must be >= 1");
    for (uint32_t c = 0; c < ncand; ++c)
        if ((cand[c] & 1u) == 0) return fail(QMC_EINVAL, "candidate %u is even (not a unit mod 2^k)", c);
    const uint32_t levels = kmax - kmin + 1;
    std::vector<double> logsum(ncand, 0.0), all(ncand), p2s((size_t)levels * ncand);
    for (uint32_t k = kmin; k <= kmax; ++k) {
        const uint64_t n = 1ull << k;
        uint64_t a;
        double p2;
        qmc_status st = qmc_korobov_search(n, d, cand, ncand, &a, &p2, all.data());
        if (st) return st;
        for (uint32_t c = 0; c < ncand; ++c) {
            p2s[(size_t)(k - kmin) * ncand + c] = all[c];
            // P2 > 0 for every lattice; a rounding to <= 0 counts as perfect
            logsum[c] += std::log(std::max(all[c], 1e-300));
        }
    }
    uint32_t best = 0;
    for (uint32_t c = 1; c < ncand; ++c)
        if (logsum[c] < logsum[best] || (logsum[c] == logsum[best] && cand[c] < cand[best])) best = c;
    *a_best = cand[best];
    *score = logsum[best] / levels;
    if (p2_levels)
        for (uint32_t l = 0; l < levels; ++l) p2_levels[l] = p2s[(size_t)l * ncand + best];
    return QMC_OK;
}

extern "C" qmc_status qmc_lattice_moved_shifts(uint64_t n2, uint32_t d, const uint64_t *g, uint32_t m,
                                              const double *shifts, double *out) {
    if (!g || !shifts || !out) return fail(QMC_EINVAL, "null argument");
    if (n2 < 2 || (n2 & (n2 - 1))) return fail(QMC_EINVAL, "n2 must be a power of two >= 2");
    if (n2 > (1ull << 32)) return fail(QMC_EUNSUPPORTED, "n2 > 2^32");
    if (d == 0 || d > kMaxDim) return fail(d ? QMC_EUNSUPPORTED : QMC_EINVAL, "d = %u outside 1..%u", d, kMaxDim);
    for (size_t i = 0; i < (size_t)m * d; ++i)
        if (!(shifts[i] >= 0.0 && shifts[i] < 1.0)) return fail(QMC_EINVAL, "shift %zu outside [0,1)", i);
    // (g_i mod n2) / n2 is exact (n2 a power of two, g_i mod n2 < 2^32);
    // the sum is rounded once, and a sum in [1, 2) wraps by an exact
    // subtraction
    const double inv = 1.0 / (double)n2;
    for (uint32_t k = 0; k < m; ++k)
        for (uint32_t i = 0; i < d; ++i) {
            double v = shifts[(size_t)k * d + i] + (double)(g[i] & (n2 - 1)) * inv;
            if (v >= 1.0) v -= 1.0;
            out[(size_t)k * d + i] = v;
        }
    return QMC_OK;
}

extern "C" qmc_status qmc_lattice_merge(uint32_t m, uint32_t np, const double *q_a, const double *q_b, double *q_out,
                                        qmc_result *out) {
    if (!q_a || !q_b || !q_out || !out) return fail(QMC_EINVAL, "null argument");
    if (m < 2) return fail(QMC_EINVAL, "m must be >= 2");
    if (np != 1 && np != 2) return fail(QMC_EINVAL, "np must be 1 (real) or 2 (complex)");
    const size_t nq = (size_t)m * np;
    bool finite = true;
    for (size_t i = 0; i < nq; ++i) {
        q_out[i] = 0.5 * q_a[i] + 0.5 * q_b[i];
        finite = finite && std::isfinite(q_out[i]);
    }
    out->is_complex = np == 2;
    out->used_cv = 0;
    out->contour_crossed = 0.0;
    if (!finite) {
        out->mean_re = out->mean_im = out->err_re = out->err_im = NAN;
        return fail(QMC_ENONFINITE, "a per-shift sum is not finite");
    }
    double mean[2] = {0.0, 0.0}, err[2] = {0.0, 0.0};
    for (uint32_t p = 0; p < np; ++p) {
        // two passes with long double accumulation (m values)
        long double s = 0.0L;
        for (uint32_t k = 0; k < m; ++k) s += q_out[(size_t)k * np + p];
        const double mu = (double)(s / m);
        long double v = 0.0L;
        for (uint32_t k = 0; k < m; ++k) {
            const long double t = (long double)q_out[(size_t)k * np + p] - mu;
            v += t * t;
        }
        mean[p] = mu;
        err[p] = std::sqrt((double)(v / ((long double)m * (m - 1))));
    }
    out->mean_re = mean[0];
    out->mean_im = np == 2 ? mean[1] : 0.0;
    out->err_re = err[0];
    out->err_im = np == 2 ? err[1] : 0.0;
    return QMC_OK;
}
