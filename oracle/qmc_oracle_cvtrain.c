/*
 * CPU ORACLE, control-variate training: the steps of one alternating
 * least-squares update of the separable Legendre model.
 *
 * TEST INFRASTRUCTURE ONLY (like qmc_oracle.c, built into the same
 * library): only the tests, the smoke check and the benchmark's CPU leg load
 * it.  It shares no source, header or helper with the GPU library.
 *
 * The control variate is not part of arXiv:1811.11722; it is the learned
 * model g(z) = sum_r c_r prod_i sum_k W[r,i,k] P~_k(z_i) on orthonormal
 * shifted Legendre polynomials that the estimator subtracts.  Training fits
 * W to samples (z_j, sw_j, y_j) of the integrand, y_j = fhat_j / scale and
 * sw_j the transform's Jacobian, by minimising
 *     J(W) = sum_j (y_j - sw_j g(z_j))^2 + lam |W[., i, .]|^2
 * over one dimension i at a time (c_r = 1 during the fit).  With every
 * other dimension fixed the model is linear in the R*K numbers W[r,i,k]:
 *     sw_j g(z_j) = sum_{r,k} rho_j[r] phi_j[k] W[r,i,k],
 *     rho_j[r] = sw_j prod_{i' != i} h_{r,i'}(z_{j,i'}),   phi_j[k] = P~_k(z_{j,i}),
 * so the step solves the ridge normal equations (A^T A + lam I) w = A^T y of
 * the design matrix A_j[u] = rho_j[r] phi_j[k], u = r K + k.
 *
 * Routines (each the plain definition, written out):
 *   or_bf16          rounding of a float to bfloat16 (nearest, ties to even)
 *   or_cv_features   rho, phi in double, and the envelope
 *                    sw_j prod_{i' != i} sum_k |W[r,i',k]| sqrt(2k+1) >= |rho_j[r]|
 *   or_cv_normal     the normal equations the GPU assembles from double
 *                    rho, phi, y: the matrix of the bfloat16 design matrix
 *                    a~_j[u] = bf16(fl32(rho) fl32(phi)) (product in single
 *                    precision) and the right-hand side sum_j (rho phi) y_j,
 *                    summed in long double; plus the sums of absolute values
 *                    (envelopes of the accumulation error); rows split over
 *                    threads only
 *   or_cv_normal_at  sampled entries of the same matrix and right-hand side
 *   or_cv_solve      (G + lam I) x = b by an unblocked Cholesky factorisation
 *                    in double, lam = ridge * trace(G) / F, escalated 100x on
 *                    a non-positive pivot (at most three times)
 *   or_cv_step       one exact ridge step in double: design matrix from
 *                    or_cv_features, normal equations in long double,
 *                    or_cv_solve; returns W with W[., i, .] replaced
 *   or_cv_objective  J(W) for dimension i (ridge term included) and
 *                    sum_j y_j^2
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_CV_MAXK 32
#define OR_CV_MAXD 64

/* Legendre P~_k(x) = sqrt(2k+1) P_k(2x - 1) from qmc_oracle.c */
void or_legendre(uint32_t K, double x, double *out);

float or_bf16(float x)
{
    uint32_t b;
    memcpy(&b, &x, 4);
    if ((b & 0x7f800000u) == 0x7f800000u) {
        if (b & 0x007fffffu)
            b |= 0x00400000u; /* NaN stays a (quiet) NaN */
        b &= 0xffff0000u;
    } else {
        /* add just under half a bfloat16 unit, plus one when the kept
           mantissa is odd, then truncate: round to nearest, ties to even */
        b += 0x7fffu + ((b >> 16) & 1u);
        b &= 0xffff0000u;
    }
    memcpy(&x, &b, 4);
    return x;
}

int or_cv_features(uint32_t n, uint32_t d, uint32_t R, uint32_t K, uint32_t i, const float *z,
                   const float *sw, const double *W, double *rho, double *phi, double *env)
{
    if (d == 0 || d > OR_CV_MAXD || K == 0 || K > OR_CV_MAXK || R == 0 || i >= d)
        return 1;
    double leg[OR_CV_MAXK];
    for (uint32_t j = 0; j < n; ++j) {
        for (uint32_t r = 0; r < R; ++r) {
            rho[(size_t)j * R + r] = (double)sw[j];
            env[(size_t)j * R + r] = fabs((double)sw[j]);
        }
        for (uint32_t ii = 0; ii < d; ++ii) {
            or_legendre(K, (double)z[(size_t)j * d + ii], leg);
            if (ii == i) {
                for (uint32_t k = 0; k < K; ++k)
                    phi[(size_t)j * K + k] = leg[k];
                continue;
            }
            for (uint32_t r = 0; r < R; ++r) {
                double h = 0.0, e = 0.0;
                for (uint32_t k = 0; k < K; ++k) {
                    const double w = W[((size_t)r * d + ii) * K + k];
                    h += w * leg[k];
                    e += fabs(w) * sqrt(2.0 * k + 1.0);
                }
                rho[(size_t)j * R + r] *= h;
                env[(size_t)j * R + r] *= e;
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
typedef struct {
    uint32_t n, R, K, F;
    const double *rho, *phi, *y;
    int exact; /* 1: the matrix of the double design matrix (no bfloat16) */
    double *gram, *rhs, *gram_abs, *rhs_abs;
    uint32_t next;
    pthread_mutex_t lock;
} or_cvn_job;

/* Feature u of point j: a16 = bf16(fl32(rho) fl32(phi)) for the matrix (in
   exact mode rho phi in double), a64 = rho phi for the right-hand side. */
static void or_cv_feat(const or_cvn_job *jb, uint32_t j, uint32_t u, double *a16, double *a64)
{
    const uint32_t r = u / jb->K, k = u % jb->K;
    const double rv = jb->rho[(size_t)j * jb->R + r], pv = jb->phi[(size_t)j * jb->K + k];
    *a64 = rv * pv;
    if (jb->exact) {
        *a16 = *a64;
        return;
    }
    const float f = (float)rv * (float)pv; /* fl32 of the single-precision factors */
    *a16 = (double)or_bf16(f);
}

static void or_cvn_row(or_cvn_job *jb, uint32_t u)
{
    const uint32_t F = jb->F;
    long double *g = (long double *)calloc((size_t)u + 1, sizeof(long double));
    long double *ga = (long double *)calloc((size_t)u + 1, sizeof(long double));
    long double b = 0.0L, ba = 0.0L;
    for (uint32_t j = 0; j < jb->n; ++j) {
        double au16, au64;
        or_cv_feat(jb, j, u, &au16, &au64);
        const long double yj = (long double)jb->y[j];
        b += (long double)au64 * yj;
        ba += fabsl((long double)au64 * yj);
        for (uint32_t v = 0; v <= u; ++v) {
            double av16, av64;
            or_cv_feat(jb, j, v, &av16, &av64);
            /* GPU mode: exact, 8-bit by 8-bit significands */
            const long double p = (long double)au16 * (long double)av16;
            g[v] += p;
            ga[v] += fabsl(p);
        }
    }
    for (uint32_t v = 0; v <= u; ++v) {
        jb->gram[(size_t)u * F + v] = jb->gram[(size_t)v * F + u] = (double)g[v];
        jb->gram_abs[(size_t)u * F + v] = jb->gram_abs[(size_t)v * F + u] = (double)ga[v];
    }
    jb->rhs[u] = (double)b;
    jb->rhs_abs[u] = (double)ba;
    free(g);
    free(ga);
}

static void *or_cvn_worker(void *arg)
{
    or_cvn_job *jb = (or_cvn_job *)arg;
    for (;;) {
        pthread_mutex_lock(&jb->lock);
        uint32_t u = jb->next++;
        pthread_mutex_unlock(&jb->lock);
        if (u >= jb->F)
            break;
        or_cvn_row(jb, u);
    }
    return NULL;
}

static void or_cvn_run(or_cvn_job *jb, int32_t nthreads)
{
    jb->next = 0;
    pthread_mutex_init(&jb->lock, NULL);
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    pthread_t th[256];
    for (int t = 1; t < nthreads; ++t)
        pthread_create(&th[t], NULL, or_cvn_worker, jb);
    or_cvn_worker(jb);
    for (int t = 1; t < nthreads; ++t)
        pthread_join(th[t], NULL);
    pthread_mutex_destroy(&jb->lock);
}

int or_cv_normal(uint32_t n, uint32_t R, uint32_t K, const double *rho, const double *phi,
                 const double *y, int32_t nthreads, double *gram, double *rhs, double *gram_abs,
                 double *rhs_abs)
{
    if (R == 0 || K == 0 || K > OR_CV_MAXK)
        return 1;
    or_cvn_job jb;
    memset(&jb, 0, sizeof jb);
    jb.n = n;
    jb.R = R;
    jb.K = K;
    jb.F = R * K;
    jb.rho = rho;
    jb.phi = phi;
    jb.y = y;
    jb.gram = gram;
    jb.rhs = rhs;
    jb.gram_abs = gram_abs;
    jb.rhs_abs = rhs_abs;
    or_cvn_run(&jb, nthreads);
    return 0;
}

/* entries (us[t], vs[t]) of the matrix and rhs[us[t]], with envelopes */
int or_cv_normal_at(uint32_t n, uint32_t R, uint32_t K, const double *rho, const double *phi,
                    const double *y, uint32_t count, const uint32_t *us, const uint32_t *vs,
                    double *gram, double *gram_abs, double *rhs, double *rhs_abs)
{
    if (R == 0 || K == 0 || K > OR_CV_MAXK)
        return 1;
    or_cvn_job jb;
    memset(&jb, 0, sizeof jb);
    jb.n = n;
    jb.R = R;
    jb.K = K;
    jb.F = R * K;
    jb.rho = rho;
    jb.phi = phi;
    jb.y = y;
    for (uint32_t t = 0; t < count; ++t) {
        if (us[t] >= jb.F || vs[t] >= jb.F)
            return 1;
        long double g = 0.0L, ga = 0.0L, b = 0.0L, ba = 0.0L;
        for (uint32_t j = 0; j < n; ++j) {
            double au16, au64, av16, av64;
            or_cv_feat(&jb, j, us[t], &au16, &au64);
            or_cv_feat(&jb, j, vs[t], &av16, &av64);
            g += (long double)au16 * (long double)av16;
            ga += fabsl((long double)au16 * (long double)av16);
            b += (long double)au64 * (long double)y[j];
            ba += fabsl((long double)au64 * (long double)y[j]);
        }
        gram[t] = (double)g;
        gram_abs[t] = (double)ga;
        rhs[t] = (double)b;
        rhs_abs[t] = (double)ba;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* (G + lam I) x = b, G symmetric F x F row-major.  Returns the number of
   escalations of the ridge (0..3), or -1 if the matrix stays indefinite. */
int or_cv_solve(uint32_t F, const double *G, const double *b, double ridge, double *lam_out,
                double *x)
{
    double *L = (double *)malloc((size_t)F * F * sizeof(double));
    double tr = 0.0;
    for (uint32_t u = 0; u < F; ++u)
        tr += G[(size_t)u * F + u];
    double rel = ridge;
    int esc;
    for (esc = 0; esc < 4; ++esc, rel *= 100.0) {
        const double lam = rel * tr / F + 1e-300;
        *lam_out = lam;
        int ok = 1;
        /* L L^T = G + lam I, column by column */
        for (uint32_t c = 0; c < F && ok; ++c) {
            double s = G[(size_t)c * F + c] + lam;
            for (uint32_t q = 0; q < c; ++q)
                s -= L[(size_t)c * F + q] * L[(size_t)c * F + q];
            if (!(s > 0.0)) {
                ok = 0;
                break;
            }
            const double dcc = sqrt(s);
            L[(size_t)c * F + c] = dcc;
            for (uint32_t r = c + 1; r < F; ++r) {
                double t = G[(size_t)r * F + c];
                for (uint32_t q = 0; q < c; ++q)
                    t -= L[(size_t)r * F + q] * L[(size_t)c * F + q];
                L[(size_t)r * F + c] = t / dcc;
            }
        }
        if (!ok)
            continue;
        /* L z = b, then L^T x = z */
        for (uint32_t u = 0; u < F; ++u) {
            double t = b[u];
            for (uint32_t q = 0; q < u; ++q)
                t -= L[(size_t)u * F + q] * x[q];
            x[u] = t / L[(size_t)u * F + u];
        }
        for (uint32_t u = F; u-- > 0;) {
            double t = x[u];
            for (uint32_t q = u + 1; q < F; ++q)
                t -= L[(size_t)q * F + u] * x[q];
            x[u] = t / L[(size_t)u * F + u];
        }
        free(L);
        return esc;
    }
    free(L);
    return -1;
}

/* ---------------------------------------------------------------------- */
int or_cv_step(uint32_t n, uint32_t d, uint32_t R, uint32_t K, uint32_t i, const float *z,
               const float *sw, const double *y, const double *W_in, double ridge, int32_t nthreads,
               double *W_out, double *lam_out)
{
    if (d == 0 || d > OR_CV_MAXD || K == 0 || K > OR_CV_MAXK || R == 0 || i >= d)
        return 1;
    const uint32_t F = R * K;
    double *rho = (double *)malloc((size_t)n * R * sizeof(double));
    double *phi = (double *)malloc((size_t)n * K * sizeof(double));
    double *env = (double *)malloc((size_t)n * R * sizeof(double));
    double *G = (double *)malloc((size_t)F * F * sizeof(double));
    double *Ga = (double *)malloc((size_t)F * F * sizeof(double));
    double *b = (double *)malloc(F * sizeof(double));
    double *ba = (double *)malloc(F * sizeof(double));
    double *x = (double *)malloc(F * sizeof(double));
    or_cv_features(n, d, R, K, i, z, sw, W_in, rho, phi, env);
    or_cvn_job jb;
    memset(&jb, 0, sizeof jb);
    jb.n = n;
    jb.R = R;
    jb.K = K;
    jb.F = F;
    jb.rho = rho;
    jb.phi = phi;
    jb.y = y;
    jb.exact = 1;
    jb.gram = G;
    jb.rhs = b;
    jb.gram_abs = Ga;
    jb.rhs_abs = ba;
    or_cvn_run(&jb, nthreads);
    const int esc = or_cv_solve(F, G, b, ridge, lam_out, x);
    memcpy(W_out, W_in, (size_t)R * d * K * sizeof(double));
    if (esc >= 0)
        for (uint32_t r = 0; r < R; ++r)
            for (uint32_t k = 0; k < K; ++k)
                W_out[((size_t)r * d + i) * K + k] = x[r * K + k];
    free(rho);
    free(phi);
    free(env);
    free(G);
    free(Ga);
    free(b);
    free(ba);
    free(x);
    return esc < 0 ? 2 : 0;
}

int or_cv_objective(uint32_t n, uint32_t d, uint32_t R, uint32_t K, uint32_t i, const float *z,
                    const float *sw, const double *y, const double *W, double lam, double *J,
                    double *sy2)
{
    if (d == 0 || d > OR_CV_MAXD || K == 0 || K > OR_CV_MAXK || R == 0 || i >= d)
        return 1;
    double *rho = (double *)malloc((size_t)n * R * sizeof(double));
    double *phi = (double *)malloc((size_t)n * K * sizeof(double));
    double *env = (double *)malloc((size_t)n * R * sizeof(double));
    or_cv_features(n, d, R, K, i, z, sw, W, rho, phi, env);
    long double e2 = 0.0L, y2 = 0.0L;
    for (uint32_t j = 0; j < n; ++j) {
        long double g = 0.0L;
        for (uint32_t r = 0; r < R; ++r)
            for (uint32_t k = 0; k < K; ++k)
                g += (long double)rho[(size_t)j * R + r] * (long double)phi[(size_t)j * K + k] *
                     (long double)W[((size_t)r * d + i) * K + k];
        const long double e = (long double)y[j] - g;
        e2 += e * e;
        y2 += (long double)y[j] * (long double)y[j];
    }
    long double w2 = 0.0L;
    for (uint32_t r = 0; r < R; ++r)
        for (uint32_t k = 0; k < K; ++k) {
            const long double w = W[((size_t)r * d + i) * K + k];
            w2 += w * w;
        }
    *J = (double)(e2 + (long double)lam * w2);
    *sy2 = (double)y2;
    free(rho);
    free(phi);
    free(env);
    return 0;
}
