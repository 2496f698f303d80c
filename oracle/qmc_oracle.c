/*
 * CPU ORACLE for the randomly shifted rank-1 lattice estimator.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  It shares no
 * source, header, table or helper with the GPU library: it is the estimator
 * written out from its definition, slowly and plainly, so that the GPU
 * results can be compared against it.
 *
 * What it computes (arXiv:1811.11722, Sec. 2):
 *   eq. (2):  Q_k = (1/n) sum_{j=1..n} fhat( {(j-1) g / n + Delta_k} ),
 *             Qbar = (1/m) sum_k Q_k
 *   eq. (3):  sigma^2 = sum_k (Q_k - Qbar)^2 / (m (m - 1))
 *   eq. (4):  Korobov transform z(x) = int_0^x w, w(u) = u^a (1-u)^a / B
 *   eq. (5):  baker's transform z(x) = 1 - |2x - 1|
 *   Sidi's sin^m transform, z(x) = int_0^x sin^m(pi u) du / int_0^1 sin^m
 *             (one of the other periodising substitutions Sec. 2 refers to)
 *   Sec. 3:   contour deformation of a sector, z = x - i lambda x (1 - x) grad F,
 *             integrand f(z) det(dz/dx) (determinant by LU with partial
 *             pivoting), and the sign-check indicator of Im(F(z) - i delta) > 0
 *   generating vectors: P2 of a rank-1 lattice, the Korobov search and the
 *             component-by-component construction for product weights
 *
 * Pins (tests/test_oracle_pins.py) tie every function to closed forms,
 * quadrature, brute force or identities; none is unpinned.
 *   fhat(x) = f(z(x)) * prod_i z_i'(x_i)   (substitution x -> z(x), Sec. 2)
 *
 * Readings taken where the paper is silent (each also listed in the design
 * notes):
 *   - the shift index runs over k = 1..m (the text's upper limit n is a typo);
 *   - points are numbered j' = j - 1 = 0..n-1, the index (j' g_i) mod n is an
 *     exact integer, the coordinate is idx/n + Delta rounded to double, and
 *     {.} subtracts 1 when that sum is >= 1;
 *   - the baker's transform is 2-to-1 with |z'| = 2, so its integrand weight is
 *     1 (the constant is integrated exactly, Sec. 2, Fig. 3 discussion);
 *   - complex integrands carry separate variances for the real and imaginary
 *     parts;
 *   - sums over points are accumulated in long double with Neumaier's
 *     compensation; the integrand itself is evaluated in double with libm.
 *
 * Threads split each shift's points into NCHUNK fixed chunks; chunk partials
 * are merged in chunk order, so results do not depend on the thread count.
 */
#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_NCHUNK 256

/* family codes used by this oracle */
enum {
    OR_F_CONST = 0,
    OR_F_TRIG = 1,
    OR_F_P2KERNEL = 2,
    OR_F_GENZ_PRODUCT_PEAK = 3,
    OR_F_GENZ_OSCILLATORY = 4,
    OR_F_GENZ_GAUSSIAN = 5,
    OR_F_GENZ_CONTINUOUS = 6,
    OR_F_GENZ_CORNER_PEAK = 7,
    OR_F_SECTOR = 8
};

/* transform codes used by this oracle */
enum { OR_T_NONE = 0, OR_T_KOROBOV = 1, OR_T_BAKER = 2, OR_T_SIDI = 3 };

typedef struct {
    int32_t family;
    /* CONST */
    double c;
    /* TRIG: f = c0 + sum_t ch[t] cos(2 pi h_t . z + phi_t), h row-major (n_terms, d) */
    uint32_t n_terms;
    double c0;
    const int64_t *h;
    const double *ch;
    const double *phi;
    /* GENZ */
    const double *a;
    const double *u;
    /* SECTOR: prod z^nu * U^pow_u * (F - i delta)^pow_f */
    uint32_t n_u, n_f;
    const double *coef_u;
    const uint8_t *exp_u; /* (n_u, d) */
    const double *coef_f;
    const uint8_t *exp_f; /* (n_f, d) */
    const uint8_t *nu;    /* d */
    double pow_u, pow_f, delta_im;
    int32_t is_complex;
    /* control variate: when cv_w != NULL the integrand becomes f - g with
       g(z) = sum_r c_r prod_i sum_k W[r,i,k] P~_k(z_i), W row-major (R, d, K);
       for a complex integrand cv_w / cv_c model the real part and
       cv_w_im / cv_c_im (same shape) the imaginary part */
    const double *cv_w;
    const double *cv_c;
    uint32_t cv_r, cv_k;
    const double *cv_w_im;
    const double *cv_c_im;
    /* expansion in a regulator e: with eps_order = k >= 1 the sector
       integrand is replaced by its coefficient of e^k when the exponents are
       pow_u + eps_u e and pow_f + eps_f e, namely f L^k / k! with
       L = eps_u ln U + eps_f ln(F - i delta) (principal branch) */
    double eps_u, eps_f;
    int32_t eps_order;
    /* contour deformation of the sector variables (lambda != 0):
       z_k = x_k - i lambda x_k (1 - x_k) dF/dx_k(x), the integrand becomes
       f(z) det(dz/dx) and is complex; delta_im applies when is_complex */
    double deform_lambda;
    /* with deform_check != 0 a deformed sector returns 1 where the deformed
       F - i delta has a positive imaginary part (the contour crosses to the
       wrong side of the -i0 prescription) and 0 elsewhere, unweighted */
    int32_t deform_check;
    /* coordinate rounding: 0 -> idx / n (IEEE division), 1 -> idx * (1/n) */
    int32_t point_mode;
    /* precise != 0: a plain (undeformed) sector is evaluated in long double
       (U, F, the monomials, the powers and logarithms), so that the
       reference's own rounding stays far below double precision even where
       the terms of a mixed-sign F cancel */
    int32_t precise;
} or_params;

/* ------------------------------------------------------------------ */
/* Lattice index and point, eq. (2)                                     */
/* ------------------------------------------------------------------ */
uint64_t or_lattice_index(uint64_t j, uint64_t gi, uint64_t n)
{
    unsigned __int128 p = (unsigned __int128)j * (unsigned __int128)gi;
    return (uint64_t)(p % n);
}

void or_lattice_indices(uint32_t d, uint64_t n, const uint64_t *g, const uint64_t *js,
                        uint64_t count, uint64_t *out)
{
    for (uint64_t t = 0; t < count; ++t)
        for (uint32_t i = 0; i < d; ++i)
            out[t * d + i] = or_lattice_index(js[t], g[i], n);
}

static double or_coord(uint64_t idx, uint64_t n, double shift, int mode)
{
    double y = (mode == 1) ? (double)idx * (1.0 / (double)n) : (double)idx / (double)n;
    double x = y + shift;
    if (x >= 1.0)
        x -= 1.0;
    return x;
}

void or_point(uint32_t d, uint64_t n, const uint64_t *g, uint64_t j, const double *shift,
              int32_t mode, double *x)
{
    for (uint32_t i = 0; i < d; ++i)
        x[i] = or_coord(or_lattice_index(j, g[i], n), n, shift[i], mode);
}

/* ------------------------------------------------------------------ */
/* Periodising transforms, eqs. (4) and (5)                             */
/* ------------------------------------------------------------------ */
static long double or_binom(int n, int k)
{
    long double r = 1.0L;
    for (int t = 1; t <= k; ++t)
        r = r * (long double)(n - k + t) / (long double)t;
    return r;
}

/* z(x) for the Korobov weight alpha: the integral of u^a (1-u)^a from 0 to x,
   divided by its value at x = 1.  Repeated integration by parts turns it into
   the binomial tail sum_{k=a+1}^{2a+1} C(2a+1,k) x^k (1-x)^(2a+1-k), which is
   what is evaluated here.  w(x) = x^a (1-x)^a / B(a+1, a+1). */
void or_transform(int32_t kind, int32_t alpha, double x, double *z, double *w)
{
    if (kind == OR_T_KOROBOV) {
        int a = alpha, nn = 2 * alpha + 1;
        long double xl = x, yl = 1.0L - (long double)x, s = 0.0L;
        for (int k = a + 1; k <= nn; ++k)
            s += or_binom(nn, k) * powl(xl, k) * powl(yl, nn - k);
        /* B(a+1, a+1) = a! a! / (2a+1)! */
        long double beta = 1.0L;
        for (int t = 1; t <= a; ++t)
            beta *= (long double)t;
        beta = beta * beta;
        for (int t = 1; t <= nn; ++t)
            beta /= (long double)t;
        *z = (double)s;
        *w = (double)(powl(xl, a) * powl(yl, a) / beta);
    } else if (kind == OR_T_BAKER) {
        *z = 1.0 - fabs(2.0 * x - 1.0);
        *w = 1.0;
    } else if (kind == OR_T_SIDI) {
        /* Sidi's sin^m transform (one of the periodising substitutions the
           paper refers to in Sec. 2): w(u) = sin^m(pi u) / T_m, T_m the
           integral of sin^m over [0, 1], z(x) = int_0^x w.  Antiderivatives:
           m = 2p:   int_0^x sin^2p(pi t) dt = binom(2p, p) x / 4^p
                     + sum_{k=1..p} (-1)^k binom(2p, p-k) sin(2 k pi x) / (4^p k pi)
           m = 2p+1: substitute u = cos(pi t): (1/pi) [P(1) - P(cos pi x)],
                     P(u) = sum_{k=0..p} binom(p, k) (-1)^k u^(2k+1) / (2k+1). */
        const int m = alpha;
        const long double pi = 3.141592653589793238462643383279502884L;
        const long double xl = x;
        long double theta, total;
        if (m % 2 == 0) {
            const int p = m / 2;
            long double four_p = powl(4.0L, p);
            theta = or_binom(2 * p, p) * xl / four_p;
            for (int k = 1; k <= p; ++k)
                theta += ((k % 2) ? -1.0L : 1.0L) * or_binom(2 * p, p - k) * sinl(2.0L * k * pi * xl) /
                         (four_p * k * pi);
            total = or_binom(2 * p, p) / four_p;
        } else {
            const int p = (m - 1) / 2;
            long double P1 = 0.0L, Pc = 0.0L, c = cosl(pi * xl);
            for (int k = 0; k <= p; ++k) {
                const long double t = or_binom(p, k) * ((k % 2) ? -1.0L : 1.0L) / (2 * k + 1);
                P1 += t;
                Pc += t * powl(c, 2 * k + 1);
            }
            theta = (P1 - Pc) / pi;
            total = 2.0L * P1 / pi;
        }
        *z = (double)(theta / total);
        *w = (double)(powl(sinl(pi * xl), m) / total);
    } else {
        *z = x;
        *w = 1.0;
    }
}

/* ------------------------------------------------------------------ */
/* Integrands                                                           */
/* ------------------------------------------------------------------ */
static double or_ipow(double v, int e)
{
    double r = 1.0;
    for (int t = 0; t < e; ++t)
        r *= v;
    return r;
}

static long double or_ipowl(long double v, int e)
{
    long double r = 1.0L;
    for (int t = 0; t < e; ++t)
        r *= v;
    return r;
}

/* sum_t coef[t] prod_i z_i^exp[t,i] in long double, and the sum of the
   terms' magnitudes */
static long double or_polyl(uint32_t d, uint32_t nt, const double *coef, const uint8_t *ex,
                            const double *z, long double *mag)
{
    long double s = 0.0L, a = 0.0L;
    for (uint32_t t = 0; t < nt; ++t) {
        long double mono = coef[t];
        for (uint32_t i = 0; i < d; ++i)
            mono *= or_ipowl((long double)z[i], ex[t * d + i]);
        s += mono;
        a += fabsl(mono);
    }
    if (mag)
        *mag = a;
    return s;
}

/* sparse polynomial sum_t coef[t] prod_i z_i^exp[t,i] */
/* sum_t coef[t] prod_i z_i^(ex[t,i] - dk[i]) * falling factor of the
   derivative: d/dz_k lowers ex[t,k] by one and multiplies by it; dk counts
   the derivatives per variable (0, 1 or 2 in total) */
static double or_poly_deriv(uint32_t d, uint32_t nt, const double *coef, const uint8_t *ex, const double *z,
                            const int *dk)
{
    double s = 0.0;
    for (uint32_t t = 0; t < nt; ++t) {
        double mono = coef[t];
        for (uint32_t i = 0; i < d && mono != 0.0; ++i) {
            int e = ex[t * d + i];
            for (int r = 0; r < dk[i]; ++r) {
                mono *= (double)e;
                e -= 1;
            }
            if (e < 0)
                mono = 0.0;
            else
                mono *= or_ipow(z[i], e);
        }
        s += mono;
    }
    return s;
}

static double complex or_cpoly(uint32_t d, uint32_t nt, const double *coef, const uint8_t *ex,
                               const double complex *z)
{
    double complex s = 0.0;
    for (uint32_t t = 0; t < nt; ++t) {
        double complex mono = coef[t];
        for (uint32_t i = 0; i < d; ++i)
            for (int r = 0; r < ex[t * d + i]; ++r)
                mono *= z[i];
        s += mono;
    }
    return s;
}

/* determinant by LU with partial pivoting (a is overwritten, n x n row-major) */
static double complex or_cdet(int n, double complex *a)
{
    double complex det = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (cabs(a[r * n + c]) > cabs(a[piv * n + c]))
                piv = r;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                double complex t = a[c * n + k];
                a[c * n + k] = a[piv * n + k];
                a[piv * n + k] = t;
            }
            det = -det;
        }
        det *= a[c * n + c];
        if (a[c * n + c] == 0.0)
            return 0.0;
        for (int r = c + 1; r < n; ++r) {
            double complex f = a[r * n + c] / a[c * n + c];
            for (int k = c; k < n; ++k)
                a[r * n + k] -= f * a[c * n + k];
        }
    }
    return det;
}

double or_poly(uint32_t d, uint32_t nt, const double *coef, const uint8_t *ex, const double *z)
{
    double s = 0.0;
    for (uint32_t t = 0; t < nt; ++t) {
        double mono = coef[t];
        for (uint32_t i = 0; i < d; ++i)
            mono *= or_ipow(z[i], ex[t * d + i]);
        s += mono;
    }
    return s;
}

/* orthonormal shifted Legendre P~_k(x) = sqrt(2k+1) P_k(2x-1), k = 0..K-1,
   from Bonnet's recurrence (k+1) P_{k+1} = (2k+1) t P_k - k P_{k-1} */
void or_legendre(uint32_t K, double x, double *out)
{
    double t = 2.0 * x - 1.0, pm = 1.0, p = t;
    for (uint32_t k = 0; k < K; ++k) {
        double pk;
        if (k == 0)
            pk = 1.0;
        else if (k == 1)
            pk = t;
        else {
            double pn = ((2.0 * (k - 1) + 1.0) * t * p - (double)(k - 1) * pm) / (double)k;
            pm = p;
            p = pn;
            pk = pn;
        }
        out[k] = sqrt(2.0 * k + 1.0) * pk;
    }
}

/* control-variate model g(z) = sum_r c_r prod_i sum_k W[r,i,k] P~_k(z_i) */
double or_cv_g(uint32_t d, uint32_t R, uint32_t K, const double *W, const double *c, const double *z)
{
    double leg[64 * 32];
    if (d > 64 || K > 32)
        return NAN; /* beyond the sizes this routine holds */
    for (uint32_t i = 0; i < d; ++i)
        or_legendre(K, z[i], leg + i * K);
    double g = 0.0;
    for (uint32_t r = 0; r < R; ++r) {
        double prod = c[r];
        for (uint32_t i = 0; i < d; ++i) {
            double h = 0.0;
            for (uint32_t k = 0; k < K; ++k)
                h += W[((size_t)r * d + i) * K + k] * leg[i * K + k];
            prod *= h;
        }
        g += prod;
    }
    return g;
}

/* integral of g over [0,1]^d: only P~_0 = 1 has a nonzero integral */
double or_cv_integral(uint32_t d, uint32_t R, uint32_t K, const double *W, const double *c)
{
    double s = 0.0;
    for (uint32_t r = 0; r < R; ++r) {
        double prod = c[r];
        for (uint32_t i = 0; i < d; ++i)
            prod *= W[((size_t)r * d + i) * K + 0];
        s += prod;
    }
    return s;
}

/* f(z) for the family in p; returns the value in (re, im) */
void or_integrand(const or_params *p, uint32_t d, const double *z, double *re, double *im)
{
    const double PI = 3.14159265358979323846;
    double vr = 0.0, vi = 0.0;
    switch (p->family) {
    case OR_F_CONST:
        vr = p->c;
        break;
    case OR_F_TRIG: {
        long double s = p->c0;
        for (uint32_t t = 0; t < p->n_terms; ++t) {
            long double arg = 0.0L;
            for (uint32_t i = 0; i < d; ++i)
                arg += (long double)p->h[(size_t)t * d + i] * (long double)z[i];
            arg -= floorl(arg);
            s += (long double)p->ch[t] * cosl(2.0L * 3.14159265358979323846264338327950288L * arg +
                                              (long double)p->phi[t]);
        }
        vr = (double)s;
        break;
    }
    case OR_F_P2KERNEL: {
        double prod = 1.0;
        for (uint32_t i = 0; i < d; ++i) {
            double b2 = z[i] * z[i] - z[i] + 1.0 / 6.0;
            prod *= 1.0 + 2.0 * PI * PI * b2;
        }
        vr = prod;
        break;
    }
    case OR_F_GENZ_PRODUCT_PEAK: {
        double prod = 1.0;
        for (uint32_t i = 0; i < d; ++i) {
            double t = z[i] - p->u[i];
            prod *= 1.0 / (1.0 / (p->a[i] * p->a[i]) + t * t);
        }
        vr = prod;
        break;
    }
    case OR_F_GENZ_OSCILLATORY: {
        double s = 2.0 * PI * p->u[0];
        for (uint32_t i = 0; i < d; ++i)
            s += p->a[i] * z[i];
        vr = cos(s);
        break;
    }
    case OR_F_GENZ_GAUSSIAN: {
        double s = 0.0;
        for (uint32_t i = 0; i < d; ++i) {
            double t = z[i] - p->u[i];
            s += p->a[i] * p->a[i] * t * t;
        }
        vr = exp(-s);
        break;
    }
    case OR_F_GENZ_CONTINUOUS: {
        double s = 0.0;
        for (uint32_t i = 0; i < d; ++i)
            s += p->a[i] * fabs(z[i] - p->u[i]);
        vr = exp(-s);
        break;
    }
    case OR_F_GENZ_CORNER_PEAK: {
        double s = 1.0;
        for (uint32_t i = 0; i < d; ++i)
            s += p->a[i] * z[i];
        vr = pow(s, -(double)(d + 1));
        break;
    }
    case OR_F_SECTOR: {
        if (p->deform_lambda != 0.0) {
            /* contour deformation: z = x - i lambda x (1 - x) grad F(x) */
            const double lam = p->deform_lambda;
            double complex zc[64], J[16 * 16];
            if (d > 16) { /* the Jacobian array holds d <= 16 */
                vr = vi = NAN;
                break;
            }
            double grad[64];
            int dk[64];
            for (uint32_t i = 0; i < d; ++i)
                dk[i] = 0;
            for (uint32_t k = 0; k < d; ++k) {
                dk[k] = 1;
                grad[k] = or_poly_deriv(d, p->n_f, p->coef_f, p->exp_f, z, dk);
                dk[k] = 0;
                zc[k] = z[k] - I * lam * z[k] * (1.0 - z[k]) * grad[k];
            }
            for (uint32_t k = 0; k < d; ++k)
                for (uint32_t l = 0; l < d; ++l) {
                    dk[k] += 1;
                    dk[l] += 1;
                    const double h = or_poly_deriv(d, p->n_f, p->coef_f, p->exp_f, z, dk);
                    dk[k] = 0;
                    dk[l] = 0;
                    double complex e = -I * lam * z[k] * (1.0 - z[k]) * h;
                    if (k == l)
                        e += 1.0 - I * lam * (1.0 - 2.0 * z[k]) * grad[k];
                    J[k * d + l] = e;
                }
            const double complex detj = or_cdet((int)d, J);
            double complex monoc = 1.0;
            for (uint32_t i = 0; i < d; ++i)
                for (int r = 0; r < p->nu[i]; ++r)
                    monoc *= zc[i];
            const double complex Uc = or_cpoly(d, p->n_u, p->coef_u, p->exp_u, zc);
            const double delta = p->is_complex ? p->delta_im : 0.0;
            const double complex Fc = or_cpoly(d, p->n_f, p->coef_f, p->exp_f, zc) - I * delta;
            if (p->deform_check) {
                vr = cimag(Fc) > 0.0 ? 1.0 : 0.0;
                vi = 0.0;
                break;
            }
            double complex v = monoc * cpow(Uc, p->pow_u) * cpow(Fc, p->pow_f) * detj;
            const double complex L = p->eps_u * clog(Uc) + p->eps_f * clog(Fc);
            for (int32_t k = 1; k <= p->eps_order; ++k)
                v = v * L / (double)k;
            vr = creal(v);
            vi = cimag(v);
            break;
        }
        if (p->precise) {
            long double monol = 1.0L;
            for (uint32_t i = 0; i < d; ++i)
                monol *= or_ipowl((long double)z[i], p->nu[i]);
            const long double Ul = or_polyl(d, p->n_u, p->coef_u, p->exp_u, z, NULL);
            const long double Fl = or_polyl(d, p->n_f, p->coef_f, p->exp_f, z, NULL);
            const long double prel = monol * powl(Ul, (long double)p->pow_u);
            long double complex vl, Ll;
            if (p->is_complex) {
                const long double complex Fcl = Fl - I * (long double)p->delta_im;
                vl = prel * cpowl(Fcl, (long double)p->pow_f);
                Ll = (long double)p->eps_u * logl(Ul) + (long double)p->eps_f * clogl(Fcl);
            } else {
                vl = prel * powl(Fl, (long double)p->pow_f);
                Ll = (long double)p->eps_u * logl(Ul) + (long double)p->eps_f * logl(Fl);
            }
            for (int32_t k = 1; k <= p->eps_order; ++k)
                vl = vl * Ll / (long double)k;
            vr = (double)creall(vl);
            vi = p->is_complex ? (double)cimagl(vl) : 0.0;
            break;
        }
        double mono = 1.0;
        for (uint32_t i = 0; i < d; ++i)
            mono *= or_ipow(z[i], p->nu[i]);
        double U = or_poly(d, p->n_u, p->coef_u, p->exp_u, z);
        double F = or_poly(d, p->n_f, p->coef_f, p->exp_f, z);
        double pre = mono * pow(U, p->pow_u);
        double complex v, L;
        if (p->is_complex) {
            double complex Fc = F - I * p->delta_im;
            v = pre * cpow(Fc, p->pow_f);
            L = p->eps_u * log(U) + p->eps_f * clog(Fc);
        } else {
            v = pre * pow(F, p->pow_f);
            L = p->eps_u * log(U) + p->eps_f * log(F);
        }
        for (int32_t k = 1; k <= p->eps_order; ++k)
            v = v * L / (double)k;
        vr = creal(v);
        vi = p->is_complex ? cimag(v) : 0.0;
        break;
    }
    default:
        vr = NAN;
        vi = NAN;
    }
    if (p->cv_w != NULL)
        vr -= or_cv_g(d, p->cv_r, p->cv_k, p->cv_w, p->cv_c, z);
    if (p->cv_w_im != NULL)
        vi -= or_cv_g(d, p->cv_r, p->cv_k, p->cv_w_im, p->cv_c_im, z);
    *re = vr;
    *im = vi;
}

/* fhat(x) = f(z(x)) * prod_i z_i'(x_i) */
void or_fhat(const or_params *p, uint32_t d, int32_t tkind, int32_t alpha, const double *x,
             double *re, double *im)
{
    double z[64], wprod = 1.0;
    for (uint32_t i = 0; i < d; ++i) {
        double w;
        or_transform(tkind, alpha, x[i], &z[i], &w);
        wprod *= w;
    }
    double vr, vi;
    or_integrand(p, d, z, &vr, &vi);
    if (p->family == OR_F_SECTOR && p->deform_lambda != 0.0 && p->deform_check)
        wprod = 1.0; /* the sign check counts points */
    *re = vr * wprod;
    *im = vi * wprod;
}

/* Samples of the lattice {j g / n + shift}, j = 0..n-1, for fitting a
   control variate: the transformed point z (n, d), the Jacobian
   J = prod_i z_i'(x_i) (n) and fhat = J f(z) (n, re and im). */
int or_cv_samples(uint32_t d, uint64_t n, const uint64_t *g, const double *shift, int32_t tkind,
                  int32_t alpha, const or_params *p, double *z, double *jac, double *f_re,
                  double *f_im)
{
    if (d == 0 || d > 64)
        return 1;
    double x[64];
    for (uint64_t j = 0; j < n; ++j) {
        or_point(d, n, g, j, shift, p->point_mode, x);
        double wprod = 1.0;
        for (uint32_t i = 0; i < d; ++i) {
            double w;
            or_transform(tkind, alpha, x[i], &z[j * d + i], &w);
            wprod *= w;
        }
        jac[j] = wprod;
        or_fhat(p, d, tkind, alpha, x, &f_re[j], &f_im[j]);
    }
    return 0;
}

/* How strongly double-precision rounding in the sums of a plain sector's
   polynomials moves its value, relative to |f|: a relative error u in every
   term of U and F changes U^pU (F - i delta)^pF by at most
   u (|pU| S_U / |U| + |pF| S_F / |F - i delta|), S the sum of the terms'
   magnitudes.  Returns that factor (without u); 0 for other families. */
double or_sector_condition(const or_params *p, uint32_t d, const double *z)
{
    if (p->family != OR_F_SECTOR || p->deform_lambda != 0.0)
        return 0.0;
    long double su, sf;
    const long double U = or_polyl(d, p->n_u, p->coef_u, p->exp_u, z, &su);
    const long double F = or_polyl(d, p->n_f, p->coef_f, p->exp_f, z, &sf);
    const long double delta = p->is_complex ? (long double)p->delta_im : 0.0L;
    const long double fmod_ = sqrtl(F * F + delta * delta);
    return (double)(fabsl((long double)p->pow_u) * su / fabsl(U) + fabsl((long double)p->pow_f) * sf / fmod_);
}

/* ------------------------------------------------------------------ */
/* Compensated long-double accumulation                                 */
/* ------------------------------------------------------------------ */
typedef struct {
    long double s, c;
} or_acc;

static void or_acc_add(or_acc *a, long double v)
{
    long double t = a->s + v;
    if (fabsl(a->s) >= fabsl(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

/* ------------------------------------------------------------------ */
/* Estimator, eq. (2)                                                   */
/* ------------------------------------------------------------------ */
typedef struct {
    uint32_t d, m;
    uint64_t n;
    const uint64_t *g;
    const double *shifts;
    int32_t tkind, alpha;
    const or_params *p;
    or_acc *part_re, *part_im, *part_abs; /* [m][NCHUNK] */
    or_acc *part_cond;                    /* [m][NCHUNK], NULL: not wanted */
    int next;                             /* next work item, guarded by lock */
    pthread_mutex_t lock;
} or_job;

static void or_work_item(or_job *jb, int item)
{
    uint32_t k = (uint32_t)(item / OR_NCHUNK);
    uint64_t c = (uint64_t)(item % OR_NCHUNK);
    uint64_t j0 = jb->n * c / OR_NCHUNK, j1 = jb->n * (c + 1) / OR_NCHUNK;
    or_acc re = {0, 0}, im = {0, 0}, ab = {0, 0}, co = {0, 0};
    double x[64], z[64];
    const double *sh = jb->shifts + (size_t)k * jb->d;
    for (uint64_t j = j0; j < j1; ++j) {
        or_point(jb->d, jb->n, jb->g, j, sh, jb->p->point_mode, x);
        double vr, vi;
        or_fhat(jb->p, jb->d, jb->tkind, jb->alpha, x, &vr, &vi);
        const double av = sqrt(vr * vr + vi * vi);
        or_acc_add(&re, vr);
        or_acc_add(&im, vi);
        or_acc_add(&ab, av);
        if (jb->part_cond) {
            for (uint32_t i = 0; i < jb->d; ++i) {
                double w;
                or_transform(jb->tkind, jb->alpha, x[i], &z[i], &w);
            }
            or_acc_add(&co, av * or_sector_condition(jb->p, jb->d, z));
        }
    }
    jb->part_re[item] = re;
    jb->part_im[item] = im;
    jb->part_abs[item] = ab;
    if (jb->part_cond)
        jb->part_cond[item] = co;
}

static void *or_worker(void *arg)
{
    or_job *jb = (or_job *)arg;
    int total = (int)jb->m * OR_NCHUNK;
    for (;;) {
        pthread_mutex_lock(&jb->lock);
        int item = jb->next++;
        pthread_mutex_unlock(&jb->lock);
        if (item >= total)
            break;
        or_work_item(jb, item);
    }
    return NULL;
}

/* Per-shift estimates Q_k (re, im) and sum_j |fhat| / n (for the condition
   number).  Returns 0, or 5 when a per-shift sum is not finite, or 1 on bad
   arguments. */
int or_estimate_cond(uint32_t d, uint64_t n, const uint64_t *g, uint32_t m, const double *shifts,
                     int32_t tkind, int32_t alpha, const or_params *p, int32_t nthreads, double *q_re,
                     double *q_im, double *q_abs, double *q_cond);

int or_estimate(uint32_t d, uint64_t n, const uint64_t *g, uint32_t m, const double *shifts,
                int32_t tkind, int32_t alpha, const or_params *p, int32_t nthreads, double *q_re,
                double *q_im, double *q_abs)
{
    return or_estimate_cond(d, n, g, m, shifts, tkind, alpha, p, nthreads, q_re, q_im, q_abs, NULL);
}

/* or_estimate, and (q_cond non-NULL) per shift (1/n) sum_j |fhat_j| c_j with
   c_j = or_sector_condition at the point's transformed coordinates: times
   the unit roundoff, a bound on how far double-precision sums of U and F
   can move Q_k */
int or_estimate_cond(uint32_t d, uint64_t n, const uint64_t *g, uint32_t m, const double *shifts,
                     int32_t tkind, int32_t alpha, const or_params *p, int32_t nthreads, double *q_re,
                     double *q_im, double *q_abs, double *q_cond)
{
    if (d == 0 || d > 64 || n < 1 || m < 1)
        return 1;
    /* the deformed sector holds its d x d Jacobian in a 16 x 16 array, the
       control-variate model at most 32 Legendre degrees */
    if (p->family == OR_F_SECTOR && p->deform_lambda != 0.0 && d > 16)
        return 1;
    if ((p->cv_w != NULL || p->cv_w_im != NULL) && p->cv_k > 32)
        return 1;
    or_job jb;
    jb.d = d;
    jb.m = m;
    jb.n = n;
    jb.g = g;
    jb.shifts = shifts;
    jb.tkind = tkind;
    jb.alpha = alpha;
    jb.p = p;
    size_t items = (size_t)m * OR_NCHUNK;
    jb.part_re = (or_acc *)calloc(items, sizeof(or_acc));
    jb.part_im = (or_acc *)calloc(items, sizeof(or_acc));
    jb.part_abs = (or_acc *)calloc(items, sizeof(or_acc));
    jb.part_cond = q_cond ? (or_acc *)calloc(items, sizeof(or_acc)) : NULL;
    jb.next = 0;
    pthread_mutex_init(&jb.lock, NULL);
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    pthread_t th[256];
    for (int t = 1; t < nthreads; ++t)
        pthread_create(&th[t], NULL, or_worker, &jb);
    or_worker(&jb);
    for (int t = 1; t < nthreads; ++t)
        pthread_join(th[t], NULL);
    pthread_mutex_destroy(&jb.lock);

    int status = 0;
    for (uint32_t k = 0; k < m; ++k) {
        or_acc re = {0, 0}, im = {0, 0}, ab = {0, 0};
        for (int c = 0; c < OR_NCHUNK; ++c) {
            or_acc *pr = &jb.part_re[(size_t)k * OR_NCHUNK + c];
            or_acc *pi = &jb.part_im[(size_t)k * OR_NCHUNK + c];
            or_acc *pa = &jb.part_abs[(size_t)k * OR_NCHUNK + c];
            or_acc_add(&re, pr->s);
            or_acc_add(&re, pr->c);
            or_acc_add(&im, pi->s);
            or_acc_add(&im, pi->c);
            or_acc_add(&ab, pa->s);
            or_acc_add(&ab, pa->c);
        }
        q_re[k] = (double)((re.s + re.c) / (long double)n);
        q_im[k] = (double)((im.s + im.c) / (long double)n);
        if (q_abs)
            q_abs[k] = (double)((ab.s + ab.c) / (long double)n);
        if (q_cond) {
            or_acc co = {0, 0};
            for (int c = 0; c < OR_NCHUNK; ++c) {
                or_acc_add(&co, jb.part_cond[(size_t)k * OR_NCHUNK + c].s);
                or_acc_add(&co, jb.part_cond[(size_t)k * OR_NCHUNK + c].c);
            }
            q_cond[k] = (double)((co.s + co.c) / (long double)n);
        }
        if (!isfinite(q_re[k]) || !isfinite(q_im[k]))
            status = 5;
    }
    free(jb.part_re);
    free(jb.part_im);
    free(jb.part_abs);
    free(jb.part_cond);
    return status;
}

/* Mean and error of eq. (2)/(3) for one real sequence: out[0] = Qbar,
   out[1] = sqrt(sum_k (Q_k - Qbar)^2 / (m (m - 1))).  Two passes. */
void or_mean_error(uint32_t m, const double *q, double *out)
{
    or_acc s = {0, 0};
    for (uint32_t k = 0; k < m; ++k)
        or_acc_add(&s, q[k]);
    long double mean = (s.s + s.c) / (long double)m;
    or_acc v = {0, 0};
    for (uint32_t k = 0; k < m; ++k) {
        long double dlt = (long double)q[k] - mean;
        or_acc_add(&v, dlt * dlt);
    }
    out[0] = (double)mean;
    out[1] = (m > 1) ? (double)sqrtl((v.s + v.c) / ((long double)m * (long double)(m - 1))) : NAN;
}

/* ------------------------------------------------------------------ */
/* Generating vector: Korobov form and the P_2 criterion                */
/* ------------------------------------------------------------------ */
void or_korobov_vector(uint64_t n, uint32_t d, uint64_t a, uint64_t *g)
{
    uint64_t v = 1 % n;
    for (uint32_t i = 0; i < d; ++i) {
        g[i] = v;
        v = or_lattice_index(v, a, n);
    }
}

typedef struct {
    uint32_t d;
    uint64_t n;
    const uint64_t *g;
    or_acc *part;
    int next;
    pthread_mutex_t lock;
} or_p2job;

static void *or_p2_worker(void *arg)
{
    const double PI = 3.14159265358979323846;
    or_p2job *jb = (or_p2job *)arg;
    for (;;) {
        pthread_mutex_lock(&jb->lock);
        int c = jb->next++;
        pthread_mutex_unlock(&jb->lock);
        if (c >= OR_NCHUNK)
            break;
        uint64_t j0 = jb->n * (uint64_t)c / OR_NCHUNK, j1 = jb->n * (uint64_t)(c + 1) / OR_NCHUNK;
        or_acc a = {0, 0};
        for (uint64_t j = j0; j < j1; ++j) {
            double prod = 1.0;
            for (uint32_t i = 0; i < jb->d; ++i) {
                double x = (double)or_lattice_index(j, jb->g[i], jb->n) / (double)jb->n;
                double b2 = x * x - x + 1.0 / 6.0;
                prod *= 1.0 + 2.0 * PI * PI * b2;
            }
            or_acc_add(&a, prod);
        }
        jb->part[c] = a;
    }
    return NULL;
}

/* P_2(g) = -1 + (1/n) sum_{j=0}^{n-1} prod_i (1 + 2 pi^2 B_2({j g_i / n})),
   B_2(x) = x^2 - x + 1/6: the worst-case error of the unshifted rule for
   the unit-weight Korobov space of smoothness 2 (Sloan and Joe). */
double or_p2(uint32_t d, uint64_t n, const uint64_t *g, int32_t nthreads)
{
    or_p2job jb;
    jb.d = d;
    jb.n = n;
    jb.g = g;
    jb.part = (or_acc *)calloc(OR_NCHUNK, sizeof(or_acc));
    jb.next = 0;
    pthread_mutex_init(&jb.lock, NULL);
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    pthread_t th[256];
    for (int t = 1; t < nthreads; ++t)
        pthread_create(&th[t], NULL, or_p2_worker, &jb);
    or_p2_worker(&jb);
    for (int t = 1; t < nthreads; ++t)
        pthread_join(th[t], NULL);
    pthread_mutex_destroy(&jb.lock);
    or_acc s = {0, 0};
    for (int c = 0; c < OR_NCHUNK; ++c) {
        or_acc_add(&s, jb.part[c].s);
        or_acc_add(&s, jb.part[c].c);
    }
    free(jb.part);
    return (double)(-1.0L + (s.s + s.c) / (long double)n);
}

/* argmin over candidates of P_2(korobov_vector(a)); ties go to the smaller
   P_2 value, then to the smaller a.  p2_all (nullable) receives every value. */
int or_korobov_search(uint64_t n, uint32_t d, const uint64_t *cand, uint32_t ncand,
                      int32_t nthreads, uint64_t *a_best, double *p2_best, double *p2_all)
{
    if (ncand == 0 || d == 0 || d > 64 || n < 2)
        return 1;
    uint64_t g[64];
    double best = INFINITY;
    uint64_t abest = 0;
    for (uint32_t c = 0; c < ncand; ++c) {
        or_korobov_vector(n, d, cand[c], g);
        double v = or_p2(d, n, g, nthreads);
        if (p2_all)
            p2_all[c] = v;
        if (v < best || (v == best && cand[c] < abest)) {
            best = v;
            abest = cand[c];
        }
    }
    *a_best = abest;
    *p2_best = best;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Component-by-component construction of a generating vector          */
/* ------------------------------------------------------------------ */
/* Sec. 2 uses rank-1 lattices and leaves the generating vector open; the
   standard construction of the lattice literature (Sloan, Kuo, Joe;
   Nuyens, Cools) fixes z_1 = 1 and, for s = 2..d, takes z_s from
   {1 <= c <= n/2, gcd(c, n) = 1} minimising the squared worst-case error of
   the weighted Korobov space of smoothness 2,
     e_s^2(c) = -1 + (1/n) sum_{j=0}^{n-1} prod_{i<s} (1 + gamma_i w({j z_i / n}))
                                        * (1 + gamma_s w({j c / n})),
   w(x) = 2 pi^2 B_2(x), B_2(x) = x^2 - x + 1/6.  Ties, taken as values
   within 1e-13 (1 + e^2) of the minimum, go to the smallest c.
   e2[s-1] receives e_s^2(z_s) (e2[0] for z_1 = 1). */
typedef struct {
    uint64_t n;
    double gamma;
    const long double *prod; /* [n] product over the chosen components */
    const uint64_t *cand;
    uint64_t ncand;
    long double *val;        /* [ncand] sums */
    uint64_t next;
    pthread_mutex_t lock;
} or_cbcjob;

static void *or_cbc_worker(void *arg)
{
    const long double PI = 3.141592653589793238462643383279502884L;
    or_cbcjob *jb = (or_cbcjob *)arg;
    for (;;) {
        pthread_mutex_lock(&jb->lock);
        uint64_t c0 = jb->next;
        jb->next += 64;
        pthread_mutex_unlock(&jb->lock);
        if (c0 >= jb->ncand)
            break;
        uint64_t c1 = c0 + 64 < jb->ncand ? c0 + 64 : jb->ncand;
        for (uint64_t t = c0; t < c1; ++t) {
            or_acc a = {0, 0};
            for (uint64_t j = 0; j < jb->n; ++j) {
                long double x = (long double)or_lattice_index(j, jb->cand[t], jb->n) / (long double)jb->n;
                long double b2 = x * x - x + 1.0L / 6.0L;
                or_acc_add(&a, jb->prod[j] * (1.0L + jb->gamma * 2.0L * PI * PI * b2));
            }
            jb->val[t] = a.s + a.c;
        }
    }
    return NULL;
}

static uint64_t or_gcd(uint64_t a, uint64_t b)
{
    while (b) {
        uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

int or_cbc(uint64_t n, uint32_t d, const double *gamma, int32_t nthreads, uint64_t *z, double *e2)
{
    const long double PI = 3.141592653589793238462643383279502884L;
    if (n < 2 || d == 0 || d > 64)
        return 1;
    long double *prod = (long double *)malloc(n * sizeof(long double));
    uint64_t *cand = (uint64_t *)malloc((n / 2 + 1) * sizeof(uint64_t));
    long double *val = (long double *)malloc((n / 2 + 1) * sizeof(long double));
    uint64_t ncand = 0;
    for (uint64_t c = 1; c <= n / 2; ++c)
        if (or_gcd(c, n) == 1)
            cand[ncand++] = c;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    for (uint64_t j = 0; j < n; ++j)
        prod[j] = 1.0L;
    for (uint32_t s = 0; s < d; ++s) {
        uint64_t best_c = 1;
        long double best = 0.0L;
        if (s == 0) {
            /* z_1 = 1: in one dimension every admissible c gives the same
               point set */
            or_cbcjob one = {n, gamma[0], prod, cand, 1, val, 0};
            pthread_mutex_init(&one.lock, NULL);
            or_cbc_worker(&one);
            pthread_mutex_destroy(&one.lock);
            best = val[0];
        } else {
            or_cbcjob jb = {n, gamma[s], prod, cand, ncand, val, 0};
            pthread_mutex_init(&jb.lock, NULL);
            pthread_t th[256];
            for (int t = 1; t < nthreads; ++t)
                pthread_create(&th[t], NULL, or_cbc_worker, &jb);
            or_cbc_worker(&jb);
            for (int t = 1; t < nthreads; ++t)
                pthread_join(th[t], NULL);
            pthread_mutex_destroy(&jb.lock);
            /* lattice symmetries make exact ties common (in two dimensions
               c and c^-1 mod n give the same error), and rounding would pick
               among them: values within 1e-13 (1 + e^2) of the minimum count
               as ties, and ties go to the smallest c */
            long double vmin = val[0];
            for (uint64_t t = 1; t < ncand; ++t)
                if (val[t] < vmin)
                    vmin = val[t];
            const long double tau = 1e-13L * (long double)n * (1.0L + fabsl(vmin / (long double)n - 1.0L));
            for (uint64_t t = 0; t < ncand; ++t)
                if (val[t] <= vmin + tau) {
                    best = val[t];
                    best_c = cand[t];
                    break;
                }
        }
        z[s] = best_c;
        e2[s] = (double)(-1.0L + best / (long double)n);
        for (uint64_t j = 0; j < n; ++j) {
            long double x = (long double)or_lattice_index(j, best_c, n) / (long double)n;
            prod[j] *= 1.0L + gamma[s] * 2.0L * PI * PI * (x * x - x + 1.0L / 6.0L);
        }
    }
    free(prod);
    free(cand);
    free(val);
    return 0;
}

