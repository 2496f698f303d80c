// Periodising transforms (arXiv:1811.11722 Sec. 2, eqs. (4)-(5)) and
// integrand families, fused so that each thread evaluates
// fhat(x) = f(z(x)) * prod_i z_i'(x_i) for T shifts of one lattice point.
//
// Parameter blobs are arrays of 8-byte words written by the host packer
// (qmc_runtime.cpp).  They are read through uniform addresses, so the
// compiler keeps them in scalar registers / the scalar cache.
#pragma once

#include "qmc_device.hpp"

namespace qmc {

// ------------------------------------------------------------ transforms
// Identity: z = x.
struct TrNone {
    static constexpr bool kJac = false;
    __device__ static double z(double x) { return x; }
    __device__ static double z_operand(double x) { return x; }
};

// Baker's transform, eq. (5): z = 1 - |2x - 1|.  The map is 2-to-1 with
// |z'| = 2 on each half, so the integrand weight is 1.  The kernels receive
// x' = {x + 1/2} (the shift tables of baker plans hold {Delta + 1/2}), and
// 1 - |2x - 1| = |2x' - 1|.  z() materialises it (one FMA and a v_max with
// an absolute-value operand, as many instructions as 1 - |2x - 1|);
// z_operand() is the FMA alone, the absolute value left as a free modifier
// of each use.  That form suits functors whose uses of z are all FMAs and
// multiplies (the run-time specialised ones: one instruction less per
// coordinate); in the table-driven functors the compiler then keeps both
// the value and its absolute value live (48 more VGPRs at d = 6 with four
// shifts, a third of the occupancy lost).
struct TrBaker {
    static constexpr bool kJac = false;
    __device__ static double z(double xh) { return __builtin_fmax(__builtin_fabs(fma_(2.0, xh, -1.0)), 0.0); }
    __device__ static double z_operand(double xh) { return __builtin_fabs(fma_(2.0, xh, -1.0)); }
};

constexpr double cfact(int k) { return k <= 1 ? 1.0 : k * cfact(k - 1); }
constexpr double cbinom(int n, int k) { return cfact(n) / (cfact(k) * cfact(n - k)); }
constexpr double cpow4(int e) {  // 4^e for e <= 0
    return e == 0 ? 1.0 : 0.25 * cpow4(e + 1);
}

// Korobov transform of weight A, eq. (4): w(x) = C_A u^A with u = x (1 - x)
// and C_A = (2A+1)!/(A!)^2, z(x) = int_0^x w.  With t = x - 1/2,
//   z = 1/2 + t * H(u),  H(u) = sum_{k=0..A} binom(2k, k) u^k.
// Differentiating (u' = -2t, t^2 = 1/4 - u), the terms of u^k from the k-th
// and (k+1)-th summands cancel because (k+1) binom(2k+2, k+1) = 2 (2k+1)
// binom(2k, k), which leaves (2A+1) binom(2A, A) u^A = C_A u^A; z(0) = 0.
// The coefficients 1, 2, 6, 20, 70, ... are positive integers and
// u <= 1/4, so every term of H lies in [0, 1] and Horner's rule sums
// positive values (no cancellation anywhere in [0, 1]).  u is needed for
// the Jacobian anyway, so z costs no separate t^2.  The constant C_A^d of
// prod_i w_i is applied once to the final sums.
template <int A>
struct TrKorobov {
    static_assert(A >= 1 && A <= 6, "Korobov weight 1..6");
    static constexpr bool kJac = true;
    static constexpr double kC = cfact(2 * A + 1) / (cfact(A) * cfact(A));
    // binom(2k, k) as a table evaluated by the compiler: calling the
    // recursive helpers from device code would leave them as run-time calls
    struct Coefs {
        double c[A + 1];
    };
    static constexpr Coefs make_coefs() {
        Coefs r{};
        for (int k = 0; k <= A; ++k) r.c[k] = cbinom(2 * k, k);
        return r;
    }
    static constexpr Coefs kCoef = make_coefs();
    // H(u), Horner from the top coefficient.  From A = 3 on the first step
    // multiplies and adds two constants that are not inline operands (20u + 6
    // at A = 3); as literals the compiler re-creates the addend with two
    // v_mov_b32 before every use, so both come from registers set once per
    // thread: the factor from an SGPR pair, the addend from a VGPR pair (one
    // FMA per use, within the one-SGPR operand limit of VOP3).
    __device__ static double h(double u) {
        double r;
        if constexpr (A == 1)
            r = fma_(u, kCoef.c[1], kCoef.c[0]);
        else if constexpr (A == 2)
            r = fma_(u, sreg_const(kCoef.c[2]), kCoef.c[1]);
        else
            r = fma_(u, sreg_const(kCoef.c[A]), vreg_const(kCoef.c[A - 1]));
#pragma unroll
        for (int k = A - 2; k >= 0; --k) r = fma_(r, u, kCoef.c[k]);
        return r;
    }
    // z and u = x (1 - x) = 1/4 - t^2
    __device__ static double z(double x, double &u) {
        const double t = x - 0.5;
        u = fma_(-t, t, 0.25);
        return fma_(t, h(u), 0.5);
    }
    // z - c, given hmc = 1/2 - c, and u
    __device__ static double z_minus(double x, double hmc, double &u) {
        const double t = x - 0.5;
        u = fma_(-t, t, 0.25);
        return fma_(t, h(u), hmc);
    }
    // prod_i w_i / C_A^d = (prod_i u_i)^A
    __device__ static double jac(double pu) {
        double r = pu;
#pragma unroll
        for (int a = 1; a < A; ++a) r *= pu;
        return r;
    }
};

// Sidi's sin^M transform: w(x) = sin^M(pi x) / T_M with T_M the integral of
// sin^M over [0, 1], z = int_0^x w.  With c = cos(pi x):
//   M = 2p+1: z = 1/2 - c sum_k d_k c^(2k), d_k = binom(p, k) (-1)^k /
//             ((2k + 1) 2 P1), P1 = sum_k binom(p, k) (-1)^k / (2k + 1)
//             (substituting u = cos(pi t) in the integral of sin^M);
//   M = 2p:   z = x + sin(2 pi x) sum_{k=1..p} e_k U_{k-1}(cos 2 pi x),
//             e_k = (-1)^k binom(2p, p-k) / (pi k binom(2p, p)), U the
//             Chebyshev polynomials of the second kind (sin(2k t) =
//             sin(2t) U_{k-1}(cos 2t)).
// u = sin(pi x); the Jacobian is (prod u)^M and 1/T_M^d is applied to the
// final sums.
template <int M>
struct TrSidi {
    static_assert(M >= 1 && M <= 6, "Sidi order 1..6");
    static constexpr bool kJac = true;
    static constexpr int P = M / 2;
    static constexpr double kPiD = 3.141592653589793;
    struct Coefs {
        double c[P + 1];
    };
    static constexpr Coefs make_coefs() {
        Coefs r{};
        if (M % 2) {
            double p1 = 0.0;
            for (int k = 0; k <= P; ++k) p1 += cbinom(P, k) * ((k & 1) ? -1.0 : 1.0) / (2 * k + 1);
            for (int k = 0; k <= P; ++k) r.c[k] = cbinom(P, k) * ((k & 1) ? -1.0 : 1.0) / ((2 * k + 1) * 2.0 * p1);
        } else {
            r.c[0] = 0.0;
            for (int k = 1; k <= P; ++k)
                r.c[k] = ((k & 1) ? -1.0 : 1.0) * cbinom(2 * P, P - k) / (kPiD * k * cbinom(2 * P, P));
        }
        return r;
    }
    static constexpr Coefs kCoef = make_coefs();
    // z = base + q r with (q, r) from the sine and cosine: odd M base 1/2,
    // q = -cos, even M base x, q = sin 2 pi x
    __device__ static void parts(double x, double &u, double &q, double &r) {
        double sn, cs;
        qsincos(kPiD * x, sn, cs);
        u = sn;
        if constexpr (M % 2) {
            const double c2 = cs * cs;
            r = kCoef.c[P];
#pragma unroll
            for (int k = P - 1; k >= 0; --k) r = fma_(r, c2, kCoef.c[k]);
            q = -cs;
        } else {
            const double C = fma_(-2.0 * sn, sn, 1.0);  // cos 2 pi x
            double um2 = 0.0, um1 = 1.0;                 // U_{-1}, U_0
            r = kCoef.c[1];
#pragma unroll
            for (int k = 2; k <= P; ++k) {
                const double uk = fma_(2.0 * C, um1, -um2);
                um2 = um1;
                um1 = uk;
                r = fma_(kCoef.c[k], uk, r);
            }
            q = 2.0 * sn * cs;
        }
    }
    __device__ static double z(double x, double &u) {
        double q, r;
        parts(x, u, q, r);
        return fma_(q, r, (M % 2) ? 0.5 : x);
    }
    // z - b given hmb = 1/2 - b, and u
    __device__ static double z_minus(double x, double hmb, double &u) {
        double q, r;
        parts(x, u, q, r);
        return fma_(q, r, (M % 2) ? hmb : (x - 0.5) + hmb);
    }
    __device__ static double jac(double pu) {
        double r = pu;
#pragma unroll
        for (int a = 1; a < M; ++a) r *= pu;
        return r;
    }
};

// z for all D coordinates of T shifts, and the Jacobian (without C_A^d);
// Operand selects z_operand() of the transforms without a Jacobian
template <class Tr, int D, int T, bool Operand = false>
__device__ __forceinline__ void apply_transform(const double (&x)[T][D], double (&z)[T][D],
                                                double (&jac)[T]) {
#pragma unroll
    for (int k = 0; k < T; ++k) {
        if constexpr (Tr::kJac) {
            double pu = 1.0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double u;
                z[k][i] = Tr::z(x[k][i], u);
                pu = (i == 0) ? u : pu * u;
            }
            jac[k] = Tr::jac(pu);
        } else {
#pragma unroll
            for (int i = 0; i < D; ++i) z[k][i] = Operand ? Tr::z_operand(x[k][i]) : Tr::z(x[k][i]);
            jac[k] = 1.0;
        }
    }
}

// ------------------------------------------------------------ families
// Every family provides NP (1 real, 2 complex) and
//   eval<Tr, D, T>(p, x, v): v[k][.] = fhat(x[k]) / (transform constant).

// constant c.  blob: [c]
struct FamConst {
    static constexpr int NP = 1;
    template <class Tr, int D, int T>
    __device__ static void eval(const double *__restrict__ p, const double (&x)[T][D],
                                double (&v)[T][NP]) {
        const double c = p[0];
        double z[T][D], jac[T];
        apply_transform<Tr, D, T>(x, z, jac);
#pragma unroll
        for (int k = 0; k < T; ++k) v[k][0] = Tr::kJac ? c * jac[k] : c;
    }
};

// prod_i (1 + 2 pi^2 B2(z_i)), B2(z) = z^2 - z + 1/6, i.e. the quadratic
// 2pi^2 z^2 - 2pi^2 z + (1 + pi^2/3) per coordinate.  No blob.
struct FamP2 {
    static constexpr int NP = 1;
    template <class Tr, int D, int T>
    __device__ static void eval(const double *__restrict__, const double (&x)[T][D],
                                double (&v)[T][NP]) {
        constexpr double c2 = 2.0 * 9.869604401089358;  // 2 pi^2
        constexpr double c0 = 1.0 + 9.869604401089358 / 3.0;
        double z[T][D], jac[T];
        apply_transform<Tr, D, T>(x, z, jac);
#pragma unroll
        for (int k = 0; k < T; ++k) {
            double prod = 1.0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const double q = fma_(fma_(c2, z[k][i], -c2), z[k][i], c0);
                prod = (i == 0) ? q : prod * q;
            }
            v[k][0] = Tr::kJac ? prod * jac[k] : prod;
        }
    }
};

// c0 + sum_t c_t cos(2 pi (h_t . z) + phi_t).
// blob: [n_terms, c0, then per term: c_t, phi_t / (2 pi), h_t[0..D-1] as doubles]
struct FamTrig {
    static constexpr int NP = 1;
    template <class Tr, int D, int T>
    __device__ static void eval(const double *__restrict__ p, const double (&x)[T][D],
                                double (&v)[T][NP]) {
        double z[T][D], jac[T];
        apply_transform<Tr, D, T>(x, z, jac);
        const uint32_t nt = (uint32_t)__double_as_longlong(p[0]);
        const double c0 = p[1];
        double acc[T];
#pragma unroll
        for (int k = 0; k < T; ++k) acc[k] = c0;
        const double *q = p + 2;
        for (uint32_t t = 0; t < nt; ++t, q += 2 + D) {
            const double c = q[0], ph = q[1];
#pragma unroll
            for (int k = 0; k < T; ++k) {
                double arg = ph;
#pragma unroll
                for (int i = 0; i < D; ++i) arg = fma_(q[2 + i], z[k][i], arg);
                acc[k] = fma_(c, cospi(2.0 * fract(arg)), acc[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < T; ++k) v[k][0] = Tr::kJac ? acc[k] * jac[k] : acc[k];
    }
};

// Genz product peak prod_i 1/(a_i^-2 + (z_i - u_i)^2).
// blob: [a^-2 (D), u (D), 1/2 - u (D), tile flag]
// The T denominators of a thread's shifts share one reciprocal when the
// tile flag is set (prefix products, the reciprocal of their total, then
// one multiply back per shift: 3 (T - 1) multiplies instead of T - 1
// quarter-rate reciprocals and their Newton steps).  The host sets the flag
// only if every product of up to 16 denominators stays within 2^-1000 ..
// 2^1000 for all z in the unit cube, from the bounds a^-2 <= q_i <=
// a^-2 + max(u^2, (1 - u)^2) of each factor.
struct FamGenzProductPeak {
    static constexpr int NP = 1;
    template <class Tr, int D, int T>
    __device__ static void eval(const double *__restrict__ p, const double (&x)[T][D],
                                double (&v)[T][NP]) {
        double den[T], w[T];
#pragma unroll
        for (int k = 0; k < T; ++k) {
            double pu = 1.0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double s;
                if constexpr (Tr::kJac) {
                    double u;
                    s = Tr::z_minus(x[k][i], p[2 * D + i], u);
                    pu = (i == 0) ? u : pu * u;
                } else {
                    s = Tr::z(x[k][i]) - p[D + i];
                }
                const double q = fma_(s, s, p[i]);
                den[k] = (i == 0) ? q : den[k] * q;
            }
            if constexpr (Tr::kJac)
                w[k] = Tr::jac(pu);
            else
                w[k] = 1.0;
        }
        if constexpr (T > 1) {
            if (p[3 * D] != 0.0) {  // the same for every thread of the launch's instance
                double r[T];
                recip_tile<T>(den, r);
#pragma unroll
                for (int k = 0; k < T; ++k) v[k][0] = w[k] * r[k];
                return;
            }
        }
#pragma unroll
        for (int k = 0; k < T; ++k) v[k][0] = w[k] * recip(den[k]);
    }
};

// Genz oscillatory cos(2 pi u_1 + sum_i a_i z_i).  blob: [a (D), 2 pi u_1]
struct FamGenzOscillatory {
    static constexpr int NP = 1;
    template <class Tr, int D, int T>
    __device__ static void eval(const double *__restrict__ p, const double (&x)[T][D],
                                double (&v)[T][NP]) {
        double z[T][D], jac[T];
        apply_transform<Tr, D, T>(x, z, jac);
#pragma unroll
        for (int k = 0; k < T; ++k) {
            double s = p[D];
#pragma unroll
            for (int i = 0; i < D; ++i) s = fma_(p[i], z[k][i], s);
            const double c = cos(s);
            v[k][0] = Tr::kJac ? c * jac[k] : c;
        }
    }
};

// Genz Gaussian exp(-sum_i a_i^2 (z_i - u_i)^2).  blob: [a^2 (D), u (D)]
struct FamGenzGaussian {
    static constexpr int NP = 1;
    template <class Tr, int D, int T>
    __device__ static void eval(const double *__restrict__ p, const double (&x)[T][D],
                                double (&v)[T][NP]) {
        double z[T][D], jac[T];
        apply_transform<Tr, D, T>(x, z, jac);
#pragma unroll
        for (int k = 0; k < T; ++k) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const double t = z[k][i] - p[D + i];
                s = fma_(p[i] * t, t, s);
            }
            const double e = qexp(-s);
            v[k][0] = Tr::kJac ? e * jac[k] : e;
        }
    }
};

// Genz continuous exp(-sum_i a_i |z_i - u_i|).  blob: [a (D), u (D)]
struct FamGenzContinuous {
    static constexpr int NP = 1;
    template <class Tr, int D, int T>
    __device__ static void eval(const double *__restrict__ p, const double (&x)[T][D],
                                double (&v)[T][NP]) {
        double z[T][D], jac[T];
        apply_transform<Tr, D, T>(x, z, jac);
#pragma unroll
        for (int k = 0; k < T; ++k) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) s = fma_(p[i], __builtin_fabs(z[k][i] - p[D + i]), s);
            const double e = qexp(-s);
            v[k][0] = Tr::kJac ? e * jac[k] : e;
        }
    }
};

// Genz corner peak (1 + sum_i a_i z_i)^-(d+1).  blob: [a (D)]
struct FamGenzCornerPeak {
    static constexpr int NP = 1;
    template <class Tr, int D, int T>
    __device__ static void eval(const double *__restrict__ p, const double (&x)[T][D],
                                double (&v)[T][NP]) {
        double z[T][D], jac[T];
        apply_transform<Tr, D, T>(x, z, jac);
#pragma unroll
        for (int k = 0; k < T; ++k) {
            double s = 1.0;
#pragma unroll
            for (int i = 0; i < D; ++i) s = fma_(p[i], z[k][i], s);
            const double r = recip(s);
            double q = r;
#pragma unroll
            for (int i = 0; i < D; ++i) q *= r;
            v[k][0] = Tr::kJac ? q * jac[k] : q;
        }
    }
};

// ---------------------------------------------------- sparse polynomials
// A monomial is coded as a 64-bit word: bits 0..3 hold the number of
// factors c (<= 12), bits 4+5f..8+5f the variable of factor f; z_i^2 is two
// factors of variable i.  The code and the coefficient are wave-uniform, so
// the factor loop and the variable selection below become scalar branches;
// only the multiplications run on the vector unit, once per shift.
// Runs f(i) for the one variable i = v in [LO, HI), choosing it by halving
// the range: ceil(log2 D) uniform branches instead of one test per variable.
template <int LO, int HI, int D, int T, class Fn>
__device__ __forceinline__ void pick_var(uint32_t v, Fn &&f) {
    if constexpr (HI - LO == 1) {
        f(LO);
    } else {
        constexpr int MID = (LO + HI) / 2;
        if (v < (uint32_t)MID)
            pick_var<LO, MID, D, T>(v, f);
        else
            pick_var<MID, HI, D, T>(v, f);
    }
}

template <int D, int T>
__device__ __forceinline__ void mul_var(double (&q)[T], const double (&z)[T][D], uint32_t v) {
    pick_var<0, D, D, T>(v, [&](int i) {
#pragma unroll
        for (int k = 0; k < T; ++k) q[k] *= z[k][i];
    });
}

template <int D, int T>
__device__ __forceinline__ void scale_var(double (&q)[T], double c, const double (&z)[T][D],
                                          uint32_t v) {
    pick_var<0, D, D, T>(v, [&](int i) {
#pragma unroll
        for (int k = 0; k < T; ++k) q[k] = c * z[k][i];
    });
}

// out[k] = sum_t coef[t] * prod_f z[k][var_f(t)]
template <int D, int T>
__device__ __forceinline__ void poly_eval(const double *__restrict__ coef,
                                          const uint64_t *__restrict__ code, uint32_t nt,
                                          const double (&z)[T][D], double (&out)[T]) {
#pragma unroll
    for (int k = 0; k < T; ++k) out[k] = 0.0;
    for (uint32_t t = 0; t < nt; ++t) {
        uint64_t c = code[t];
        const double cf = coef[t];
        const uint32_t cnt = (uint32_t)(c & 15u);
        if (cnt == 0) {
#pragma unroll
            for (int k = 0; k < T; ++k) out[k] += cf;
            continue;
        }
        c >>= 4;
        double q[T];
        scale_var<D, T>(q, cf, z, (uint32_t)(c & 31u));
        for (uint32_t f = 1; f < cnt; ++f) {
            c >>= 5;
            mul_var<D, T>(q, z, (uint32_t)(c & 31u));
        }
#pragma unroll
        for (int k = 0; k < T; ++k) out[k] += q[k];
    }
}

// out[k] = init[k] * prod_i z[k][i]^e_i with e_i = bits 2i..2i+1 of code
// (the z^nu prefactor; e_i <= 2)
template <int D, int T>
__device__ __forceinline__ void nu_eval(uint32_t code, const double (&init)[T], const double (&z)[T][D],
                                        double (&out)[T]) {
#pragma unroll
    for (int k = 0; k < T; ++k) out[k] = init[k];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const uint32_t e = (code >> (2 * i)) & 3u;
        if (e >= 1) {
#pragma unroll
            for (int k = 0; k < T; ++k) out[k] *= z[k][i];
        }
        if (e == 2) {
#pragma unroll
            for (int k = 0; k < T; ++k) out[k] *= z[k][i];
        }
    }
}

// Sector integrand prod_i z_i^nu_i * U^pow_u * (F - i delta)^pow_f (eq. (6)
// with the two Symanzik-type polynomials; -i delta as in eq. (7)).
// blob: [n_u, n_f, flags, pow_u, pow_f, delta, nu (2 bits per variable),
//        coef_u (n_u), code_u (n_u), coef_f (n_f), code_f (n_f)]
// flags bit 0: complex, bit 1: pow_u == -2 (U^-2 by reciprocal).
enum : uint32_t { kSectorComplex = 1u, kSectorPowUm2 = 2u };
// Expansion orders (qmc_integrate_orders, flag 4): three words after the F
// exponent codes hold eps_u, eps_f and the number of orders.
enum : uint32_t { kSectorOrders = 4u };
constexpr uint32_t kSectorMaxOrders = 4;
constexpr int kSectorHeader = 7;

// fhat from the polynomial values: mono = jac * prod z^nu, then
// mono * U^pow_u * (F - i delta)^pow_f with the principal branch.
template <bool Complex>
__device__ __forceinline__ void sector_finish(double mono, double U, double F, uint32_t flags,
                                              double pow_u, double pow_f, double delta,
                                              double (&v)[Complex ? 2 : 1]) {
    double pre = mono;
    double lu = 0.0;
    if (flags & kSectorPowUm2) {
        const double r = recip(U);
        pre = pre * (r * r);
    } else {
        lu = pow_u * qlog(U);
    }
    if constexpr (!Complex) {
        v[0] = pre * qexp(fma_(pow_f, qlog(F), lu));
    } else {
        // log(F - i delta) = ln|F - i delta| + i atan2(-delta, F)
        const double mod2 = fma_(F, F, delta * delta);
        const double e = fma_(0.5 * pow_f, qlog(mod2), lu);
        const double ph = pow_f * qatan2(-delta, F);
        double s, c;
        qsincos(ph, s, c);
        const double mag = pre * qexp(e);
        v[0] = mag * c;
        v[1] = mag * s;
    }
}

// Coefficients of the expansion in a regulator e of
// mono * U^(pow_u + eps_u e) * (F - i delta)^(pow_f + eps_f e):
// with f the value at e = 0 and L = eps_u ln U + eps_f ln(F - i delta)
// (principal branch), the coefficient of e^k is f L^k / k!.  Part k (real)
// or parts (2k, 2k+1) (complex) receive order k, k < NO.
template <bool Complex, int NO>
__device__ __forceinline__ void sector_orders(double mono, double U, double F, uint32_t flags, double pow_u,
                                              double pow_f, double delta, double eps_u, double eps_f,
                                              double (&v)[(Complex ? 2 : 1) * NO]) {
    const double lnu = qlog(U);
    double pre = mono;
    if (flags & kSectorPowUm2) {
        const double r = recip(U);
        pre = pre * (r * r);
    } else {
        pre = pre * qexp(pow_u * lnu);
    }
    if constexpr (!Complex) {
        const double lnf = qlog(F);
        double f = pre * qexp(pow_f * lnf);
        const double L = fma_(eps_u, lnu, eps_f * lnf);
        v[0] = f;
#pragma unroll
        for (int k = 1; k < NO; ++k) {
            f = (f * L) * (1.0 / k);
            v[k] = f;
        }
    } else {
        const double lnm = 0.5 * qlog(fma_(F, F, delta * delta));  // ln|F - i delta|
        const double th = qatan2(-delta, F);                        // arg(F - i delta)
        double s, c;
        qsincos(pow_f * th, s, c);
        const double mag = pre * qexp(pow_f * lnm);
        double fr = mag * c, fi = mag * s;
        const double lr = fma_(eps_u, lnu, eps_f * lnm), li = eps_f * th;
        v[0] = fr;
        v[1] = fi;
#pragma unroll
        for (int k = 1; k < NO; ++k) {
            const double nr = fma_(fr, lr, -fi * li), ni = fma_(fr, li, fi * lr);
            fr = nr * (1.0 / k);
            fi = ni * (1.0 / k);
            v[2 * k] = fr;
            v[2 * k + 1] = fi;
        }
    }
}

// ------------------------------------------------ contour deformation
// Sec. 3: a sector whose F changes sign inside the cube is integrated along
// z_k = x_k - i lam x_k (1 - x_k) dF/dx_k (x), which keeps the faces of the
// cube fixed and gives F(z) a negative imaginary part to first order (the
// -i0 prescription).  The integrand gains det(dz/dx).
enum : uint32_t { kSectorDeform = 8u };
// Sign check of a deformation (with flag 8): the functor returns 1 where the
// deformed F - i delta has a positive imaginary part, else 0, unweighted.
enum : uint32_t { kSectorDeformCheck = 16u };

// det(dz/dx) = det(I + i B), B_kl = -lam [s_k H_kl + delta_kl (1 - 2 x_k) g_k],
// s_k = x_k (1 - x_k), g = grad F, H = Hessian of F.  With r_k = sqrt(s_k),
// B is similar to the symmetric Bs_kl = -lam [r_k r_l H_kl + delta_kl (1 - 2 x_k) g_k]
// (a diagonal similarity, so every leading block keeps its determinant;
// r_k = 0 follows by continuity; each term of det holds r_k r_k, so a
// rounded s_k slightly below 0 may use r_k = sqrt(|s_k|)).  I + i Bs is complex symmetric with
// Hermitian part I: each leading block is nonsingular, so the LDL^T
// factorisation without pivoting exists and det = prod of the pivots.
// a holds the lower triangle of I + i Bs, row-major packed: (i, j), j <= i, at
// i (i + 1) / 2 + j; it is overwritten.
template <int D>
__device__ __forceinline__ void csym_det(double (&ar)[D * (D + 1) / 2], double (&ai)[D * (D + 1) / 2],
                                         double &dr, double &di) {
    double pr = 1.0, pi = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int kk = k * (k + 1) / 2 + k;
        const double a = ar[kk], b = ai[kk];
        {
            const double nr = fma_(pr, a, -pi * b), ni = fma_(pr, b, pi * a);
            pr = nr;
            pi = ni;
        }
        const double h = recip(fma_(a, a, b * b));
        const double vr = a * h, vi = -b * h;  // 1 / pivot
#pragma unroll
        for (int i = k + 1; i < D; ++i) {
            const int ik = i * (i + 1) / 2 + k;
            const double lr = fma_(ar[ik], vr, -ai[ik] * vi), li = fma_(ar[ik], vi, ai[ik] * vr);
#pragma unroll
            for (int j = k + 1; j <= i; ++j) {
                const int ij = i * (i + 1) / 2 + j, jk = j * (j + 1) / 2 + k;
                ar[ij] = ar[ij] - fma_(lr, ar[jk], -li * ai[jk]);
                ai[ij] = ai[ij] - fma_(lr, ai[jk], li * ar[jk]);
            }
        }
    }
    dr = pr;
    di = pi;
}

// Value (and expansion orders) of the deformed sector integrand:
// mono * det * U^pow_u * (F - i delta)^pow_f at complex mono, det, U, F, with
// the principal branch of each power; order k multiplies by L^k / k!,
// L = eps_u ln U + eps_f ln(F - i delta).  Parts (2k, 2k+1) hold order k.
template <int NO>
__device__ __forceinline__ void sector_deformed(double mr, double mi, double dr, double di, double ur, double ui,
                                                double fr, double fi, uint32_t flags, double pow_u, double pow_f,
                                                double delta, double eps_u, double eps_f, double (&v)[2 * NO]) {
    fi = fi - delta;
    // pre = mono * det
    double pr = fma_(mr, dr, -mi * di), pim = fma_(mr, di, mi * dr);
    const double lmf = 0.5 * qlog(fma_(fr, fr, fi * fi)), thf = qatan2(fi, fr);  // ln(F - i delta)
    double lmu = 0.0, thu = 0.0;
    double lm = pow_f * lmf, th = pow_f * thf;
    if ((flags & kSectorPowUm2) == 0 || NO >= 2) {
        lmu = 0.5 * qlog(fma_(ur, ur, ui * ui));
        thu = qatan2(ui, ur);
    }
    if (flags & kSectorPowUm2) {
        // 1 / U^2 = conj(U)^2 / |U|^4
        const double h = recip(fma_(ur, ur, ui * ui));
        const double qr = ur * h, qi = -ui * h;
        const double sr = fma_(qr, qr, -qi * qi), si = 2.0 * qr * qi;
        const double nr = fma_(pr, sr, -pim * si), ni = fma_(pr, si, pim * sr);
        pr = nr;
        pim = ni;
    } else {
        lm = fma_(pow_u, lmu, lm);
        th = fma_(pow_u, thu, th);
    }
    double s, c;
    qsincos(th, s, c);
    const double mag = qexp(lm);
    double wr = mag * fma_(pr, c, -pim * s), wi = mag * fma_(pr, s, pim * c);
    v[0] = wr;
    v[1] = wi;
    if constexpr (NO >= 2) {
        const double lr = fma_(eps_u, lmu, eps_f * lmf), li = fma_(eps_u, thu, eps_f * thf);
#pragma unroll
        for (int k = 1; k < NO; ++k) {
            const double nr = fma_(wr, lr, -wi * li), ni = fma_(wr, li, wi * lr);
            wr = nr * (1.0 / k);
            wi = ni * (1.0 / k);
            v[2 * k] = wr;
            v[2 * k + 1] = wi;
        }
    }
}

template <bool Complex>
struct FamSector {
    static constexpr int NP = Complex ? 2 : 1;
    template <class Tr, int D, int T>
    __device__ static void eval(const double *__restrict__ p, const double (&x)[T][D],
                                double (&v)[T][NP]) {
        double z[T][D], jac[T];
        apply_transform<Tr, D, T>(x, z, jac);
        const uint32_t nu = (uint32_t)__double_as_longlong(p[0]);
        const uint32_t nf = (uint32_t)__double_as_longlong(p[1]);
        const uint32_t flags = (uint32_t)__double_as_longlong(p[2]);
        const double pow_u = p[3], pow_f = p[4], delta = p[5];
        const uint32_t nucode = (uint32_t)__double_as_longlong(p[6]);
        const double *cu = p + kSectorHeader;
        const uint64_t *eu = reinterpret_cast<const uint64_t *>(cu + nu);
        const double *cf = cu + 2 * nu;
        const uint64_t *ef = reinterpret_cast<const uint64_t *>(cf + nf);
        double U[T], F[T], mono[T];
        poly_eval<D, T>(cu, eu, nu, z, U);
        poly_eval<D, T>(cf, ef, nf, z, F);
        nu_eval<D, T>(nucode, jac, z, mono);
#pragma unroll
        for (int k = 0; k < T; ++k) sector_finish<Complex>(mono[k], U[k], F[k], flags, pow_u, pow_f, delta, v[k]);
    }
};

}  // namespace qmc
