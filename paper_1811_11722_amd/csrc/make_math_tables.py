"""Writes the table of the device logarithm and exponential (qlog and qexp
in qmc_device.hpp): the initialiser of kMathTab.

Entries 2j and 2j + 1, j = 0..255 (qlog): the mantissa interval
[1/2 + j/512, 1/2 + (j+1)/512) has the midpoint c_j = 1/2 + (j + 1/2)/512;
entry 2j is ic_j = 1 / c_j rounded to double and entry 2j + 1 is
L_j = -ln(ic_j) (of the rounded ic_j) rounded to double from 40-digit
arithmetic.  For a mantissa m in that interval r = m ic_j - 1 lies in
[-1/512, 1/512] up to the rounding of ic_j, and ln m = L_j + ln(1 + r).

Entry 512 + j, j = 0..511 (qexp): 2^(j/512) rounded to double from 40-digit
arithmetic; exp(x) = 2^(k >> 9) 2^((k & 511)/512) exp(r) with
k = rint(512 x / ln 2).

With --poly it writes instead the polynomial coefficients of qatan2 and
qsincos: Chebyshev interpolants (mpmath.chebyfit, 50 digits; near-minimax)
of the smooth remainders
  atan:  P(s) = (atan(sqrt s) - sqrt s) / s^(3/2),  s in [0, tan^2(pi/8)], degree 10
  sin:   S(u) = (sin(sqrt u) - sqrt u) / u^(3/2),   u in [0, (pi/4)^2],     degree 5
  cos:   C(u) = (cos(sqrt u) - 1 + u/2) / u^2,      u in [0, (pi/4)^2],     degree 5
(highest degree first, each rounded to double), and the three-part split of
pi/2 that reduces the sine and cosine argument: two parts of 33 significant
bits and a remainder rounded to double.

    python make_math_tables.py [--poly]
"""
import sys

import mpmath

mpmath.mp.dps = 40


def main():
    print("    // qlog: {1/(1/2 + (j + 1/2)/512), -ln of it}, j = 0..255")
    for j in range(256):
        ic = 1.0 / (0.5 + (j + 0.5) / 512.0)  # IEEE division: correctly rounded
        lj = float(-mpmath.log(mpmath.mpf(ic)))
        print(f"    {ic.hex()}, {lj.hex()},")
    print("    // qexp: 2^(j/512), j = 0..511")
    for j in range(0, 512, 2):
        a = float(mpmath.power(2, mpmath.mpf(j) / 512))
        b = float(mpmath.power(2, mpmath.mpf(j + 1) / 512))
        print(f"    {a.hex()}, {b.hex()},")


def _remainder(f, at0):
    return lambda v: at0 if v == 0 else f(v)


def polynomials():
    """{name: coefficients (highest degree first) as doubles} and the
    pi/2 split, as qmc_device.hpp uses them."""
    with mpmath.workdps(50):
        def atan_p(v):
            r = mpmath.sqrt(v)
            return (mpmath.atan(r) - r) / (v * r)

        def sin_s(v):
            r = mpmath.sqrt(v)
            return (mpmath.sin(r) - r) / (v * r)

        def cos_c(v):
            r = mpmath.sqrt(v)
            return (mpmath.cos(r) - 1 + v / 2) / (v * v)

        q = (mpmath.pi / 4) ** 2
        fits = {
            "atan": (_remainder(atan_p, mpmath.mpf(-1) / 3), mpmath.tan(mpmath.pi / 8) ** 2, 10),
            "sin": (_remainder(sin_s, mpmath.mpf(-1) / 6), q, 5),
            "cos": (_remainder(cos_c, mpmath.mpf(1) / 24), q, 5),
        }
        out = {}
        for name, (f, hi, deg) in fits.items():
            coef = mpmath.chebyfit(f, [0, hi], deg + 1)
            out[name] = [float(c) for c in coef]
        half_pi = mpmath.pi / 2

        def top_bits(v, bits):
            e = int(mpmath.floor(mpmath.log(abs(v), 2)))
            scale = mpmath.mpf(2) ** (bits - 1 - e)
            return float(mpmath.nint(v * scale) / scale)

        p1 = top_bits(half_pi, 33)
        p2 = top_bits(half_pi - p1, 33)
        p3 = float(half_pi - p1 - p2)
        out["half_pi_split"] = [p1, p2, p3]
        out["two_over_pi"] = [float(2 / mpmath.pi)]
    return out


def main_poly():
    for name, vals in polynomials().items():
        print(f"{name}: " + ", ".join(v.hex() for v in vals))


if __name__ == "__main__":
    main_poly() if "--poly" in sys.argv[1:] else main()
