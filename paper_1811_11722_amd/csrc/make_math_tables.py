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

    python make_math_tables.py
"""
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


if __name__ == "__main__":
    main()
