"""Parity bounds shared by the GPU tests (no tests here)."""
import os

import numpy as np

from oracle import oracle as O

THREADS = min(16, os.cpu_count() or 1)


U64 = 2.0 ** -53


def complex_sector_check(q_gpu, n, g, sh, tab, tk="baker", alpha=0, label=""):
    """GPU Q_k of a mixed-sign complex sector against the oracle in long
    double (precise mode), within a bound derived from the rounding
    condition of the sector at every point.

    In double precision U and F are sums of terms up to ~100 that cancel to
    |F - i delta| ~ 0.01 near F's zero set.  The GPU forms F by multivariate
    Horner: every term passes at most d + deg + 1 fused multiply-adds (deg
    <= 3 is the monomials' total degree), and its coordinates are within two
    units of the oracle's, moving each term by at most 2 deg units; so
    |dF| <= (d + 3 deg + 2) u S_F, S_F the sum of the terms' magnitudes, and
    likewise U.  The value moves by (|pU| dU / |U| + |pF| dF / |F - i delta|)
    relative, plus a few units for the transform, the logarithm and
    exponential and the products (32 u counted).  Summed over the points:
      |dQ_k| <= u ((d + 11) q_cond_k + 32 q_abs_k),
    q_cond_k = (1/n) sum_j |fhat_j| c_j and c_j the condition the oracle
    computes per point (O.sector_condition).  The achieved difference is
    printed beside the bound."""
    d = tab.d
    est = O.estimate(n, g, sh, O.Params("sector", d, sector=tab, precise=True), tk, alpha, threads=THREADS,
                     condition=True)
    assert est.status == 0
    qo = est.q
    bound = U64 * ((d + 11) * est.q_cond + 32 * est.q_abs)
    diff = np.abs(np.asarray(q_gpu) - qo)
    print(f"  {label} max |dQ|/|Q| {np.max(diff / np.abs(qo)):.3g}, max |dQ|/bound {np.max(diff / bound):.3g}, "
          f"bound/|Q| up to {np.max(bound / np.abs(qo)):.3g}")
    assert np.all(diff <= bound), (np.max(diff / bound), np.max(diff / np.abs(qo)))
    return est
