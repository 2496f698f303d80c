"""Embedded lattices in base 2 (host logic, no GPU): the nesting that the
ladder relies on, checked in exact rationals, and the merge of two
half-lattice estimates."""
from fractions import Fraction

import numpy as np
import pytest

from paper_1811_11722_amd import synth


def _points(n, g, shift):
    return sorted(tuple((Fraction(j * gi % n, n) + s) % 1 for gi, s in zip(g, shift)) for j in range(n))


@pytest.mark.parametrize("k", [1, 3, 5])
def test_odd_points_are_the_moved_half_lattice(k):
    """{j g / 2n + D} over j < 2n equals {j g / n + D} together with
    {j g / n + D + (g mod 2n) / 2n}, as exact point sets."""
    n = 1 << k
    g_full = [1, 13, 13 * 13 % 256, 13 ** 3 % 256]
    D = [Fraction(3, 7), Fraction(1, 5), Fraction(0), Fraction(6, 11)]
    g2 = [v % (2 * n) for v in g_full]
    g1 = [v % n for v in g_full]
    moved = [(d + Fraction(v, 2 * n)) % 1 for d, v in zip(D, g2)]
    assert _points(2 * n, g2, D) == sorted(_points(n, g1, D) + _points(n, g1, moved))


def test_lattice_merge_matches_the_estimator():
    from paper_1811_11722_amd import qmc
    rng = np.random.default_rng(3)
    m = 7
    for np_ in (1, 2):
        a, b = rng.normal(size=m * np_), rng.normal(size=m * np_)
        out = np.zeros(m * np_)
        res = qmc.qmc_result()
        qmc.check(qmc.lib().qmc_lattice_merge(m, np_, qmc._p(a), qmc._p(b), qmc._p(out), qmc.C.byref(res)), "merge")
        q = (a + b) / 2
        assert np.allclose(out, q, rtol=0, atol=1e-16)
        for p, (mean, err) in enumerate([(res.mean_re, res.err_re), (res.mean_im, res.err_im)][:np_]):
            col = q[p::np_]
            assert abs(mean - col.mean()) < 1e-15
            assert abs(err - col.std(ddof=1) / np.sqrt(m)) < 1e-15
    st = qmc.lib().qmc_lattice_merge(1, 1, qmc._p(a), qmc._p(b), qmc._p(out), qmc.C.byref(res))
    assert st == qmc.QMC_EINVAL
