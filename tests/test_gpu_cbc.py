"""GPU component-by-component generating vectors against the oracle's.

The chosen components are integers decided by floating-point sums, computed
in FP64 double-double on the GPU and in long double on the host; they must be
equal, and the squared worst-case errors must agree on the scale of 1 + e^2
(the criterion is a mean of products near 1 minus 1).
"""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def Q():
    O.build(force=False)
    from paper_1811_11722_amd import qmc
    qmc.lib()
    return qmc


@pytest.mark.parametrize("n,d", [(2, 3), (31, 4), (1021, 6), (4093, 8), (16381, 8)])
@pytest.mark.parametrize("weights", ["unit", "decaying"])
def test_cbc_matches_oracle(Q, n, d, weights):
    gam = np.ones(d) if weights == "unit" else 1.0 / np.arange(1, d + 1) ** 2
    _say(f"cbc n={n} d={d} {weights}")
    z, e2 = Q.cbc_search(n, d, gamma=gam)
    zo, e2o = O.cbc(n, d, gamma=gam, threads=THREADS)
    assert list(z) == list(zo), (z, zo)
    assert np.all(np.abs(e2 - e2o) <= 1e-14 * (1 + np.abs(e2o))), np.abs(e2 - e2o).max()


def test_cbc_candidate_subset_and_composite_n(Q):
    """A caller's candidate subset (unsorted, with a duplicate) and a
    composite n (only units are admissible)."""
    n, d = 4096, 5
    cand = np.array([1001, 3, 1001, 517, 2047, 77, 1235], dtype=np.uint64)
    _say("cbc subset n=4096")
    z, e2 = Q.cbc_search(n, d, cand=cand)
    assert z[0] == 1 and all(int(c) in set(int(v) for v in cand) for c in z[1:])
    for s in range(1, d):
        vals = [O.p2(n, np.concatenate([z[:s], [c]])) for c in sorted(set(int(v) for v in cand))]
        assert abs(e2[s] - min(vals)) <= 1.1e-13 * (1 + min(vals))
    with pytest.raises(Q.QMCError) as e:
        Q.cbc_search(n, d, cand=np.array([2, 3], dtype=np.uint64))
    assert e.value.status == Q.QMC_EINVAL


def test_cbc_full_size_against_p2(Q):
    """n = 2^20 - 3, d = 10, every candidate: the final unit-weight error is
    the P2 of the vector (oracle P2 over all n points), it grows with s, and
    sampled other candidates for the last component are no better."""
    n, d = 1048573, 10
    _say("cbc full n=1048573 d=10")
    z, e2 = Q.cbc_search(n, d)
    assert np.all(np.diff(e2) > 0)
    p2 = O.p2(n, z, threads=THREADS)
    assert abs(e2[-1] - p2) <= 1e-13 * (1 + p2)
    rng = np.random.default_rng(5)
    for c in rng.integers(1, n // 2, size=3):
        other = O.p2(n, np.concatenate([z[:-1], [c]]), threads=THREADS)
        assert other >= e2[-1] - 1e-13 * (1 + other)
