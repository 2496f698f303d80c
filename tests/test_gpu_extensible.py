"""Embedded base-2 lattice ladders on the GPU: every rung of the ladder
(which evaluates each point once) against the oracle's direct estimate on
the same 2^k-point lattice and shifts, and the rung-wise generator search
against the oracle's P2 values."""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1811_11722_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12
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


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(b), 1e-300)


def test_ladder_product_peak(Q):
    d, m, kmin, kmax = 4, 8, 8, 14
    a_, u_ = synth.genz_params(41, d)
    lat = Q.ExtensibleLattice(d, 1093, kmax, synth.shifts(41, m, d), "korobov", 3)
    params = Q.Params("genz_product_peak", d, a=a_, u=u_)
    _say("ladder product peak")
    rungs = lat.ladder(params, kmin)
    assert [n for n, _, _ in rungs] == [1 << k for k in range(kmin, kmax + 1)]
    for n, res, q in rungs:
        est = O.estimate(n, O.korobov_vector(n, d, lat.a), lat.shifts,
                         O.Params("genz_product_peak", d, a=a_, u=u_), "korobov", 3, threads=THREADS)
        assert np.all(_rel(q, est.q_re) < TOL), (n, _rel(q, est.q_re).max())
        mean, err, _ = est.mean_error()
        assert abs(res.mean_re - mean.real) <= TOL * abs(mean.real)
    # the top rung against a direct plan on the GPU
    plan = Q.Plan(d, 1 << kmax, lat.g, lat.shifts, "korobov", 3)
    _, qd = plan.integrate(params)
    plan.close()
    assert np.all(_rel(rungs[-1][2], qd) < 1e-13)


@pytest.mark.parametrize("cplx", [False, True])
def test_ladder_sector(Q, cplx):
    """The sector family through the ladder (specialised kernel), real and
    complex (constant -i delta with positive F: no cancellation, so the
    per-shift bar stays 1e-12 although the ladder's moved shifts round the
    points differently from the direct lattice by an ulp)."""
    d, m, kmin, kmax = 6, 6, 10, 15
    tab = synth.sector_tables(77, d, 12, 30)
    if cplx:
        tab.delta_im, tab.is_complex = 0.05, True
    lat = Q.ExtensibleLattice(d, 40503, kmax, synth.shifts(77, m, d), "baker")
    _say(f"ladder sector complex={cplx}")
    rungs = lat.ladder(Q.Params("sector", d, sector=tab), kmin)
    n, res, q = rungs[-1]
    est = O.estimate(n, O.korobov_vector(n, d, lat.a), lat.shifts, O.Params("sector", d, sector=tab), "baker",
                     threads=THREADS)
    assert np.all(_rel(q, est.q) < TOL), _rel(q, est.q).max()


def test_extensible_search_against_oracle_p2(Q):
    d, kmin, kmax = 5, 8, 12
    cand = np.array([3, 5, 77, 1093, 2041, 3001, 40503, 12345], dtype=np.uint64)
    _say("extensible search")
    a, score, p2 = Q.korobov_search_extensible(kmin, kmax, d, cand)
    logs = np.zeros(cand.size)
    for k in range(kmin, kmax + 1):
        _, _, allp = O.korobov_search(1 << k, d, cand, threads=THREADS)
        logs += np.log(allp)
        assert abs(p2[k - kmin] - allp[list(cand).index(a)]) <= 1e-12 * (1 + allp.max())
    want = int(cand[int(np.argmin(logs))])
    assert a == want and abs(score - logs.min() / (kmax - kmin + 1)) < 1e-9
    with pytest.raises(Q.QMCError) as e:
        Q.korobov_search_extensible(kmin, kmax, d, np.array([4], dtype=np.uint64))
    assert e.value.status == Q.QMC_EINVAL


def test_choose_transform_rule(Q):
    """The automatic choice keeps the transform with the smallest error, and
    each candidate's estimate is the plain estimate under that transform."""
    from paper_1811_11722_amd import drivers
    d, n = 4, 16381
    tab = synth.sector_tables(88, d, 6, 10)
    params = Q.Params("sector", d, sector=tab)
    _say("choose transform")
    out = drivers.choose_transform(params, d, n, m=8, seed=88)
    errs = [r["err"] for r in out["rows"]]
    assert len(out["rows"]) == len(drivers.TRANSFORM_CHOICES)
    assert out["best"]["err"] == min(errs)
    g = drivers.GeneratingVectors(88)(n, d)
    r0 = out["rows"][3]
    plan = Q.Plan(d, n, g, synth.shifts(88, 8, d), r0["transform"], r0["alpha"])
    res, _ = plan.integrate(params)
    plan.close()
    assert res.mean_re == r0["mean_re"]
