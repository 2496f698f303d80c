"""The estimate that allocates no device memory (qmc_integrate_static)
against the plan-based entry point and the oracle.

Calls run back to back on the library's one static device array, the later
ones with smaller inputs (fewer shifts, smaller n and d), so a stale region
from an earlier call would show up as a mismatch."""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1811_11722_amd import synth

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


def _check(q_static, q_plan, q_oracle):
    qs, qp, qo = np.asarray(q_static), np.asarray(q_plan), np.asarray(q_oracle)
    rel_plan = np.max(np.abs(qs - qp) / np.abs(qp))
    rel_or = np.max(np.abs(qs - qo) / np.abs(qo))
    print(f"  static vs plan {rel_plan:.3g} (bitwise {np.array_equal(qs, qp)}), vs oracle {rel_or:.3g}")
    assert rel_plan <= 1e-12
    assert rel_or <= 1e-12


def test_static_matches_plan_twice_shrinking(Q):
    # 1: workload 1 (product peak, d = 4, Korobov 3, n = 131071, m = 16)
    w = synth.product_peak_workload()
    g = O.korobov_vector(w.n, w.d, 5029)
    pq = Q.Params("genz_product_peak", w.d, a=w.genz_a, u=w.genz_u)
    _say("static product peak n=131071 m=16")
    r1, q1 = Q.integrate_static(w.d, w.n, g, w.shifts, pq, "korobov", 3)
    plan = Q.Plan(w.d, w.n, g, w.shifts, "korobov", 3)
    rp, qp = plan.integrate(pq)
    eo = O.estimate(w.n, g, w.shifts, O.Params("genz_product_peak", w.d, a=w.genz_a, u=w.genz_u), "korobov", 3,
                    threads=THREADS)
    _check(q1, qp, eo.q_re)
    assert abs(r1.mean_re - rp.mean_re) <= 1e-12 * abs(rp.mean_re)
    assert abs(r1.err_re - rp.err_re) <= 1e-9 * rp.err_re

    # 2: smaller -- a real sector, d = 3, n = 4093, m = 8, baker, against the
    # plan's table-driven kernel (the same one the static entry runs)
    d, n, m = 3, 4093, 8
    tab = synth.sector_tables(91, d, 6, 9)
    g2 = O.korobov_vector(n, d, 1077)
    sh = synth.shifts(91, m, d)
    ps = Q.Params("sector", d, sector=tab)
    _say("static sector d=3 n=4093 m=8")
    r2, q2 = Q.integrate_static(d, n, g2, sh, ps, "baker")
    plan2 = Q.Plan(d, n, g2, sh, "baker")
    plan2.set_jit(0)
    rp2, qp2 = plan2.integrate(ps)
    eo2 = O.estimate(n, g2, sh, O.Params("sector", d, sector=tab), "baker", threads=THREADS)
    _check(q2, qp2, eo2.q_re)

    # 3: smaller again and complex -- d = 2, n = 1021, m = 4
    d, n, m = 2, 1021, 4
    tab = synth.sector_tables(92, d, 3, 5, complex_kinematics=True)
    g3 = O.korobov_vector(n, d, 76)
    sh = synth.shifts(92, m, d)
    pc = Q.Params("sector", d, sector=tab)
    _say("static complex sector d=2 n=1021 m=4")
    r3, q3 = Q.integrate_static(d, n, g3, sh, pc, "baker")
    assert r3.is_complex == 1
    plan3 = Q.Plan(d, n, g3, sh, "baker")
    plan3.set_jit(0)
    rp3, qp3 = plan3.integrate(pc)
    eo3 = O.estimate(n, g3, sh, O.Params("sector", d, sector=tab), "baker", threads=THREADS)
    _check(q3, qp3, eo3.q)


def test_static_limits(Q):
    d, n = 2, 1021
    g = O.korobov_vector(n, d, 76)
    pg = Q.Params("genz_gaussian", d, a=[1.0, 2.0], u=[0.2, 0.3])
    _say("static limits")
    st, _, _ = Q.integrate_static(d, n, g, synth.shifts(1, 65, d), pg, "baker", status_only=True)
    assert st == Q.QMC_EUNSUPPORTED  # m > 64
    terms = 3000  # 2 + 3000 (2 + d) doubles > 8192
    rng = np.random.default_rng(1)
    trig = (1.0, rng.integers(1, 5, (terms, d)), rng.random(terms), rng.random(terms))
    st, _, _ = Q.integrate_static(d, n, g, synth.shifts(1, 4, d), Q.Params("trig", d, trig=trig), "baker",
                                  status_only=True)
    assert st == Q.QMC_EUNSUPPORTED
    st, _, _ = Q.integrate_static(d, n, g, synth.shifts(1, 1, d), pg, "baker", status_only=True)
    assert st == Q.QMC_EINVAL  # m = 1
    # a valid call after the rejected ones still works
    r, q = Q.integrate_static(d, n, g, synth.shifts(1, 4, d), pg, "baker")
    eo = O.estimate(n, g, synth.shifts(1, 4, d), O.Params("genz_gaussian", d, a=[1.0, 2.0], u=[0.2, 0.3]),
                    "baker")
    assert np.max(np.abs(q - eo.q_re) / np.abs(eo.q_re)) <= 1e-12
