"""Parity at the workloads' own sizes.

- Workload 3: all 2000 pilot estimates (n = 16381, m = 16, per-sector shifts)
  run as one batch and compared per shift with the oracle; then the
  error-goal rule's lattice size for every sector, and 50 seeded sectors at
  their final size on two sampled shifts each.
- Workload 5: the complex d = 10 sector at n = 16777213, m = 32, two sampled
  shifts against the long-double oracle within the bound of its rounding
  condition.
- Control-variate residuals at workload 4's model (d = 8, R = 32, K = 12, the
  two-waves-per-SIMD kernel) and workload 5's (d = 10, complex, R = 64,
  K = 12), with seeded model weights.
"""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1811_11722_amd import drivers, synth
from parity_bounds import complex_sector_check

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
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(np.asarray(b)), 1e-300)


def test_workload3_all_pilots_and_sampled_final_sizes(Q):
    seed, count, m, goal = synth.SEED_BASE + 3, 2000, 16, 1e-8
    tabs = synth.sector_batch(seed, count)
    gv = drivers.GeneratingVectors(seed, candidates=16)
    n0 = drivers.LADDER[0]
    _say(f"workload 3: {count} pilots at n = {n0}")
    plans, params, cases = [], [], []
    for s, t in enumerate(tabs):
        g = gv(n0, t.d)
        sh = synth.shifts(seed, m, t.d, stream=16 + s, sub=3)
        plans.append(Q.Plan(t.d, n0, g, sh, "baker"))
        params.append(Q.Params("sector", t.d, sector=t))
        cases.append((g, sh))
    res = Q.integrate_batch(plans, params)
    per = Q.batch_per_shift(plans)
    worst = 0.0
    for s, (t, (g, sh), q) in enumerate(zip(tabs, cases, per)):
        est = O.estimate(n0, g, sh, O.Params("sector", t.d, sector=t), "baker", threads=THREADS)
        r = _rel(q, est.q_re)
        worst = max(worst, float(r.max()))
        assert np.all(r < TOL), (s, t.d, r.max())
    print(f"  pilots: max per-shift relative difference {worst:.3g}")
    for p in plans:
        p.close()

    # the error-goal rule, then 50 seeded sectors at their final size
    ns = [drivers.allocate_n(abs(r.err_re) / abs(r.mean_re), n0, goal) for r in res]
    pick = np.random.default_rng(31).choice(count, 50, replace=False)
    _say(f"workload 3: 50 sectors at their final n (max {max(ns[i] for i in pick)})")
    worst = 0.0
    for s in pick:
        t, n = tabs[s], ns[s]
        g = gv(n, t.d)
        sh = synth.sector_batch_shifts(seed, int(s), m, t.d)
        plan = Q.Plan(t.d, n, g, sh, "baker")
        _, q = plan.integrate(Q.Params("sector", t.d, sector=t))
        plan.close()
        rows = [0, 11]
        est = O.estimate(n, g, sh[rows], O.Params("sector", t.d, sector=t), "baker", threads=THREADS)
        r = _rel(np.asarray(q)[rows], est.q_re)
        worst = max(worst, float(r.max()))
        assert np.all(r < TOL), (int(s), t.d, n, r.max())
    print(f"  final sizes: max per-shift relative difference {worst:.3g}")


def test_workload5_shape_full_n_sampled_shifts(Q):
    n, m, d = 16777213, 32, 10
    w = synth.sector_workload(n=n, m=m, d=d, n_u=20, n_f=60, seed=synth.SEED_BASE + 5, complex_kinematics=True)
    a, _, _ = Q.korobov_search(n, d, w.candidates[:8])
    g = Q.korobov_vector(n, d, a)
    plan = Q.Plan(d, n, g, w.shifts, "baker")
    _say(f"workload 5 shape at n = {n}, m = {m}")
    res, q = plan.integrate(Q.Params("sector", d, sector=w.sector))
    plan.close()
    rows = [0, 17]
    complex_sector_check(np.asarray(q)[rows], n, g, w.shifts[rows], w.sector, label="workload 5, n = 2^24 - 3")


def _seeded_model(seed, nm, R, d, K):
    rng = np.random.default_rng(seed)
    W = rng.normal(size=(nm, R, d, K)) / np.sqrt(K)
    W[:, :, :, 0] += 1.0
    c = rng.normal(size=(nm, R)) * 1e-3
    return (W[0], c[0]) if nm == 1 else (W, c)


def test_cv_residual_workload4_model(Q):
    """Real d = 8 sector of workload 4's family, R = 32, K = 12 (the
    two-waves-per-SIMD residual kernel), seeded weights."""
    d, n, m, R, K = 8, 65521, 8, 32, 12
    seed = synth.SEED_BASE + 4
    tab = synth.sector_tables(seed, d, 12, 30)
    g = O.korobov_vector(n, d, 17364)
    sh = synth.shifts(seed, m, d)
    W, c = _seeded_model(81, 1, R, d, K)
    plan = Q.Plan(d, n, g, sh, "baker")
    _say(f"cv residual d={d} R={R} K={K} n={n}")
    out, plain, qp, qr = plan.integrate_cv(Q.Params("sector", d, sector=tab), W, c)
    plan.close()
    ep = O.estimate(n, g, sh, O.Params("sector", d, sector=tab), "baker", threads=THREADS)
    er = O.estimate(n, g, sh, O.Params("sector", d, sector=tab, cv=(W, c)), "baker", threads=THREADS)
    scale = np.maximum(np.abs(ep.q_re), np.abs(er.q_re))
    print(f"  plain {np.max(_rel(qp, ep.q_re)):.3g}, residual {np.max(np.abs(qr - er.q_re) / scale):.3g}")
    assert np.all(_rel(qp, ep.q_re) <= TOL)
    assert np.all(np.abs(qr - er.q_re) <= TOL * scale)


def test_cv_residual_workload5_model(Q):
    """Complex d = 10 sector of workload 5's family, one model per component,
    R = 64, K = 12, seeded weights: the plain part against the long-double
    oracle within its rounding-condition bound, the residual within the same
    bound plus 1e-12 of the model's share."""
    d, n, m, R, K = 10, 16381, 6, 64, 12
    w = synth.sector_workload(n=n, m=m, d=d, n_u=20, n_f=60, seed=synth.SEED_BASE + 5, complex_kinematics=True)
    g = O.korobov_vector(n, d, 5029)
    W, c = _seeded_model(82, 2, R, d, K)
    plan = Q.Plan(d, n, g, w.shifts, "baker")
    _say(f"cv residual complex d={d} R={R} K={K}")
    out, plain, qp, qr = plan.integrate_cv(Q.Params("sector", d, sector=w.sector), W, c)
    plan.close()
    est = complex_sector_check(qp, n, g, w.shifts, w.sector, label="cv plain part")
    er = O.estimate(n, g, w.shifts, O.Params("sector", d, sector=w.sector, cv=(W, c), precise=True), "baker",
                    threads=THREADS)
    u = 2.0 ** -53
    bound = u * ((d + 11) * est.q_cond + 32 * est.q_abs) + TOL * np.abs(er.q - est.q)
    diff = np.abs(qr - er.q)
    print(f"  residual max |dQ|/bound {np.max(diff / bound):.3g}")
    assert np.all(diff <= bound)
