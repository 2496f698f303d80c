"""Batched persistent launch and autotuner on the GPU, against the oracle."""
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
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(np.asarray(b)), 1e-300)


def _sector_plans(Q, count, seed, ns, m):
    draws = synth.sector_batch_draws(seed, count)
    tabs = synth.sector_batch(seed, count)
    plans, params, cases = [], [], []
    for s, ((d, _, _), tab) in enumerate(zip(draws, tabs)):
        n = ns[s % len(ns)]
        g = O.korobov_vector(n, d, 3 + 2 * s)
        sh = synth.sector_batch_shifts(seed, s, m, d)
        plans.append(Q.Plan(d, n, g, sh, "baker"))
        params.append(Q.Params("sector", d, sector=tab))
        cases.append((d, n, g, sh, tab))
    return plans, params, cases


@pytest.mark.parametrize("use_graph,schedule", [(True, "default"), (False, "default"), (True, "persistent"),
                                               (False, "persistent"), (True, "per_tile")])
def test_sector_batch_parity(Q, use_graph, schedule):
    """Sectors of d = 2..9 and uneven n in one launch per dimension."""
    plans, params, cases = _sector_plans(Q, 24, 77, [1021, 4093, 16381, 257, 65521], 6)
    _say(f"sector batch graph={use_graph} schedule={schedule}")
    res = Q.integrate_batch(plans, params, use_graph=use_graph, tile_points=1024, schedule=schedule)
    per = Q.batch_per_shift(plans)
    for (d, n, g, sh, tab), q, r in zip(cases, per, res):
        est = O.estimate(n, g, sh, O.Params("sector", d, sector=tab), "baker", threads=THREADS)
        assert np.all(_rel(q, est.q_re) < TOL), (d, n, _rel(q, est.q_re).max())
        mean, err, _ = est.mean_error()
        assert abs(r.mean_re - mean.real) <= TOL * abs(mean.real)


def test_batch_graph_replay_and_per_plan_mode(Q):
    plans, params, cases = _sector_plans(Q, 16, 78, [4093, 16381], 8)
    _say("graph replays")
    first = Q.integrate_batch(plans, params, use_graph=True)
    q1 = Q.batch_per_shift(plans)
    for rep in range(3):
        again = Q.integrate_batch(plans, params, use_graph=True)
        qa = Q.batch_per_shift(plans)
        assert all(np.array_equal(a, b) for a, b in zip(q1, qa))
        assert [r.mean_re for r in again] == [r.mean_re for r in first]
    eager = Q.integrate_batch(plans, params, use_graph=False)
    assert [r.mean_re for r in eager] == [r.mean_re for r in first]
    # the two schedules write the same tile slots and add them in the same
    # order, so they agree bit for bit
    persist = Q.integrate_batch(plans, params, use_graph=True, schedule="persistent")
    assert [r.mean_re for r in persist] == [r.mean_re for r in first]
    _say("per-plan launches")
    pp = Q.integrate_batch(plans, params, per_plan_launches=True)
    for a, b in zip(pp, first):
        assert abs(a.mean_re - b.mean_re) <= TOL * abs(b.mean_re)
        assert abs(a.err_re - b.err_re) <= 1e-6 * abs(b.err_re) + 1e-300


def test_genz_batch(Q):
    """Product peak instances (shared g and shifts, own a and u), Korobov 3."""
    d, n, m = 4, 16381, 16
    g = O.korobov_vector(n, d, 1234)
    sh = synth.shifts(5, m, d)
    plans, params, cases = [], [], []
    for b in range(12):
        a, u = synth.genz_params(1000 + b, d)
        plans.append(Q.Plan(d, n, g, sh, "korobov", 3))
        params.append(Q.Params("genz_product_peak", d, a=a, u=u))
        cases.append((a, u))
    _say("genz batch")
    Q.integrate_batch(plans, params, tile_points=2048)
    for (a, u), q in zip(cases, Q.batch_per_shift(plans)):
        est = O.estimate(n, g, sh, O.Params("genz_product_peak", d, a=a, u=u), "korobov", 3,
                         threads=THREADS)
        assert np.all(_rel(q, est.q_re) < TOL)


@pytest.mark.parametrize("use_graph", [True, False])
def test_uniform_batch_instances(Q, use_graph):
    """Plans with one (d, n, m) run as instances of a single lattice launch.
    Every third instance has its a scaled by 1e-4 and every third by 100, so
    that instances whose shifts share one reciprocal and instances with one
    reciprocal per shift run in the same launch.  (A scale of 1e3 makes the
    peaks so sharp, a up to 8000, that one rounding of z moves f by about
    a x 1e-16 per dimension, above the 1e-12 bar whichever path runs.)"""
    d, n, m = 4, 16381, 16
    plans, params, cases = [], [], []
    for b in range(40):
        a, u = synth.genz_params(2000 + b, d)
        a = a * (1.0, 1e-4, 100.0)[b % 3]
        g = O.korobov_vector(n, d, 76 + 2 * b)
        sh = synth.shifts(2000 + b, m, d)
        plans.append(Q.Plan(d, n, g, sh, "korobov", 3))
        params.append(Q.Params("genz_product_peak", d, a=a, u=u))
        cases.append((a, u, g, sh))
    _say(f"uniform batch graph={use_graph}")
    res = Q.integrate_batch(plans, params, use_graph=use_graph)
    per = Q.batch_per_shift(plans)
    for (a, u, g, sh), q, r in zip(cases, per, res):
        est = O.estimate(n, g, sh, O.Params("genz_product_peak", d, a=a, u=u), "korobov", 3,
                         threads=THREADS)
        assert np.all(_rel(q, est.q_re) < TOL)
        assert abs(r.mean_re - est.mean_error()[0].real) <= TOL * abs(r.mean_re)


def test_complex_batch(Q):
    d, m = 4, 4
    plans, params, cases = [], [], []
    for s in range(5):
        tab = synth.sector_tables(900 + s, d, 6, 9, complex_kinematics=True)
        n = [1021, 2039][s % 2]
        g = O.korobov_vector(n, d, 5 + s)
        sh = synth.shifts(900 + s, m, d)
        plans.append(Q.Plan(d, n, g, sh, "baker"))
        params.append(Q.Params("sector", d, sector=tab))
        cases.append((n, g, sh, tab))
    _say("complex batch")
    Q.integrate_batch(plans, params, tile_points=512)
    for (n, g, sh, tab), q in zip(cases, Q.batch_per_shift(plans, complex_parts=True)):
        est = O.estimate(n, g, sh, O.Params("sector", d, sector=tab), "baker", threads=THREADS)
        assert np.all(np.abs(q - est.q) <= 1e-11 * np.abs(est.q))


def test_batch_validation(Q):
    g = O.korobov_vector(1021, 2, 5)
    p1 = Q.Plan(2, 1021, g, synth.shifts(1, 2, 2), "baker")
    p2 = Q.Plan(2, 1021, g, synth.shifts(1, 2, 2), "korobov", 3)
    prm = Q.Params("genz_gaussian", 2, a=[1.0, 2.0], u=[0.3, 0.4])
    with pytest.raises(Q.QMCError) as e:
        Q.integrate_batch([p1, p2], [prm, prm])
    assert e.value.status == Q.QMC_EINVAL
    with pytest.raises(Q.QMCError) as e:
        Q.integrate_batch([p1], [prm], tile_points=100)
    assert e.value.status == Q.QMC_EINVAL


def test_autotune(Q, tmp_path, monkeypatch):
    """The tuner picks a shape; estimates with it still match the oracle."""
    w = synth.product_peak_workload(n=65521, m=16)
    g = O.korobov_vector(w.n, w.d, 17364)
    plan = Q.Plan(w.d, w.n, g, w.shifts, "korobov", 3)
    p = Q.Params("genz_product_peak", w.d, a=w.genz_a, u=w.genz_u)
    _say("autotune product peak")
    T, bpc = plan.autotune(p)
    assert T in (2, 4, 8) and bpc in (2, 4, 8, 16, 32)
    _, q = plan.integrate(p)
    assert plan.last_launch()[0] == T
    est = O.estimate(w.n, g, w.shifts, O.Params("genz_product_peak", w.d, a=w.genz_a, u=w.genz_u),
                     "korobov", 3, threads=THREADS)
    assert np.all(_rel(q, est.q_re) < TOL)
    ws = synth.sector_workload(n=65521, m=8)
    gs = O.korobov_vector(ws.n, ws.d, 17364)
    sp = Q.Plan(ws.d, ws.n, gs, ws.shifts, "baker")
    _say("autotune sector")
    T2, _ = sp.autotune(Q.Params("sector", ws.d, sector=ws.sector))
    assert T2 in (1, 2, 4)
    _, q2 = sp.integrate(Q.Params("sector", ws.d, sector=ws.sector))
    est2 = O.estimate(ws.n, gs, ws.shifts, O.Params("sector", ws.d, sector=ws.sector), "baker",
                      threads=THREADS)
    assert np.all(_rel(q2, est2.q_re) < TOL)


def test_batch_specialised_schedule_matches_default(Q):
    """The specialised schedule (one launch per sector of its run-time
    specialised kernel) against the table-driven batch and the oracle."""
    from oracle import oracle as O
    from paper_1811_11722_amd import synth
    tabs = synth.sector_batch(synth.SEED_BASE + 3, 12)
    plans, params, lat = [], [], []
    for s, t in enumerate(tabs):
        n = 4093 if s % 2 else 16381
        g = O.korobov_vector(n, t.d, 17364 % n)
        sh = synth.sector_batch_shifts(synth.SEED_BASE + 3, s, 4, t.d)
        plans.append(Q.Plan(t.d, n, g, sh, "baker"))
        params.append(Q.Params("sector", t.d, sector=t))
        lat.append((n, g, sh))
    print("[gpu-case] batch specialised", flush=True)
    sp = Q.integrate_batch(plans, params, schedule="specialised")
    df = Q.integrate_batch(plans, params, use_graph=False, tile_points=8192)
    for a, b in zip(sp, df):
        assert abs(a.mean_re - b.mean_re) <= 1e-12 * abs(b.mean_re)
        assert abs(a.err_re - b.err_re) <= 1e-9 * abs(b.err_re) + 1e-18
    t, (n, g, sh) = tabs[3], lat[3]
    est = O.estimate(n, g, sh, O.Params("sector", t.d, sector=t), "baker")
    mean, _, _ = est.mean_error()
    assert abs(sp[3].mean_re - mean.real) <= 1e-12 * abs(mean.real)
    with pytest.raises(Q.QMCError) as e:
        Q.integrate_batch(plans[:1], [Q.Params("genz_gaussian", plans[0].d, a=np.ones(plans[0].d),
                                               u=np.full(plans[0].d, 0.5))], schedule="specialised")
    assert e.value.status == Q.QMC_EUNSUPPORTED
    for p in plans:
        p.close()


def test_batch_specialised_graph_replays(Q):
    """The specialised schedule captured into a graph: every replay (with
    eager work on the same plans between replays, and new coefficients of the
    same exponent structures, uploaded before a replay) equals the eager
    launches bit for bit; per-plan standalone calls in between, which move
    a plan's launch shape, make the next call capture afresh."""
    import dataclasses
    tabs = synth.sector_batch(synth.SEED_BASE + 3, 10)
    plans, params = [], []
    for s, t in enumerate(tabs):
        n = 4093 if s % 2 else 16381
        g = O.korobov_vector(n, t.d, 17364 % n)
        plans.append(Q.Plan(t.d, n, g, synth.sector_batch_shifts(synth.SEED_BASE + 3, s, 4, t.d), "baker"))
        params.append(Q.Params("sector", t.d, sector=t))
    _say("batch specialised graph")
    key = lambda rs: [(r.mean_re, r.err_re) for r in rs]
    eager = key(Q.integrate_batch(plans, params, use_graph=False, schedule="specialised"))
    for rep in range(3):
        got = key(Q.integrate_batch(plans, params, use_graph=True, schedule="specialised"))
        assert got == eager, rep
        # eager work on the same plans between replays
        for p, pa in zip(plans[:3], params[:3]):
            p.integrate(pa)
    # new coefficients, same structures: the graph is replayed with the new blobs
    scaled = [Q.Params("sector", t.d, sector=dataclasses.replace(t, coef_f=t.coef_f * 1.5)) for t in tabs]
    eager2 = key(Q.integrate_batch(plans, scaled, use_graph=False, schedule="specialised"))
    assert eager2 != eager
    assert key(Q.integrate_batch(plans, scaled, use_graph=True, schedule="specialised")) == eager2
    # a plan whose launch shape changed: captured again, same results
    plans[0].set_launch(2, 4)
    assert key(Q.integrate_batch(plans, scaled, use_graph=True, schedule="specialised")) == \
        key(Q.integrate_batch(plans, scaled, use_graph=False, schedule="specialised"))
    for p in plans:
        p.close()


def test_batch_context_reused(Q):
    """A repeated batch over the same plans and options replays its context
    and graph: one context built, one graph launch per call, identical
    results; another tile-size option or launch shape builds its own.
    (A context key that never matched once rebuilt buffers and graph on
    every call.)"""
    w = synth.product_peak_workload(n=16381, m=8)
    g = O.korobov_vector(w.n, w.d, 3993)
    plans, params = [], []
    for b in range(3):
        aa, uu = synth.genz_params(synth.SEED_BASE + 1, w.d, stream=16 + b)
        plans.append(Q.Plan(w.d, w.n, g, w.shifts, "korobov", 3))
        params.append(Q.Params("genz_product_peak", w.d, a=aa, u=uu))
    _say("batch context reuse")
    key = lambda rs: [(r.mean_re, r.err_re) for r in rs]
    s0 = Q.batch_stats()
    first = key(Q.integrate_batch(plans, params))
    for _ in range(3):
        assert key(Q.integrate_batch(plans, params)) == first
    s1 = Q.batch_stats()
    assert s1["contexts_built"] - s0["contexts_built"] == 1
    assert s1["graph_launches"] - s0["graph_launches"] == 4
    Q.integrate_batch(plans, params, tile_points=1024)  # tiled layout: its own context
    Q.integrate_batch(plans, params, tile_points=1024)
    plans[0].set_launch(2, 4)                            # new launch shape: rebuilt
    # another grid sums in another order: means within 1e-12; the errors come
    # from differences of the Q_k (about 1e-6 apart here, each within an ulp
    # of 2.5e3, so ~3e-7 relative), checked to 1e-5
    again = np.array(key(Q.integrate_batch(plans, params)))
    ref = np.array(first)
    assert np.all(_rel(again[:, 0], ref[:, 0]) < TOL) and np.all(_rel(again[:, 1], ref[:, 1]) < 1e-5)
    s2 = Q.batch_stats()
    assert s2["contexts_built"] - s1["contexts_built"] == 2
    assert s2["graph_launches"] - s1["graph_launches"] == 3
    for p in plans:
        p.close()


def test_batch_autotune(Q):
    """The batch autotuner returns a table-driven configuration whose graph
    batch matches the oracle within 1e-12 per shift."""
    plans, params, cases = _sector_plans(Q, 24, synth.SEED_BASE + 3, [4093, 16381], 4)
    _say("batch autotune")
    opts, ms = Q.batch_autotune(plans, params)
    assert opts["schedule"] in ("default", "persistent") and opts["use_graph"]
    assert opts["tile_points"] in (4096, 8192, 16384, 32768) and ms > 0
    Q.integrate_batch(plans, params, **opts)
    per = Q.batch_per_shift(plans)
    for (d, n, g, sh, tab), q in zip(cases, per):
        est = O.estimate(n, g, sh, O.Params("sector", d, sector=tab), "baker", threads=THREADS)
        assert np.all(_rel(q, est.q_re) < TOL)
    for p in plans:
        p.close()


def test_jit_code_object_store(Q, tmp_path):
    """With QMC_JIT_CACHE set, a compiled sector kernel is written to disk and
    a second process loads it: same per-shift sums, bit for bit."""
    import json
    import subprocess
    from paper_1811_11722_amd import synth
    os.environ["QMC_JIT_CACHE"] = str(tmp_path)
    try:
        tab = synth.sector_tables(4242, 5, 9, 17)
        g = O.korobov_vector(4093, 5, 1234)
        sh = synth.shifts(4242, 4, 5)
        plan = Q.Plan(5, 4093, g, sh, "korobov", 2)
        print("[gpu-case] jit store parent", flush=True)
        _, q = plan.integrate(Q.Params("sector", 5, sector=tab))
        plan.close()
        files = [f for f in os.listdir(tmp_path) if f.endswith(".co")]
        assert files, "no code object written"
        code = (
            "import json, numpy as np\n"
            "from oracle import oracle as O\n"
            "from paper_1811_11722_amd import qmc, synth\n"
            "tab = synth.sector_tables(4242, 5, 9, 17)\n"
            "plan = qmc.Plan(5, 4093, O.korobov_vector(4093, 5, 1234), synth.shifts(4242, 4, 5), 'korobov', 2)\n"
            "_, q = plan.integrate(qmc.Params('sector', 5, sector=tab))\n"
            "print(json.dumps([float(v) for v in q]))\n")
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        print("[gpu-case] jit store child", flush=True)
        out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=120,
                             env=dict(os.environ))
        assert out.returncode == 0, out.stderr[-2000:]
        q2 = np.array(json.loads(out.stdout.strip().splitlines()[-1]))
        assert np.array_equal(q2, q)
        assert sorted(files) == sorted(f for f in os.listdir(tmp_path) if f.endswith(".co"))
    finally:
        del os.environ["QMC_JIT_CACHE"]
