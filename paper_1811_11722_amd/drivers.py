"""Drivers above the estimator: batches of sectors with an error-goal lattice
size rule, and throughput batches of small instances.

Every estimate runs in the HIP library (qmc_integrate / qmc_integrate_batch);
this module only chooses lattice sizes and generating vectors, builds plans
and times calls.

    python -m paper_1811_11722_amd.drivers sector_batch [--count 2000] [--out rows.jsonl]
    python -m paper_1811_11722_amd.drivers product_peak_batch [--count 512]
    python -m paper_1811_11722_amd.drivers product_peak_latency [--reps 1000]
    python -m paper_1811_11722_amd.drivers time_to_error
    python -m paper_1811_11722_amd.drivers convergence [--out rows.jsonl]
    python -m paper_1811_11722_amd.drivers cv_estimate
    python -m paper_1811_11722_amd.drivers cv_train [--workload 4|5] [--sweeps 12]
    python -m paper_1811_11722_amd.drivers fig3
    python -m paper_1811_11722_amd.drivers allocation_compare [--count 2000]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time
from typing import Dict, List, Tuple

import numpy as np

from . import qmc, synth

LADDER = synth.prime_ladder(14, 24)  # largest prime below 2^k, k = 14..24


class GeneratingVectors:
    """Korobov generating vectors chosen on the GPU by the P2 criterion, one
    per (n, d), cached."""

    def __init__(self, seed: int, candidates: int = 64):
        self.seed, self.candidates = seed, candidates
        self.cache: Dict[Tuple[int, int], np.ndarray] = {}

    def __call__(self, n: int, d: int) -> np.ndarray:
        key = (n, d)
        if key not in self.cache:
            a, _, _ = qmc.korobov_search(n, d, synth.korobov_candidates(self.seed, n, self.candidates))
            self.cache[key] = qmc.korobov_vector(n, d, a)
        return self.cache[key]


class JsonlRows:
    """Append-only JSON-lines record of finished results, one object per
    line, keyed by `key_fields`.  A rerun with the same file reuses every row
    already written, so an interrupted sweep resumes where it stopped; a last
    line cut short by a crash is dropped."""

    def __init__(self, path, key_fields):
        self.path, self.key_fields = path, tuple(key_fields)
        self.rows = {}
        if path and os.path.exists(path):
            with open(path, "rb") as f:
                data = f.read()
            keep = data[: data.rfind(b"\n") + 1]
            if len(keep) != len(data):
                with open(path, "wb") as f:
                    f.write(keep)
            for line in keep.decode().splitlines():
                if line.strip():
                    r = json.loads(line)
                    self.rows[self.key(r)] = r
        self.resumed = len(self.rows)

    def key(self, row):
        return tuple(row[f] for f in self.key_fields)

    def get(self, *key):
        return self.rows.get(tuple(key))

    def add(self, row):
        self.rows[self.key(row)] = row
        if self.path:
            with open(self.path, "a") as f:
                f.write(json.dumps(row) + "\n")
                f.flush()
                os.fsync(f.fileno())
        return row


def allocate_n(rel_err0: float, n0: int, goal: float, rate: float = 2.0) -> int:
    """Smallest ladder prime >= n0 (r0 / goal)^(1/rate), clamped to the ladder:
    the error of the baker-transformed rule falls like n^-2 (Sec. 2)."""
    if not np.isfinite(rel_err0) or rel_err0 <= goal:
        return LADDER[0]
    want = n0 * (rel_err0 / goal) ** (1.0 / rate)
    for n in LADDER:
        if n >= want:
            return n
    return LADDER[-1]


def allocate_total(sigma0, cost, n0: int, goal: float, rate=2.0, ladder=None):
    """Lattice sizes for a sum of sectors with a total error goal.

    With sector s's error sigma_s(n) = sigma0_s (n0 / n)^rate_s (a pilot at
    n0 and the sector's rate) and its time cost_s * n, minimise
    sum_s cost_s n_s subject to sum_s sigma_s(n_s)^2 <= goal^2.  The Lagrange
    condition cost_s = lam * 2 rate_s sigma_s(n_s)^2 / n_s gives
    n_s(lam) = (2 rate_s lam sigma0_s^2 n0^(2 rate_s) / cost_s)^(1 / (2 rate_s + 1));
    the total error falls as lam grows, and lam is found by bisection on
    log lam (closed form when all rates are equal).  Each n_s is then rounded
    up to the ladder (which only lowers the error) and clamped to its ends.
    rate: a scalar or one value per sector.
    Returns (sizes, continuous sizes, predicted total error of the sizes)."""
    ladder = list(LADDER if ladder is None else ladder)
    s0 = np.asarray(sigma0, dtype=np.float64)
    c = np.asarray(cost, dtype=np.float64)
    r = np.broadcast_to(np.asarray(rate, dtype=np.float64), s0.shape)
    if np.any(~np.isfinite(s0)) or np.any(c <= 0) or goal <= 0 or np.any(r <= 0):
        raise ValueError("sigma0 must be finite; cost, goal and rate positive")
    live = s0 > 0
    cont = np.full(s0.shape, float(ladder[0]))
    if np.any(live):
        sl, cl, rl = s0[live], c[live], r[live]
        b = 2.0 * rl
        ln0 = math.log(n0)

        def log_n(loglam):  # log n_s(lam), in logarithms (n0^(2 rate) overflows)
            return (np.log(b) + loglam + 2.0 * np.log(sl) + b * ln0 - np.log(cl)) / (b + 1.0)

        def log_err2(loglam):  # log of sum_s sigma_s(n_s(lam))^2
            t = 2.0 * np.log(sl) + b * (ln0 - log_n(loglam))
            mx = t.max()
            return mx + math.log(np.sum(np.exp(t - mx)))

        target = 2.0 * math.log(goal)
        lo, hi = -200.0, 200.0
        for _ in range(200):  # log err^2 is decreasing in log lam
            mid = 0.5 * (lo + hi)
            if log_err2(mid) > target:
                lo = mid
            else:
                hi = mid
        cont[live] = np.exp(log_n(hi))
    sizes = np.asarray([next((n for n in ladder if n >= v), ladder[-1]) for v in cont], dtype=np.int64)
    pred = float(np.sqrt(np.sum((s0 * (n0 / sizes.astype(np.float64)) ** r) ** 2)))
    return sizes, cont, pred


def estimate_rates(sigma_a, sigma_b, n_a: int, n_b: int, lo: float = 0.25, hi: float = 2.5):
    """Per-sector convergence rates from error estimates at two lattice
    sizes, sigma ~ n^-rate, clamped to [lo, hi] (the estimates are noisy:
    lattices of similar size can differ by orders of magnitude, Sec. 2)."""
    a = np.asarray(sigma_a, dtype=np.float64)
    b = np.asarray(sigma_b, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        rate = np.log(a / b) / math.log(n_b / n_a)
    return np.clip(np.nan_to_num(rate, nan=lo, posinf=hi, neginf=lo), lo, hi)


def _timed(fn, reps: int):
    fn()  # warm-up (uploads, graph capture)
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        ts.append(time.perf_counter() - t0)
    return out, float(np.median(ts))


def sector_batch(count: int = 2000, m: int = 16, goal: float = 1e-8, seed: int = synth.SEED_BASE + 3,
                 tile_points: int = 8192, reps: int = 3, compare: bool = True, log=None) -> dict:
    """Batched sectors: pilot estimates at n0 = 16381, the error-goal rule for
    each sector's n, then graph-replayed launches (per-tile and persistent
    schedules at tile_points, and the tiling the autotuner picks) against one
    launch per sector."""
    say = log or (lambda msg: None)
    tabs = synth.sector_batch(seed, count)
    gv = GeneratingVectors(seed)
    n0 = LADDER[0]
    params = [qmc.Params("sector", t.d, sector=t) for t in tabs]

    pilots = [qmc.Plan(t.d, n0, gv(n0, t.d), synth.shifts(seed, m, t.d, stream=16 + s, sub=3),
                       "baker") for s, t in enumerate(tabs)]
    t0 = time.perf_counter()
    pres = qmc.integrate_batch(pilots, params, tile_points=tile_points)
    t_pilot = time.perf_counter() - t0
    rel0 = [abs(r.err_re) / abs(r.mean_re) for r in pres]
    ns = [allocate_n(r, n0, goal) for r in rel0]
    for p in pilots:
        p.close()

    t0 = time.perf_counter()
    plans = [qmc.Plan(t.d, n, gv(n, t.d), synth.sector_batch_shifts(seed, s, m, t.d), "baker")
             for s, (t, n) in enumerate(zip(tabs, ns))]
    t_setup = time.perf_counter() - t0
    evals = int(sum(n * m for n in ns))
    say(f"  {count} sectors, {evals} evaluations; graph batch")
    res, t_graph = _timed(lambda: qmc.integrate_batch(plans, params, use_graph=True,
                                                     tile_points=tile_points), reps)
    say(f"  graph batch {t_graph:.3f} s; persistent")
    res_ps, t_persist = _timed(lambda: qmc.integrate_batch(plans, params, use_graph=True, tile_points=tile_points,
                                                          schedule="persistent"), reps)
    # the tiling and schedule the autotuner picks
    say(f"  persistent {t_persist:.3f} s; autotuning")
    t0 = time.perf_counter()
    tuned, tuned_device_ms = qmc.batch_autotune(plans, params)
    t_tune = time.perf_counter() - t0
    say(f"  autotuner: {tuned} ({t_tune:.1f} s)")
    _, t_tuned = _timed(lambda: qmc.integrate_batch(plans, params, **tuned), reps)
    say(f"  tuned batch {t_tuned:.3f} s")
    out = {
        "sectors": count, "m": m, "goal": goal, "tile_points": tile_points,
        "pilot_n": n0, "pilot_seconds": t_pilot,
        "n_histogram": {str(n): int(sum(1 for v in ns if v == n)) for n in sorted(set(ns))},
        "sectors_at_cap": int(sum(1 for v in ns if v == LADDER[-1])),
        "evals": evals, "setup_seconds": t_setup,
        "graph_seconds": t_graph, "graph_evals_per_s": evals / t_graph,
        "graph_persistent_seconds": t_persist, "graph_persistent_evals_per_s": evals / t_persist,
        "autotuned": dict(tuned, seconds=t_tuned, evals_per_s=evals / t_tuned, device_ms=tuned_device_ms,
                          tuning_seconds=t_tune),
        "max_rel_diff_per_tile_vs_persistent": float(max(
            abs(a.mean_re - b.mean_re) / abs(b.mean_re) for a, b in zip(res, res_ps))),
        "rel_err_max": float(max(abs(r.err_re) / abs(r.mean_re) for r in res)),
        "rel_err_median": float(np.median([abs(r.err_re) / abs(r.mean_re) for r in res])),
    }
    if compare:
        res_pp, t_pp = _timed(lambda: qmc.integrate_batch(plans, params, per_plan_launches=True),
                              reps)
        out["per_plan_seconds"] = t_pp
        out["per_plan_evals_per_s"] = evals / t_pp
        out["speedup_graph_vs_per_plan"] = t_pp / t_graph
        out["max_rel_diff_graph_vs_per_plan"] = float(max(
            abs(a.mean_re - b.mean_re) / abs(b.mean_re) for a, b in zip(res, res_pp)))
    for p in plans:
        p.close()
    return out


def sector_batch_rows(path: str, count: int = 2000, m: int = 16, goal: float = 1e-8,
                      seed: int = synth.SEED_BASE + 3, chunk: int = 250, tile_points: int = 8192,
                      log=None) -> dict:
    """Configuration 3 as a resumable sweep: pilot estimates at n0 = 16381 and
    then every sector at the lattice size the error-goal rule gives it, each
    in graph-replayed batches of `chunk` sectors, with one JSON line per
    sector and phase appended to `path` (JsonlRows: a rerun skips every
    sector already written).  Pilot rows: sector, d, pilot rel_err, allocated
    n; final rows: sector, d, n, mean, err, per-shift Q_k."""
    say = log or (lambda msg: None)
    rows = JsonlRows(path, ("phase", "sector"))
    tabs = synth.sector_batch(seed, count)
    gv = GeneratingVectors(seed)
    n0 = LADDER[0]
    t0 = time.perf_counter()
    computed = 0

    def run_chunks(phase, todo, plan_for, row_for):
        nonlocal computed
        for c0 in range(0, len(todo), chunk):
            part = todo[c0:c0 + chunk]
            plans = [plan_for(s) for s in part]
            params = [qmc.Params("sector", tabs[s].d, sector=tabs[s]) for s in part]
            res = qmc.integrate_batch(plans, params, use_graph=True, tile_points=tile_points)
            per = qmc.batch_per_shift(plans)
            for s, p, r, q in zip(part, plans, res, per):
                rows.add(row_for(s, p, r, q))
                p.close()
            computed += len(part)
            say(f"  {phase}: {c0 + len(part)}/{len(todo)} sectors, {time.perf_counter() - t0:.1f} s")

    todo = [s for s in range(count) if rows.get("pilot", s) is None]
    run_chunks("pilot", todo,
               lambda s: qmc.Plan(tabs[s].d, n0, gv(n0, tabs[s].d),
                                  synth.shifts(seed, m, tabs[s].d, stream=16 + s, sub=3), "baker"),
               lambda s, p, r, q: {"phase": "pilot", "sector": s, "d": tabs[s].d, "n": n0,
                                   "rel_err": abs(r.err_re) / abs(r.mean_re),
                                   "n_alloc": allocate_n(abs(r.err_re) / abs(r.mean_re), n0, goal)})
    todo = [s for s in range(count) if rows.get("final", s) is None]
    n_of = {s: rows.get("pilot", s)["n_alloc"] for s in range(count)}
    run_chunks("final", todo,
               lambda s: qmc.Plan(tabs[s].d, n_of[s], gv(n_of[s], tabs[s].d),
                                  synth.sector_batch_shifts(seed, s, m, tabs[s].d), "baker"),
               lambda s, p, r, q: {"phase": "final", "sector": s, "d": tabs[s].d, "n": n_of[s],
                                   "mean": r.mean_re, "err": r.err_re, "q": [float(v) for v in q]})
    finals = [rows.get("final", s) for s in range(count)]
    return {"sectors": count, "m": m, "goal": goal, "path": path, "rows_resumed": rows.resumed,
            "sectors_computed": computed, "seconds": time.perf_counter() - t0,
            "evals": int(sum(r["n"] * m for r in finals)),
            "rel_err_max": float(max(abs(r["err"]) / abs(r["mean"]) for r in finals))}


def _precompile_worker(args):
    """Compile the specialised kernels of a slice of sectors by integrating
    each once on a tiny lattice (the compiled code objects land in the
    on-disk code-object cache of the ROCm compiler, shared with the parent)."""
    seed, count, first, step, transform = args
    tabs = synth.sector_batch(seed, count)
    for s in range(first, count, step):
        t = tabs[s]
        plan = qmc.Plan(t.d, 1021, qmc.korobov_vector(1021, t.d, 76), np.full((2, t.d), 0.5), transform)
        plan.integrate(qmc.Params("sector", t.d, sector=t))
        plan.close()
    return (count - first + step - 1) // step


def precompile(seed: int, count: int, workers: int = 8, transform: str = "baker", log=None) -> float:
    """Compile the 2000 sectors' specialised kernels in `workers` processes
    (hipRTC serialises compiles inside one process); returns the wall time."""
    import multiprocessing as mp
    say = log or (lambda msg: None)
    t0 = time.perf_counter()
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        done = 0
        for k in pool.imap_unordered(_precompile_worker, [(seed, count, w, workers, transform)
                                                          for w in range(workers)]):
            done += k
            say(f"  precompiled {done}/{count} sector kernels, {time.perf_counter() - t0:.1f} s")
    return time.perf_counter() - t0


def sector_batch_specialised(count: int = 2000, m: int = 16, goal: float = 1e-8, seed: int = synth.SEED_BASE + 3,
                             tile_points: int = 8192, reps: int = 3, workers: int = 0, log=None) -> dict:
    """Configuration 3 with the run-time specialised sector kernels: the same
    pilots, lattice sizes and shifts as sector_batch; every distinct exponent
    structure is compiled once (timed separately, with progress lines), then
    the batch runs as one launch per sector of its specialised kernel, against
    the graph-replayed table-driven batch."""
    say = log or (lambda msg: None)
    if workers > 1 and not os.environ.get("QMC_JIT_CACHE"):
        import tempfile
        # compiled code objects shared between the compile processes and this one
        os.environ["QMC_JIT_CACHE"] = tempfile.mkdtemp(prefix="qmc_jit_")
    t_pre = precompile(seed, count, workers, log=log) if workers > 1 else 0.0
    tabs = synth.sector_batch(seed, count)
    gv = GeneratingVectors(seed)
    n0 = LADDER[0]
    params = [qmc.Params("sector", t.d, sector=t) for t in tabs]
    pilots = [qmc.Plan(t.d, n0, gv(n0, t.d), synth.shifts(seed, m, t.d, stream=16 + s, sub=3),
                       "baker") for s, t in enumerate(tabs)]
    pres = qmc.integrate_batch(pilots, params, tile_points=tile_points)
    ns = [allocate_n(abs(r.err_re) / abs(r.mean_re), n0, goal) for r in pres]
    # compile every structure on the small pilot lattices, reporting progress
    t0 = time.perf_counter()
    for i, (pl, pa) in enumerate(zip(pilots, params)):
        pl.integrate(pa)
        if (i + 1) % 100 == 0:
            say(f"  compiled {i + 1}/{count} sector kernels, {time.perf_counter() - t0:.1f} s")
    t_compile = time.perf_counter() - t0
    for p in pilots:
        p.close()
    plans = [qmc.Plan(t.d, n, gv(n, t.d), synth.sector_batch_shifts(seed, s, m, t.d), "baker")
             for s, (t, n) in enumerate(zip(tabs, ns))]
    evals = int(sum(n * m for n in ns))
    res_sp, t_sp = _timed(lambda: qmc.integrate_batch(plans, params, schedule="specialised"), reps)
    say(f"  specialised batch (graph) {t_sp:.3f} s")
    _, t_sp_eager = _timed(lambda: qmc.integrate_batch(plans, params, use_graph=False, schedule="specialised"), reps)
    say(f"  specialised batch (launches) {t_sp_eager:.3f} s")
    res_g, t_g = _timed(lambda: qmc.integrate_batch(plans, params, use_graph=True, tile_points=tile_points), reps)
    say(f"  table-driven graph batch {t_g:.3f} s")
    for p in plans:
        p.close()
    return {"sectors": count, "m": m, "goal": goal, "evals": evals, "precompile_workers": workers,
            "precompile_seconds": t_pre, "compile_seconds": t_compile,
            "specialised_seconds": t_sp, "specialised_evals_per_s": evals / t_sp,
            "specialised_launches_seconds": t_sp_eager,
            "graph_seconds": t_g, "graph_evals_per_s": evals / t_g,
            "max_rel_diff_specialised_vs_graph": float(max(
                abs(a.mean_re - b.mean_re) / abs(b.mean_re) for a, b in zip(res_sp, res_g)))}


def allocation_compare(count: int = 2000, m: int = 16, goal: float = 1e-8, seed: int = synth.SEED_BASE + 3,
                       tile_points: int = 8192, reps: int = 2) -> dict:
    """The per-sector error-goal rule against the total-error allocation on
    the same sectors.  Rule 1: each sector to goal relative to its own pilot
    mean (sizes from its pilot error at the assumed rate 2).  Rule 2: sizes
    minimising the modelled time sum_s cost_s n_s for the total error rule 1
    achieves, with each sector's rate estimated from pilots at two sizes and
    cost_s = 100 + 4 (n_u + n_f) FP64 flops per point.  Both run as
    graph-replayed batches."""
    tabs = synth.sector_batch(seed, count)
    gv = GeneratingVectors(seed)
    n0, n1 = LADDER[0], LADDER[2]
    params = [qmc.Params("sector", t.d, sector=t) for t in tabs]

    def pilot(n):
        plans = [qmc.Plan(t.d, n, gv(n, t.d), synth.shifts(seed, m, t.d, stream=16 + s, sub=3), "baker")
                 for s, t in enumerate(tabs)]
        res = qmc.integrate_batch(plans, params, tile_points=tile_points)
        for p in plans:
            p.close()
        return np.array([r.err_re for r in res]), np.array([r.mean_re for r in res])

    s0, q0 = pilot(n0)
    s1, _ = pilot(n1)
    rates = estimate_rates(s0, s1, n0, n1)
    cost = np.array([100.0 + 4.0 * (t.n_u + t.n_f) for t in tabs])

    def run(ns, label):
        plans = [qmc.Plan(t.d, int(n), gv(int(n), t.d), synth.sector_batch_shifts(seed, s, m, t.d), "baker")
                 for s, (t, n) in enumerate(zip(tabs, ns))]
        res, t = _timed(lambda: qmc.integrate_batch(plans, params, use_graph=True, tile_points=tile_points), reps)
        for p in plans:
            p.close()
        total = float(np.sqrt(np.sum([r.err_re ** 2 for r in res])))
        value = float(np.sum([r.mean_re for r in res]))
        return {"rule": label, "evals": int(sum(int(n) * m for n in ns)), "seconds": t,
                "modelled_cost": float(np.sum(cost * np.asarray(ns, dtype=np.float64))),
                "total": value, "total_err": total, "total_rel_err": total / abs(value),
                "sectors_at_cap": int(sum(1 for n in ns if n == LADDER[-1]))}

    per_sector = [allocate_n(abs(e) / abs(q), n0, goal) for e, q in zip(s0, q0)]
    r1 = run(per_sector, "per-sector relative goal (rate 2)")
    sizes, _, pred = allocate_total(s1, cost, n1, r1["total_err"], rates)
    r2 = run(sizes, "total-error allocation (estimated rates)")
    r2["predicted_total_err"] = pred
    return {"sectors": count, "m": m, "pilot_n": [n0, n1], "rate_median": float(np.median(rates)),
            "rate_quartiles": [float(np.percentile(rates, 25)), float(np.percentile(rates, 75))],
            "rules": [r1, r2]}


def product_peak_batch(count: int = 512, n: int = 131071, m: int = 16, d: int = 4,
                       seed: int = synth.SEED_BASE + 1, tile_points: int = 0, reps: int = 5,
                       shift_tile: int = 0, blocks_per_cu: int = 0) -> dict:
    """Throughput on many Genz product-peak instances (Korobov weight 3):
    shared generating vector and shifts, own a_i and u_i per instance.
    shift_tile / blocks_per_cu (0 = default) set the instance launch."""
    w = synth.product_peak_workload(n=n, m=m, d=d, seed=seed)
    a, _, _ = qmc.korobov_search(n, d, w.candidates)
    g = qmc.korobov_vector(n, d, a)
    plans, params = [], []
    for b in range(count):
        aa, uu = synth.genz_params(seed, d, stream=16 + b)
        plans.append(qmc.Plan(d, n, g, w.shifts, "korobov", 3))
        if shift_tile or blocks_per_cu:
            plans[-1].set_launch(shift_tile, blocks_per_cu)
        params.append(qmc.Params("genz_product_peak", d, a=aa, u=uu))
    qmc.integrate_batch(plans, params, tile_points=tile_points)  # builds and captures the batch
    plans[0].set_timing(True)
    plans[0].kernel_time(reset=True)
    res, t = _timed(lambda: qmc.integrate_batch(plans, params, tile_points=tile_points), reps)
    kms, launches = plans[0].kernel_time()
    evals = count * n * m
    for p in plans:
        p.close()
    return {"instances": count, "n": n, "m": m, "d": d, "evals": evals, "seconds": t,
            "evals_per_s": evals / t, "device_seconds": kms / max(launches, 1) / 1e3, "generator_a": a,
            "shift_tile": shift_tile, "blocks_per_cu": blocks_per_cu}


def product_peak_latency(reps: int = 1000, n: int = 131071, m: int = 16, d: int = 4,
                         seed: int = synth.SEED_BASE + 1) -> dict:
    """Latency of one Genz product-peak estimate (config 1, one instance,
    about 2 million evaluations): the estimate as a graph-replayed batch of
    one (captured by the first call), as the same batch launched without the
    graph, and as a plain qmc_integrate call; the wall time of each of
    `reps` calls (host packing, launch or replay, result copy and
    synchronisation included; median and 10th / 90th percentiles), and the
    device time of the replayed graph (HIP events on the batch stream, mean
    over the calls)."""
    w = synth.product_peak_workload(n=n, m=m, d=d, seed=seed)
    a, _, _ = qmc.korobov_search(n, d, w.candidates)
    plan = qmc.Plan(d, n, qmc.korobov_vector(n, d, a), w.shifts, "korobov", 3)
    params = qmc.Params("genz_product_peak", d, a=w.genz_a, u=w.genz_u)

    def wall(fn):
        fn()  # warm-up: uploads, graph capture
        ts = np.empty(reps)
        for r in range(reps):
            t0 = time.perf_counter()
            fn()
            ts[r] = time.perf_counter() - t0
        return {"median_us": float(np.median(ts)) * 1e6, "p10_us": float(np.percentile(ts, 10)) * 1e6,
                "p90_us": float(np.percentile(ts, 90)) * 1e6}

    graph = wall(lambda: qmc.integrate_batch([plan], [params]))
    plan.set_timing(True)
    plan.kernel_time(reset=True)
    for _ in range(reps):
        qmc.integrate_batch([plan], [params])
    kms, launches = plan.kernel_time()
    plan.set_timing(False)
    graph["device_us"] = kms / max(launches, 1) * 1e3
    batch_direct = wall(lambda: qmc.integrate_batch([plan], [params], use_graph=False))
    direct = wall(lambda: plan.integrate(params))
    res, _ = plan.integrate(params)
    plan.close()
    return {"workload": f"genz_product_peak_d{d}_korobov3_n{n}_m{m}", "evals": n * m, "reps": reps,
            "graph_replay": graph, "batch_no_graph": batch_direct, "integrate": direct, "mean": res.mean_re,
            "err": res.err_re}


def _sync():
    import torch
    torch.cuda.synchronize()  # the library calls return synchronously; kept as a guard


class CvLadderPolicy:
    """Which pass a rung of the control variate's ladder runs: the residual
    pass until `drop_after` consecutive rungs have fallen back to the plain
    estimate (the model no longer lowers the error at that resolution), the
    plain kernel from then on; drop_after = 0 keeps the residual pass."""

    def __init__(self, drop_after: int):
        self.drop_after = drop_after
        self.fallbacks = 0

    def residual_pass(self) -> bool:
        return not (self.drop_after and self.fallbacks >= self.drop_after)

    def record(self, used_cv: bool) -> None:
        self.fallbacks = 0 if used_cv else self.fallbacks + 1


def time_to_error(d: int = 8, n_u: int = 12, n_f: int = 30, seed: int = synth.SEED_BASE + 4,
                  goal: float = 1e-7, m: int = 32, R: int = 32, K: int = 12, n_train: int = 1048573,
                  kmin: int = 14, kmax: int = 30, cv_kmax: int = 28, max_sweeps: int = 12, transform=None,
                  pilot_n: int = 65521, candidates: int = 64, choices=None, cv_drop_after: int = 2,
                  log=None) -> dict:
    """Time to a relative error goal, plain estimator against the control
    variate (real sector integrand).  The periodising transform is
    `transform` = (kind, alpha), or (None) the one choose_transform picks on
    a pilot lattice of pilot_n points, timed and reported on its own.  Each
    form runs the ladder of primes below 2^k upwards (plain to kmax, the
    control variate to cv_kmax) until err / |mean| <= goal; reported: the
    wall time of the first lattice size that meets the goal (CV training
    included for the CV form) or of the last rung, the cumulative ladder
    time, and every rung.  Generating vectors (P2 search over `candidates`
    Korobov multipliers) are searched once per (n, d) beforehand (tabulated
    in practice) and their time is reported on its own; the first call of
    each form compiles its specialised kernel and is not timed.  choices:
    the candidate transforms (None: every transform choose_transform
    knows).  cv_drop_after: once that many consecutive rungs of the CV form
    have fallen back to the plain estimate (the model no longer lowers the
    error at that resolution), its later rungs run the plain kernel instead
    of the residual pass (0: never); each rung records which it ran."""
    tab = synth.sector_tables(seed, d, n_u, n_f)
    params = qmc.Params("sector", d, sector=tab)
    ladder = synth.prime_ladder(kmin, kmax)
    sh = synth.shifts(seed, m, d)
    gv = GeneratingVectors(seed, candidates=candidates)
    say = log or (lambda msg: None)
    t0 = time.perf_counter()
    for n in ladder:
        gv(n, d)
    t_search = time.perf_counter() - t0
    say(f"generating vectors for {len(ladder)} rungs: {t_search:.2f} s")
    choice, t_choice = None, 0.0
    if transform is None:
        t0 = time.perf_counter()
        choice = choose_transform(params, d, pilot_n, m=16, seed=seed, choices=choices, gv=gv)
        t_choice = time.perf_counter() - t0
        transform = (choice["best"]["transform"], choice["best"]["alpha"])
        say(f"transform choice at n={pilot_n}: {transform} ({t_choice:.2f} s)")
    tk, alpha = transform

    warm = qmc.Plan(d, ladder[0], gv(ladder[0], d), sh, tk, alpha)
    warm.integrate(params)

    def ladder_run(step, top):
        rows, cum, hit = [], 0.0, None
        for n in ladder:
            if n >= (1 << top):
                break
            plan = qmc.Plan(d, n, gv(n, d), sh, tk, alpha)
            _sync()
            t = time.perf_counter()
            res = step(plan)
            _sync()
            t = time.perf_counter() - t
            plan.close()
            cum += t
            rel = abs(res.err_re) / abs(res.mean_re)
            rows.append({"n": n, "mean": res.mean_re, "err": res.err_re, "rel_err": rel,
                         "seconds": t, "used_cv": res.used_cv, "cv_pass": getattr(res, "cv_pass", False)})
            say(f"  n={n} mean={res.mean_re!r} rel_err={rel:.3e} used_cv={res.used_cv} {t * 1e3:.2f} ms")
            if rel <= goal:
                hit = rows[-1]
                break
        return rows, cum, hit

    say("plain")
    rows_p, cum_p, hit_p = ladder_run(lambda plan: plan.integrate(params)[0], kmax)

    say("control variate: training")
    # the training sampler is specialised to the integrand like the lattice
    # kernels: compile it outside the timed region
    warm_train = qmc.Plan(d, ladder[0], gv(ladder[0], d), synth.shifts(seed, 2, d, stream=3), tk, alpha)
    warm_train.cv_samples(params)
    warm_train.close()
    train = qmc.Plan(d, n_train, gv(n_train, d), synth.shifts(seed, 2, d, stream=3), tk, alpha)
    _sync()
    t = time.perf_counter()
    W, c, rep = train.cv_train(params, R, K, max_sweeps=max_sweeps)
    _sync()
    t_train = time.perf_counter() - t
    train.close()
    say(f"  sweeps={rep.sweeps} rel_loss={rep.rel_loss:.3e} {t_train:.3f} s")
    warm.integrate_cv(params, W, c)
    warm.close()
    say("control variate: ladder")
    policy = CvLadderPolicy(cv_drop_after)

    def cv_step(plan):
        if not policy.residual_pass():
            return plan.integrate(params)[0]
        res = plan.integrate_cv(params, W, c)[0]
        res.cv_pass = True
        policy.record(bool(res.used_cv))
        return res

    rows_c, cum_c, hit_c = ladder_run(cv_step, cv_kmax)

    def summary(rows, cum, hit, extra):
        return {"goal_met": hit is not None, "n": (hit or rows[-1])["n"],
                "rel_err": (hit or rows[-1])["rel_err"],
                "seconds_at_n": (hit or rows[-1])["seconds"] + extra,
                "ladder_seconds": cum + extra, "rungs": rows}

    return {"d": d, "n_u": n_u, "n_f": n_f, "m": m, "goal": goal, "transform": f"{tk}{alpha or ''}",
            "transform_choice": None if choice is None else
            {"pilot_n": pilot_n, "seconds": t_choice,
             "rel_err": {f"{r['transform']}{r['alpha'] or ''}": r["rel_err"] for r in choice["rows"]}},
            "generating_vector_search_seconds": t_search,
            "plain": summary(rows_p, cum_p, hit_p, 0.0),
            "cv": dict(summary(rows_c, cum_c, hit_c, t_train), R=R, K=K, n_train=n_train,
                       train_seconds=t_train, train_sweeps=rep.sweeps, train_rel_loss=rep.rel_loss,
                       drop_after=cv_drop_after)}


def convergence(d: int = 10, n_u: int = 20, n_f: int = 60, seed: int = synth.SEED_BASE + 5, m: int = 32,
                kmin: int = 16, kmax: int = 30, cv_kmax: int = 30, R: int = 64, K: int = 12,
                n_train: int = 1048573, max_sweeps: int = 12, out_path: str = None, log=None) -> dict:
    """Convergence table of the complex sector integrand (F - 0.01 i,
    mixed-sign F, baker's transform) over the ladder of primes below 2^k:
    n, mean, error, relative error, wall time and lattice-point evaluations
    per second for every rung, for the plain estimator and (up to 2^cv_kmax)
    the control variate (one model per component, trained on n_train points
    of an independent lattice).  With out_path every rung and the trained
    model are appended there as JSON lines (JsonlRows), and a rerun resumes:
    rungs already written are reused, and so is the model."""
    log_rows = JsonlRows(out_path, ("form", "n"))
    w = synth.sector_workload(n=synth.largest_prime_below(1 << kmax), m=m, d=d, n_u=n_u, n_f=n_f,
                              seed=seed, complex_kinematics=True)
    params = qmc.Params("sector", d, sector=w.sector)
    gv = GeneratingVectors(seed, candidates=32)
    say = log or (lambda msg: None)

    def row(n, res, t, t_search):
        mean = complex(res.mean_re, res.mean_im)
        err = math.hypot(res.err_re, res.err_im)
        return {"n": n, "mean_re": res.mean_re, "mean_im": res.mean_im, "err_re": res.err_re,
                "err_im": res.err_im, "rel_err": err / abs(mean), "seconds": t,
                "evals_per_s": n * m / t, "search_seconds": t_search, "used_cv": res.used_cv}

    def ladder(step, top, label):
        rows = []
        for n in synth.prime_ladder(kmin, top):
            done = log_rows.get(label, n)
            if done is not None:
                rows.append({k: v for k, v in done.items() if k != "form"})
                say(f"  {label} n={n} resumed")
                continue
            ts = time.perf_counter()
            g = gv(n, d)
            t_search = time.perf_counter() - ts
            plan = qmc.Plan(d, n, g, w.shifts, "baker")
            if not rows:
                step(plan)  # compiles the specialised kernel
            _sync()
            t = time.perf_counter()
            res = step(plan)
            _sync()
            t = time.perf_counter() - t
            plan.close()
            rows.append(row(n, res, t, t_search))
            log_rows.add(dict(rows[-1], form=label))
            r = rows[-1]
            say(f"  {label} n={n} mean={complex(res.mean_re, res.mean_im)!r} rel_err={r['rel_err']:.3e} "
                f"used_cv={res.used_cv} {t * 1e3:.2f} ms {n * m / t:.3e} evals/s")
        return rows

    say("plain")
    rows_p = ladder(lambda plan: plan.integrate(params)[0], kmax, "plain")
    out = {"d": d, "n_u": n_u, "n_f": n_f, "m": m, "transform": "baker", "complex": True,
           "name": w.name, "rows": rows_p}
    if cv_kmax >= kmin:
        model = log_rows.get("cv_model", n_train)
        if model is None:
            say("control variate: training")
            train = qmc.Plan(d, n_train, gv(n_train, d), synth.shifts(seed, 2, d, stream=3), "baker")
            _sync()
            t = time.perf_counter()
            W, c, rep = train.cv_train(params, R, K, max_sweeps=max_sweeps)
            _sync()
            t_train = time.perf_counter() - t
            train.close()
            say(f"  sweeps={rep.sweeps} rel_loss={rep.rel_loss:.3e} {t_train:.3f} s")
            model = log_rows.add({"form": "cv_model", "n": n_train, "R": R, "K": K, "train_seconds": t_train,
                                  "train_sweeps": rep.sweeps, "train_rel_loss": rep.rel_loss,
                                  "W": np.asarray(W).ravel().tolist(), "c": np.asarray(c).ravel().tolist(),
                                  "W_shape": list(np.shape(W)), "c_shape": list(np.shape(c))})
        else:
            say("control variate: model resumed")
        W = np.array(model["W"]).reshape(model["W_shape"])
        c = np.array(model["c"]).reshape(model["c_shape"])
        out["cv"] = {"R": R, "K": K, "n_train": n_train, "train_seconds": model["train_seconds"],
                     "train_sweeps": model["train_sweeps"], "train_rel_loss": model["train_rel_loss"],
                     "rows": ladder(lambda plan: plan.integrate_cv(params, W, c)[0], cv_kmax, "cv")}
    out["rows_resumed"] = log_rows.resumed
    return out


def cv_estimate(d: int = 8, n_u: int = 12, n_f: int = 30, seed: int = synth.SEED_BASE + 4, n: int = 4194301,
                m: int = 32, R: int = 32, K: int = 12, n_train: int = 1048573, max_sweeps: int = 12,
                reps: int = 3) -> dict:
    """One control-variate estimate of the d = 8 sector integrand: training on
    the independent lattice, then plain and residual sums in one pass at n;
    the timed pass is the median of reps."""
    tab = synth.sector_tables(seed, d, n_u, n_f)
    params = qmc.Params("sector", d, sector=tab)
    gv = GeneratingVectors(seed)
    train = qmc.Plan(d, n_train, gv(n_train, d), synth.shifts(seed, 2, d, stream=3), "baker")
    t0 = time.perf_counter()
    W, c, rep = train.cv_train(params, R, K, max_sweeps=max_sweeps)
    t_train = time.perf_counter() - t0
    train.close()
    plan = qmc.Plan(d, n, gv(n, d), synth.shifts(seed, m, d), "baker")
    (out, plain, _, _), t_cv = _timed(lambda: plan.integrate_cv(params, W, c), reps)
    _, t_plain = _timed(lambda: plan.integrate(params), reps)
    plan.close()
    return {"d": d, "n": n, "m": m, "R": R, "K": K, "n_train": n_train, "train_seconds": t_train,
            "train_device_seconds": rep.seconds, "train_sweeps": rep.sweeps, "train_rel_loss": rep.rel_loss,
            "cv_pass_seconds": t_cv, "plain_seconds": t_plain, "used_cv": out.used_cv,
            "err_cv": out.err_re, "err_plain": plain.err_re, "mean_cv": out.mean_re, "mean_plain": plain.mean_re}


def cv_train(workload: int = 4, reps: int = 2, max_sweeps: int = 12, n_train: int = 1048573, log=None) -> dict:
    """Control-variate training alone, timed: workload 4's real d = 8 sector
    (R = 32, K = 12, the Korobov-2 transform the time-to-error run picks) or
    workload 5's complex d = 10 sector (R = 64, K = 12, baker, one model per
    component), on n_train points of the independent training lattice.  The
    first call compiles the sampler and is reported as rep 0."""
    say = log or (lambda msg: None)
    if workload == 4:
        d, R, K, seed, tk, alpha = 8, 32, 12, synth.SEED_BASE + 4, "korobov", 2
        tab = synth.sector_tables(seed, d, 12, 30)
    else:
        d, R, K, seed, tk, alpha = 10, 64, 12, synth.SEED_BASE + 5, "baker", 0
        tab = synth.sector_workload(n=16381, m=2, d=d, n_u=20, n_f=60, seed=seed, complex_kinematics=True).sector
    params = qmc.Params("sector", d, sector=tab)
    gv = GeneratingVectors(seed, candidates=8)
    plan = qmc.Plan(d, n_train, gv(n_train, d), synth.shifts(seed, 2, d, stream=3), tk, alpha)
    rows = []
    for r in range(reps):
        _sync()
        t = time.perf_counter()
        _, _, rep = plan.cv_train(params, R, K, max_sweeps=max_sweeps)
        _sync()
        t = time.perf_counter() - t
        rows.append({"wall_seconds": t, "device_seconds": rep.seconds, "sweeps": rep.sweeps,
                     "rel_loss": rep.rel_loss})
        say(f"  rep {r}: {t:.4f} s wall, {rep.seconds:.4f} s device, {rep.sweeps} sweeps, "
            f"rel_loss {rep.rel_loss:.3e}")
    plan.close()
    return {"workload": workload, "d": d, "R": R, "K": K, "n_train": n_train, "transform": f"{tk}{alpha or ''}",
            "reps": rows}


def fig3(dims=(6, 9, 10), alphas=(3, 6), kmin: int = 10, kmax: int = 26, m: int = 32,
         seed: int = synth.SEED_BASE + 6, log=None) -> dict:
    """The error study of Sec. 2 (Fig. 3): the constant 1 integrated with the
    Korobov transform of weight alpha in d dimensions, for the ladder of
    primes below 2^k.  The exact value is 1; for every (d, alpha, n) the
    reported relative error sigma / |mean| and the true error |mean - 1|.
    (The baker transform integrates a constant exactly for any lattice.)"""
    say = log or (lambda msg: None)
    rows = []
    for d in dims:
        gv = GeneratingVectors(seed + d)
        sh = synth.shifts(seed + d, m, d)
        for alpha in alphas:
            for n in synth.prime_ladder(kmin, kmax):
                plan = qmc.Plan(d, n, gv(n, d), sh, "korobov", alpha)
                res, _ = plan.integrate(qmc.Params("const", d, c=1.0))
                plan.close()
                rows.append({"d": d, "alpha": alpha, "n": n, "mean": res.mean_re, "err": res.err_re,
                             "rel_err": res.err_re / abs(res.mean_re), "true_err": abs(res.mean_re - 1.0)})
                say(f"  d={d} alpha={alpha} n={n} err={res.err_re:.3e} true={abs(res.mean_re - 1.0):.3e}")
    return {"m": m, "rows": rows}


TRANSFORM_CHOICES = [("baker", 0)] + [("korobov", a) for a in range(1, 7)] + [("sidi", m_) for m_ in range(1, 7)]


def choose_transform(params, d: int, n: int, m: int = 16, seed: int = synth.SEED_BASE + 8,
                     choices=None, gv=None) -> dict:
    """Automatic transform choice (the paper's Fig. 3 observation that the
    best periodisation depends on d and n): integrate the same lattice and
    shifts under every candidate transform and keep the smallest estimated
    error sqrt(err_re^2 + err_im^2); kernel times are reported beside it."""
    choices = TRANSFORM_CHOICES if choices is None else choices
    gv = gv or GeneratingVectors(seed)
    g = gv(n, d)
    sh = synth.shifts(seed, m, d)
    rows = []
    for tk, alpha in choices:
        plan = qmc.Plan(d, n, g, sh, tk, alpha)
        plan.integrate(params)  # compile / warm up
        plan.set_timing(True)
        plan.kernel_time(reset=True)
        res, _ = plan.integrate(params)
        ms = plan.kernel_time()[0]
        plan.close()
        err = math.hypot(res.err_re, res.err_im)
        rows.append({"transform": tk, "alpha": alpha, "mean_re": res.mean_re, "mean_im": res.mean_im,
                     "err": err, "rel_err": err / max(abs(complex(res.mean_re, res.mean_im)), 1e-300),
                     "kernel_ms": ms})
    best = min(range(len(rows)), key=lambda i: (rows[i]["err"], i))
    return {"d": d, "n": n, "m": m, "best": rows[best], "rows": rows}


def transform_study(n_list=(65521, 1048573), log=None) -> dict:
    """choose_transform on the real d = 6 sector (configuration 2's shape) and
    the complex d = 10 sector (configuration 5's shape) at two lattice sizes."""
    say = log or (lambda msg: None)
    out = []
    for label, d, n_u, n_f, cplx, seed in (("sector_real_d6", 6, 12, 30, False, synth.SEED_BASE + 2),
                                           ("sector_complex_d10", 10, 20, 60, True, synth.SEED_BASE + 5)):
        w = synth.sector_workload(n=n_list[0], m=16, d=d, n_u=n_u, n_f=n_f, seed=seed, complex_kinematics=cplx)
        params = qmc.Params("sector", d, sector=w.sector)
        for n in n_list:
            r = choose_transform(params, d, n, m=16, seed=seed)
            r["workload"] = label
            say(f"  {label} n={n}: best {r['best']['transform']}{r['best']['alpha']} rel_err={r['best']['rel_err']:.3e}")
            out.append(r)
    return {"studies": out}


def lattice_study(n: int = 1048573, d: int = 10, m: int = 32, seed: int = synth.SEED_BASE + 5, log=None) -> dict:
    """Generating vectors for the complex d = 10 sector (configuration 5's
    shape) at one n: the Korobov P2 search over 64 candidates against
    component-by-component vectors with unit and with decaying (1/s^2)
    weights.  For each: construction time, P2, and the relative error of the
    sector (baker) and of the constant under Korobov weight 3 (Fig. 3's test)."""
    say = log or (lambda msg: None)
    w = synth.sector_workload(n=n, m=m, d=d, n_u=20, n_f=60, seed=seed, complex_kinematics=True)
    params = qmc.Params("sector", d, sector=w.sector)
    vecs = []
    # the process's first library call loads the code objects: keep it out of
    # the construction times
    qmc.korobov_search(n, d, synth.korobov_candidates(seed, n, 1))
    _sync()
    t = time.perf_counter()
    a, p2k, _ = qmc.korobov_search(n, d, synth.korobov_candidates(seed, n, 64))
    vecs.append(("korobov_p2_64", qmc.korobov_vector(n, d, a), time.perf_counter() - t, p2k))
    for label, gam in (("cbc_unit", None), ("cbc_decay2", 1.0 / np.arange(1, d + 1) ** 2)):
        _sync()
        t = time.perf_counter()
        z, e2 = qmc.cbc_search(n, d, gamma=gam)
        vecs.append((label, z, time.perf_counter() - t, float(e2[-1])))
    rows = []
    for label, g, t_build, crit in vecs:
        plan = qmc.Plan(d, n, g, w.shifts, "baker")
        res, _ = plan.integrate(params)
        plan.close()
        plan = qmc.Plan(d, n, g, w.shifts, "korobov", 3)
        one, _ = plan.integrate(qmc.Params("const", d, c=1.0))
        plan.close()
        row = {"vector": label, "g": [int(v) for v in g], "build_seconds": t_build, "criterion": crit,
               "sector_rel_err": math.hypot(res.err_re, res.err_im) / abs(complex(res.mean_re, res.mean_im)),
               "const_kor3_rel_err": one.err_re / abs(one.mean_re), "const_kor3_true_err": abs(one.mean_re - 1.0)}
        rows.append(row)
        say(f"  {label}: build {t_build:.3f} s, sector rel_err {row['sector_rel_err']:.3e}, "
            f"constant (Korobov 3) rel_err {row['const_kor3_rel_err']:.3e}")
    return {"n": n, "d": d, "m": m, "korobov_p2": p2k, "rows": rows}


def sector_sum(count: int = 8, d: int = 6, n: int = 16777213, m: int = 32, seed: int = synth.SEED_BASE + 9,
               reps: int = 5, log=None) -> dict:
    """The sum of `count` d = 6 sectors (configuration 2's shape, own tables
    each) in one pass against one pass per sector; kernel times from HIP
    events, median of reps."""
    say = log or (lambda msg: None)
    tabs = [synth.sector_tables(seed + 97 * s, d, 12, 30) for s in range(count)]
    params = [qmc.Params("sector", d, sector=t) for t in tabs]
    gv = GeneratingVectors(seed)
    plan = qmc.Plan(d, n, gv(n, d), synth.shifts(seed, m, d), "baker")
    plan.integrate_sum(params)
    for pa in params:
        plan.integrate(pa)
    plan.set_timing(True)

    def kernel_ms(fn):
        ts = []
        for _ in range(reps):
            plan.kernel_time(reset=True)
            out = fn()
            ts.append(plan.kernel_time()[0])
        return out, float(np.median(ts))

    (res, _), t_sum = kernel_ms(lambda: plan.integrate_sum(params))
    singles, t_sep = kernel_ms(lambda: [plan.integrate(pa)[0] for pa in params])
    plan.close()
    total = sum(r.mean_re for r in singles)
    say(f"  sum of {count}: {t_sum:.3f} ms in one pass, {t_sep:.3f} ms in {count} passes")
    return {"count": count, "d": d, "n": n, "m": m, "sum_pass_ms": t_sum, "separate_passes_ms": t_sep,
            "sector_evals_per_s": count * n * m / (t_sum * 1e-3), "mean_sum": res.mean_re, "err_sum": res.err_re,
            "mean_of_separate": total,
            "err_of_separate_quadrature": float(np.sqrt(sum(r.err_re ** 2 for r in singles)))}


def deform(d: int = 6, n_u: int = 12, n_f: int = 30, seed: int = synth.SEED_BASE + 7, n: int = 16777213,
           m: int = 32, n_pilot: int = 65521, lam_max: float = 0.8, shrink: float = 0.5, count: int = 8,
           reps: int = 5, log=None) -> dict:
    """Contour deformation (Sec. 3) of a mixed-sign sector (F vanishes inside
    the cube) at delta = 0: lambda chosen on a pilot lattice by the sign check
    and the smallest error, then the full lattice.  For comparison the same
    sector regulated by a constant -i delta (delta = 1e-2, 1e-3) instead.
    Kernel times from HIP events on the plan's stream (median of reps)."""
    say = log or (lambda msg: None)
    tab = synth.sector_tables(seed, d, n_u, n_f, complex_kinematics=True)
    tab0 = dataclasses.replace(tab, delta_im=0.0, is_complex=True)
    gv = GeneratingVectors(seed)
    sh = synth.shifts(seed, m, d)
    pilot = qmc.Plan(d, n_pilot, gv(n_pilot, d), sh[:8], "korobov", 3)
    t0 = time.perf_counter()
    lam, pres = pilot.deform_select(qmc.Params("sector", d, sector=tab0), lam_max, shrink, count)
    t_select = time.perf_counter() - t0
    ladder = []
    for i in range(count):
        L = lam_max * shrink ** i
        frac, _ = pilot.deform_check(qmc.Params("sector", d, sector=tab0, deform=L))
        ladder.append({"lambda": L, "violations": frac})
    pilot.close()
    say(f"  selected lambda={lam} pilot mean={complex(pres.mean_re, pres.mean_im)!r} ({t_select:.2f} s)")

    def run(params, label):
        plan = qmc.Plan(d, n, gv(n, d), sh, "korobov", 3)
        plan.integrate(params)  # compiles the specialised kernel
        plan.set_timing(True)
        ks, ws = [], []
        for _ in range(reps):
            plan.kernel_time(reset=True)
            _sync()
            t = time.perf_counter()
            res, _ = plan.integrate(params)
            ws.append(time.perf_counter() - t)
            ks.append(plan.kernel_time()[0])
        launch = plan.last_launch()
        plan.close()
        k_ms, w_s = float(np.median(ks)), float(np.median(ws))
        mean = complex(res.mean_re, res.mean_im)
        row = {"label": label, "kernel_ms": k_ms, "wall_s": w_s, "evals_per_s": n * m / (k_ms * 1e-3),
               "mean_re": res.mean_re, "mean_im": res.mean_im, "err_re": res.err_re, "err_im": res.err_im,
               "rel_err": math.hypot(res.err_re, res.err_im) / abs(mean), "launch": list(launch)}
        say(f"  {label}: {k_ms:.3f} ms kernel, {row['evals_per_s']:.3e} evals/s, mean={mean!r} "
            f"rel_err={row['rel_err']:.3e}")
        return row

    rows = [run(qmc.Params("sector", d, sector=tab0, deform=lam), f"deformed lambda={lam}")]
    for delta in (1e-2, 1e-3):
        rows.append(run(qmc.Params("sector", d, sector=dataclasses.replace(tab, delta_im=delta, is_complex=True)),
                        f"-i delta, delta={delta}"))
    return {"d": d, "n_u": n_u, "n_f": n_f, "n": n, "m": m, "transform": "korobov3", "lambda": lam,
            "select_seconds": t_select, "ladder": ladder, "rows": rows}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["sector_batch", "product_peak_batch", "product_peak_latency",
                                     "time_to_error", "convergence",
                                     "cv_estimate", "fig3", "allocation_compare", "deform", "transforms",
                                     "lattices", "sector_batch_specialised", "sector_sum", "cv_train"])
    ap.add_argument("--kmax", type=int, default=0)
    ap.add_argument("--cv-kmax", type=int, default=-1, help="largest 2^k of the CV ladder (convergence)")
    ap.add_argument("--shift-tile", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--count", type=int, default=0)
    ap.add_argument("--tile-points", type=int, default=-1)
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--workers", type=int, default=0, help="compile processes (sector_batch_specialised)")
    ap.add_argument("--workload", type=int, default=4, help="4 or 5 (cv_train)")
    ap.add_argument("--reps", type=int, default=2,
                    help="training runs (cv_train); timed calls (product_peak_latency, default 1000)")
    ap.add_argument("--sweeps", type=int, default=12, help="ALS sweeps at most (cv_train)")
    ap.add_argument("--out", default=None, help="JSON-lines file of results; a rerun resumes from it "
                                                "(sector_batch, convergence)")
    args = ap.parse_args(argv)
    if args.what == "sector_batch" and args.out:
        out = sector_batch_rows(args.out, count=args.count or 2000,
                                tile_points=8192 if args.tile_points < 0 else args.tile_points,
                                log=lambda msg: print(msg, file=sys.stderr, flush=True))
    elif args.what == "sector_batch":
        out = sector_batch(count=args.count or 2000,
                           tile_points=8192 if args.tile_points < 0 else args.tile_points,
                           compare=not args.no_compare, log=lambda msg: print(msg, file=sys.stderr, flush=True))
    elif args.what == "product_peak_batch":
        out = product_peak_batch(count=args.count or 512,
                                 tile_points=0 if args.tile_points < 0 else args.tile_points,
                                 shift_tile=args.shift_tile, blocks_per_cu=args.blocks_per_cu)
    elif args.what == "product_peak_latency":
        out = product_peak_latency(reps=args.reps if args.reps > 2 else 1000)
    elif args.what == "cv_estimate":
        out = cv_estimate()
    elif args.what == "cv_train":
        out = cv_train(workload=args.workload, reps=args.reps, max_sweeps=args.sweeps,
                       log=lambda msg: print(msg, file=sys.stderr, flush=True))
    elif args.what == "allocation_compare":
        out = allocation_compare(count=args.count or 2000)
    elif args.what == "sector_sum":
        out = sector_sum(log=lambda msg: print(msg, file=sys.stderr, flush=True))
    elif args.what == "sector_batch_specialised":
        out = sector_batch_specialised(count=args.count or 2000, workers=args.workers,
                                       log=lambda msg: print(msg, file=sys.stderr, flush=True))
    elif args.what == "lattices":
        out = lattice_study(log=lambda msg: print(msg, file=sys.stderr, flush=True))
    elif args.what == "transforms":
        out = transform_study(log=lambda msg: print(msg, file=sys.stderr, flush=True))
    elif args.what == "deform":
        out = deform(log=lambda msg: print(msg, file=sys.stderr, flush=True))
    elif args.what == "fig3":
        out = fig3(kmax=args.kmax or 26, log=lambda msg: print(msg, file=sys.stderr, flush=True))
    elif args.what == "time_to_error":
        out = time_to_error(kmax=args.kmax or 30, log=lambda msg: print(msg, file=sys.stderr, flush=True))
    else:
        kmax = args.kmax or 30
        out = convergence(kmax=kmax, cv_kmax=kmax if args.cv_kmax < 0 else args.cv_kmax, out_path=args.out,
                          log=lambda msg: print(msg, file=sys.stderr, flush=True))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
