#!/usr/bin/env python3
"""Throughput of the randomly shifted rank-1 lattice estimator on one MI355X.

One step = one full estimate (eqs. (2)-(3) of arXiv:1811.11722): all n*m
lattice-point evaluations of the periodised integrand, the compensated
per-shift reductions, Q_k, the mean and the error, for one resident plan.
Inputs (generating vector, shifts, integrand tables) are in HBM before the
timed region; each step copies back m + 4 doubles.

Default workload: sector-decomposed Feynman-parameter integrand
x^nu U^-2 F^-1.3, d = 6, U with 12 and F with 30 monomials (positive
coefficients), baker's transform, n = 16777213 (largest prime < 2^24),
m = 32 shifts; synthetic seeded inputs.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "lattice-point evals/sec (FP64) + % FP64 peak; time-to-error plain vs control-variate"
FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CU x 64 FMA/clk x 2 x 2.4 GHz


def flops_per_eval(workload: str) -> float:
    """Modelled algorithmic FP64 flops per lattice-point evaluation (FMA = 2)."""
    return {"sector": 280.0, "product_peak": 91.0}[workload]


# HBM bytes per lattice-kernel launch from rocprofv3 FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0 (factors from a 256 MiB copy of known size); recorded for
# the kernel as profiled (profiles/k_lattice_sector_jit_d6_n16777213_m32.md).
TRAFFIC_BYTES = {"sector": 803840}


def make_workload(name: str):
    from paper_1811_11722_amd import synth
    if name == "sector":
        w = synth.sector_workload()
        return w, "baker", 0
    if name == "product_peak":
        w = synth.product_peak_workload()
        return w, "korobov", 3
    raise SystemExit(f"unknown workload {name}")


def params_for(qmc, w):
    if w.family == "sector":
        return qmc.Params("sector", w.d, sector=w.sector)
    return qmc.Params(w.family, w.d, a=w.genz_a, u=w.genz_u)


def oracle_params(O, w):
    if w.family == "sector":
        return O.Params("sector", w.d, sector=w.sector)
    return O.Params(w.family, w.d, a=w.genz_a, u=w.genz_u)


def cpu_baseline(w, tk, alpha, g, seconds: float):
    """The CPU oracle on a bounded sample of the same workload: the first k
    shifts at the full lattice size, k chosen to take about `seconds`."""
    from oracle import oracle as O
    O.build(force=False)
    threads = os.cpu_count() or 1
    p = oracle_params(O, w)
    t0 = time.perf_counter()
    O.estimate(w.n, g, w.shifts[:1], p, tk, alpha, threads=threads)
    t1 = time.perf_counter() - t0
    k = int(max(1, min(w.m, seconds / max(t1, 1e-6))))
    if k > 1:
        t0 = time.perf_counter()
        O.estimate(w.n, g, w.shifts[:k], p, tk, alpha, threads=threads)
        t1 = time.perf_counter() - t0
    return {"value": w.n * k / t1, "unit": "lattice-point evals/s", "cores": threads,
            "kind": "oracle", "sample": f"first {k} of {w.m} shifts at full n={w.n}, "
                                        f"{t1:.2f} s wall on {threads} threads"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sector", choices=["sector", "product_peak"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-error", action="store_true",
                    help="skip the time-to-error comparison of the plain estimator and the control variate")
    ap.add_argument("--tte-goal", type=float, default=1e-4, help="relative error goal of the time-to-error leg")
    ap.add_argument("--tile", type=int, default=0, help="shift tile override (0 = tuned/default)")
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer 4 times (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the estimator "
              "would shard the lattice points across GPUs, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_mib": args.copy_probe, "copies": 4}))
        return
    from paper_1811_11722_amd import qmc

    w, tk, alpha = make_workload(args.workload)
    print(f"[bench] workload {w.name}", file=sys.stderr, flush=True)
    a, p2, _ = qmc.korobov_search(w.n, w.d, w.candidates)
    g = qmc.korobov_vector(w.n, w.d, a)
    plan = qmc.Plan(w.d, w.n, g, w.shifts, tk, alpha)
    stream = torch.cuda.current_stream()
    plan.set_stream(stream.cuda_stream)
    if args.tile or args.blocks_per_cu:
        plan.set_launch(args.tile, args.blocks_per_cu)
    params = params_for(qmc, w)

    for _ in range(args.warmup):
        res, q = plan.integrate(params)
    print(f"[bench] warmup done: mean {res.mean_re!r} err {res.err_re!r}", file=sys.stderr,
          flush=True)
    plan.set_timing(True)
    plan.kernel_time(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res, q = plan.integrate(params)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms, launches = plan.kernel_time()
    evals = w.n * w.m
    value = evals * args.steps / wall
    avg_kernel_s = kernel_ms / max(launches, 1) / 1e3
    fpe = flops_per_eval(args.workload)
    achieved = fpe * evals / avg_kernel_s / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "lattice-point evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "d": w.d, "n": w.n, "m": w.m,
                   "transform": tk if tk != "korobov" else f"korobov{alpha}",
                   "family": w.family, "evals_per_step": evals, "generator_a": a},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": TRAFFIC_BYTES.get(args.workload), "kernel": "k_lattice",
                     "kernel_ms": avg_kernel_s * 1e3,
                     "flops_per_eval": fpe},
        "result": {"mean": res.mean_re, "err": res.err_re},
    }
    if not args.no_time_to_error and args.workload == "sector":
        # the metric's second part: wall time to a relative error goal, plain
        # estimator against the learned control variate (training included),
        # on the d = 8 sector workload, each up the ladder of primes below 2^k
        from paper_1811_11722_amd import drivers
        print("[bench] time-to-error ladders", file=sys.stderr, flush=True)
        tte = drivers.time_to_error(goal=args.tte_goal, kmax=26)
        out["time_to_error"] = {
            "goal_rel_err": args.tte_goal, "workload": f"sector_real_d{tte['d']}_nu{tte['n_u']}_nf{tte['n_f']}_baker",
            "m": tte["m"],
            "plain": {k: tte["plain"][k] for k in ("goal_met", "n", "rel_err", "seconds_at_n", "ladder_seconds")},
            "cv": {k: tte["cv"][k] for k in ("goal_met", "n", "rel_err", "seconds_at_n", "ladder_seconds",
                                             "train_seconds", "R", "K")}}
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, tk, alpha, g, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
