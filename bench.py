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
m = 32 shifts; synthetic seeded inputs.  Prints one JSON line, which also
carries the metric's other parts, each on its own workload:
- product_peak_batch512: 512 Genz product-peak instances (d = 4,
  Korobov weight 3, n = 131071, m = 16) in one launch, and the latency of
  one instance (graph replay and plain call, median of 1000);
- sector_complex_d10: the complex sector (d = 10, U 20 / F 60 monomials,
  mixed-sign F - 0.01i, baker) at n = 1073741789, m = 32;
- time_to_error: wall time to a relative error of 1e-7 on the d = 8 sector,
  plain estimator against the learned control variate, with the transform
  picked automatically (the control variate's ladder runs the plain kernel
  once two consecutive rungs have fallen back; `cv_pass` marks the rungs
  that ran the residual pass);
- cpu_baseline: the CPU oracle at 1 thread and at the machine's CPU share.
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
CPU_THREADS_MAX = 16            # the host CPU share of one GPU on the measurement boxes

# Modelled algorithmic FP64 flops per evaluation (FMA = 2) and the FP64 flops
# the counters count per evaluation (SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes per
# wave-evaluation, rocprofv3 --pmc on the same launches; profiles/ holds the
# runs), per workload.
FLOPS_MODEL = {"sector": 280.0, "product_peak": 91.0, "sector_complex": 540.0}
FLOPS_COUNTED = {"sector": 163.95, "product_peak": 71.4, "sector_complex": 371.8}
# engine cycles of one launch of the headline kernel: GRBM_GUI_ACTIVE per XCD
# (rocprofv3 --pmc, profiles/); divided by the kernel time measured here it
# gives the clock the kernel ran at
CYCLES_PER_XCD = {"sector": 4.678e6}

# HBM bytes per lattice-kernel launch from rocprofv3 FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0 (factors from a 256 MiB copy of known size); recorded for
# the kernel as profiled (profiles/k_lattice_sector_jit_d6_n16777213_m32.md).
TRAFFIC_BYTES = {"sector": 803226}


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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, tk, alpha, g, seconds: float):
    """The CPU oracle on a bounded sample of the same workload: the first k
    shifts at the full lattice size, k chosen to take about `seconds`, at the
    box's CPU share of threads; and one shift on one thread."""
    from oracle import oracle as O
    O.build(force=False)
    threads = max(1, min(CPU_THREADS_MAX, os.cpu_count() or 1))
    p = oracle_params(O, w)
    t0 = time.perf_counter()
    O.estimate(w.n, g, w.shifts[:1], p, tk, alpha, threads=1)
    t_one = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.estimate(w.n, g, w.shifts[:1], p, tk, alpha, threads=threads)
    t1 = time.perf_counter() - t0
    k = int(max(1, min(w.m, seconds / max(t1, 1e-6))))
    if k > 1:
        t0 = time.perf_counter()
        O.estimate(w.n, g, w.shifts[:k], p, tk, alpha, threads=threads)
        t1 = time.perf_counter() - t0
    return {"value": w.n * k / t1, "unit": "lattice-point evals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {k} of {w.m} shifts at full n={w.n}, {t1:.2f} s wall on {threads} threads; "
                      f"1 shift on 1 thread {t_one:.2f} s",
            "value_1thread": w.n / t_one, "cpu_model": cpu_model(), "cpu_count": os.cpu_count()}


def roofline_fields(workload: str, evals: float, seconds: float) -> dict:
    fm, fc = FLOPS_MODEL[workload], FLOPS_COUNTED[workload]
    return {"flops_per_eval_model": fm, "counted_flops_per_eval": fc,
            "frac_model": fm * evals / seconds / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
            "frac_counted": fc * evals / seconds / 1e12 / FP64_VECTOR_PEAK_TFLOPS}


def leg_product_peak_batch(qmc, drivers):
    """Workload 1 on 512 seeded instances (own a_i, u_i; shared g and shifts)
    in one multi-instance launch: median wall time of 5 batches, and the
    batch's device time (HIP events around its graph on the batch stream)
    for the roofline."""
    r = drivers.product_peak_batch(count=512, reps=5)
    out = {"workload": "genz_product_peak_d4_korobov3_n131071_m16_x512", "evals": r["evals"],
           "seconds": r["seconds"], "evals_per_s": r["evals_per_s"], "device_ms": r["device_seconds"] * 1e3,
           "device_evals_per_s": r["evals"] / r["device_seconds"]}
    out.update(roofline_fields("product_peak", r["evals"], r["device_seconds"]))
    # one instance: latency of a graph replay and of a plain call, median of 1000
    lat = drivers.product_peak_latency(reps=1000)
    out["single_instance"] = {k: lat[k] for k in ("workload", "evals", "reps", "graph_replay", "batch_no_graph",
                                                   "integrate")}
    return out


def leg_complex_d10(qmc, steps: int):
    """Workload 5 (complex sector, d = 10) at its full lattice size, plain
    estimator: the plan's kernel time (HIP events) and wall time per
    estimate over `steps` estimates after one warm-up."""
    import torch
    from paper_1811_11722_amd import synth
    w = synth.sector_workload(n=1073741789, m=32, d=10, n_u=20, n_f=60, seed=synth.SEED_BASE + 5,
                              complex_kinematics=True)
    a, _, _ = qmc.korobov_search(w.n, w.d, w.candidates[:8])
    plan = qmc.Plan(w.d, w.n, qmc.korobov_vector(w.n, w.d, a), w.shifts, "baker")
    params = qmc.Params("sector", w.d, sector=w.sector)
    res, _ = plan.integrate(params)
    if not plan.last_launch()[2]:
        raise SystemExit("the complex sector did not run its run-time specialised kernel")
    plan.set_timing(True)
    plan.kernel_time(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res, _ = plan.integrate(params)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    kms, launches = plan.kernel_time()
    ks = kms / max(launches, 1) / 1e3
    evals = w.n * w.m
    out = {"workload": w.name, "evals": evals, "seconds_per_estimate": wall, "kernel_ms": ks * 1e3,
           "evals_per_s": evals / wall, "mean": [res.mean_re, res.mean_im], "err": [res.err_re, res.err_im]}
    out.update(roofline_fields("sector_complex", evals, ks))
    plan.close()
    return out


def leg_time_to_error(drivers, goal: float):
    tte = drivers.time_to_error(goal=goal, kmax=30, cv_kmax=28, candidates=16,
                                choices=[("baker", 0), ("korobov", 2), ("korobov", 3), ("korobov", 4)])
    keep = ("goal_met", "n", "rel_err", "seconds_at_n", "ladder_seconds")
    return {"goal_rel_err": goal, "transform": tte["transform"],
            "workload": f"sector_real_d{tte['d']}_nu{tte['n_u']}_nf{tte['n_f']}", "m": tte["m"],
            "transform_choice": tte["transform_choice"],
            "plain": {k: tte["plain"][k] for k in keep},
            "cv": dict({k: tte["cv"][k] for k in keep},
                       **{k: tte["cv"][k] for k in ("train_seconds", "train_rel_loss", "R", "K", "drop_after")},
                       used_cv=[r["used_cv"] for r in tte["cv"]["rungs"]],
                       cv_pass=[int(r["cv_pass"]) for r in tte["cv"]["rungs"]])}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sector", choices=["sector", "product_peak"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-error", action="store_true",
                    help="skip the time-to-error comparison of the plain estimator and the control variate")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the product-peak batch and the complex d = 10 legs")
    ap.add_argument("--tte-goal", type=float, default=1e-7, help="relative error goal of the time-to-error leg")
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
    from paper_1811_11722_amd import drivers, qmc

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
    if w.family == "sector" and not plan.last_launch()[2]:
        raise SystemExit("the sector estimate did not run its run-time specialised kernel "
                         "(hipRTC unavailable?): refusing to report the table-driven fallback")
    print(f"[bench] warmup done: mean {res.mean_re!r} err {res.err_re!r}", file=sys.stderr, flush=True)
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
    fpe = FLOPS_MODEL[args.workload]
    achieved = fpe * evals / avg_kernel_s / 1e12
    rf = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
          "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
          "traffic": TRAFFIC_BYTES.get(args.workload), "kernel": "k_lattice",
          "kernel_ms": avg_kernel_s * 1e3, "flops_per_eval": fpe,
          "counted_flops_per_eval": FLOPS_COUNTED[args.workload],
          "achieved_counted": FLOPS_COUNTED[args.workload] * evals / avg_kernel_s / 1e12,
          "frac_counted": FLOPS_COUNTED[args.workload] * evals / avg_kernel_s / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
          "cycles_per_xcd": CYCLES_PER_XCD.get(args.workload),
          "clock_ghz_implied": (CYCLES_PER_XCD[args.workload] / avg_kernel_s / 1e9
                                if args.workload in CYCLES_PER_XCD else None)}
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
                   "family": w.family, "evals_per_step": evals, "generator_a": a,
                   "kernel_specialised": bool(plan.last_launch()[2]) if w.family == "sector" else None},
        "roofline": rf,
        "result": {"mean": res.mean_re, "err": res.err_re},
    }
    plan.close()
    if not args.no_legs and args.workload == "sector":
        print("[bench] product-peak batch of 512", file=sys.stderr, flush=True)
        out["product_peak_batch512"] = leg_product_peak_batch(qmc, drivers)
        print("[bench] complex sector d = 10 at n = 2^30 - 35", file=sys.stderr, flush=True)
        out["sector_complex_d10"] = leg_complex_d10(qmc, steps=3)
    if not args.no_time_to_error and args.workload == "sector":
        print("[bench] time-to-error ladders", file=sys.stderr, flush=True)
        out["time_to_error"] = leg_time_to_error(drivers, args.tte_goal)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, tk, alpha, g, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
