#!/usr/bin/env python3
"""Benchmark of the Cell2Fire hot path on one MI355X.

A step is one complete simulation request on inputs already resident in
HBM: FBP rates per (burning cell, period), elliptical 8-axis propagation
over every period, and the reduction into burn counts and per-rep outputs,
all in the HIP library (one hipGraph launch of the fused kernel).

Prints one JSON line.  value = cell-updates/s = reps x cells x periods per
second (whole job).  The roofline object describes the propagation kernel:
algorithmic bytes per launch (per-unit byte figures x the kernel's own
event counters) over its HIP-event duration.  cpu_baseline times the FP64
reference oracle on the same workload on the host (one core).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Per-unit algorithmic bytes of the propagation kernel:
#   rate evaluation (a burning cell in a period): 5 B landscape (fuel + slope)
#     + 16 B work-list entry read + 16 B entry write           = 37 B
#   arrival candidate offered to a neighbour: 1 B fuel + 8 B label RMW = 9 B
#   ignition: 16 B list append + 8 B burn-count RMW              = 24 B
#   per cell of the grid: 4 B burn-count initialisation
#   per cell per rep of dense outputs: 4 B label read + 1 B scar + 4 B period
B_EVAL, B_CAND, B_IGN, B_CELL, B_DENSE = 37, 9, 24, 4, 9
HBM_PEAK_GBS = 8000.0


def make_workload(name: str):
    from paper_1905_09317_amd import inputs
    if name == "single":
        return inputs.single_large_fire(side=2048, n_periods=48, precision=1)
    if name == "single64":
        return inputs.single_large_fire(side=2048, n_periods=48, precision=0)
    if name == "batched":
        return inputs.batched_monte_carlo(side=1024, reps=2048, n_scenarios=100, n_periods=48)
    if name == "large":
        return inputs.large_landscape(side=8192, reps=64, n_periods=72)
    if name == "tiny":
        return inputs.tiny_c2()
    raise SystemExit(f"unknown workload {name}")


def dense_outputs(w) -> tuple:
    # a single fire returns its scar and arrival periods; Monte-Carlo runs
    # return burn counts and per-rep burned areas
    if w.reps == 1:
        return ("scar", "arrival_period", "burn_count", "burned_cells")
    return ("burn_count", "burned_cells")


def cpu_baseline(w, budget_s: float) -> dict:
    import numpy as np

    import oracle
    reps_done = 0
    t0 = time.perf_counter()
    n_runs = 0
    chunk = 1 if w.reps == 1 else max(1, min(w.reps, 4))
    while True:
        off = reps_done % w.reps if w.reps > 1 else 0
        n = min(chunk, w.reps - off) if w.reps > 1 else 1
        oracle.simulate(w.fuel, w.elev, w.weather, cell_m=w.cell_m, n_periods=w.n_periods, reps=n,
                        rep_offset=off, seed=w.seed, sigma=np.float32(w.sigma).item(),
                        threshold=w.threshold, rounding=w.rounding, ignition_mode=w.ignition_mode,
                        ignition_cell=w.ignition_cell, scenario_mode=w.scenario_mode,
                        scenario=w.scenario, period_min=w.period_min, want_rep_outputs=(w.reps == 1))
        reps_done += n
        n_runs += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    cu = reps_done * w.rows * w.cols * w.n_periods
    what = (f"the full workload simulated {n_runs} times" if w.reps == 1
            else f"{reps_done} of the {w.reps} replications")
    return {"value": cu / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{what} by the single-threaded FP64 oracle in {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="single",
                    choices=["single", "single64", "batched", "large", "tiny"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--autotune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; the simulation of one GPU's share "
                          "is what is measured (run with --gpus 1)"}))
        sys.exit(2)

    import torch

    from paper_1905_09317_amd import Request, Simulator

    w = make_workload(args.workload)
    print(f"[bench] workload {w.name}: {w.rows}x{w.cols}, reps {w.reps}, periods {w.n_periods}",
          file=sys.stderr, flush=True)
    sim = Simulator(0)
    stream = torch.cuda.current_stream()
    sim.set_stream(stream)
    land = sim.load_landscape(w.fuel, w.elev, cell_m=w.cell_m, pc=w.pc, curing=w.curing)
    wx = sim.set_weather(w.weather, period_min=w.period_min)
    req = Request(landscape=land, weather=wx, n_periods=w.n_periods, reps=w.reps, seed=w.seed,
                  sigma=w.sigma, threshold=w.threshold, rounding=w.rounding,
                  precision=w.precision, ignition_mode=w.ignition_mode,
                  ignition_cell=w.ignition_cell, scenario_mode=w.scenario_mode,
                  scenario=w.scenario, outputs=dense_outputs(w), device_out=True)
    if args.autotune:
        sim.autotune(req)
    if args.block:
        sim.set_tuning(args.block, 0)

    for _ in range(args.warmup):
        sim.simulate(req)
    torch.cuda.synchronize()
    kms, stats = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = sim.simulate(req)
        st = sim.stats()
        kms.append(st["kernel_ms"])
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    cell_updates = w.reps * w.rows * w.cols * w.n_periods
    value = cell_updates / (ms / 1e3)

    st = stats[-1]
    n = w.rows * w.cols
    dense = w.reps * n * B_DENSE if "scar" in dense_outputs(w) else 0
    alg_bytes = (B_EVAL * st["rate_evals"] + B_CAND * st["candidates"] + B_IGN * st["ignitions"]
                 + B_CELL * n + dense)
    kernel_ms = sum(kms) / len(kms)
    achieved = alg_bytes / (kernel_ms / 1e3) / 1e9
    burned = int(out["burned_cells"].sum().item())

    line = {
        "metric": "cell-updates/s (reps x cells x periods)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.precision == 1 else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "rows": w.rows, "cols": w.cols, "cell_m": w.cell_m,
                   "reps": w.reps, "n_periods": w.n_periods, "period_min": w.period_min,
                   "scenarios": int(w.weather.shape[0]), "ros_sigma": w.sigma,
                   "rounding": ["nearest", "stochastic"][w.rounding],
                   "rate_precision": ["fp64", "fp32"][w.precision],
                   "ignition": ["fixed", "uniform-burnable", "nearest-centre"][w.ignition_mode],
                   "block_threads": st["block_threads"], "grid_blocks": st["grid_blocks"],
                   "list_capacity": st["list_capacity"]},
        "burn_maps_per_s": w.reps / (ms / 1e3),
        "burned_cells": burned,
        "counters": {k: st[k] for k in ("ignitions", "entries", "continuations", "rounds",
                                        "rate_evals", "candidates", "improvements", "relaunches")},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "c2f::propagate_kernel", "kernel_ms": kernel_ms,
                     "alg_bytes_per_launch": alg_bytes},
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(line), flush=True)
    sim.close()


if __name__ == "__main__":
    main()
