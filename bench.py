#!/usr/bin/env python3
"""Benchmark of the Cell2Fire hot path on one MI355X.

A step is one complete simulation request on inputs already resident in
HBM: FBP rates per (burning cell, period), elliptical 8-axis propagation
over every period, and the reduction into burn counts and per-rep outputs,
all in the HIP library (one hipGraph launch of the fused kernel).

Prints one JSON line.  value = cell-updates/s = reps x cells x periods per
second (whole job).  The default workload is the largest single-GPU one:
an 8192 x 8192 landscape, 64 replications, 72 hourly periods, FP64 rates.
The roofline object describes the propagation kernel: algorithmic bytes per
launch over its HIP-event duration, where the bytes are per-unit figures
times the work units of the minute-stepping method (burning-cell-periods,
axis reach events, ignitions) counted from the run's final arrival minutes
by the library (c2f_count_work), not the kernel's own work counters (those
are reported beside them as a redundancy ratio).  roofline.step adds the
burn-count array and the requested outputs over the whole step.
cpu_baseline times the FP64 reference oracle on a bounded sample of the
same workload on the host.
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
#   burning-cell-period: 5 B landscape (fuel + slope) + 16 B work-list entry
#     read + 16 B entry write                                     = 37 B
#   axis reach event: 1 B neighbour fuel + 8 B arrival label RMW   = 9 B
#   ignition: 16 B list append + 8 B burn-count RMW                 = 24 B
# A step adds 4 B per cell of burn counts and the requested per-rep outputs
# (1 B scar, 4 B arrival period, 8 B burned cells).
B_EVAL, B_CAND, B_IGN = 37, 9, 24
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the propagation kernel measured with rocprofv3
# (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, factors from a plain 256 MiB
# copy), valid for the kernel sources whose digest is given; reported as
# roofline.traffic only while the sources are unchanged.
KERNEL_SOURCES = ("propagate.hip", "device.h", "ln64.h", "types.h", "fuel_table.h")
TRAFFIC = {
    "single-fire-2048x2048-48h": ("688daae243f8835b", 10_503_435),
    "batched-mc-1024x1024-2048reps": ("688daae243f8835b", 46_238_681_485),
    "large-8192x8192-64reps-72h": ("688daae243f8835b", 825_783_656),
}


# The same for the scar comparison kernel (one launch per comparison of the
# 2048^2 x 48-period workload).
SCAR_SOURCES = ("metrics.hip",)
SCAR_TRAFFIC = ("80d01cc9a8a45579", 219_159_903)


def kernel_digest(sources=KERNEL_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_1905_09317_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


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


def work_units(sim, req) -> dict:
    """The method's work units of the request (c2f_count_work), from the final
    arrival minutes of one more, untimed run of the same request."""
    import dataclasses

    import torch
    o = sim.simulate(dataclasses.replace(req, outputs=("arrival_minute",), device_out=True))
    units = sim.count_work(req, o["arrival_minute"])
    del o
    torch.cuda.empty_cache()
    return units


def dense_outputs(w) -> tuple:
    # a single fire returns its scar and arrival periods; Monte-Carlo runs
    # return burn counts and per-rep burned areas
    if w.reps == 1:
        return ("scar", "arrival_period", "burn_count", "burned_cells")
    return ("burn_count", "burned_cells")


def _oracle_kwargs(w) -> dict:
    import numpy as np
    return dict(cell_m=w.cell_m, n_periods=w.n_periods, seed=w.seed,
                sigma=np.float32(w.sigma).item(), threshold=w.threshold, rounding=w.rounding,
                ignition_mode=w.ignition_mode, ignition_cell=w.ignition_cell,
                scenario_mode=w.scenario_mode, scenario=w.scenario, period_min=w.period_min)


def _oracle_shard(arg) -> tuple:
    """One CPU worker: simulate replications first, first + stride, ... one at
    a time with the oracle until the time budget is spent."""
    folder, kw, first, stride, reps, budget_s = arg
    import numpy as np

    import oracle
    fuel = np.load(os.path.join(folder, "fuel.npy"), mmap_mode="r")
    elev = np.load(os.path.join(folder, "elev.npy"), mmap_mode="r")
    weather = np.load(os.path.join(folder, "weather.npy"))
    fuel, elev = np.ascontiguousarray(fuel), np.ascontiguousarray(elev)
    t0 = time.perf_counter()
    done, r = 0, first
    while True:
        oracle.simulate(fuel, elev, weather, reps=1, rep_offset=r % reps, want_rep_outputs=False,
                        **kw)
        done += 1
        r += stride
        if time.perf_counter() - t0 >= budget_s:
            break
    return done, time.perf_counter() - t0


def cpu_baseline(w, budget_s: float, procs: int) -> dict:
    """The FP64 oracle on this host: a single fire repeated on one core, or
    the replications sharded over `procs` worker processes."""
    import multiprocessing
    import tempfile

    import numpy as np

    import oracle
    kw = _oracle_kwargs(w)
    if w.reps == 1 or procs <= 1:
        t0 = time.perf_counter()
        runs = 0
        while True:
            oracle.simulate(w.fuel, w.elev, w.weather, reps=1, rep_offset=runs % w.reps,
                            want_rep_outputs=(w.reps == 1), **kw)
            runs += 1
            if time.perf_counter() - t0 >= budget_s:
                break
        dt = time.perf_counter() - t0
        what = (f"the full workload simulated {runs} times" if w.reps == 1
                else f"{runs} replications (cycling through the workload's {w.reps})")
        return {"value": runs * w.rows * w.cols * w.n_periods / dt, "unit": "cell-updates/s",
                "cores": 1, "kind": "oracle",
                "sample": f"{what} by the single-threaded FP64 oracle in {dt:.1f} s"}
    with tempfile.TemporaryDirectory() as folder:
        np.save(os.path.join(folder, "fuel.npy"), w.fuel)
        np.save(os.path.join(folder, "elev.npy"),
                w.elev if w.elev is not None else np.zeros_like(w.fuel, dtype=np.int16))
        np.save(os.path.join(folder, "weather.npy"), w.weather)
        args = [(folder, kw, k, procs, w.reps, budget_s) for k in range(procs)]
        # spawned workers: fresh interpreters that never touch the GPU
        with multiprocessing.get_context("spawn").Pool(procs) as pool:
            res = pool.map(_oracle_shard, args)
    reps_done = sum(r[0] for r in res)
    dt = max(r[1] for r in res)
    return {"value": reps_done * w.rows * w.cols * w.n_periods / dt, "unit": "cell-updates/s",
            "cores": procs, "kind": "oracle",
            "sample": (f"{reps_done} replications (cycling through the workload's {w.reps}) "
                       f"sharded over {procs} single-threaded FP64 oracle processes, in {dt:.1f} s")}


def one_per_launch(sim, req, w, n: int, batched: dict, ms_batched: float) -> dict:
    """Time the same replications one simulation per launch (reps=1 with
    rep_offset r) and check each against the batched launch."""
    import dataclasses

    import torch
    n = min(n, w.reps)
    counts = None
    same = True
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(n):
        o = sim.simulate(dataclasses.replace(req, reps=1, rep_offset=r,
                                             outputs=("burn_count", "burned_cells")))
        same &= bool(o["burned_cells"][0].item() == batched["burned_cells"][r].item())
        counts = o["burn_count"].clone() if counts is None else counts + o["burn_count"]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) * 1e3
    if n == w.reps:
        same &= bool(torch.equal(counts, batched["burn_count"]))
    ms_rep = dt / n
    return {"reps_timed": n, "ms_per_rep": ms_rep, "est_ms_all_reps": ms_rep * w.reps,
            "batched_speedup": ms_rep * w.reps / ms_batched, "identical_to_batched": same}


def copy_calibration(args) -> None:
    """Plain copy of known size: each launch reads and writes args.copy_mib MiB."""
    import torch
    n = args.copy_mib << 20
    src = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "steps": args.steps,
                      "ms_per_copy": ms, "GB_per_s": 2 * n / (ms / 1e3) / 1e9}), flush=True)


def served_bench(args) -> None:
    """Continuous-batching service: a Poisson stream of Monte-Carlo queries
    (side log-uniform 128..4096 cells, 1..256 reps, 48 h, FP64 rates) on
    landscapes already resident in HBM; latency from submission to delivered
    burn counts, by the library's clock."""
    import torch  # noqa: F401  (HIP runtime shared with torch)

    from paper_1905_09317_amd import Simulator, inputs
    from paper_1905_09317_amd.serve import load_stream, run_stream

    st = inputs.served_stream(n_queries=args.queries, rate_per_s=args.rate)
    if args.precision >= 0:
        import dataclasses
        st = dataclasses.replace(st, precision=args.precision)
    print(f"[bench] {st.name}: {len(st.queries)} queries, loading landscapes", file=sys.stderr,
          flush=True)
    sim = Simulator(0)
    sim.set_serving(lanes=args.lanes)
    wx, lands = load_stream(sim, st)
    print("[bench] landscapes resident; warming the lanes", file=sys.stderr, flush=True)
    warm = sorted(st.queries, key=lambda q: q.side * q.side * q.reps)[:max(0, args.warmup) * 4]
    if warm:
        run_stream(sim, st, wx, lands, queries=warm, pace=False)
    print("[bench] replaying the stream", file=sys.stderr, flush=True)
    s = run_stream(sim, st, wx, lands)
    line = {
        "metric": "cell-updates/s (reps x cells x periods), served stream",
        "value": s["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": len(warm),
        "ms_per_step": s["span_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ["f32+f64", "f32"][st.precision],
        "data": "synthetic",
        "config": {"workload": st.name, "queries": len(st.queries), "rate_per_s": args.rate,
                   "side": [128, 4096], "reps": [1, 256], "n_periods": st.n_periods,
                   "lanes": args.lanes, "ros_sigma": st.sigma, "rounding": "stochastic",
                   "rate_precision": ["fp64 results (fp32 first, fp64 near rounding boundaries)", "fp32"][st.precision],
                   "ignition": "uniform-burnable"},
        "latency_ms": {"p50": s["latency_ms_p50"], "p99": s["latency_ms_p99"],
                       "mean": s["latency_ms_mean"], "max": s["latency_ms_max"]},
        "queue_ms": {"p50": s["queue_ms_p50"], "p99": s["queue_ms_p99"]},
        "served": {k: s[k] for k in ("completed", "failed", "errors", "offered_cell_updates_per_s",
                                     "arrival_span_s", "drain_ms", "sustained", "batches",
                                     "mean_batch_requests", "lanes_used")},
        "roofline": None,
    }
    print(json.dumps(line), flush=True)
    sim.close()


def treatment_plans(w, n_plans: int, seed: int = 77):
    """Fuel-treatment plans of a landscape: plan 0 is the landscape itself;
    plan k > 0 cuts a 3-cell fuel break along a column and harvests 5 % of
    the cells at random (both set to non-fuel)."""
    import numpy as np

    rng = np.random.default_rng(seed)
    rows, cols = w.rows, w.cols
    plans = [(np.zeros(0, np.int32), np.zeros(0, np.uint8))]
    for _ in range(1, n_plans):
        c0 = int(rng.integers(8, cols - 11))
        strip = (np.arange(rows)[:, None] * cols + np.arange(c0, c0 + 3)[None, :]).ravel().astype(np.int32)
        cut = rng.choice(rows * cols, rows * cols // 20, replace=False).astype(np.int32)
        cells = np.concatenate([strip, cut])
        plans.append((cells, np.zeros(cells.size, np.uint8)))
    return plans


def treatment_bench(args) -> None:
    """Fuel-treatment batch: the batched Monte-Carlo landscape and 7 derived
    plans, 256 replications each, in one fused launch (burn probability per
    plan), against the same plans one launch each."""
    import torch

    from paper_1905_09317_amd import Request, Simulator

    n_plans, reps = 8, 256
    w = make_workload("batched")
    sim = Simulator(0)
    sim.set_stream(torch.cuda.current_stream())
    base = sim.load_landscape(w.fuel, w.elev, cell_m=w.cell_m, pc=w.pc, curing=w.curing)
    wx = sim.set_weather(w.weather, period_min=w.period_min)
    lids = [base] + [sim.derive_landscape(base, c, f) for c, f in treatment_plans(w, n_plans)[1:]]
    print(f"[bench] {n_plans} treatment plans of {w.rows}x{w.cols}, {reps} reps each", file=sys.stderr,
          flush=True)
    reqs = [Request(landscape=lid, weather=wx, n_periods=w.n_periods, reps=reps, seed=w.seed, sigma=w.sigma,
                    rounding=w.rounding, precision=w.precision, ignition_mode=w.ignition_mode,
                    scenario_mode=w.scenario_mode, outputs=("burn_count", "burned_cells"), device_out=True)
            for lid in lids]
    for _ in range(args.warmup):
        sim.simulate_batch(reqs)
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        outs = sim.simulate_batch(reqs)
        st = sim.stats()
        kms.append(st["kernel_ms"])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # the same plans, one launch each
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    alone = [sim.simulate(r) for r in reqs]
    torch.cuda.synchronize()
    ms_alone = (time.perf_counter() - t0) * 1e3
    same = all(torch.equal(a["burn_count"], b["burn_count"]) for a, b in zip(alone, outs))
    units = {"burning_cell_periods": 0, "axis_reaches": 0, "ignitions": 0}
    for r in reqs:
        for k, v in work_units(sim, r).items():
            units[k] += v
    alg_bytes = (B_EVAL * units["burning_cell_periods"] + B_CAND * units["axis_reaches"]
                 + B_IGN * units["ignitions"])
    kernel_ms = sum(kms) / len(kms)
    achieved = alg_bytes / (kernel_ms / 1e3) / 1e9
    cell_updates = n_plans * reps * w.rows * w.cols * w.n_periods
    p_burn = [float(o["burn_count"].double().mean().item()) / reps for o in outs]
    line = {
        "metric": "cell-updates/s (reps x cells x periods), fuel-treatment batch",
        "value": cell_updates / (ms / 1e3),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"treatments-{n_plans}plans-{w.rows}x{w.cols}-{reps}reps", "plans": n_plans,
                   "reps_per_plan": reps, "n_periods": w.n_periods, "scenarios": int(w.weather.shape[0]),
                   "ros_sigma": w.sigma, "block_threads": st["block_threads"],
                   "grid_blocks": st["grid_blocks"], "rep_order": st["rep_order"]},
        "one_launch_per_plan": {"ms": ms_alone, "speedup": ms_alone / ms, "identical": bool(same)},
        "mean_burn_probability": p_burn,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "c2f::propagate_kernel",
                     "kernel_ms": kernel_ms, "alg_bytes_per_launch": alg_bytes, "units": units},
    }
    sim.close()
    if not args.no_cpu_baseline:
        # the untreated plan's replications as the bounded sample
        import dataclasses
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(dataclasses.replace(w, reps=reps), args.cpu_seconds,
                                            args.cpu_procs or min(16, os.cpu_count() or 1))
        line["cpu_baseline"]["sample"] += " (the untreated plan)"
    print(json.dumps(line), flush=True)


def scar_bench(args) -> None:
    """Scar comparison (Section 4 metrics): the 2048^2 x 48 h single fire in
    FP32 against its FP64 run, period by period (48 reference scars of
    4.2M cells resident in HBM)."""
    import numpy as np
    import torch

    from paper_1905_09317_amd import Request, Simulator

    w = make_workload("single")
    sim = Simulator(0)
    sim.set_stream(torch.cuda.current_stream())
    land = sim.load_landscape(w.fuel, w.elev, cell_m=w.cell_m, pc=w.pc, curing=w.curing)
    wx = sim.set_weather(w.weather, period_min=w.period_min)
    kw = dict(n_periods=w.n_periods, ignition_mode=w.ignition_mode, outputs=("arrival_minute",),
              device_out=True)
    a64 = sim.simulate(Request(landscape=land, weather=wx, precision=0, **kw))["arrival_minute"][0]
    a32 = sim.simulate(Request(landscape=land, weather=wx, precision=1, **kw))["arrival_minute"][0]
    t = torch.arange(1, w.n_periods + 1, device=a64.device, dtype=torch.int32)[:, None] * w.period_min
    ref = ((a64[None] >= 0) & (a64[None] <= t)).to(torch.uint8).contiguous()
    res = torch.empty(2 * w.n_periods + 1, dtype=torch.float64, device=a64.device)
    for _ in range(args.warmup):
        sim.compare_scars_async(a32, ref, res, period_min=w.period_min)
    # the comparisons queue back to back on torch's stream (results stay in
    # HBM); HIP events on that stream time the device work
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        sim.compare_scars_async(a32, ref, res, period_min=w.period_min)
    ev1.record()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    ms = ev0.elapsed_time(ev1) / args.steps
    r = res.cpu().numpy()
    m = {"mse": r[:w.n_periods], "ssim": r[w.n_periods:2 * w.n_periods], "delta_norm": float(r[-1])}
    t0 = time.perf_counter()
    sync = sim.compare_scars(a32, ref, period_min=w.period_min)
    sync_ms = (time.perf_counter() - t0) * 1e3
    n = w.rows * w.cols
    alg = w.n_periods * n + 4 * n            # every reference scar once, the arrival field once
    line = {
        "metric": "scar comparisons/s (cells x periods)",
        "value": w.n_periods * n / (ms / 1e3),
        "unit": "cell-periods/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "wall_ms_per_step": wall_ms, "sync_call_ms": sync_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"scars-{w.rows}x{w.cols}-{w.n_periods}periods", "periods": w.n_periods,
                   "cells": n},
        "final": {"mse": float(m["mse"][-1]), "ssim": float(m["ssim"][-1]), "delta_norm": m["delta_norm"]},
        "sync_equals_async": bool(np.array_equal(sync["mse"], m["mse"]) and np.array_equal(sync["ssim"], m["ssim"])),
        "roofline": {"bound": "hbm", "achieved": alg / (ms / 1e3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": SCAR_TRAFFIC[1] if kernel_digest(SCAR_SOURCES) == SCAR_TRAFFIC[0] else None,
                     "kernel": "c2f::scar_counts_rows_kernel<16> (the whole comparison in one launch)",
                     "kernel_ms": ms, "alg_bytes_per_launch": alg},
    }
    if not args.no_cpu_baseline:
        # the FP64 oracle on the same inputs, repeated for about the CPU budget
        import oracle
        a_h, r_h = a32.cpu().numpy(), ref.cpu().numpy()
        runs, t0 = 0, time.perf_counter()
        while True:
            o = oracle.scar_metrics(a_h, r_h, period_min=w.period_min)
            runs += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": runs * w.n_periods * n / dt, "unit": "cell-periods/s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"the full comparison {runs} times by the single-threaded FP64 oracle "
                                          f"in {dt:.1f} s"}
        line["oracle_equals_gpu"] = bool(np.array_equal(o["mse"], m["mse"]) and
                                         np.allclose(o["ssim"], m["ssim"], rtol=1e-9, atol=1e-12) and
                                         o["delta_norm"] == m["delta_norm"])
    print(json.dumps(line), flush=True)
    sim.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large",
                    choices=["single", "single64", "batched", "large", "tiny", "served", "treatments",
                             "scars"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="oracle worker processes for multi-replication workloads "
                         "(default: min(16, host CPUs))")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--precision", type=int, default=-1, choices=[-1, 0, 1],
                    help="rate precision: 0 FP64, 1 FP32 (default: the workload's)")
    ap.add_argument("--per-launch", type=int, default=-1,
                    help="also time this many replications one per launch (default: 64 for "
                         "multi-replication workloads, 0 = off)")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--tuning", default="",
                    help="tuning cache file: loaded when it exists; written after --autotune")
    ap.add_argument("--rep-order", type=int, default=1, choices=[0, 1],
                    help="1: groups running several replications take the longest predicted "
                         "first (default); 0: index order")
    ap.add_argument("--queries", type=int, default=1000, help="served: queries in the stream")
    ap.add_argument("--rate", type=float, default=50.0, help="served: Poisson arrivals per second")
    ap.add_argument("--lanes", type=int, default=4, help="served: concurrent serving lanes")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="instead of the simulation, run a plain device-to-device copy of this "
                         "many MiB per step (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU per run: the measurement covers one GPU's share of the work "
                          "(run with --gpus 1)"}))
        sys.exit(2)

    import torch

    from paper_1905_09317_amd import Request, Simulator

    if args.copy_mib:
        copy_calibration(args)
        return

    if args.workload == "served":
        served_bench(args)
        return
    if args.workload == "treatments":
        treatment_bench(args)
        return
    if args.workload == "scars":
        scar_bench(args)
        return

    w = make_workload(args.workload)
    default_precision = w.precision
    if args.precision >= 0 and args.precision != w.precision:
        import dataclasses
        w = dataclasses.replace(w, precision=args.precision)
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
    sim.set_rep_order(args.rep_order)
    if args.tuning and os.path.exists(args.tuning):
        sim.load_tuning(args.tuning)
    if args.autotune:
        sim.autotune(req)
        if args.tuning:
            sim.save_tuning(args.tuning)
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
    kernel_ms = sum(kms) / len(kms)
    burned = int(out["burned_cells"].sum().item())
    print("[bench] counting the work units", file=sys.stderr, flush=True)
    units = work_units(sim, req)
    alg_bytes = (B_EVAL * units["burning_cell_periods"] + B_CAND * units["axis_reaches"]
                 + B_IGN * units["ignitions"])
    per_rep_out = {"scar": 1, "arrival_period": 4, "arrival_minute": 4}
    step_bytes = (alg_bytes + 4 * n + 8 * w.reps
                  + w.reps * n * sum(per_rep_out.get(k, 0) for k in dense_outputs(w)))
    traffic = None
    # counters were taken at the workload's own precision
    if w.name in TRAFFIC and TRAFFIC[w.name][0] == kernel_digest() and w.precision == default_precision:
        traffic = TRAFFIC[w.name][1]
    achieved = alg_bytes / (kernel_ms / 1e3) / 1e9
    step_achieved = step_bytes / (ms / 1e3) / 1e9

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
        # precision 0: FP32 evaluation, FP64 where a rounding decision is close
        "dtype": "f32" if w.precision == 1 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "rows": w.rows, "cols": w.cols, "cell_m": w.cell_m,
                   "reps": w.reps, "n_periods": w.n_periods, "period_min": w.period_min,
                   "scenarios": int(w.weather.shape[0]), "ros_sigma": w.sigma,
                   "rounding": ["nearest", "stochastic"][w.rounding],
                   "rate_precision": ["fp64 results (fp32 first, fp64 near rounding boundaries)",
                                      "fp32"][w.precision],
                   "ignition": ["fixed", "uniform-burnable", "nearest-centre"][w.ignition_mode],
                   "block_threads": st["block_threads"], "grid_blocks": st["grid_blocks"],
                   "rep_order": st["rep_order"],
                   "list_capacity": st["list_capacity"]},
        "burn_maps_per_s": w.reps / (ms / 1e3),
        "burned_cells": burned,
        "counters": {k: st[k] for k in ("ignitions", "entries", "continuations", "rounds",
                                        "rate_evals", "candidates", "improvements", "relaunches")},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "c2f::propagate_kernel", "kernel_ms": kernel_ms,
                     "alg_bytes_per_launch": alg_bytes,
                     "alg_bytes_per_cell_update": alg_bytes / (w.reps * w.rows * w.cols * w.n_periods),
                     "units": units,
                     "step": {"alg_bytes": step_bytes, "ms": ms, "achieved": step_achieved,
                              "frac": step_achieved / HBM_PEAK_GBS},
                     "redundancy": {
                         "rate_evals_per_burning_cell_period":
                             st["rate_evals"] / max(1, units["burning_cell_periods"]),
                         "candidates_per_axis_reach": st["candidates"] / max(1, units["axis_reaches"])}},
    }
    n_single = args.per_launch if args.per_launch >= 0 else (64 if w.reps > 1 else 0)
    if n_single > 0 and w.reps > 1:
        print("[bench] timing one replication per launch", file=sys.stderr, flush=True)
        line["one_per_launch"] = one_per_launch(sim, req, w, n_single, out, ms)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        procs = args.cpu_procs or min(16, os.cpu_count() or 1)
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, procs)
    print(json.dumps(line), flush=True)
    sim.close()


if __name__ == "__main__":
    main()
