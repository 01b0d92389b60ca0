"""Shared helpers for the GPU parity tests (not collected by pytest)."""
import numpy as np

import oracle
from paper_1905_09317_amd import Request

OUTS = ("scar", "arrival_period", "arrival_minute", "burn_count", "burned_cells", "ignition_cell",
        "scenario")


def oracle_run(fuel, elev, weather, *, n_periods, reps=1, rep_offset=0, seed=0, sigma=0.0,
               threshold=0.0, rounding=0, ignition_mode=0, ignition_cell=0, scenario_mode=0,
               scenario=0, period_min=60, cell_m=100, pc=50.0, curing=80.0, overrides=None,
               want_rep_outputs=True, ignition_weights=None, ignition_period=0, burn_hours=0,
               burnout=0.0, ignitions=None, fmc=97.0, pdf=50.0, hfi_min=0.0):
    return oracle.simulate(fuel, elev, weather, cell_m=cell_m, n_periods=n_periods, reps=reps,
                           rep_offset=rep_offset, seed=seed, sigma=np.float32(sigma).item(),
                           threshold=np.float32(threshold).item(), rounding=rounding,
                           ignition_mode=ignition_mode, ignition_cell=ignition_cell,
                           scenario_mode=scenario_mode, scenario=scenario, period_min=period_min,
                           pc=np.float32(pc).item(), curing=np.float32(curing).item(),
                           overrides=overrides, want_rep_outputs=want_rep_outputs,
                           ignition_weights=ignition_weights, ignition_period=ignition_period,
                           burn_hours=burn_hours, burnout=np.float32(burnout).item(), ignitions=ignitions,
                           fmc=np.float32(fmc).item(), pdf=np.float32(pdf).item(),
                           hfi_min=np.float32(hfi_min).item())


def assert_same_outputs(gpu: dict, ref: dict, names=OUTS, where=""):
    for k in names:
        if k not in gpu:
            continue
        g = np.asarray(gpu[k])
        r = np.asarray(ref[k])
        if k == "burn_count":
            g = g.view(np.uint32) if g.dtype == np.int32 else g
        assert g.shape == r.shape, (where, k, g.shape, r.shape)
        if not np.array_equal(g, r):
            bad = np.argwhere(g != r)
            first = tuple(bad[0])
            raise AssertionError(f"{where} {k}: {len(bad)} mismatches, first at {first}: "
                                 f"gpu={g[first]} oracle={r[first]}")


def request_kwargs(w, **over):
    kw = dict(n_periods=w.n_periods, reps=w.reps, seed=w.seed, sigma=w.sigma,
              threshold=w.threshold, rounding=w.rounding, precision=w.precision,
              ignition_mode=w.ignition_mode, ignition_cell=w.ignition_cell,
              scenario_mode=w.scenario_mode, scenario=w.scenario)
    kw.update(over)
    return kw


def oracle_kwargs(w, **over):
    kw = dict(n_periods=w.n_periods, reps=w.reps, seed=w.seed, sigma=w.sigma,
              threshold=w.threshold, rounding=w.rounding, ignition_mode=w.ignition_mode,
              ignition_cell=w.ignition_cell, scenario_mode=w.scenario_mode, scenario=w.scenario,
              period_min=w.period_min, cell_m=w.cell_m, pc=w.pc, curing=w.curing)
    kw.update(over)
    kw.pop("precision", None)
    return kw


def boundary_case(xu: np.ndarray, x: np.ndarray, tol_rel: float) -> np.ndarray:
    """True where the oracle's floored value sits within tol of an integer."""
    return np.abs(xu - np.rint(xu)) <= tol_rel * np.maximum(1.0, np.abs(x))


def fp32_overrides(sim, land, wx, fuel, elev, weather, *, reps, n_periods, seed, sigma, rounding,
                   scenarios, cell_m=100, pc=50.0, curing=80.0, tol_rel=1e-5, cells=None, rep_ids=None):
    """Audit FP32 integer rates against the FP64 oracle for every (rep, period)
    (on `cells` only, if given) and return (override keys, q) for the cells
    where they differ; every difference must be a boundary case of the
    oracle's value.  Replications are 0..reps-1, or the global indices
    rep_ids (scenarios[i] belongs to the i-th of them)."""
    keys, qs, n_checked = [], [], 0
    sel = None if cells is None else np.asarray(cells, np.int64)
    for i, r in enumerate(range(reps) if rep_ids is None else rep_ids):
        for p in range(n_periods):
            g = sim.eval_ros(land, wx, scenario=int(scenarios[i]), period=p, rep=int(r), seed=seed,
                             sigma=sigma, rounding=rounding, precision=1)
            o = oracle.eval_ros(fuel, elev, weather, cell_m=cell_m, scenario=int(scenarios[i]),
                                period=p, rep=r, seed=seed, sigma=np.float32(sigma).item(),
                                rounding=rounding, pc=pc, curing=curing,
                                cells=None if sel is None else sel.astype(np.int32))
            gq = g["q8"] if sel is None else g["q8"][sel]
            diff = np.any(gq != o["q8"], axis=1)
            n_checked += gq.size
            if diff.any():
                pos = np.nonzero(diff)[0]
                ok = boundary_case(o["xu8"][pos], o["x8"][pos], tol_rel) | (gq[pos] == o["q8"][pos])
                assert ok.all(), f"rep {r} period {p}: non-boundary integer-rate mismatch at {pos[~ok.all(axis=1)][:5]}"
                for ix in pos:
                    c = int(ix) if sel is None else int(sel[ix])
                    keys.append((int(r), p, c))
                    qs.append(gq[ix])
    k = np.array(keys, np.int32).reshape(-1, 3)
    q = np.array(qs, np.int32).reshape(-1, 8)
    return k, q, n_checked


def dilate(mask2d: np.ndarray, steps: int = 1) -> np.ndarray:
    """8-neighbour dilation of a boolean grid."""
    m = mask2d.copy()
    for _ in range(steps):
        p = np.pad(m, 1)
        m = (p[:-2, :-2] | p[:-2, 1:-1] | p[:-2, 2:] | p[1:-1, :-2] | p[1:-1, 1:-1] | p[1:-1, 2:]
             | p[2:, :-2] | p[2:, 1:-1] | p[2:, 2:])
    return m


def _oracle_shard(arg):
    """One worker process: the oracle over replications first, first +
    stride, ... of a request (per-rep areas and the summed burn counts)."""
    folder, kw, first, stride, reps = arg
    import os

    import numpy as np

    import oracle
    fuel = np.load(os.path.join(folder, "fuel.npy"))
    elev = np.load(os.path.join(folder, "elev.npy"))
    weather = np.load(os.path.join(folder, "weather.npy"))
    counts = np.zeros(fuel.size, np.uint64)
    areas = {}
    for r in range(first, reps, stride):
        ref = oracle_run(fuel, elev, weather, want_rep_outputs=False, **dict(kw, reps=1, rep_offset=r))
        counts += ref["burn_count"]
        areas[r] = int(ref["burned_cells"][0])
    return counts, areas


def oracle_sharded(fuel, elev, weather, reps, procs=None, **kw):
    """The oracle over replications 0..reps-1 of one request, sharded over
    spawned worker processes (fresh interpreters that never touch the GPU):
    returns burn_count [cells] (uint32) and burned_cells [reps]."""
    import multiprocessing
    import os
    import tempfile
    procs = procs or min(16, os.cpu_count() or 1, reps)
    with tempfile.TemporaryDirectory() as folder:
        np.save(os.path.join(folder, "fuel.npy"), np.ascontiguousarray(fuel))
        np.save(os.path.join(folder, "elev.npy"),
                np.ascontiguousarray(elev) if elev is not None else np.zeros_like(fuel, dtype=np.int16))
        np.save(os.path.join(folder, "weather.npy"), np.ascontiguousarray(weather))
        with multiprocessing.get_context("spawn").Pool(procs) as pool:
            parts = pool.map(_oracle_shard, [(folder, kw, k, procs, reps) for k in range(procs)])
    counts = np.zeros(np.asarray(fuel).size, np.uint64)
    burned = np.zeros(reps, np.int64)
    for c, a in parts:
        counts += c
        for r, v in a.items():
            burned[r] = v
    return {"burn_count": counts.astype(np.uint32), "burned_cells": burned}
