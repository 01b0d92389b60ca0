"""Cell2Fire reference oracle -- TEST INFRASTRUCTURE ONLY.

A ctypes binding to ``oracle.c``: a plain single-threaded FP64 CPU simulator
that follows the paper's Algorithm 1 minute by minute.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg use it.  It imports nothing
from the simulator package and the simulator never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C11, -O2, no fast-math)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-Wall", "-Wextra", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i32, i64, u64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        L.oracle_philox4x32_10.argtypes = [P, P, P]
        L.oracle_philox4x32_10.restype = None
        L.oracle_horn.argtypes = [i32, i32, P, P, P]
        L.oracle_fuel_coefficients.argtypes = [i32, P]
        L.oracle_fuel_coefficients.restype = ctypes.c_int
        L.oracle_fbp_point.argtypes = [i32, f64, f64, f64, f64, f64, f64, f64, f64, P]
        L.oracle_fbp_point_ext.argtypes = [i32, f64, f64, f64, f64, f64, f64, f64, f64, f64, f64, P]
        L.oracle_crown_coefficients.argtypes = [i32, P]
        L.oracle_crown_coefficients.restype = ctypes.c_int
        L.oracle_axis_ros.argtypes = [f64, f64, f64, f64, P]
        L.oracle_axis_ros.restype = None
        L.oracle_eval_ros.argtypes = [i32, i32, i32, P, P, f64, f64, i32, i32, P, i32, i32, i32,
                                      u64, f64, i32, P, P, P, P, P, P, P, P]
        L.oracle_eval_ros_cells.argtypes = [i32, i32, i32, P, P, f64, f64, f64, f64, i32, i32, P, i32,
                                            i32, i32, u64, f64, i32, i64, P, P, P, P, P, P, P, P, P, P,
                                            P]
        L.oracle_simulate.argtypes = [i32, i32, i32, P, P, f64, f64, i32, i32, i32, P,
                                      i32, i32, i32, u64, f64, f64, i32, i32, i32, i32, i32,
                                      i32, P, P, P, P, P, P, P, P, P, P]
        L.oracle_simulate_ext.argtypes = [i32, i32, i32, P, P, f64, f64, f64, f64, i32, i32, i32, P,
                                          i32, i32, i32, u64, f64, f64, i32, i32, i32, P, i32, i32,
                                          f64, f64, i32, P, i32, i32, i32, P, P, P, P, P, P, P, P, P, P]
        L.oracle_scar_metrics.argtypes = [i64, i32, i32, P, P, P, P, P]
        for fn in ("oracle_horn", "oracle_fbp_point", "oracle_fbp_point_ext", "oracle_eval_ros", "oracle_eval_ros_cells",
                   "oracle_simulate", "oracle_simulate_ext", "oracle_scar_metrics"):
            getattr(L, fn).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def fuel_coefficients(fuel: int) -> np.ndarray:
    out = np.zeros(5, np.float64)
    if _load().oracle_fuel_coefficients(int(fuel), _ptr(out)) != 0:
        raise ValueError("bad fuel code")
    return out


def crown_coefficients(fuel: int) -> np.ndarray:
    """Crown base height (m) and crown fuel load (kg/m^2) of a fuel code."""
    out = np.zeros(2, np.float64)
    if _load().oracle_crown_coefficients(int(fuel), _ptr(out)) != 0:
        raise ValueError("bad fuel code")
    return out


def horn(elev: np.ndarray):
    e = np.ascontiguousarray(elev, dtype=np.int16)
    r, c = e.shape
    gx = np.zeros((r, c), np.int32)
    gn = np.zeros((r, c), np.int32)
    if _load().oracle_horn(r, c, _ptr(e), _ptr(gx), _ptr(gn)) != 0:
        raise ValueError("oracle_horn: bad input")
    return gx, gn


FBP_FIELDS = ("hros", "bros", "fros", "lb", "raz", "isi", "wsv", "be", "rsi", "wse", "sfc", "cfb",
              "tfc", "hfi")


def fbp_point(fuel: int, ffmc: float, bui: float, ws: float, wd: float, slope_pct: float = 0.0,
              upslope_az: float = 0.0, pc: float = 50.0, curing: float = 80.0, fmc: float = 97.0,
              pdf: float = 50.0) -> dict:
    out = np.zeros(14, np.float64)
    rc = _load().oracle_fbp_point_ext(int(fuel), float(ffmc), float(bui), float(ws), float(wd),
                                      float(slope_pct), float(upslope_az), float(pc), float(curing),
                                      float(fmc), float(pdf), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_fbp_point: bad input")
    return dict(zip(FBP_FIELDS, out.tolist()))


def axis_ros(hros: float, bros: float, fros: float, raz_deg: float) -> np.ndarray:
    out = np.zeros(8, np.float64)
    _load().oracle_axis_ros(float(hros), float(bros), float(fros), float(raz_deg), _ptr(out))
    return out


def _land(fuel, elev, weather):
    f = np.ascontiguousarray(fuel, dtype=np.uint8)
    e = None if elev is None else np.ascontiguousarray(elev, dtype=np.int16)
    w = np.ascontiguousarray(weather, dtype=np.float32)
    if w.ndim == 2:
        w = w[None]
    if e is not None and e.shape != f.shape:
        raise ValueError("elevation shape differs from fuel shape")
    return f, e, w


def eval_ros(fuel, elev, weather, *, cell_m=100, scenario=0, period=0, rep=0, seed=0, sigma=0.0,
             rounding=0, pc=50.0, curing=80.0, fmc=97.0, pdf=50.0, cells=None) -> dict:
    """Per-cell rate field; with `cells` (grid indices) only those cells,
    outputs indexed by position in `cells`."""
    f, e, w = _land(fuel, elev, weather)
    rows, cols = f.shape
    sel = None if cells is None else np.ascontiguousarray(cells, dtype=np.int32)
    n = rows * cols if sel is None else sel.size
    out = {k: np.zeros(n, np.float64) for k in ("hros", "bros", "fros", "lb", "raz", "cfb", "hfi")}
    out["x8"] = np.zeros((n, 8), np.float64)
    out["xu8"] = np.zeros((n, 8), np.float64)
    out["q8"] = np.zeros((n, 8), np.int32)
    rc = _load().oracle_eval_ros_cells(rows, cols, int(cell_m), _ptr(f), _ptr(e), float(pc),
                                       float(curing), float(fmc), float(pdf), w.shape[0], w.shape[1],
                                       _ptr(w), int(scenario),
                                       int(period), int(rep), int(seed) & (2**64 - 1), float(sigma),
                                       int(rounding), -1 if sel is None else int(sel.size),
                                       _ptr(sel), _ptr(out["hros"]), _ptr(out["bros"]),
                                       _ptr(out["fros"]), _ptr(out["lb"]), _ptr(out["raz"]),
                                       _ptr(out["x8"]), _ptr(out["xu8"]), _ptr(out["q8"]),
                                       _ptr(out["cfb"]), _ptr(out["hfi"]))
    if rc != 0:
        raise ValueError("oracle_eval_ros: bad input")
    return out


def simulate(fuel, elev, weather, *, cell_m=100, n_periods, reps=1, rep_offset=0, seed=0,
             sigma=0.0, threshold=0.0, rounding=0, ignition_mode=0, ignition_cell=0,
             scenario_mode=0, scenario=0, period_min=60, pc=50.0, curing=80.0, fmc=97.0, pdf=50.0,
             overrides=None, want_rep_outputs=True, ignition_weights=None, ignition_period=0,
             burn_hours=0, burnout=0.0, hfi_min=0.0, ignitions=None) -> dict:
    """Run the minute-stepping reference simulation.

    overrides: optional (keys int32 [n,3] of (rep, period, cell), q int32 [n,8]).
    ignition_mode 3 draws the ignition from ignition_weights (uint32 per
    cell); ignition_period starts the fire at that period; burn_hours (1..24)
    is the daily burning window (0 = always); burnout (m/min, 0 = off) is the
    rate below which a burning cell burns out; hfi_min (kW/m, 0 = off) the
    head fire intensity below which it does.  ignitions: (cell, period)
    pairs [k, 2] lit as the clock reaches their periods (ignition_mode 4,
    set by passing them).
    Returns scar/arrival_period/arrival_minute [reps, rows*cols] (if wanted),
    burn_count [rows*cols], burned_cells/ignition_cell/scenario [reps], stats [5]
    (ignitions, burning-cell-minutes, rate evaluations, burning-cell-periods,
    axis reach events).
    """
    f, e, w = _land(fuel, elev, weather)
    rows, cols = f.shape
    n = rows * cols
    res = {}
    if want_rep_outputs:
        res["scar"] = np.zeros((reps, n), np.uint8)
        res["arrival_period"] = np.zeros((reps, n), np.int32)
        res["arrival_minute"] = np.zeros((reps, n), np.int32)
    res["burn_count"] = np.zeros(n, np.uint32)
    res["burned_cells"] = np.zeros(reps, np.int64)
    res["ignition_cell"] = np.zeros(reps, np.int32)
    res["scenario"] = np.zeros(reps, np.int32)
    res["stats"] = np.zeros(5, np.int64)
    n_ov, ok, oq = 0, None, None
    if overrides is not None and len(overrides[0]) > 0:
        ok = np.ascontiguousarray(overrides[0], dtype=np.int32).reshape(-1, 3)
        oq = np.ascontiguousarray(overrides[1], dtype=np.int32).reshape(-1, 8)
        n_ov = ok.shape[0]
    iw = None
    if ignition_weights is not None:
        iw = np.ascontiguousarray(ignition_weights, dtype=np.uint32).reshape(-1)
        if iw.size != n:
            raise ValueError("ignition_weights must hold one weight per cell")
    seeds = None
    if ignitions is not None:
        seeds = np.ascontiguousarray(ignitions, dtype=np.int32).reshape(-1, 2)
        ignition_mode = 4
    rc = _load().oracle_simulate_ext(
        rows, cols, int(cell_m), _ptr(f), _ptr(e), float(pc), float(curing), float(fmc), float(pdf),
        w.shape[0], w.shape[1], int(period_min), _ptr(w), int(reps), int(rep_offset), int(n_periods),
        int(seed) & (2**64 - 1), float(sigma), float(threshold), int(rounding),
        int(ignition_mode), int(ignition_cell), _ptr(iw), int(ignition_period), int(burn_hours),
        float(burnout), float(hfi_min), 0 if seeds is None else seeds.shape[0], _ptr(seeds),
        int(scenario_mode), int(scenario), n_ov,
        _ptr(ok), _ptr(oq), _ptr(res.get("scar")), _ptr(res.get("arrival_period")),
        _ptr(res.get("arrival_minute")), _ptr(res["burn_count"]), _ptr(res["burned_cells"]),
        _ptr(res["ignition_cell"]), _ptr(res["scenario"]), _ptr(res["stats"]))
    if rc != 0:
        raise ValueError("oracle_simulate_ext: bad input")
    return res


def scar_metrics(arrival_minute, reference, *, period_min=60) -> dict:
    """MSE and SSIM per period and the final delta_norm of the scars given by
    arrival minutes [cells] against reference 0-1 scars [periods, cells]."""
    a = np.ascontiguousarray(arrival_minute, dtype=np.int32).reshape(-1)
    r = np.ascontiguousarray(reference, dtype=np.uint8)
    r = r.reshape(r.shape[0], -1)
    if r.shape[1] != a.size:
        raise ValueError("reference scars must have one value per cell")
    T = r.shape[0]
    out = {"mse": np.zeros(T), "ssim": np.zeros(T), "delta_norm": np.zeros(1)}
    rc = _load().oracle_scar_metrics(a.size, T, int(period_min), _ptr(a), _ptr(r), _ptr(out["mse"]),
                                     _ptr(out["ssim"]), _ptr(out["delta_norm"]))
    if rc != 0:
        raise ValueError("oracle_scar_metrics: bad input")
    out["delta_norm"] = float(out["delta_norm"][0])
    return out
