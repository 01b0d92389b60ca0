"""Python front end of libc2f: argument marshalling only.

Every step of the simulation runs in the HIP library; this module converts
numpy arrays and torch tensors to the C ABI of include/c2f.h and back.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

from . import _lib
from ._lib import Outputs, RunStats, SimParams, TicketInfo, WeatherRow

OUTPUT_NAMES = ("scar", "arrival_period", "arrival_minute", "burn_count", "burned_cells",
                "ignition_cell", "scenario")
_PER_REP_CELLS = {"scar": np.uint8, "arrival_period": np.int32, "arrival_minute": np.int32}
_PER_REP = {"burned_cells": np.int64, "ignition_cell": np.int32, "scenario": np.int32}


class C2FError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_lib.STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


@dataclass
class Request:
    """One Monte-Carlo simulation request (mirrors c2f_sim_params)."""
    landscape: int
    weather: int
    n_periods: int
    reps: int = 1
    seed: int = 0
    sigma: float = 0.0
    threshold: float = 0.0
    rounding: int = 0
    precision: int = 0
    ignition_mode: int = 0
    ignition_cell: int = 0
    scenario_mode: int = 0
    scenario: int = 0
    rep_offset: int = 0
    ignition_period: int = 0
    burn_hours: int = 0
    burnout: float = 0.0
    hfi_min: float = 0.0      # head fire intensity below which a burning cell burns out (kW/m; 0 = off)
    outputs: tuple = OUTPUT_NAMES
    device_out: bool = False
    ignitions: object = None   # (cell, period) pairs: the ignition-point list (ignition_mode 4)

    def params(self) -> SimParams:
        mode, n, ptr = self.ignition_mode, 0, None
        if self.ignitions is not None:
            arr = np.ascontiguousarray(self.ignitions, dtype=np.int32).reshape(-1, 2)
            self._ignition_array = arr   # alive as long as the request
            mode, n, ptr = 4, arr.shape[0], arr.ctypes.data
        return SimParams(self.landscape, self.weather, self.reps, self.n_periods,
                         int(self.seed) & (2**64 - 1), float(self.sigma), float(self.threshold),
                         self.rounding, self.precision, mode, self.ignition_cell,
                         self.scenario_mode, self.scenario, self.rep_offset, self.ignition_period,
                         self.burn_hours, float(self.burnout), n, ptr, float(self.hfi_min))


@dataclass
class _Landscape:
    rows: int
    cols: int
    cell_m: int


class Simulator:
    """A device context holding landscapes and weather streams in HBM."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self._L = _lib.load()
        self._ctx = ctypes.c_void_p()
        st = self._L.c2f_create(int(device), int(hbm_budget_bytes), ctypes.byref(self._ctx))
        if st != 0:
            raise C2FError(st, f"c2f_create(device={device}) failed (a gfx950 GPU is required)")
        self._lands: dict[int, _Landscape] = {}
        self._device = device
        self._keep = {}

    # ----------------------------------------------------------- plumbing
    def _check(self, st: int):
        if st != 0:
            msg = self._L.c2f_last_error(self._ctx)
            raise C2FError(st, msg.decode() if msg else "")

    def close(self):
        if self._ctx:
            self._L.c2f_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream=None):
        """Order library work on a HIP stream (a torch.cuda.Stream, an int handle, or None)."""
        handle = None
        if stream is not None:
            handle = getattr(stream, "cuda_stream", stream)
        self._check(self._L.c2f_set_stream(self._ctx, ctypes.c_void_p(handle)))

    # ------------------------------------------------------------- inputs
    def load_landscape(self, fuel, elev=None, cell_m: int = 100, pc: float = 50.0,
                       curing: float = 80.0) -> int:
        f = np.ascontiguousarray(fuel, dtype=np.uint8)
        if f.ndim != 2:
            raise ValueError("fuel must be a 2-D grid")
        e = None
        if elev is not None:
            e = np.ascontiguousarray(elev, dtype=np.int16)
            if e.shape != f.shape:
                raise ValueError("elevation shape differs from fuel shape")
        lid = ctypes.c_int32()
        self._check(self._L.c2f_load_landscape(
            self._ctx, f.shape[0], f.shape[1], int(cell_m), f.ctypes.data_as(ctypes.c_void_p),
            None if e is None else e.ctypes.data_as(ctypes.c_void_p), float(pc), float(curing),
            ctypes.byref(lid)))
        self._lands[lid.value] = _Landscape(f.shape[0], f.shape[1], int(cell_m))
        return lid.value

    def unload_landscape(self, landscape: int):
        self._check(self._L.c2f_unload_landscape(self._ctx, int(landscape)))
        self._lands.pop(landscape, None)

    def compare_scars(self, arrival_minute, reference, period_min: int = 60) -> dict:
        """MSE and SSIM per period and the last period's Frobenius norm of the
        scars given by one replication's arrival minutes against reference
        0-1 scars [periods, cells].  torch tensors on the device stay there."""
        on_dev = hasattr(arrival_minute, "is_cuda") and arrival_minute.is_cuda
        if on_dev:
            import torch
            a = arrival_minute.contiguous().view(-1).to(torch.int32)
            r = reference.contiguous().to(torch.uint8)
            r = r.view(r.shape[0], -1)
            self.set_stream(torch.cuda.current_stream(self._device))
            pa, pr, n, T = a.data_ptr(), r.data_ptr(), a.numel(), r.shape[0]
            if r.shape[1] != n:
                raise ValueError("reference scars must have one value per cell")
        else:
            a = np.ascontiguousarray(arrival_minute, dtype=np.int32).reshape(-1)
            r = np.ascontiguousarray(reference, dtype=np.uint8)
            r = r.reshape(r.shape[0], -1)
            if r.shape[1] != a.size:
                raise ValueError("reference scars must have one value per cell")
            pa, pr, n, T = a.ctypes.data, r.ctypes.data, a.size, r.shape[0]
        out = {"mse": np.zeros(T), "ssim": np.zeros(T)}
        dn = ctypes.c_double()
        self._check(self._L.c2f_compare_scars(
            self._ctx, ctypes.c_int64(n), int(T), int(period_min), ctypes.c_void_p(pa), ctypes.c_void_p(pr),
            1 if on_dev else 0, out["mse"].ctypes.data_as(ctypes.c_void_p),
            out["ssim"].ctypes.data_as(ctypes.c_void_p), ctypes.byref(dn)))
        out["delta_norm"] = dn.value
        return out

    def compare_scars_async(self, arrival_minute, reference, results, period_min: int = 60):
        """compare_scars on device tensors, ordered on torch's current stream
        without waiting: results (float64, 2 T + 1 elements on the device)
        receives mse[T], then ssim[T], then the Frobenius norm."""
        import torch
        a = arrival_minute.contiguous().view(-1).to(torch.int32)
        r = reference.contiguous().to(torch.uint8)
        r = r.view(r.shape[0], -1)
        n, T = a.numel(), r.shape[0]
        if r.shape[1] != n:
            raise ValueError("reference scars must have one value per cell")
        if (not results.is_cuda or results.dtype != torch.float64 or not results.is_contiguous()
                or results.numel() < 2 * T + 1):
            raise ValueError("results must be a contiguous float64 device tensor of 2 T + 1 elements")
        self.set_stream(torch.cuda.current_stream(self._device))
        self._check(self._L.c2f_compare_scars_async(
            self._ctx, ctypes.c_int64(n), int(T), int(period_min), ctypes.c_void_p(a.data_ptr()),
            ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(results.data_ptr())))
        return results

    def derive_landscape(self, base: int, cells, fuels) -> int:
        """A treatment variant of `base`: fuel[cells[k]] = fuels[k] (0 =
        harvested / non-fuel); same grid, slopes and constants."""
        c = np.ascontiguousarray(cells, dtype=np.int32).reshape(-1)
        f = np.ascontiguousarray(np.broadcast_to(np.asarray(fuels, dtype=np.uint8), c.shape))
        out = ctypes.c_int32()
        self._check(self._L.c2f_derive_landscape(self._ctx, int(base), ctypes.c_int64(c.size),
                                                 c.ctypes.data_as(ctypes.c_void_p),
                                                 f.ctypes.data_as(ctypes.c_void_p), ctypes.byref(out)))
        self._lands[out.value] = self._lands[base]
        return out.value

    def set_ignition_map(self, landscape: int, weights):
        """Ignition probability per cell (ignition_mode 3): integer weights of
        the landscape's shape; None removes the map."""
        if weights is None:
            self._check(self._L.c2f_set_ignition_map(self._ctx, int(landscape), None))
            return
        lm = self._lands[landscape]
        w = np.ascontiguousarray(weights, dtype=np.uint32).reshape(-1)
        if w.size != lm.rows * lm.cols:
            raise ValueError(f"ignition map needs {lm.rows * lm.cols} weights, got {w.size}")
        self._check(self._L.c2f_set_ignition_map(self._ctx, int(landscape),
                                                 w.ctypes.data_as(ctypes.c_void_p)))

    def set_weather(self, weather, period_min: int = 60) -> int:
        w = np.ascontiguousarray(weather, dtype=np.float32)
        if w.ndim == 2:
            w = w[None]
        if w.ndim != 3 or w.shape[2] != 4:
            raise ValueError("weather must be [scenarios, periods, 4]")
        wid = ctypes.c_int32()
        self._check(self._L.c2f_set_weather(self._ctx, w.shape[0], w.shape[1], int(period_min),
                                            w.ctypes.data_as(ctypes.c_void_p), ctypes.byref(wid)))
        return wid.value

    def unset_weather(self, weather: int):
        self._check(self._L.c2f_unset_weather(self._ctx, int(weather)))

    # ------------------------------------------------------------ outputs
    def _alloc_outputs(self, req: Request):
        lm = self._lands[req.landscape]
        n = lm.rows * lm.cols
        shapes = {"scar": (req.reps, n), "arrival_period": (req.reps, n),
                  "arrival_minute": (req.reps, n), "burn_count": (n,), "burned_cells": (req.reps,),
                  "ignition_cell": (req.reps,), "scenario": (req.reps,)}
        dtypes = {**_PER_REP_CELLS, **_PER_REP, "burn_count": np.uint32}
        res = {}
        o = Outputs()
        o.on_device = 1 if req.device_out else 0
        for name in req.outputs:
            if req.device_out:
                import torch
                tdt = {np.uint8: torch.uint8, np.int32: torch.int32, np.int64: torch.int64,
                       np.uint32: torch.int32}[dtypes[name]]
                t = torch.empty(shapes[name], dtype=tdt, device=f"cuda:{self._device}")
                res[name] = t
                setattr(o, name, t.data_ptr())
            else:
                a = np.empty(shapes[name], dtype=dtypes[name])
                res[name] = a
                setattr(o, name, a.ctypes.data)
        return res, o

    def simulate(self, req: Request | None = None, **kw) -> dict:
        """Run one request; returns the wanted outputs (numpy, or torch tensors
        on the device with device_out=True; burn_count then has dtype int32
        holding the uint32 bits)."""
        req = req or Request(**kw)
        if req.device_out:
            import torch
            self.set_stream(torch.cuda.current_stream(self._device))
        res, o = self._alloc_outputs(req)
        p = req.params()
        self._check(self._L.c2f_simulate(self._ctx, ctypes.byref(p), ctypes.byref(o)))
        return res

    def simulate_noalloc(self, req: Request | None = None, **kw) -> dict:
        """simulate() through c2f_simulate_noalloc: device outputs only, no
        device allocation inside the library (the outputs are torch tensors
        allocated here, before the call)."""
        req = req or Request(**kw)
        if not req.device_out:
            raise ValueError("simulate_noalloc needs device outputs (device_out=True)")
        import torch
        self.set_stream(torch.cuda.current_stream(self._device))
        res, o = self._alloc_outputs(req)
        p = req.params()
        self._check(self._L.c2f_simulate_noalloc(self._ctx, ctypes.byref(p), ctypes.byref(o)))
        return res

    def count_work(self, req: Request, arrival_minute) -> dict:
        """Work counts of a finished request from its arrival minutes (a device
        tensor [reps, rows*cols] int32, as simulate returns with
        device_out=True): burning-cell-periods, axis reach events, ignitions."""
        import torch
        a = arrival_minute
        lm = self._lands[req.landscape]
        if (not isinstance(a, torch.Tensor) or not a.is_cuda or a.dtype != torch.int32
                or not a.is_contiguous() or a.numel() != req.reps * lm.rows * lm.cols):
            raise ValueError("arrival_minute must be a contiguous int32 device tensor [reps, cells]")
        self.set_stream(torch.cuda.current_stream(self._device))
        out = np.zeros(3, np.int64)
        p = req.params()
        self._check(self._L.c2f_count_work(self._ctx, ctypes.byref(p), ctypes.c_void_p(a.data_ptr()),
                                           out.ctypes.data_as(ctypes.c_void_p)))
        return {"burning_cell_periods": int(out[0]), "axis_reaches": int(out[1]), "ignitions": int(out[2])}

    def simulate_batch(self, reqs: list[Request]) -> list[dict]:
        """Run several requests (any landscapes/weather) in one fused launch."""
        if any(r.device_out for r in reqs):
            import torch
            self.set_stream(torch.cuda.current_stream(self._device))
        allocs = [self._alloc_outputs(r) for r in reqs]
        P = (SimParams * len(reqs))(*[r.params() for r in reqs])
        O = (Outputs * len(reqs))(*[a[1] for a in allocs])
        self._check(self._L.c2f_simulate_batch(self._ctx, len(reqs), P, O))
        return [a[0] for a in allocs]

    def eval_ros(self, landscape: int, weather: int, *, scenario=0, period=0, rep=0, seed=0,
                 sigma=0.0, rounding=0, precision=0) -> dict:
        lm = self._lands[landscape]
        n = lm.rows * lm.cols
        out = {k: np.empty(n, np.float64) for k in ("hros", "bros", "fros", "lb", "raz", "cfb", "hfi")}
        out["x8"] = np.empty((n, 8), np.float64)
        out["q8"] = np.empty((n, 8), np.int32)
        ptr = {k: v.ctypes.data_as(ctypes.c_void_p) for k, v in out.items()}
        self._check(self._L.c2f_eval_ros(
            self._ctx, int(landscape), int(weather), int(scenario), int(period), int(rep),
            int(seed) & (2**64 - 1), float(sigma), int(rounding), int(precision), ptr["hros"],
            ptr["bros"], ptr["fros"], ptr["lb"], ptr["raz"], ptr["x8"], ptr["q8"], ptr["cfb"],
            ptr["hfi"]))
        return out

    def set_landscape_fbp(self, landscape: int, fmc: float = 97.0, pdf: float = 50.0):
        """Foliar moisture content and percent dead fir of a landscape."""
        self._check(self._L.c2f_set_landscape_fbp(self._ctx, int(landscape), float(fmc), float(pdf)))

    # ------------------------------------------------------------- tuning
    def set_tuning(self, block_threads: int = 0, list_capacity: int = 0):
        self._check(self._L.c2f_set_tuning(self._ctx, int(block_threads), int(list_capacity)))

    def set_rep_order(self, mode: int = 1):
        """1: work groups that run several replications take the longest
        predicted first (default); 0: in index order.  Same results."""
        self._check(self._L.c2f_set_rep_order(self._ctx, int(mode)))

    def autotune(self, req: Request | None = None, **kw):
        req = req or Request(**kw)
        p = req.params()
        self._check(self._L.c2f_autotune(self._ctx, ctypes.byref(p)))

    def save_tuning(self, path: str):
        """Write the context's tuning entries (block size and list capacity
        per grid size, replication count and precision) to a text file."""
        self._check(self._L.c2f_save_tuning(self._ctx, os.fsencode(path)))

    def load_tuning(self, path: str):
        """Add the entries of a tuning file written on the same kind of device."""
        self._check(self._L.c2f_load_tuning(self._ctx, os.fsencode(path)))

    def stats(self) -> dict:
        s = RunStats()
        self._check(self._L.c2f_get_stats(self._ctx, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in RunStats._fields_}

    # ------------------------------------------------------------ serving
    def set_serving(self, lanes: int = 4, max_batch_reps: int = 2048, max_batch_grid: int = 0,
                    admit_bytes: int = 0):
        """Serving lanes, batch limits and admission memory; call before the
        first submit."""
        self._check(self._L.c2f_set_serving(self._ctx, int(lanes), int(max_batch_reps),
                                            int(max_batch_grid), int(admit_bytes)))

    def memory(self) -> tuple[int, int]:
        """(device bytes held by the context, serving admission limit)."""
        held, limit = ctypes.c_uint64(), ctypes.c_uint64()
        self._check(self._L.c2f_get_memory(self._ctx, ctypes.byref(held), ctypes.byref(limit)))
        return held.value, limit.value

    def submit(self, req: Request) -> tuple[int, dict]:
        """Queue a request; returns (ticket, outputs that fill in when done)."""
        res, o = self._alloc_outputs(req)
        if req.device_out:
            # serving lanes run on their own streams: work of the caller's
            # stream that may still use these (possibly reused) buffers
            # must finish first
            import torch
            torch.cuda.current_stream(self._device).synchronize()
        p = req.params()
        t = ctypes.c_uint64()
        self._check(self._L.c2f_submit(self._ctx, ctypes.byref(p), ctypes.byref(o), ctypes.byref(t)))
        self._keep[t.value] = res
        return t.value, res

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int32()
        self._check(self._L.c2f_poll(self._ctx, ctypes.c_uint64(ticket), ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int) -> dict:
        return self.wait_info(ticket)[0]

    def wait_info(self, ticket: int) -> tuple[dict, dict]:
        """Block until the request completes; returns (outputs, timing)."""
        info = TicketInfo()
        try:
            self._check(self._L.c2f_wait_info(self._ctx, ctypes.c_uint64(ticket), ctypes.byref(info)))
        finally:
            res = self._keep.pop(ticket, None)
        return res, {k: getattr(info, k) for k, _ in TicketInfo._fields_}


def fbp_crown_coefficients(fuel: int) -> np.ndarray:
    """Crown base height (m) and crown fuel load (kg/m^2) of a fuel code."""
    out = np.zeros(2, np.float64)
    st = _lib.load().c2f_fbp_crown_coefficients(int(fuel), out.ctypes.data_as(ctypes.c_void_p))
    if st != 0:
        raise C2FError(st, f"bad fuel code {fuel}")
    return out


def fbp_coefficients(fuel: int) -> np.ndarray:
    out = np.zeros(5, np.float64)
    st = _lib.load().c2f_fbp_coefficients(int(fuel), out.ctypes.data_as(ctypes.c_void_p))
    if st != 0:
        raise C2FError(st, f"bad fuel code {fuel}")
    return out


def request_for(sim: Simulator, workload, landscape: int, weather: int, **over) -> Request:
    """A Request reproducing a synthetic workload's settings."""
    kw = dict(landscape=landscape, weather=weather, n_periods=workload.n_periods,
              reps=workload.reps, seed=workload.seed, sigma=workload.sigma,
              threshold=workload.threshold, rounding=workload.rounding,
              precision=workload.precision, ignition_mode=workload.ignition_mode,
              ignition_cell=workload.ignition_cell, scenario_mode=workload.scenario_mode,
              scenario=workload.scenario)
    kw.update(over)
    return Request(**kw)
