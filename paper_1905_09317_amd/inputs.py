"""Seeded synthetic inputs: landscapes, weather streams, query streams.

This module holds no fire-spread arithmetic.  It only draws random rasters
and weather tables of the shapes the paper works with (100 m cells, hourly
weather; Section 3.5 "Main Inputs" and Appendix A "Instances") so that the
simulator and its CPU reference can be fed identical inputs.

Landscape recipe (fuel): white Gaussian noise on the grid, smoothed with a
periodic Gaussian filter of standard deviation ``corr_len`` cells, rescaled
to zero mean and unit variance, then cut at the 15 standard-normal quantiles
Phi^-1(k/16), k = 1..15, into 16 equiprobable classes numbered 0..15.  The
class number is used directly as the fuel code (0 = non-fuel, 1 C-1, 2 C-2,
3 C-3, 4 C-4, 5 C-5, 6 C-6, 7 C-7, 8 D-1, 9 M-1, 10 M-2, 11 S-1, 12 S-2,
13 S-3, 14 O-1a, 15 O-1b).

Landscape recipe (elevation): spectral synthesis with power spectrum
proportional to |f|^-3 (zero mean component), rescaled to [0, elev_max] m
and rounded to int16.

Weather recipe (hourly, per scenario): FFMC random walk (step N(0, 0.5))
clipped to [85, 94]; BUI drawn U[40, 120] once per 24 h; wind speed random
walk (step N(0, 2) km/h) clipped to [5, 40]; wind direction (meteorological
"from" azimuth) random walk with N(0, 20 deg) steps, wrapped to [0, 360).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.fft
from scipy.special import ndtri

N_FUEL_CODES = 16


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def gaussian_random_field(rows: int, cols: int, seed: int, corr_len: float) -> np.ndarray:
    """Standardised periodic Gaussian random field (float32, rows x cols)."""
    rng = _rng(seed)
    noise = rng.standard_normal((rows, cols), dtype=np.float32)
    ky = np.fft.fftfreq(rows).astype(np.float32)
    kx = np.fft.rfftfreq(cols).astype(np.float32)
    s2 = np.float32(2.0 * math.pi**2 * corr_len**2)
    spec = scipy.fft.rfft2(noise, workers=8)
    del noise
    spec *= np.exp(-s2 * ky[:, None] ** 2)
    spec *= np.exp(-s2 * kx[None, :] ** 2)
    field = scipy.fft.irfft2(spec, s=(rows, cols), workers=8).astype(np.float32)
    del spec
    field -= field.mean(dtype=np.float64)
    sd = field.std(dtype=np.float64)
    if sd > 0:
        field /= np.float32(sd)
    return field


def fuel_grid(rows: int, cols: int, seed: int, corr_len: float = 30.0) -> np.ndarray:
    """uint8 fuel codes 0..15 from a thresholded random field (row 0 = north)."""
    field = gaussian_random_field(rows, cols, seed, corr_len)
    cuts = ndtri(np.arange(1, N_FUEL_CODES, dtype=np.float64) / N_FUEL_CODES).astype(np.float32)
    return np.searchsorted(cuts, field.ravel()).astype(np.uint8).reshape(rows, cols)


def elevation_grid(rows: int, cols: int, seed: int, elev_max: float = 800.0) -> np.ndarray:
    """int16 elevation in metres from 1/f^3 spectral synthesis, range [0, elev_max]."""
    rng = _rng(seed)
    ky = np.fft.fftfreq(rows).astype(np.float32)
    kx = np.fft.rfftfreq(cols).astype(np.float32)
    f2 = ky[:, None] ** 2 + kx[None, :] ** 2
    f2[0, 0] = np.inf
    amp = f2 ** np.float32(-0.75)  # power ~ |f|^-3  =>  amplitude ~ |f|^-1.5
    del f2
    spec = (rng.standard_normal(amp.shape, dtype=np.float32)
            + 1j * rng.standard_normal(amp.shape, dtype=np.float32)).astype(np.complex64)
    spec *= amp
    del amp
    z = scipy.fft.irfft2(spec, s=(rows, cols), workers=8).astype(np.float32)
    del spec
    lo, hi = float(z.min()), float(z.max())
    if hi > lo:
        z = (z - lo) * np.float32(elev_max / (hi - lo))
    else:
        z[:] = 0
    return np.rint(z).astype(np.int16)


def weather_stream(n_periods: int, seed: int) -> np.ndarray:
    """float32 [n_periods, 4] hourly rows (FFMC, BUI, WS km/h, WD deg 'from')."""
    rng = _rng(seed)
    out = np.empty((n_periods, 4), dtype=np.float32)
    ffmc = rng.uniform(85.0, 94.0)
    ws = rng.uniform(5.0, 40.0)
    wd = rng.uniform(0.0, 360.0)
    bui = rng.uniform(40.0, 120.0)
    for p in range(n_periods):
        if p > 0:
            ffmc = min(94.0, max(85.0, ffmc + rng.normal(0.0, 0.5)))
            ws = min(40.0, max(5.0, ws + rng.normal(0.0, 2.0)))
            wd = (wd + rng.normal(0.0, 20.0)) % 360.0
            if p % 24 == 0:
                bui = rng.uniform(40.0, 120.0)
        out[p] = (ffmc, bui, ws, wd)
    return out


def weather_scenarios(n_scenarios: int, n_periods: int, seed0: int) -> np.ndarray:
    """float32 [n_scenarios, n_periods, 4]; scenario k uses seed seed0 + k."""
    return np.stack([weather_stream(n_periods, seed0 + k) for k in range(n_scenarios)])


def constant_weather(n_periods: int, ffmc: float, bui: float, ws: float, wd: float,
                     n_scenarios: int = 1) -> np.ndarray:
    row = np.array([ffmc, bui, ws, wd], dtype=np.float32)
    return np.broadcast_to(row, (n_scenarios, n_periods, 4)).copy()


@dataclass
class Workload:
    """A named synthetic workload: landscape, weather and simulation settings."""
    name: str
    fuel: np.ndarray            # uint8 [rows, cols]
    elev: np.ndarray | None     # int16 [rows, cols] or None (flat)
    weather: np.ndarray         # float32 [S, P, 4]
    cell_m: int
    n_periods: int
    reps: int
    seed: int
    sigma: float
    rounding: int               # 0 nearest, 1 stochastic
    precision: int              # 0 fp64, 1 fp32
    ignition_mode: int          # 0 fixed, 1 uniform burnable, 2 nearest centre
    ignition_cell: int
    scenario_mode: int          # 0 fixed, 1 uniform
    scenario: int = 0
    period_min: int = 60
    threshold: float = 0.0
    pc: float = 50.0
    curing: float = 80.0

    @property
    def rows(self) -> int:
        return int(self.fuel.shape[0])

    @property
    def cols(self) -> int:
        return int(self.fuel.shape[1])

    @property
    def cell_updates(self) -> int:
        return self.reps * self.rows * self.cols * self.n_periods


def tiny_c2(rows: int = 20, cols: int = 20, n_periods: int = 10, ws: float = 20.0,
            wd: float = 270.0, ffmc: float = 90.0, bui: float = 80.0) -> Workload:
    """20x20 all C-2, flat, one centre ignition, constant weather, no noise."""
    fuel = np.full((rows, cols), 2, dtype=np.uint8)
    return Workload("tiny-c2-20x20", fuel, None,
                    constant_weather(n_periods, ffmc, bui, ws, wd), 100, n_periods,
                    reps=1, seed=0, sigma=0.0, rounding=0, precision=0,
                    ignition_mode=0, ignition_cell=(rows // 2) * cols + cols // 2,
                    scenario_mode=0)


def single_large_fire(side: int = 2048, n_periods: int = 48, precision: int = 1,
                      fuel_seed: int = 2, elev_seed: int = 3, wx_seed: int = 4) -> Workload:
    """One fire on a random heterogeneous landscape with hourly weather."""
    return Workload(f"single-fire-{side}x{side}-{n_periods}h",
                    fuel_grid(side, side, fuel_seed), elevation_grid(side, side, elev_seed),
                    weather_stream(n_periods, wx_seed)[None], 100, n_periods,
                    reps=1, seed=1, sigma=0.0, rounding=0, precision=precision,
                    ignition_mode=2, ignition_cell=0, scenario_mode=0)


def batched_monte_carlo(side: int = 1024, reps: int = 2048, n_scenarios: int = 100,
                        n_periods: int = 48, land_seed: int = 5, wx_seed0: int = 6,
                        seed: int = 7, precision: int = 0) -> Workload:
    """Many replications: uniform ignitions, scenario draws, lognormal ROS noise."""
    return Workload(f"batched-mc-{side}x{side}-{reps}reps",
                    fuel_grid(side, side, land_seed), elevation_grid(side, side, land_seed + 1000),
                    weather_scenarios(n_scenarios, n_periods, wx_seed0), 100, n_periods,
                    reps=reps, seed=seed, sigma=0.15, rounding=1, precision=precision,
                    ignition_mode=1, ignition_cell=0, scenario_mode=1)


def large_landscape(side: int = 8192, reps: int = 64, n_periods: int = 72,
                    land_seed: int = 9, wx_seed: int = 10, seed: int = 11,
                    precision: int = 0) -> Workload:
    return Workload(f"large-{side}x{side}-{reps}reps-{n_periods}h",
                    fuel_grid(side, side, land_seed), elevation_grid(side, side, land_seed + 1000),
                    weather_stream(n_periods, wx_seed)[None], 100, n_periods,
                    reps=reps, seed=seed, sigma=0.15, rounding=1, precision=precision,
                    ignition_mode=1, ignition_cell=0, scenario_mode=0)


def query_stream(n_queries: int, rate_per_s: float, seed: int, side_min: int = 128,
                 side_max: int = 4096, reps_max: int = 256):
    """Poisson arrivals; side log-uniform in [side_min, side_max]; reps U{1..reps_max}."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_queries)
    t = np.cumsum(gaps) - gaps[0]
    sides = np.rint(np.exp(rng.uniform(math.log(side_min), math.log(side_max), size=n_queries)))
    reps = rng.integers(1, reps_max + 1, size=n_queries)
    return [(float(t[i]), int(sides[i]), int(reps[i])) for i in range(n_queries)]


@dataclass
class Query:
    """One served request: arrival time, its landscape crop and settings."""
    qid: int
    t: float          # arrival, seconds after the stream starts
    side: int         # landscape side, cells
    reps: int
    row0: int         # top-left corner of the crop in the base landscape
    col0: int
    seed: int         # Philox key of the request (the query id)


@dataclass
class ServedStream:
    """A Poisson stream of Monte-Carlo queries over crops of one base
    landscape, sharing one set of weather scenarios."""
    name: str
    fuel: np.ndarray          # uint8 [base, base]
    elev: np.ndarray          # int16 [base, base]
    weather: np.ndarray       # float32 [S, P, 4]
    queries: list
    cell_m: int = 100
    n_periods: int = 48
    sigma: float = 0.15
    rounding: int = 1
    precision: int = 0

    def crop(self, q: Query) -> tuple:
        r, c, s = q.row0, q.col0, q.side
        return (np.ascontiguousarray(self.fuel[r:r + s, c:c + s]),
                np.ascontiguousarray(self.elev[r:r + s, c:c + s]))

    @property
    def cell_updates(self) -> int:
        return sum(q.reps * q.side * q.side for q in self.queries) * self.n_periods


def served_stream(n_queries: int = 1000, rate_per_s: float = 50.0, seed: int = 8,
                  base_side: int = 4096, side_min: int = 128, side_max: int = 4096,
                  reps_max: int = 256, n_scenarios: int = 100, n_periods: int = 48,
                  land_seed: int = 12, wx_seed0: int = 6) -> ServedStream:
    """Query stream of query_stream(); each query's landscape is the crop of
    its side at a position drawn from a generator seeded by the query id, and
    its Philox key is the query id.  Uniform-burnable ignitions, uniform
    scenarios, lognormal ROS noise sigma 0.15, stochastic rounding."""
    base = max(base_side, side_max)
    qs = []
    for i, (t, side, reps) in enumerate(query_stream(n_queries, rate_per_s, seed, side_min,
                                                     side_max, reps_max)):
        rng = _rng(1_000_003 * (seed + 1) + i)
        r0 = int(rng.integers(0, base - side + 1))
        c0 = int(rng.integers(0, base - side + 1))
        qs.append(Query(i, t, side, reps, r0, c0, i))
    return ServedStream(f"served-{n_queries}q-{rate_per_s:g}qps-{side_min}to{side_max}",
                        fuel_grid(base, base, land_seed),
                        elevation_grid(base, base, land_seed + 1000),
                        weather_scenarios(n_scenarios, n_periods, wx_seed0), qs,
                        n_periods=n_periods)
