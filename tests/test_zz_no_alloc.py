"""The no-allocation entry point (c2f_simulate_noalloc) against c2f_simulate.

Both calls go through the C ABI on the same context and the same inputs;
every output must be bit-identical (scars, arrival minutes and periods,
burn counts, per-rep areas, ignition cells and scenarios).  Two calls in a
row use the scratch, the second with a smaller grid and fewer replications,
so that what the first call left in the scratch cannot leak into the second.
"""
import sys

import numpy as np
import pytest

from paper_1905_09317_amd import C2FError, Request, Simulator, inputs

from _helpers import assert_same_outputs, oracle_run

pytestmark = pytest.mark.gpu

ALL = ("scar", "arrival_period", "arrival_minute", "burn_count", "burned_cells", "ignition_cell",
       "scenario")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _host(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


def _case(seed, rows, cols, n_periods):
    rng = np.random.default_rng(seed)
    fuel = inputs.fuel_grid(rows, cols, seed)
    elev = inputs.elevation_grid(rows, cols, seed + 1)
    wx = np.zeros((3, n_periods, 4), np.float32)
    wx[..., 0] = rng.uniform(85, 95, (3, n_periods))
    wx[..., 1] = rng.uniform(40, 120, (3, n_periods))
    wx[..., 2] = rng.uniform(5, 40, (3, n_periods))
    wx[..., 3] = rng.uniform(0, 360, (3, n_periods))
    return fuel, elev, wx


def _both(sim, fuel, elev, wx, **kw):
    land = sim.load_landscape(fuel, elev)
    w = sim.set_weather(wx)
    req = Request(landscape=land, weather=w, outputs=ALL, device_out=True, **kw)
    a = _host(sim.simulate_noalloc(req))
    st = sim.stats()
    b = _host(sim.simulate(req))
    sim.unload_landscape(land)
    sim.unset_weather(w)
    return a, b, st


def test_noalloc_equals_simulate_twice_second_smaller():
    with Simulator(0) as sim:
        _say("noalloc call 1: 96x80, 24 reps")
        f1, e1, w1 = _case(3, 96, 80, 10)
        kw1 = dict(n_periods=10, reps=24, seed=41, sigma=0.15, rounding=1, ignition_mode=1,
                   scenario_mode=1)
        a, b, st = _both(sim, f1, e1, w1, **kw1)
        assert_same_outputs(a, b, ALL, where="noalloc call 1")
        assert st["grid_blocks"] >= 1 and st["relaunches"] == 0
        r = oracle_run(f1, e1, w1, **kw1)
        assert_same_outputs(a, r, ALL, where="noalloc call 1 vs oracle")
        _say("noalloc call 2: 40x31, 5 reps")
        f2, e2, w2 = _case(4, 40, 31, 6)
        kw2 = dict(n_periods=6, reps=5, seed=42, sigma=0.3, rounding=1, threshold=2.0,
                   ignition_mode=2, scenario_mode=1)
        a, b, _ = _both(sim, f2, e2, w2, **kw2)
        assert_same_outputs(a, b, ALL, where="noalloc call 2")
        r = oracle_run(f2, e2, w2, **kw2)
        assert_same_outputs(a, r, ALL, where="noalloc call 2 vs oracle")


def test_noalloc_list_overflow_grows_and_matches():
    with Simulator(0) as sim:
        _say("noalloc forced list overflow")
        f, e, w = _case(5, 64, 64, 8)
        sim.set_tuning(0, 1)
        try:
            a, b, st = _both(sim, f, e, w, n_periods=8, reps=3, seed=7, sigma=0.1, rounding=1,
                             ignition_mode=1)
        finally:
            sim.set_tuning(0, 0)
        assert st["relaunches"] >= 1
        assert_same_outputs(a, b, ALL, where="noalloc overflow")


def test_noalloc_rejects_what_the_scratch_cannot_hold():
    with Simulator(0) as sim:
        _say("noalloc argument checks")
        # one arrival plane of 6000 x 6000 cells (144 MB) exceeds the 128 MiB scratch
        fuel = np.full((6000, 6000), 2, np.uint8)
        land = sim.load_landscape(fuel)
        w = sim.set_weather(np.tile(np.array([90, 80, 10, 0], np.float32), (2, 1)))
        req = Request(landscape=land, weather=w, n_periods=1, ignition_cell=0, outputs=("burn_count",),
                      device_out=True)
        with pytest.raises(C2FError) as ei:
            sim.simulate_noalloc(req)
        assert ei.value.status == -1 and "scratch" in str(ei.value)
        with pytest.raises(ValueError):
            sim.simulate_noalloc(Request(landscape=land, weather=w, n_periods=1, outputs=("burn_count",)))
