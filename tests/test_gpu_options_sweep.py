"""Seeded sweep over combinations of the simulation options, each case
bit-exact against the FP64 oracle: grid shapes from strips to small
landscapes, every ignition mode (fixed, uniform, nearest the centre, map,
list), later ignitions, noise and rounding modes, thresholds, daily burning
windows, burn-out, scenario draws and period lengths.  Rates are evaluated
in FP64 so that every integer rate equals the oracle's."""
import sys

import numpy as np
import pytest

from paper_1905_09317_amd import Request, Simulator, inputs

from _helpers import assert_same_outputs, oracle_run

pytestmark = pytest.mark.gpu

N_CASES = 32


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim():
    s = Simulator(0)
    yield s
    s.close()


def _case(i):
    """Options and inputs of case i, drawn from a generator seeded by i."""
    rng = np.random.default_rng(1000 + i)
    shape = [(1, 40), (40, 1), (3, 3), (17, 23), (48, 48), (64, 40), (96, 96)][int(rng.integers(0, 7))]
    rows, cols = shape
    period_min = int(rng.choice([15, 20, 30, 60]))
    n_periods = int(rng.integers(2, 24 if period_min == 60 else 40))
    n_scen = int(rng.integers(1, 4))
    fuel = inputs.fuel_grid(rows, cols, 7 * i + 1) if min(rows, cols) > 3 else \
        rng.choice(np.arange(1, 16, dtype=np.uint8), size=(rows, cols))
    elev = inputs.elevation_grid(rows, cols, 7 * i + 2, elev_max=float(rng.choice([0.0, 300.0, 900.0])))
    wx = inputs.weather_scenarios(n_scen, n_periods, 7 * i + 3)
    kw = dict(n_periods=n_periods, reps=int(rng.integers(1, 20)), seed=int(rng.integers(0, 2**40)),
              sigma=float(rng.choice([0.0, 0.1, 0.3])), rounding=int(rng.integers(0, 2)),
              threshold=float(rng.choice([0.0, 0.0, 1.0, 3.0])), scenario_mode=int(rng.integers(0, 2)),
              scenario=int(rng.integers(0, n_scen)), burnout=float(rng.choice([0.0, 0.0, 1.0, 4.0])),
              burn_hours=int(rng.choice([0, 0, 6, 13])))
    burnable = np.flatnonzero(fuel.ravel() != 0)
    mode = int(rng.integers(0, 5))
    weights = None
    if mode == 0:
        kw.update(ignition_mode=0, ignition_cell=int(rng.integers(0, rows * cols)),
                  ignition_period=int(rng.integers(0, n_periods)))
    elif mode in (1, 2):
        kw.update(ignition_mode=mode, ignition_period=int(rng.integers(0, min(3, n_periods))))
    elif mode == 3:
        weights = rng.integers(0, 50, rows * cols).astype(np.uint32)
        weights[rng.random(rows * cols) < 0.5] = 0
        kw.update(ignition_mode=3)
    else:
        k = int(rng.integers(1, 6))
        cells = rng.integers(0, rows * cols, k) if burnable.size == 0 else rng.choice(burnable, k)
        kw.update(ignitions=np.stack([cells, rng.integers(0, n_periods, k)], axis=1).astype(np.int32))
    return fuel, elev, wx, period_min, weights, kw


@pytest.mark.parametrize("i", range(N_CASES))
def test_option_combination_equals_oracle(sim, i):
    fuel, elev, wx, period_min, weights, kw = _case(i)
    desc = {k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in kw.items()}
    _say(f"case {i}: grid {fuel.shape}, period {period_min} min, {desc}")
    land = sim.load_landscape(fuel, elev)
    x = sim.set_weather(wx, period_min=period_min)
    if weights is not None:
        sim.set_ignition_map(land, weights)
    try:
        g = sim.simulate(Request(landscape=land, weather=x, **kw))
    finally:
        sim.unload_landscape(land)
        sim.unset_weather(x)
    ref = oracle_run(fuel, elev, wx, period_min=period_min, ignition_weights=weights, **kw)
    assert_same_outputs(g, ref, where=f"case {i}")
