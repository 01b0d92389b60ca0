"""GPU parity of the burn-out threshold (assumption A5 (i)) against the
FP64 oracle, bit-exact, alone and with noise, stochastic rounding, an
ignition threshold and the daily burning window."""
import sys

import numpy as np
import pytest

from paper_1905_09317_amd import C2FError, Request, Simulator, inputs

from _helpers import assert_same_outputs, oracle_run

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim():
    s = Simulator(0)
    yield s
    s.close()


def _run(sim, fuel, elev, wx, period_min=60, **kw):
    land = sim.load_landscape(fuel, elev)
    x = sim.set_weather(wx, period_min=period_min)
    g = sim.simulate(Request(landscape=land, weather=x, **kw))
    sim.unload_landscape(land)
    sim.unset_weather(x)
    return g


@pytest.mark.parametrize("delta", [1.0, 2.5, 6.0, 15.0])
def test_burnout_equals_oracle(sim, delta):
    _say(f"burn-out delta {delta}")
    fuel = inputs.fuel_grid(88, 72, 230)
    elev = inputs.elevation_grid(88, 72, 231, elev_max=900.0)
    wx = inputs.weather_scenarios(3, 14, 232)
    kw = dict(n_periods=14, reps=16, seed=8, sigma=0.2, rounding=1, ignition_mode=1, scenario_mode=1,
              burnout=delta)
    g = _run(sim, fuel, elev, wx, **kw)
    ref = oracle_run(fuel, elev, wx, **kw)
    assert_same_outputs(g, ref, where=f"delta {delta}")


def test_burnout_with_threshold_and_burning_window(sim):
    _say("burn-out with threshold and window")
    fuel = inputs.fuel_grid(64, 64, 240)
    elev = inputs.elevation_grid(64, 64, 241, elev_max=600.0)
    wx = inputs.weather_scenarios(2, 96, 242)
    kw = dict(n_periods=96, reps=10, seed=5, sigma=0.15, rounding=1, threshold=1.0, ignition_mode=1,
              scenario_mode=1, burn_hours=10, burnout=3.0)
    g = _run(sim, fuel, elev, wx, period_min=30, **kw)
    ref = oracle_run(fuel, elev, wx, period_min=30, **kw)
    assert_same_outputs(g, ref, where="delta + window")


def test_calm_period_stops_the_fire(sim):
    fuel = np.full((61, 61), 2, np.uint8)
    elev = np.zeros((61, 61), np.int16)
    windy, calm = [91.0, 90.0, 30.0, 250.0], [80.0, 40.0, 0.0, 0.0]
    wx = np.asarray([windy, calm, windy, windy], np.float32)[None]
    c = 30 * 61 + 30
    free = _run(sim, fuel, elev, wx, n_periods=4, ignition_cell=c)
    cut = _run(sim, fuel, elev, wx, n_periods=4, ignition_cell=c, burnout=4.0)
    ref = oracle_run(fuel, elev, wx, n_periods=4, ignition_cell=c, burnout=4.0)
    assert_same_outputs(cut, ref, where="calm")
    assert int(np.asarray(free["burned_cells"])[0]) > int(np.asarray(cut["burned_cells"])[0])


def test_negative_burnout_is_rejected(sim):
    fuel = np.full((8, 8), 2, np.uint8)
    with pytest.raises(C2FError) as e:
        _run(sim, fuel, None, np.asarray([[[90.0, 80.0, 10.0, 0.0]]], np.float32), n_periods=1, burnout=-1.0)
    assert e.value.status == -1
