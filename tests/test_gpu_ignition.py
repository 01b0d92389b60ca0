"""GPU parity of the ignition and burning-window options against the FP64
oracle, bit-exact: the ignition-probability map (Section 3.1, uncertainty
(1)), ignition at a later period (the ignition-point input of Section 3.2),
and the daily burning window (assumption A5).  Rates are evaluated in FP64
so that every integer rate equals the oracle's."""
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


def _land(side_r, side_c, seed, n_scen, n_periods):
    fuel = inputs.fuel_grid(side_r, side_c, seed)
    elev = inputs.elevation_grid(side_r, side_c, seed + 1, elev_max=700.0)
    wx = inputs.weather_scenarios(n_scen, n_periods, seed + 2)
    return fuel, elev, wx


def _weights(fuel, seed, zero_frac=0.6):
    rng = np.random.default_rng(seed)
    w = rng.integers(1, 1000, fuel.size, dtype=np.uint32)
    w[rng.random(fuel.size) < zero_frac] = 0
    return w


def _run(sim, fuel, elev, wx, weights=None, period_min=60, **kw):
    land = sim.load_landscape(fuel, elev)
    x = sim.set_weather(wx, period_min=period_min)
    if weights is not None:
        sim.set_ignition_map(land, weights)
    g = sim.simulate(Request(landscape=land, weather=x, **kw))
    st = sim.stats()
    sim.unload_landscape(land)
    sim.unset_weather(x)
    return g, st


def _ref(fuel, elev, wx, weights=None, period_min=60, **kw):
    return oracle_run(fuel, elev, wx, period_min=period_min, ignition_weights=weights, **kw)


@pytest.mark.parametrize("seed", [0, 1])
def test_ignition_map_equals_oracle(sim, seed):
    _say(f"ignition map seed {seed}")
    fuel, elev, wx = _land(96, 80, 70 + seed, 4, 10)
    w = _weights(fuel, 5 + seed)
    kw = dict(n_periods=10, reps=40, seed=11 + seed, sigma=0.15, rounding=1, ignition_mode=3,
              scenario_mode=1)
    g, _ = _run(sim, fuel, elev, wx, weights=w, **kw)
    ref = _ref(fuel, elev, wx, weights=w, **kw)
    assert_same_outputs(g, ref, where=f"map {seed}")
    assert (w[np.asarray(g["ignition_cell"])] > 0).all()


def test_ignition_map_with_more_replications_than_slots(sim):
    """Groups run several replications in predicted-length order; the
    predictor draws ignitions from the map as well."""
    _say("ignition map, 700 reps")
    fuel, elev, wx = _land(48, 48, 80, 3, 6)
    w = _weights(fuel, 9, zero_frac=0.3)
    kw = dict(n_periods=6, reps=700, seed=4, sigma=0.1, rounding=1, ignition_mode=3, scenario_mode=1)
    outs = ("burn_count", "burned_cells", "ignition_cell", "scenario")
    g, st = _run(sim, fuel, elev, wx, weights=w, outputs=outs, **kw)
    assert st["rep_order"] == 1 and st["grid_blocks"] < 700
    ref = _ref(fuel, elev, wx, weights=w, want_rep_outputs=False, **kw)
    assert_same_outputs(g, ref, outs, where="map 700 reps")


@pytest.mark.parametrize("p0,period_min,threshold", [(3, 60, 0.0), (5, 30, 2.0), (11, 20, 0.0)])
def test_later_ignition_equals_oracle(sim, p0, period_min, threshold):
    _say(f"later ignition p0={p0} period {period_min}")
    fuel, elev, wx = _land(72, 72, 90, 3, 16)
    kw = dict(n_periods=16, reps=12, seed=7, sigma=0.2, rounding=1, threshold=threshold,
              ignition_mode=1, scenario_mode=1, ignition_period=p0)
    g, _ = _run(sim, fuel, elev, wx, period_min=period_min, **kw)
    ref = _ref(fuel, elev, wx, period_min=period_min, **kw)
    assert_same_outputs(g, ref, where=f"p0 {p0}")
    on = np.asarray(g["scar"]) == 1
    assert (np.asarray(g["arrival_minute"])[on] >= p0 * period_min).all()


@pytest.mark.parametrize("hours,period_min,threshold,sigma", [(6, 60, 0.0, 0.15), (3, 20, 0.0, 0.0),
                                                              (9, 30, 1.5, 0.1), (1, 60, 0.0, 0.2)])
def test_burning_window_equals_oracle(sim, hours, period_min, threshold, sigma):
    _say(f"burning window {hours} h, period {period_min}")
    n_periods = 3 * 1440 // period_min          # three days
    fuel, elev, wx = _land(64, 64, 100 + hours, 2, n_periods)
    kw = dict(n_periods=n_periods, reps=8, seed=13, sigma=sigma, rounding=1 if sigma else 0,
              threshold=threshold, ignition_mode=1, scenario_mode=1, burn_hours=hours)
    g, _ = _run(sim, fuel, elev, wx, period_min=period_min, **kw)
    ref = _ref(fuel, elev, wx, period_min=period_min, **kw)
    assert_same_outputs(g, ref, where=f"{hours} h")
    m = np.asarray(g["arrival_minute"])
    lit = m > 0
    assert (((m[lit] - 1) % 1440) < hours * 60).all()   # every ignition inside a window


def test_ignition_outside_the_window_waits_for_the_next_day(sim):
    """A fire lit in the seventh hour with a five-hour window spreads from
    the first minute of the next day; combined with the ignition map."""
    _say("ignition outside the window")
    fuel, elev, wx = _land(64, 64, 120, 2, 72)
    w = _weights(fuel, 21, zero_frac=0.5)
    kw = dict(n_periods=72, reps=10, seed=17, sigma=0.1, rounding=1, ignition_mode=3,
              scenario_mode=1, ignition_period=7, burn_hours=5)
    g, _ = _run(sim, fuel, elev, wx, weights=w, **kw)
    ref = _ref(fuel, elev, wx, weights=w, **kw)
    assert_same_outputs(g, ref, where="outside window")
    m = np.asarray(g["arrival_minute"])
    assert (m[m > 7 * 60] > 1440).all()


def test_served_requests_with_ignition_options():
    fuel, elev, wx = _land(80, 80, 140, 3, 48)
    w = _weights(fuel, 31)
    kws = [dict(n_periods=12, reps=6, seed=1, sigma=0.1, rounding=1, ignition_mode=3, scenario_mode=1),
           dict(n_periods=48, reps=5, seed=2, sigma=0.1, rounding=1, ignition_mode=1, scenario_mode=1,
                ignition_period=2, burn_hours=8),
           dict(n_periods=24, reps=7, seed=3, ignition_mode=3, scenario_mode=1, burn_hours=10,
                ignition_period=11)]
    with Simulator(0) as s:
        land = s.load_landscape(fuel, elev)
        s.set_ignition_map(land, w)
        x = s.set_weather(wx)
        tickets = [s.submit(Request(landscape=land, weather=x, **kw))[0] for kw in kws]
        got = [s.wait(t) for t in tickets]
    for kw, g in zip(kws, got):
        ref = _ref(fuel, elev, wx, weights=w, **kw)
        assert_same_outputs(g, ref, where=str(kw))


def test_ignition_options_are_validated(sim):
    fuel, elev, wx = _land(32, 32, 150, 1, 8)
    land = sim.load_landscape(fuel, elev)
    x = sim.set_weather(wx)
    x45 = sim.set_weather(wx, period_min=45)
    bad = [dict(weather=x, n_periods=8, ignition_mode=3),            # no map
           dict(weather=x, n_periods=8, ignition_period=8),
           dict(weather=x, n_periods=8, burn_hours=25),
           dict(weather=x45, n_periods=8, burn_hours=6)]              # 45 min does not divide an hour
    for kw in bad:
        with pytest.raises(C2FError) as e:
            sim.simulate(Request(landscape=land, **kw))
        assert e.value.status == -1
    with pytest.raises(ValueError):
        sim.set_ignition_map(land, np.ones(10, np.uint32))
    sim.set_ignition_map(land, np.zeros(fuel.size, np.uint32))
    g = sim.simulate(Request(landscape=land, weather=x, n_periods=8, reps=3, ignition_mode=3))
    assert (np.asarray(g["burned_cells"]) == 0).all()
    sim.set_ignition_map(land, None)
    with pytest.raises(C2FError):
        sim.simulate(Request(landscape=land, weather=x, n_periods=8, ignition_mode=3))
    sim.unload_landscape(land)
    sim.unset_weather(x)
    sim.unset_weather(x45)
