"""GPU parity of the ignition-point list (Section 3.2 (iii): cells paired
with their ignition periods, several fires per replication) against the FP64
oracle, bit-exact.  Rates are evaluated in FP64 so that every integer rate
equals the oracle's."""
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


def _seeds(fuel, periods, seed, with_nonfuel=False):
    rng = np.random.default_rng(seed)
    cells = rng.choice(np.flatnonzero(fuel.ravel() != 0), size=len(periods), replace=False)
    s = [[int(c), int(p)] for c, p in zip(cells, periods)]
    if with_nonfuel and (fuel == 0).any():
        s.append([int(np.flatnonzero(fuel.ravel() == 0)[0]), int(periods[0])])
    return np.array(s, np.int32)


def _run(sim, fuel, elev, wx, period_min=60, **kw):
    land = sim.load_landscape(fuel, elev)
    x = sim.set_weather(wx, period_min=period_min)
    g = sim.simulate(Request(landscape=land, weather=x, **kw))
    st = sim.stats()
    sim.unload_landscape(land)
    sim.unset_weather(x)
    return g, st


CASES = [
    dict(periods=[0, 0], kw=dict(sigma=0.0), period_min=60, n_periods=10),
    dict(periods=[0, 3, 3, 7], kw=dict(sigma=0.2, rounding=1, scenario_mode=1), period_min=60, n_periods=12),
    dict(periods=[5, 1, 9], kw=dict(sigma=0.15, rounding=1, threshold=2.0, scenario_mode=1), period_min=30,
         n_periods=16),
    dict(periods=[2, 20, 40], kw=dict(sigma=0.1, rounding=0, burn_hours=7, scenario_mode=1), period_min=20,
         n_periods=144),
    dict(periods=[0, 4, 6], kw=dict(sigma=0.2, rounding=1, burnout=3.0, scenario_mode=1), period_min=60,
         n_periods=12),
    dict(periods=list(range(0, 32)), kw=dict(sigma=0.1, rounding=1, scenario_mode=1), period_min=60, n_periods=36),
]


@pytest.mark.parametrize("i", range(len(CASES)))
def test_ignition_list_equals_oracle(sim, i):
    c = CASES[i]
    _say(f"ignition list case {i}: periods {c['periods']}")
    fuel, elev, wx = _land(80, 72, 200 + i, 3, c["n_periods"])
    seeds = _seeds(fuel, c["periods"], 7 + i, with_nonfuel=(i % 2 == 1))[:32]
    kw = dict(n_periods=c["n_periods"], reps=10, seed=3 + i, **c["kw"])
    g, _ = _run(sim, fuel, elev, wx, period_min=c["period_min"], ignitions=seeds, **kw)
    ref = oracle_run(fuel, elev, wx, period_min=c["period_min"], ignitions=seeds, **kw)
    assert_same_outputs(g, ref, where=f"list case {i}")


def test_a_later_fire_after_the_first_has_stopped(sim):
    """The first fire is closed in by a fuel break and is out by minute 914;
    the run goes on to light the second, beyond the break, at period 20."""
    _say("ignition list, later fire")
    fuel = np.full((48, 48), 2, np.uint8)
    fuel[:, 12] = 0
    elev = np.zeros((48, 48), np.int16)
    wx = np.tile(np.array([[90.0, 80.0, 10.0, 90.0]], np.float32), (24, 1))[None]
    seeds = np.array([[24 * 48 + 4, 0], [24 * 48 + 40, 20]], np.int32)
    kw = dict(n_periods=24, reps=2)
    g, _ = _run(sim, fuel, elev, wx, ignitions=seeds, **kw)
    ref = oracle_run(fuel, elev, wx, ignitions=seeds, **kw)
    assert_same_outputs(g, ref, where="later fire")
    m = np.asarray(g["arrival_minute"])[0]
    assert m[24 * 48 + 40] == 20 * 60
    left = m.reshape(48, 48)[:, :12]
    assert (left >= 0).all() and left.max() < 19 * 60                  # out before the second is lit
    assert (m.reshape(48, 48)[:, 13:] > 20 * 60).sum() > 1


def test_ignition_list_with_more_replications_than_slots(sim):
    """Groups run several replications in predicted-length order; the
    predictor starts from the earliest entry."""
    _say("ignition list, 700 reps")
    fuel, elev, wx = _land(48, 48, 260, 3, 8)
    seeds = _seeds(fuel, [2, 0, 5], 4)
    kw = dict(n_periods=8, reps=700, seed=4, sigma=0.15, rounding=1, scenario_mode=1, threshold=1.0)
    outs = ("burn_count", "burned_cells", "ignition_cell", "scenario")
    g, st = _run(sim, fuel, elev, wx, ignitions=seeds, outputs=outs, **kw)
    assert st["rep_order"] == 1 and st["grid_blocks"] < 700
    ref = oracle_run(fuel, elev, wx, ignitions=seeds, want_rep_outputs=False, **kw)
    assert_same_outputs(g, ref, outs, where="list 700 reps")


def test_lists_fused_with_other_requests_and_served():
    """A list request fused in one launch with single-ignition requests, and
    the same requests through serving lanes, each equal to the oracle."""
    _say("ignition list, batched and served")
    fuel, elev, wx = _land(64, 64, 280, 3, 12)
    seeds_a = _seeds(fuel, [0, 2, 2, 6], 11)
    seeds_b = _seeds(fuel, [3], 12)
    kws = [dict(n_periods=12, reps=6, seed=1, sigma=0.1, rounding=1, scenario_mode=1, ignitions=seeds_a),
           dict(n_periods=10, reps=5, seed=2, sigma=0.1, rounding=1, ignition_mode=1, scenario_mode=1),
           dict(n_periods=12, reps=4, seed=3, scenario_mode=1, burn_hours=9, ignitions=seeds_b)]
    refs = [oracle_run(fuel, elev, wx, **kw) for kw in kws]
    with Simulator(0) as s:
        land = s.load_landscape(fuel, elev)
        x = s.set_weather(wx)
        fused = s.simulate_batch([Request(landscape=land, weather=x, **kw) for kw in kws])
        tickets = [s.submit(Request(landscape=land, weather=x, **kw))[0] for kw in kws]
        served = [s.wait(t) for t in tickets]
    for i, (f, sv, r) in enumerate(zip(fused, served, refs)):
        assert_same_outputs(f, r, where=f"fused {i}")
        assert_same_outputs(sv, r, where=f"served {i}")


def test_ignition_lists_are_validated(sim):
    fuel, elev, wx = _land(32, 32, 300, 1, 8)
    land = sim.load_landscape(fuel, elev)
    x = sim.set_weather(wx)
    bad = [np.zeros((0, 2), np.int32), np.array([[-1, 0]]), np.array([[32 * 32, 0]]),
           np.array([[5, 8]]), np.array([[5, -1]]), np.tile(np.array([[5, 0]]), (33, 1))]
    for s in bad:
        with pytest.raises(C2FError) as e:
            sim.simulate(Request(landscape=land, weather=x, n_periods=8, ignitions=s))
        assert e.value.status == -1
    sim.unload_landscape(land)
    sim.unset_weather(x)
