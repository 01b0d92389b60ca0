"""Pins of the oracle's ignition-point list (Section 3.2 (iii): cells paired
with their ignition periods, several fires in one replication).

Arrival minutes are the least fixed point of a rule that is monotone in the
neighbours' arrivals: a cell's rates depend on (cell, period, replication)
only, so a fire lit earlier never arrives anywhere later.  Several fires lit
together therefore reach each cell at the earliest of the times the single
fires reach it on their own.  The single-fire runs are pinned elsewhere, so
the elementwise minimum checks the list without retyping its code.  The
burn-out threshold is left out of that check: a cell that burns out stays
out, so an earlier ignition can stop a spread that a later one would make."""
import numpy as np
import pytest

import oracle
from paper_1905_09317_amd import inputs

OUTS = ("scar", "arrival_minute", "arrival_period", "burn_count", "burned_cells", "ignition_cell",
        "scenario")


def _small(side=40, seed=31, n_wp=12):
    fuel = inputs.fuel_grid(side, side, seed)
    elev = inputs.elevation_grid(side, side, seed + 1, elev_max=600.0)
    wx = inputs.weather_scenarios(3, n_wp, seed + 2)
    return fuel, elev, wx


def _same(a, b, names=OUTS):
    for k in names:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def _burnable(fuel, k, seed):
    cells = np.flatnonzero(fuel.ravel() != 0)
    return np.random.default_rng(seed).choice(cells, size=k, replace=False)


def _min_arrivals(runs):
    big = np.iinfo(np.int32).max
    a = np.stack([np.where(r["arrival_minute"] < 0, big, r["arrival_minute"]) for r in runs]).min(axis=0)
    return np.where(a == big, -1, a).astype(np.int32)


@pytest.mark.parametrize("p", [0, 3])
def test_one_entry_equals_the_single_ignition(p):
    fuel, elev, wx = _small()
    c = int(_burnable(fuel, 1, 4)[0])
    kw = dict(n_periods=9, reps=5, seed=2, sigma=0.2, rounding=1, scenario_mode=1, threshold=1.5,
              burn_hours=10, burnout=2.0)
    single = oracle.simulate(fuel, elev, wx, ignition_mode=0, ignition_cell=c, ignition_period=p, **kw)
    listed = oracle.simulate(fuel, elev, wx, ignitions=[[c, p]], **kw)
    _same(single, listed)


@pytest.mark.parametrize("case", [
    dict(periods=[0, 0], kw=dict(sigma=0.0, rounding=0)),
    dict(periods=[0, 2, 5], kw=dict(sigma=0.25, rounding=1, threshold=2.0)),
    dict(periods=[1, 1, 4, 6], kw=dict(sigma=0.15, rounding=0, burn_hours=9), period_min=30),
    dict(periods=[3, 0], kw=dict(sigma=0.1, rounding=1, threshold=0.5, burn_hours=14), period_min=20),
])
def test_fires_lit_together_arrive_at_the_earliest_single_time(case):
    period_min = case.get("period_min", 60)
    fuel, elev, wx = _small(n_wp=20)
    cells = _burnable(fuel, len(case["periods"]), 11 + len(case["periods"]))
    kw = dict(n_periods=12, reps=4, seed=7, scenario_mode=1, period_min=period_min, **case["kw"])
    seeds = [[int(c), p] for c, p in zip(cells, case["periods"])]
    multi = oracle.simulate(fuel, elev, wx, ignitions=seeds, **kw)
    singles = [oracle.simulate(fuel, elev, wx, ignitions=[s], **kw) for s in seeds]
    arr = _min_arrivals(singles)
    np.testing.assert_array_equal(multi["arrival_minute"], arr)
    np.testing.assert_array_equal(multi["scar"], (arr >= 0).astype(np.uint8))
    np.testing.assert_array_equal(multi["burned_cells"], (arr >= 0).sum(axis=1))
    np.testing.assert_array_equal(multi["burn_count"], (arr >= 0).sum(axis=0).astype(np.uint32))
    P = period_min
    np.testing.assert_array_equal(multi["arrival_period"], np.where(arr < 0, -1, np.maximum(arr - 1, 0) // P))
    # the earliest entry names the replication's ignition
    first = min(seeds, key=lambda s: s[1])[0]
    assert (multi["ignition_cell"] == first).all()


def test_an_entry_on_a_burned_or_fuel_free_cell_changes_nothing():
    fuel, elev, wx = _small()
    a, b = (int(x) for x in _burnable(fuel, 2, 21))
    kw = dict(n_periods=10, reps=3, seed=8, sigma=0.2, rounding=1, scenario_mode=1)
    alone = oracle.simulate(fuel, elev, wx, ignitions=[[a, 0]], **kw)
    # a cell burned by period 6 in every replication, lit again at period 6
    burned = np.flatnonzero((alone["arrival_minute"] >= 0).all(axis=0) &
                            (alone["arrival_minute"] <= 6 * 60).all(axis=0))
    burned = burned[burned != a]
    assert burned.size > 0
    nonfuel = int(np.flatnonzero(fuel.ravel() == 0)[0])
    extra = oracle.simulate(fuel, elev, wx, ignitions=[[a, 0], [int(burned[-1]), 6], [nonfuel, 2]], **kw)
    _same(alone, extra)


def test_list_order_within_and_across_periods():
    fuel, elev, wx = _small()
    c = [int(x) for x in _burnable(fuel, 3, 31)]
    kw = dict(n_periods=8, reps=3, seed=12, sigma=0.2, rounding=1, scenario_mode=1, threshold=1.0)
    base = oracle.simulate(fuel, elev, wx, ignitions=[[c[0], 1], [c[1], 1], [c[2], 4]], **kw)
    shuffled = oracle.simulate(fuel, elev, wx, ignitions=[[c[2], 4], [c[0], 1], [c[1], 1]], **kw)
    _same(base, shuffled)
    swapped = oracle.simulate(fuel, elev, wx, ignitions=[[c[1], 1], [c[0], 1], [c[2], 4]], **kw)
    _same(base, swapped, names=OUTS[:-2] + ("scenario",))
    assert (swapped["ignition_cell"] == c[1]).all()


def test_a_later_fire_joins_after_the_first_has_stopped():
    """A fuel break closes the first grass fire in, and it is out hours
    before the second is lit beyond the break: the run goes on while
    entries remain, and the second fire still burns."""
    fuel = np.full((40, 40), 2, np.uint8)
    fuel[:, 20] = 0                      # a fuel break splits the grid
    elev = np.zeros((40, 40), np.int16)
    wx = np.tile(np.array([[90.0, 80.0, 10.0, 90.0]], np.float32), (24, 1))[None]
    kw = dict(n_periods=24, seed=1)
    left = oracle.simulate(fuel, elev, wx, ignitions=[[20 * 40 + 5, 0]], **kw)
    right = oracle.simulate(fuel, elev, wx, ignitions=[[20 * 40 + 30, 16]], **kw)
    both = oracle.simulate(fuel, elev, wx, ignitions=[[20 * 40 + 5, 0], [20 * 40 + 30, 16]], **kw)
    assert 0 < left["arrival_minute"].max() < 16 * 60 - 60   # out at least an hour before
    assert right["burned_cells"][0] > 1
    assert both["burned_cells"][0] == left["burned_cells"][0] + right["burned_cells"][0]
    np.testing.assert_array_equal(both["arrival_minute"], _min_arrivals([left, right]))
    assert both["arrival_minute"][0, 20 * 40 + 30] == 16 * 60


@pytest.mark.parametrize("bad", [[], [[-1, 0]], [[1600, 0]], [[5, -1]], [[5, 8]]])
def test_invalid_lists_are_rejected(bad):
    fuel, elev, wx = _small()
    with pytest.raises(ValueError):
        oracle.simulate(fuel, elev, wx, n_periods=8, ignitions=np.array(bad, np.int32).reshape(-1, 2))
