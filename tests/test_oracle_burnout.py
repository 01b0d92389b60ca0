"""Pins of the oracle's burn-out threshold (assumption A5 (i)): a burning
cell whose integer rates toward every burnable neighbour are below delta
spreads no further.  Checked by reductions: delta at or below 1 m/min only
removes cells that could not spread anyway; above the ignition cell's
fastest rate nothing spreads; a calm period after a windy one freezes the
scar where the unrestricted fire stood; more delta never burns more."""
import numpy as np
import pytest

import oracle
from paper_1905_09317_amd import inputs

OUTS = ("scar", "arrival_minute", "arrival_period", "burn_count", "burned_cells")


def _uniform(side=41):
    return np.full((side, side), 2, np.uint8), np.zeros((side, side), np.int16)


def _wx(rows):
    return np.asarray(rows, np.float32)[None]


def test_delta_of_one_changes_nothing_when_rates_are_constant():
    """With constant weather, no noise and nearest rounding a cell's rates
    are the same in every period, so a cell whose rates are all below
    1 m/min (all zero) could never spread; burning it out changes nothing.
    (Under changing weather it does: burn-out is permanent, while a stalled
    cell would otherwise resume when its rates rise.)"""
    fuel = inputs.fuel_grid(48, 48, 201)
    elev = inputs.elevation_grid(48, 48, 202, elev_max=700.0)
    wx = np.repeat(inputs.weather_scenarios(1, 1, 203), 10, axis=1)
    kw = dict(n_periods=10, reps=12, seed=4, ignition_mode=1)
    a = oracle.simulate(fuel, elev, wx, burnout=1.0, **kw)
    b = oracle.simulate(fuel, elev, wx, **kw)
    for k in OUTS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_a_stalled_cell_burns_out_for_good():
    """A calm period between windy ones: without delta the fire waits and
    resumes; with delta above the calm rates it ends at the calm period."""
    fuel, elev = _uniform(41)
    windy, calm = [91.0, 90.0, 30.0, 250.0], [80.0, 40.0, 0.0, 0.0]
    wx = _wx([windy, calm, windy, windy])
    c = 20 * 41 + 20
    qc = oracle.eval_ros(fuel, elev, wx, period=1)["q8"][c].max()
    free = oracle.simulate(fuel, elev, wx, n_periods=4, ignition_cell=c)
    cut = oracle.simulate(fuel, elev, wx, n_periods=4, ignition_cell=c, burnout=float(qc) + 1.0)
    m = free["arrival_minute"][0]
    assert (m > 120).any()                           # the free fire grows after the calm period
    np.testing.assert_array_equal(cut["scar"][0].astype(bool), (m >= 0) & (m <= 60))


def test_delta_above_the_fastest_rate_keeps_the_fire_in_its_cell():
    fuel, elev = _uniform()
    wx = _wx([[90.0, 80.0, 20.0, 270.0]] * 4)
    c = 20 * 41 + 20
    q = oracle.eval_ros(fuel, elev, wx, period=0)["q8"][c]
    o = oracle.simulate(fuel, elev, wx, n_periods=4, ignition_cell=c, burnout=float(q.max()) + 0.5)
    assert o["burned_cells"][0] == 1
    o2 = oracle.simulate(fuel, elev, wx, n_periods=4, ignition_cell=c, burnout=float(q.max()))
    o3 = oracle.simulate(fuel, elev, wx, n_periods=4, ignition_cell=c)
    np.testing.assert_array_equal(o2["arrival_minute"], o3["arrival_minute"])   # every cell's max is q.max()


def test_calm_period_freezes_the_scar():
    """Flat uniform C-2: windy periods then calm ones.  With delta between
    the calm and the windy fastest rates, every burning cell burns out when
    the calm period starts: the scar is the unrestricted fire's at that time."""
    fuel, elev = _uniform(61)
    windy, calm = [91.0, 90.0, 30.0, 250.0], [86.0, 90.0, 0.0, 0.0]
    wx = _wx([windy] * 3 + [calm] * 3)
    c = 30 * 61 + 30
    qw = oracle.eval_ros(fuel, elev, wx, period=0)["q8"][c].max()
    qc = oracle.eval_ros(fuel, elev, wx, period=3)["q8"][c].max()
    assert qc < qw
    delta = (qc + qw) / 2.0
    free = oracle.simulate(fuel, elev, wx, n_periods=6, ignition_cell=c)
    cut = oracle.simulate(fuel, elev, wx, n_periods=6, ignition_cell=c, burnout=float(delta))
    m = free["arrival_minute"][0]
    expect = (m >= 0) & (m <= 3 * 60)
    np.testing.assert_array_equal(cut["scar"][0].astype(bool), expect)
    np.testing.assert_array_equal(cut["arrival_minute"][0][expect], m[expect])
    assert free["burned_cells"][0] > cut["burned_cells"][0] > 50


def test_more_delta_never_burns_more():
    fuel = inputs.fuel_grid(48, 48, 211)
    elev = inputs.elevation_grid(48, 48, 212, elev_max=900.0)
    wx = inputs.weather_scenarios(1, 12, 213)
    kw = dict(n_periods=12, ignition_mode=2)
    prev = None
    for d in (0.0, 2.0, 4.0, 8.0, 16.0):
        o = oracle.simulate(fuel, elev, wx, burnout=d, **kw)
        s = o["scar"][0].astype(bool)
        if prev is not None:
            assert not (s & ~prev).any()
        prev = s


def test_negative_delta_is_rejected():
    fuel, elev = _uniform(11)
    with pytest.raises(ValueError):
        oracle.simulate(fuel, elev, _wx([[90.0, 80.0, 10.0, 0.0]]), n_periods=1, burnout=-1.0)
