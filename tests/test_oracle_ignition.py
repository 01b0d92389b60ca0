"""Pins of the oracle's ignition and burning-window options (Section 3.1,
uncertainty source (1): a spatial ignition probability; the ignition-point
input with its ignition period; assumption A5, general fire dynamics (1):
maximum burning hours per day).  Each check reduces an option to another
mode or to a closed form: none retypes the option's own formula."""
import numpy as np
import pytest

import oracle
from paper_1905_09317_amd import inputs

OUTS = ("scar", "arrival_minute", "arrival_period", "burn_count", "burned_cells", "ignition_cell",
        "scenario")


def _small(side=40, seed=31):
    fuel = inputs.fuel_grid(side, side, seed)
    elev = inputs.elevation_grid(side, side, seed + 1, elev_max=600.0)
    wx = inputs.weather_scenarios(3, 12, seed + 2)
    return fuel, elev, wx


def _same(a, b, names=OUTS):
    for k in names:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_unit_weights_on_burnable_cells_equal_uniform_ignition():
    fuel, elev, wx = _small()
    kw = dict(n_periods=8, reps=24, seed=5, sigma=0.2, rounding=1, scenario_mode=1)
    uni = oracle.simulate(fuel, elev, wx, ignition_mode=1, **kw)
    w = (fuel.ravel() != 0).astype(np.uint32)
    mapped = oracle.simulate(fuel, elev, wx, ignition_mode=3, ignition_weights=w, **kw)
    _same(uni, mapped)


def test_single_weight_equals_fixed_ignition():
    fuel, elev, wx = _small()
    c = int(np.flatnonzero(fuel.ravel() != 0)[123])
    w = np.zeros(fuel.size, np.uint32)
    w[c] = 7
    kw = dict(n_periods=8, reps=6, seed=9, sigma=0.1, rounding=1, scenario_mode=1)
    fixed = oracle.simulate(fuel, elev, wx, ignition_mode=0, ignition_cell=c, **kw)
    mapped = oracle.simulate(fuel, elev, wx, ignition_mode=3, ignition_weights=w, **kw)
    _same(fixed, mapped)


def test_ignition_frequencies_follow_the_weights():
    fuel = np.full((6, 6), 2, np.uint8)
    elev = np.zeros((6, 6), np.int16)
    wx = np.array([[[90.0, 80.0, 0.0, 0.0]]], np.float32)
    w = np.zeros(36, np.uint32)
    w[[3, 10, 20, 35]] = [1, 2, 3, 4]
    reps = 20000
    o = oracle.simulate(fuel, elev, wx, n_periods=1, reps=reps, seed=3, ignition_mode=3,
                        ignition_weights=w, want_rep_outputs=False)
    got = np.bincount(o["ignition_cell"], minlength=36)
    assert set(np.flatnonzero(got)) == {3, 10, 20, 35}
    expect = reps * w / w.sum()
    chi2 = float(((got - expect)[w > 0] ** 2 / expect[w > 0]).sum())
    assert chi2 < 16.3    # 3 degrees of freedom, p = 0.001


def test_zero_weights_burn_nothing():
    fuel, elev, wx = _small()
    o = oracle.simulate(fuel, elev, wx, n_periods=4, reps=3, ignition_mode=3,
                        ignition_weights=np.zeros(fuel.size, np.uint32))
    assert (o["burned_cells"] == 0).all() and (o["ignition_cell"] == -1).all()


@pytest.mark.parametrize("p0", [1, 3, 7])
def test_later_ignition_equals_shifted_weather(p0):
    """Without random draws tied to the period (no noise, nearest rounding),
    a fire lit at the start of period p0 is the fire lit at minute 0 under
    the weather from p0 on, every arrival delayed by p0 periods."""
    fuel, elev, wx = _small(seed=41)
    c = int(np.flatnonzero(fuel.ravel() != 0)[700])
    kw = dict(ignition_mode=0, ignition_cell=c, period_min=60)
    late = oracle.simulate(fuel, elev, wx, n_periods=12, ignition_period=p0, **kw)
    early = oracle.simulate(fuel, elev, np.ascontiguousarray(wx[:, p0:]), n_periods=12 - p0, **kw)
    np.testing.assert_array_equal(late["scar"], early["scar"])
    on = early["scar"][0] == 1
    np.testing.assert_array_equal(late["arrival_minute"][0][on], early["arrival_minute"][0][on] + 60 * p0)
    assert (late["arrival_minute"][0][~on] == -1).all()
    # a minute m belongs to period (m - 1) div P: the ignition itself, at
    # minute 60 p0, reads as period p0 - 1
    assert late["arrival_period"][0][c] == p0 - 1


def _constant_weather(n_periods, ffmc=91.0, bui=90.0, ws=18.0, wd=250.0):
    w = np.zeros((1, n_periods, 4), np.float32)
    w[0, :] = (ffmc, bui, ws, wd)
    return w


@pytest.mark.parametrize("hours,period_min", [(4, 60), (9, 30), (1, 20)])
def test_burning_window_maps_the_clock(hours, period_min):
    """Under constant weather, no noise and nearest rounding, the rates are
    the same in every period, so a fire that only spreads during the first
    `hours` hours of each day reaches a cell at the real minute of the
    k-th burning minute, where k is the minute the unrestricted fire reaches
    it; over D days the windowed run has exactly the D hours-long spans."""
    fuel = inputs.fuel_grid(48, 48, 51)
    elev = inputs.elevation_grid(48, 48, 52, elev_max=500.0)
    days = 3
    per_day = 1440 // period_min
    n_win = days * per_day
    n_cont = days * hours * 60 // period_min
    c = int(np.flatnonzero(fuel.ravel() != 0)[1100])
    kw = dict(ignition_mode=0, ignition_cell=c, period_min=period_min)
    win = oracle.simulate(fuel, elev, _constant_weather(n_win), n_periods=n_win, burn_hours=hours, **kw)
    cont = oracle.simulate(fuel, elev, _constant_weather(n_win), n_periods=n_cont, **kw)
    np.testing.assert_array_equal(win["scar"], cont["scar"])
    k = cont["arrival_minute"][0]
    on = k >= 0
    span = hours * 60
    real = np.where(k == 0, 0, ((k - 1) // span) * 1440 + (k - 1) % span + 1)
    np.testing.assert_array_equal(win["arrival_minute"][0][on], real[on])
    assert cont["burned_cells"][0] > 30


def test_burning_window_of_24_hours_is_no_limit():
    fuel, elev, wx = _small(seed=61)
    kw = dict(n_periods=10, reps=5, seed=2, sigma=0.2, rounding=1, scenario_mode=1, ignition_mode=1)
    _same(oracle.simulate(fuel, elev, wx, burn_hours=24, **kw), oracle.simulate(fuel, elev, wx, **kw))


def test_option_bounds_are_checked():
    fuel, elev, wx = _small()
    with pytest.raises(ValueError):
        oracle.simulate(fuel, elev, wx, n_periods=4, ignition_period=4)
    with pytest.raises(ValueError):
        oracle.simulate(fuel, elev, wx, n_periods=4, burn_hours=25)
    with pytest.raises(ValueError):
        oracle.simulate(fuel, elev, wx, n_periods=4, ignition_mode=3)
