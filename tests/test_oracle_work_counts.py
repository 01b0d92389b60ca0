"""Pins for the oracle's work counts: burning-cell-periods, axis reach events
and ignitions (the units of the sending stage of Section 3.8 and App. A,
counted as the minute-stepping loop of Algorithm 1 meets them).

Hand traces on 1 x 3 strips of C-2 with no wind and no slope: the rate of
spread is 4.469 m/min on every axis, so the integer rate is 4 m/min and the
100 m between two centres take 25 minutes.
"""
import numpy as np
import pytest

import oracle

WX_CALM = np.tile(np.array([90.0, 80.0, 0.0, 0.0], np.float32), (8, 1))[None]


def _stats(ignition_cell, n_periods, period_min, **kw):
    fuel = np.full((1, 3), 2, np.uint8)
    r = oracle.simulate(fuel, None, WX_CALM, n_periods=n_periods, period_min=period_min,
                        ignition_cell=ignition_cell, **kw)
    return r, dict(zip(("ign", "bcm", "evals", "bp", "ax"), r["stats"].tolist()))


def test_calm_rate_is_four_metres_per_minute():
    q = oracle.eval_ros(np.full((1, 3), 2, np.uint8), None, WX_CALM)["q8"]
    assert q[1, 0] == 4 and q[1, 4] == 4


def test_centre_ignition_one_period_two_reaches():
    # cell 1 burns from minute 0, reaches cells 0 and 2 at minute 25; they
    # have no available neighbour left, so only cell 1 takes rates (once)
    r, s = _stats(1, n_periods=2, period_min=60)
    assert r["arrival_minute"][0].tolist() == [25, 0, 25]
    assert (s["ign"], s["bp"], s["ax"]) == (3, 1, 2)


def test_chain_hour_periods():
    # cell 0 takes rates in period 0 and reaches cell 1 at 25; cell 1 takes
    # rates at minute 26 (still period 0) and reaches cell 2 at 50
    r, s = _stats(0, n_periods=4, period_min=60)
    assert r["arrival_minute"][0].tolist() == [0, 25, 50]
    assert (s["ign"], s["bp"], s["ax"]) == (3, 2, 2)


def test_chain_half_hour_periods():
    # with 30-minute periods cell 1 burns across the period end: it takes
    # rates in period 0 (minutes 26-30) and again in period 1 (31-50)
    r, s = _stats(0, n_periods=4, period_min=30)
    assert r["arrival_minute"][0].tolist() == [0, 25, 50]
    assert (s["ign"], s["bp"], s["ax"]) == (3, 3, 2)


def test_ignition_with_no_available_neighbour_takes_no_burning_period():
    fuel = np.array([[0, 2, 0]], np.uint8)
    r = oracle.simulate(fuel, None, WX_CALM, n_periods=2, ignition_cell=1)
    ign, _, evals, bp, ax = r["stats"].tolist()
    assert (ign, bp, ax) == (1, 0, 0)
    assert evals == 1          # its rates are still taken once, at minute 1


def test_burned_out_cell_counts_its_period_and_no_reach():
    # delta above every rate: the ignition takes rates once and spreads nowhere
    r, s = _stats(1, n_periods=3, period_min=60, burnout=5.0)
    assert (s["ign"], s["bp"], s["ax"]) == (1, 1, 0)


@pytest.mark.parametrize("seed", range(4))
def test_counts_against_outputs(seed):
    """Ignitions equal the burned cells; every burned cell other than a
    replication's ignition was reached at least once (an axis reach event);
    a burning-cell-period needs a burned cell."""
    rng = np.random.default_rng(seed)
    fuel = rng.integers(0, 16, (24, 30)).astype(np.uint8)
    elev = rng.integers(0, 300, (24, 30)).astype(np.int16)
    wx = rng.uniform([84, 30, 0, 0], [96, 120, 40, 360], (2, 12, 4)).astype(np.float32)
    r = oracle.simulate(fuel, elev, wx, n_periods=12, period_min=[60, 30, 20, 60][seed], reps=5,
                        seed=seed, sigma=0.2, rounding=1, ignition_mode=1, scenario_mode=1,
                        threshold=[0.0, 1.0, 0.0, 3.0][seed])
    ign, _, evals, bp, ax = r["stats"].tolist()
    assert ign == int(r["burned_cells"].sum())
    assert ax >= ign - 5
    assert 0 < bp <= evals
    assert bp <= ign * 12
