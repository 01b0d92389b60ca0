"""GPU parity for the FBP System's crown fire, fuel consumption and head fire
intensity (Section 2.3), the intensity burn-out of assumption A5 (iv), and
fuels D-2, M-3, M-4: rate fields (with crown fraction burned and intensity)
against the oracle within 1e-11 relative in FP64 and 1e-5 in FP32, and
propagation outputs bit-exact in FP64."""
import sys

import numpy as np
import pytest

import oracle
from paper_1905_09317_amd import Request, Simulator, inputs

from _helpers import assert_same_outputs, boundary_case, oracle_run

pytestmark = pytest.mark.gpu

ALL = ("scar", "arrival_period", "arrival_minute", "burn_count", "burned_cells", "ignition_cell",
       "scenario")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim():
    s = Simulator(0)
    yield s
    s.close()


def _all_fuels(seed, rows, cols, nonfuel=0.05):
    rng = np.random.default_rng(seed)
    fuel = rng.integers(1, 19, (rows, cols)).astype(np.uint8)
    fuel[rng.random((rows, cols)) < nonfuel] = 0
    return fuel


def _crowning_weather(seed, n_scen, n_periods):
    rng = np.random.default_rng(seed)
    w = np.zeros((n_scen, n_periods, 4), np.float32)
    w[..., 0] = rng.uniform(84, 98, (n_scen, n_periods))
    w[..., 1] = rng.uniform(0, 200, (n_scen, n_periods))
    w[..., 2] = rng.uniform(0, 60, (n_scen, n_periods))
    w[..., 3] = rng.uniform(0, 360, (n_scen, n_periods))
    w[0, 0] = (88.0, 0.0, 0.0, 0.0)       # no build-up: no surface consumption
    return w


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("sigma,rounding", [(0.0, 0), (0.2, 1)])
def test_crown_rate_field_parity(sim, precision, sigma, rounding):
    _say(f"crown rate field precision={precision} sigma={sigma}")
    fuel = _all_fuels(31, 90, 70)
    elev = inputs.elevation_grid(90, 70, 32, elev_max=1200.0)
    wx = _crowning_weather(33, 2, 5)
    land = sim.load_landscape(fuel, elev, pc=60.0, curing=85.0)
    sim.set_landscape_fbp(land, fmc=112.0, pdf=35.0)
    w = sim.set_weather(wx)
    tol = 1e-5 if precision == 1 else 1e-11
    qtol = 1e-5 if precision == 1 else 1e-12
    n_audit = 0
    burn = fuel.ravel() != 0
    crowned = 0
    for s in range(2):
        for p in range(5):
            g = sim.eval_ros(land, w, scenario=s, period=p, rep=4, seed=77, sigma=sigma, rounding=rounding,
                             precision=precision)
            o = oracle.eval_ros(fuel, elev, wx, scenario=s, period=p, rep=4, seed=77,
                                sigma=np.float32(sigma).item(), rounding=rounding, pc=60.0, curing=85.0,
                                fmc=112.0, pdf=35.0)
            for k in ("hros", "bros", "fros", "lb", "hfi"):
                np.testing.assert_allclose(g[k], o[k], rtol=tol, atol=1e-9, err_msg=k)
            np.testing.assert_allclose(g["cfb"], o["cfb"], rtol=0, atol=10 * tol, err_msg="cfb")
            np.testing.assert_allclose(g["x8"], o["x8"], rtol=tol, atol=1e-9)
            crowned += int((o["cfb"][burn] > 0).sum())
            diff = g["q8"] != o["q8"]
            if diff.any():
                assert np.all(boundary_case(o["xu8"][diff], o["x8"][diff], qtol))
                n_audit += int(diff.sum())
    assert crowned > 100
    if precision == 0:
        assert n_audit == 0
    sim.unload_landscape(land)
    sim.unset_weather(w)


def test_every_fuel_code_flat(sim):
    """Each of the 19 codes at one weather row that crowns the conifers."""
    fuel = np.arange(19, dtype=np.uint8).reshape(1, 19)
    wx = np.array([[[95.0, 110.0, 30.0, 200.0]]], np.float32)
    land = sim.load_landscape(fuel, None)
    w = sim.set_weather(wx)
    g = sim.eval_ros(land, w)
    o = oracle.eval_ros(fuel, None, wx)
    for k in ("hros", "bros", "lb", "cfb", "hfi"):
        np.testing.assert_allclose(g[k], o[k], rtol=1e-12, atol=1e-12, err_msg=k)
    assert np.all(o["cfb"][[1, 2, 3, 4, 6, 9, 10, 17, 18]] > 0)


def _run_both(sim, fuel, elev, wx, period_min=60, fmc=97.0, pdf=50.0, **kw):
    land = sim.load_landscape(fuel, elev)
    sim.set_landscape_fbp(land, fmc=fmc, pdf=pdf)
    w = sim.set_weather(wx, period_min=period_min)
    g = sim.simulate(Request(landscape=land, weather=w, **kw))
    okw = {k: v for k, v in kw.items() if k != "precision"}
    r = oracle_run(fuel, elev, wx, period_min=period_min, fmc=fmc, pdf=pdf, **okw)
    sim.unload_landscape(land)
    sim.unset_weather(w)
    return g, r


@pytest.mark.parametrize("seed", range(8))
def test_propagation_with_new_fuels_and_intensity_cutoff(sim, seed):
    rows, cols = [(40, 50), (64, 64), (30, 90), (50, 40)][seed % 4]
    fuel = _all_fuels(400 + seed, rows, cols)
    elev = inputs.elevation_grid(rows, cols, 500 + seed, elev_max=600.0)
    wx = _crowning_weather(600 + seed, 3, 10)
    P = [60, 30, 20, 60, 15, 60, 30, 60][seed]
    kw = dict(n_periods=10, reps=5, seed=70 + seed, sigma=[0.0, 0.15, 0.3][seed % 3], rounding=seed % 2,
              threshold=[0.0, 0.0, 1.5, 0.0][seed % 4], ignition_mode=[1, 2][seed % 2], scenario_mode=1,
              hfi_min=[0.0, 300.0, 1500.0, 6000.0][seed % 4], precision=0)
    if seed == 5:
        kw["burnout"] = 2.0
    _say(f"crown propagation seed={seed} {rows}x{cols} P={P} hfi_min={kw['hfi_min']}")
    g, r = _run_both(sim, fuel, elev, wx, period_min=P, fmc=[97.0, 85.0, 120.0, 100.0][seed % 4],
                     pdf=[50.0, 20.0, 80.0, 100.0][seed % 4], **kw)
    assert_same_outputs(g, r, ALL, where=f"crown seed {seed}")


def test_huge_intensity_threshold_stops_every_fire_at_its_ignition(sim):
    fuel = _all_fuels(9, 48, 48, nonfuel=0.0)
    wx = _crowning_weather(10, 1, 6)
    g, r = _run_both(sim, fuel, None, wx, n_periods=6, reps=7, seed=3, ignition_mode=1, hfi_min=1e9)
    assert_same_outputs(g, r, ALL, where="huge hfi_min")
    assert np.all(g["burned_cells"] == 1)


def test_work_counts_with_intensity_cutoff(sim):
    fuel = _all_fuels(12, 60, 60)
    elev = inputs.elevation_grid(60, 60, 13, elev_max=400.0)
    wx = _crowning_weather(14, 2, 8)
    land = sim.load_landscape(fuel, elev)
    w = sim.set_weather(wx)
    req = Request(landscape=land, weather=w, n_periods=8, reps=4, seed=5, sigma=0.2, rounding=1,
                  ignition_mode=1, scenario_mode=1, hfi_min=800.0, outputs=("arrival_minute",),
                  device_out=True)
    got = sim.count_work(req, sim.simulate(req)["arrival_minute"])
    r = oracle_run(fuel, elev, wx, n_periods=8, reps=4, seed=5, sigma=0.2, rounding=1, ignition_mode=1,
                   scenario_mode=1, hfi_min=800.0)
    assert got == {"ignitions": int(r["stats"][0]), "burning_cell_periods": int(r["stats"][3]),
                   "axis_reaches": int(r["stats"][4])}
    sim.unload_landscape(land)
    sim.unset_weather(w)


def test_landscape_fbp_argument_checks(sim):
    land = sim.load_landscape(np.full((4, 4), 6, np.uint8))
    for fmc, pdf in ((0.0, 50.0), (301.0, 50.0), (97.0, -1.0), (97.0, 101.0)):
        with pytest.raises(Exception):
            sim.set_landscape_fbp(land, fmc=fmc, pdf=pdf)
    w = sim.set_weather(np.tile(np.array([90, 80, 10, 0], np.float32), (2, 1)))
    with pytest.raises(Exception):
        sim.simulate(Request(landscape=land, weather=w, n_periods=1, hfi_min=-1.0))
    sim.unload_landscape(land)
    sim.unset_weather(w)
