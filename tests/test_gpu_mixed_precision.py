"""FP64 results from the FP32-first evaluation (precision 0): on inputs chosen
to be hard for it (steep slopes, crowning weather, build-up up to 250, all
18 fuels, winds exactly at the 40 km/h switch of f(W), grass at 1 km/h),
the integer rates equal floor(x + 1/2) of the same call's FP64 rates, and
the oracle's integer rates, with noise and with stochastic rounding."""
import sys

import numpy as np
import pytest

import oracle
from paper_1905_09317_amd import Simulator, inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim():
    s = Simulator(0)
    yield s
    s.close()


def _self_consistent(out, burn):
    """q8 of a nearest-rounding call against floor(x8 + 1/2) of its FP64 x8."""
    x = out["x8"][burn]
    want = np.floor(x + 0.5)
    want = np.where(want < 2 ** 30, want, 2 ** 30).astype(np.int64)
    bad = np.argwhere(out["q8"][burn] != want)
    assert bad.size == 0, (len(bad), x[tuple(bad[0])], out["q8"][burn][tuple(bad[0])])


@pytest.mark.parametrize("trial", range(4))
def test_harsh_landscapes_integer_rates_are_fp64(sim, trial):
    rng = np.random.default_rng(700 + trial)
    rows, cols = 384, 320
    fuel = rng.integers(1, 19, (rows, cols)).astype(np.uint8)
    elev = inputs.elevation_grid(rows, cols, 710 + trial, elev_max=[800.0, 3000.0, 2000.0, 5000.0][trial])
    cell_m = [100, 100, 30, 50][trial]
    land = sim.load_landscape(fuel, elev, cell_m=cell_m, pc=float(rng.uniform(0, 100)),
                              curing=float(rng.uniform(30, 100)))
    sim.set_landscape_fbp(land, fmc=[97.0, 85.0, 120.0, 100.0][trial], pdf=[50.0, 20.0, 80.0, 100.0][trial])
    wx = np.zeros((2, 6, 4), np.float32)
    wx[..., 0] = rng.uniform(80, 99, (2, 6))
    wx[..., 1] = rng.uniform(0, 250, (2, 6))
    wx[..., 2] = rng.uniform(0, 80, (2, 6))
    wx[..., 3] = rng.uniform(0, 360, (2, 6))
    wx[1, :3, 2] = 40.0                       # wind exactly at the f(W) switch
    w = sim.set_weather(wx)
    burn = fuel.ravel() != 0
    _say(f"mixed precision: harsh trial {trial}")
    for s in range(2):
        for p in range(6):
            for sigma in (0.0, 0.3):
                out = sim.eval_ros(land, w, scenario=s, period=p, rep=p + 1, seed=23, sigma=sigma, rounding=0,
                                   precision=0)
                _self_consistent(out, burn)
    sim.unload_landscape(land)
    sim.unset_weather(w)


def test_winds_at_the_switch_and_grass_at_one_kmh_match_the_oracle(sim):
    """Flat ground, so the effective wind is the weather's own: 40 km/h from
    96 directions for every fuel, and about 1 km/h for the grasses, where
    FP32 and FP64 may round the speed to different sides of the switch."""
    fuel = np.tile(np.arange(1, 19, dtype=np.uint8), (4, 1))
    n = 96
    wx = np.zeros((1, n, 4), np.float32)
    wx[0, :, 0] = np.resize([88.0, 92.0, 95.0, 98.0], n)
    wx[0, :, 1] = np.resize([40.0, 80.0, 120.0, 200.0], n)
    wx[0, :, 2] = 40.0
    wx[0, :, 3] = 3.75 * np.arange(n)
    land = sim.load_landscape(fuel, None)
    w = sim.set_weather(wx)
    burn = fuel.ravel() != 0
    _say("mixed precision: 40 km/h winds")
    for p in range(n):
        out = sim.eval_ros(land, w, period=p, precision=0)
        _self_consistent(out, burn)
        assert np.array_equal(out["q8"], oracle.eval_ros(fuel, None, wx, period=p)["q8"]), p
    sim.unload_landscape(land)
    sim.unset_weather(w)
    grass = np.tile(np.array([[14, 15]], np.uint8), (4, 4))
    wg = np.zeros((1, 6, 4), np.float32)
    wg[0, :, 0] = 90.0
    wg[0, :, 1] = 60.0
    wg[0, :, 2] = (1.0, np.nextafter(np.float32(1.0), np.float32(2.0)), np.nextafter(np.float32(1.0),
                                                                                     np.float32(0.0)),
                   1.0, 1.0, 1.0)
    wg[0, :, 3] = (10.0, 100.0, 250.0, 33.3, 123.4, 301.7)
    land_g = sim.load_landscape(grass, None, curing=90.0)
    w = sim.set_weather(wg)
    for p in range(6):
        out = sim.eval_ros(land_g, w, period=p, precision=0)
        _self_consistent(out, grass.ravel() != 0)
        assert np.array_equal(out["q8"], oracle.eval_ros(grass, None, wg, period=p, curing=90.0)["q8"]), p
    sim.unload_landscape(land_g)
    sim.unset_weather(w)


def test_stochastic_rounding_on_steep_ground_matches_the_oracle(sim):
    rng = np.random.default_rng(811)
    fuel = rng.integers(1, 19, (96, 80)).astype(np.uint8)
    elev = inputs.elevation_grid(96, 80, 812, elev_max=2500.0)
    land = sim.load_landscape(fuel, elev, cell_m=40, pc=35.0, curing=70.0)
    sim.set_landscape_fbp(land, fmc=105.0, pdf=60.0)
    wx = np.zeros((1, 4, 4), np.float32)
    wx[0, :, 0] = (86.0, 91.0, 96.0, 99.0)
    wx[0, :, 1] = (30.0, 90.0, 150.0, 240.0)
    wx[0, :, 2] = (10.0, 40.0, 25.0, 65.0)
    wx[0, :, 3] = (20.0, 140.0, 250.0, 330.0)
    w = sim.set_weather(wx)
    for p in range(4):
        g = sim.eval_ros(land, w, period=p, rep=9, seed=31, sigma=0.25, rounding=1, precision=0)
        o = oracle.eval_ros(fuel, elev, wx, period=p, rep=9, seed=31, sigma=np.float32(0.25).item(), rounding=1,
                            cell_m=40, pc=35.0, curing=70.0, fmc=105.0, pdf=60.0)
        assert np.array_equal(g["q8"], o["q8"]), p
    sim.unload_landscape(land)
    sim.unset_weather(w)


@pytest.mark.parametrize("seed", range(12))
def test_random_settings_match_the_oracle(sim, seed):
    """Random grids, slopes, landscape settings and weather (including calm,
    40 km/h and storm winds), noise and stochastic rounding: the integer
    rates of precision 0 equal the oracle's."""
    rng = np.random.default_rng(900 + seed)
    rows, cols = int(rng.integers(24, 72)), int(rng.integers(24, 72))
    fuel = rng.integers(1, 19, (rows, cols)).astype(np.uint8)
    elev = inputs.elevation_grid(rows, cols, 950 + seed, elev_max=float(rng.choice([0.0, 400.0, 2500.0, 6000.0])))
    cell_m = int(rng.choice([25, 50, 100, 250]))
    pc, curing = float(rng.uniform(0, 100)), float(rng.uniform(0, 100))
    fmc, pdf = float(rng.uniform(80, 130)), float(rng.uniform(0, 100))
    land = sim.load_landscape(fuel, elev, cell_m=cell_m, pc=pc, curing=curing)
    sim.set_landscape_fbp(land, fmc=fmc, pdf=pdf)
    n_p = 6
    wx = np.zeros((1, n_p, 4), np.float32)
    wx[0, :, 0] = rng.uniform(70, 99, n_p)
    wx[0, :, 1] = rng.uniform(0, 300, n_p)
    wx[0, :, 2] = rng.choice([0.0, 1.0, 5.0, 39.99, 40.0, 40.01, 60.0, 120.0], n_p)
    wx[0, :, 3] = rng.uniform(0, 360, n_p)
    w = sim.set_weather(wx)
    sigma = float(np.float32(rng.choice([0.0, 0.15, 0.4])))
    rounding = int(rng.integers(0, 2))
    _say(f"mixed precision: random settings seed {seed} {rows}x{cols} cell {cell_m}")
    for p in range(n_p):
        g = sim.eval_ros(land, w, period=p, rep=seed, seed=77 + seed, sigma=sigma, rounding=rounding, precision=0)
        o = oracle.eval_ros(fuel, elev, wx, period=p, rep=seed, seed=77 + seed, sigma=sigma, rounding=rounding,
                            cell_m=cell_m, pc=pc, curing=curing, fmc=fmc, pdf=pdf)
        assert np.array_equal(g["q8"], o["q8"]), (p, int((g["q8"] != o["q8"]).sum()))
    sim.unload_landscape(land)
    sim.unset_weather(w)
