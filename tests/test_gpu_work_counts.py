"""c2f_count_work against the oracle's own counts: burning-cell-periods, axis
reach events and ignitions (the sending stage's units, Section 3.8 and
App. A) must be equal, on grids with noise, stochastic rounding,
thresholds, burning windows, burn-out, later ignitions, ignition lists and
scenario draws.  The arrival minutes come from the GPU run, which the
parity tests show equal to the oracle's."""
import sys

import numpy as np
import pytest

from paper_1905_09317_amd import Request, Simulator, inputs

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


def _check(sim, fuel, elev, wx, period_min, **kw):
    land = sim.load_landscape(fuel, elev)
    w = sim.set_weather(wx, period_min=period_min)
    req = Request(landscape=land, weather=w, outputs=("arrival_minute", "burned_cells"), device_out=True,
                  **kw)
    g = sim.simulate(req)
    got = sim.count_work(req, g["arrival_minute"])
    okw = {k: v for k, v in kw.items() if k != "precision"}
    r = oracle_run(fuel, elev, wx, period_min=period_min, **okw)
    assert_same_outputs({k: v.cpu().numpy() for k, v in g.items()}, r, ("arrival_minute", "burned_cells"))
    want = {"ignitions": int(r["stats"][0]), "burning_cell_periods": int(r["stats"][3]),
            "axis_reaches": int(r["stats"][4])}
    sim.unload_landscape(land)
    sim.unset_weather(w)
    assert got == want, (got, want)
    return got


def test_strip_hand_traces(sim):
    _say("work counts: 1x3 strips")
    wx = np.tile(np.array([90.0, 80.0, 0.0, 0.0], np.float32), (8, 1))[None]
    fuel = np.full((1, 3), 2, np.uint8)
    assert _check(sim, fuel, None, wx, 60, n_periods=2, ignition_cell=1) == {
        "burning_cell_periods": 1, "axis_reaches": 2, "ignitions": 3}
    assert _check(sim, fuel, None, wx, 30, n_periods=4, ignition_cell=0) == {
        "burning_cell_periods": 3, "axis_reaches": 2, "ignitions": 3}


def test_tiny_workload(sim):
    w = inputs.tiny_c2()
    _say("work counts: 20x20")
    got = _check(sim, w.fuel, w.elev, w.weather, w.period_min, n_periods=w.n_periods,
                 ignition_cell=w.ignition_cell)
    assert got["ignitions"] == 226


@pytest.mark.parametrize("seed", range(10))
def test_random_cases(sim, seed):
    rng = np.random.default_rng(500 + seed)
    rows, cols = [(37, 29), (64, 48), (20, 90), (50, 50)][seed % 4]
    fuel = rng.integers(1, 16, (rows, cols)).astype(np.uint8)
    fuel[rng.random((rows, cols)) < 0.1] = 0
    elev = rng.integers(0, 300, (rows, cols)).astype(np.int16)
    n_periods = 12
    wx = rng.uniform([84, 30, 0, 0], [96, 120, 45, 360], (3, n_periods, 4)).astype(np.float32)
    P = [60, 30, 20, 15, 60, 12, 60, 30, 10, 60][seed]
    kw = dict(n_periods=n_periods, reps=4, seed=900 + seed, sigma=[0.0, 0.15, 0.3][seed % 3],
              rounding=seed % 2, threshold=[0.0, 0.0, 2.0, 5.0][seed % 4], ignition_mode=[1, 2][seed % 2],
              scenario_mode=1, precision=0)
    if seed in (2, 5):
        kw["burn_hours"] = 3 if P <= 30 else 1
    if seed in (3, 6):
        kw["burnout"] = 3.0
    if seed == 4:
        kw["ignition_period"] = 2
    if seed in (7, 9):
        kw.pop("ignition_mode")
        kw["ignitions"] = [[rows * cols // 3, 0], [rows * cols // 2 + 5, 1], [7, 1], [rows * cols - 3, 4]]
    _say(f"work counts: random seed={seed} {rows}x{cols} P={P}")
    _check(sim, fuel, elev, wx, P, **kw)
