"""Parity at the full sizes of the measured workloads, in the launch
configuration bench.py times: the whole single fire against the oracle, and
the burn-count maps and every replication's area of the batched (2048
replications) and large (64 replications) launches against the oracle run
over all their replications, sharded over host processes."""
import sys

import numpy as np
import pytest

from paper_1905_09317_amd import Request, Simulator, inputs

from _helpers import (assert_same_outputs, dilate, fp32_overrides, oracle_kwargs, oracle_run, oracle_sharded,
                      request_kwargs)

pytestmark = pytest.mark.gpu

SINGLE_OUTS = ("scar", "arrival_period", "burn_count", "burned_cells")
MC_OUTS = ("burn_count", "burned_cells")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim():
    s = Simulator(0)
    yield s
    s.close()


def _run(sim, w, outputs, **over):
    land = sim.load_landscape(w.fuel, w.elev, cell_m=w.cell_m, pc=w.pc, curing=w.curing)
    wx = sim.set_weather(w.weather, period_min=w.period_min)
    g = sim.simulate(Request(landscape=land, weather=wx, outputs=outputs, **request_kwargs(w, **over)))
    return land, wx, g


def test_single_fire_2048_fp64_full():
    w = inputs.single_large_fire(side=2048, n_periods=48, precision=0)
    with Simulator(0) as sim:
        _say(f"[fullsize] {w.name} fp64")
        _, _, g = _run(sim, w, SINGLE_OUTS)
        st = sim.stats()
    assert st["grid_blocks"] == 1 and st["block_threads"] == 512
    ref = oracle_run(w.fuel, w.elev, w.weather, **oracle_kwargs(w))
    assert_same_outputs(g, ref, SINGLE_OUTS, where="single fire fp64")
    assert int(g["burned_cells"][0]) > 10000


def test_single_fire_2048_fp32_full_with_audited_rates():
    """The bench's single-fire workload (FP32 rates).  Integer rates are
    audited on every cell that burns in either run and its neighbours, for
    every period; audited boundary cases are replayed into the oracle."""
    w = inputs.single_large_fire(side=2048, n_periods=48, precision=1)
    with Simulator(0) as sim:
        _say(f"[fullsize] {w.name} fp32")
        land, wx, g = _run(sim, w, SINGLE_OUTS)
        ref0 = oracle_run(w.fuel, w.elev, w.weather, **oracle_kwargs(w))
        burnt = (np.asarray(g["scar"][0]) | ref0["scar"][0]).reshape(w.rows, w.cols).astype(bool)
        cells = np.nonzero(dilate(burnt, 1).ravel())[0]
        _say(f"[fullsize] auditing {cells.size} cells x {w.n_periods} periods")
        keys, qs, n = fp32_overrides(sim, land, wx, w.fuel, w.elev, w.weather, reps=1,
                                     n_periods=w.n_periods, seed=w.seed, sigma=w.sigma,
                                     rounding=w.rounding, scenarios=[0], cells=cells)
    _say(f"[fullsize] {len(keys)} boundary cases in {n} audited integer rates")
    ref = oracle_run(w.fuel, w.elev, w.weather, overrides=(keys, qs), **oracle_kwargs(w))
    assert_same_outputs(g, ref, SINGLE_OUTS, where="single fire fp32")


def _full_mc(sim, w):
    """The workload's launch (as bench.py times it) against the oracle over
    every replication: burn counts element by element and every area."""
    _, _, g = _run(sim, w, MC_OUTS)
    st = sim.stats()
    _say(f"[fullsize] {w.name}: oracle over all {w.reps} replications, sharded")
    ref = oracle_sharded(w.fuel, w.elev, w.weather, w.reps,
                         **{k: v for k, v in oracle_kwargs(w).items() if k != "reps"})
    assert_same_outputs(g, ref, MC_OUTS, where=w.name)
    assert (np.asarray(g["burned_cells"]) >= 1).all()   # every replication ignites a burnable cell
    return g, st


def test_batched_mc_1024_2048reps_full(sim):
    w = inputs.batched_monte_carlo(side=1024, reps=2048, n_scenarios=100, n_periods=48)
    _, st = _full_mc(sim, w)
    assert st["grid_blocks"] == 512 and st["relaunches"] == 0 and st["rep_order"] == 1


def test_large_8192_64reps_full(sim):
    w = inputs.large_landscape(side=8192, reps=64, n_periods=72)
    _, st = _full_mc(sim, w)
    assert st["grid_blocks"] == 64 and st["block_threads"] == 512


def test_single_fire_2048_fp64_ignition_list_window_burnout():
    """The 2048^2 x 48 h fire (FP64 rates, one 512-thread group) lit from five
    listed cells at periods 0 to 30, with a 12 h daily burning window and a
    burn-out threshold, element by element against the oracle."""
    w = inputs.single_large_fire(side=2048, n_periods=48, precision=0)
    rng = np.random.default_rng(41)
    cells = rng.choice(np.flatnonzero(w.fuel.ravel() != 0), 5, replace=False)
    seeds = np.stack([cells, [0, 6, 12, 20, 30]], axis=1).astype(np.int32)
    over = dict(ignitions=seeds, burn_hours=12, burnout=1.0)
    outs = SINGLE_OUTS + ("arrival_minute",)
    with Simulator(0) as sim:
        _say(f"[fullsize] {w.name} fp64, ignition list, window, burn-out")
        _, _, g = _run(sim, w, outs, **over)
        st = sim.stats()
    assert st["grid_blocks"] == 1 and st["block_threads"] == 512
    ref = oracle_run(w.fuel, w.elev, w.weather, **oracle_kwargs(w, **over))
    assert_same_outputs(g, ref, outs, where="single fire, ignition list")
    m = np.asarray(g["arrival_minute"])[0]
    assert (m[seeds[:, 0]] <= seeds[:, 1] * w.period_min).all()


def test_batched_mc_1024_2048reps_ignition_map_sampled(sim):
    """The batched workload with ignitions drawn from a map, lit at period 2,
    and a burn-out threshold: properties at full size and sampled
    replications against the oracle."""
    w = inputs.batched_monte_carlo(side=1024, reps=2048, n_scenarios=100, n_periods=48)
    rng = np.random.default_rng(43)
    weights = np.where(w.fuel.ravel() != 0, rng.integers(0, 1000, w.fuel.size), 0).astype(np.uint32)
    over = dict(ignition_mode=3, ignition_period=2, burnout=2.0)
    land = sim.load_landscape(w.fuel, w.elev, cell_m=w.cell_m, pc=w.pc, curing=w.curing)
    sim.set_ignition_map(land, weights)
    wx = sim.set_weather(w.weather, period_min=w.period_min)
    _say(f"[fullsize] {w.name}, ignition map")
    outs = MC_OUTS + ("ignition_cell",)
    g = sim.simulate(Request(landscape=land, weather=wx, outputs=outs, **request_kwargs(w, **over)))
    st = sim.stats()
    assert st["grid_blocks"] == 512 and st["relaunches"] == 0
    burned = np.asarray(g["burned_cells"])
    counts = np.asarray(g["burn_count"]).view(np.uint32)
    assert int(counts.sum(dtype=np.int64)) == int(burned.sum())
    assert (weights[np.asarray(g["ignition_cell"])] > 0).all()
    for r in (0, 1023, 2047):
        _say(f"[fullsize] {w.name}, ignition map: oracle replication {r}")
        ref = oracle_run(w.fuel, w.elev, w.weather, want_rep_outputs=False, ignition_weights=weights,
                         **oracle_kwargs(w, reps=1, rep_offset=r, **over))
        assert int(burned[r]) == int(ref["burned_cells"][0]), f"replication {r}"
        assert int(np.asarray(g["ignition_cell"])[r]) == int(ref["ignition_cell"][0])
    sim.unload_landscape(land)
    sim.unset_weather(wx)


def test_treatment_plans_1024_fused_sampled(sim):
    """Two fuel-treatment plans of the batched landscape (a 3-cell fuel break
    and 5 % harvested cells each) fused with the untreated landscape in one
    launch of 3 x 256 replications; sampled replications of each plan against
    the oracle on the edited grid."""
    w = inputs.batched_monte_carlo(side=1024, reps=256, n_scenarios=100, n_periods=48)
    rng = np.random.default_rng(47)
    base = sim.load_landscape(w.fuel, w.elev, cell_m=w.cell_m, pc=w.pc, curing=w.curing)
    wx = sim.set_weather(w.weather, period_min=w.period_min)
    lids, grids = [base], [w.fuel]
    for _ in range(2):
        c0 = int(rng.integers(8, w.cols - 11))
        strip = (np.arange(w.rows)[:, None] * w.cols + np.arange(c0, c0 + 3)[None, :]).ravel()
        cut = rng.choice(w.rows * w.cols, w.rows * w.cols // 20, replace=False)
        cells = np.concatenate([strip, cut]).astype(np.int32)
        lids.append(sim.derive_landscape(base, cells, 0))
        f = w.fuel.copy().ravel()
        f[cells] = 0
        grids.append(f.reshape(w.fuel.shape))
    _say("[fullsize] treatment plans, fused launch")
    outs = sim.simulate_batch([Request(landscape=lid, weather=wx, outputs=MC_OUTS, **request_kwargs(w))
                               for lid in lids])
    for k, r in ((0, 5), (1, 0), (1, 200), (2, 255)):
        _say(f"[fullsize] treatment plan {k}: oracle replication {r}")
        ref = oracle_run(grids[k], w.elev, w.weather, want_rep_outputs=False,
                         **oracle_kwargs(w, reps=1, rep_offset=r))
        assert int(np.asarray(outs[k]["burned_cells"])[r]) == int(ref["burned_cells"][0]), (k, r)
    for k in range(3):
        c = np.asarray(outs[k]["burn_count"]).view(np.uint32)
        assert int(c.sum(dtype=np.int64)) == int(np.asarray(outs[k]["burned_cells"]).sum())
        if k:
            assert (c.reshape(w.fuel.shape)[grids[k] == 0] == 0).all()   # treated cells never burn
    for lid in lids[1:]:
        sim.unload_landscape(lid)
    sim.unload_landscape(base)
    sim.unset_weather(wx)


def test_batched_mc_1024_2048reps_fp32_audited_in_launch(sim):
    """The batched workload with FP32 rates (2048 replications in one launch,
    as `bench.py --workload batched --precision 1` times it).  The launch
    fuses two requests of the one landscape, replications 0..2039 and
    2040..2047, the second returning its scars: 2048 work items in one
    launch.  Every cell that burns in either precision, and
    its neighbours, has its integer rates audited against the FP64 oracle
    for every period; the audited boundary cases are replayed into the
    oracle, which must then give the same scars and areas."""
    w = inputs.batched_monte_carlo(side=1024, reps=2048, n_scenarios=100, n_periods=48, precision=1)
    _say(f"[fullsize] {w.name} fp32")
    land = sim.load_landscape(w.fuel, w.elev, cell_m=w.cell_m, pc=w.pc, curing=w.curing)
    wx = sim.set_weather(w.weather, period_min=w.period_min)
    head = Request(landscape=land, weather=wx, outputs=MC_OUTS, **request_kwargs(w, reps=2040))
    tail = Request(landscape=land, weather=wx, outputs=("scar", "burned_cells", "scenario", "burn_count"),
                   **request_kwargs(w, reps=8, rep_offset=2040))
    g0, g1 = sim.simulate_batch([head, tail])
    st = sim.stats()
    # one launch whose groups each run several replications, longest first
    assert st["relaunches"] == 0 and st["grid_blocks"] < 2048 and st["rep_order"] == 1
    burned = np.concatenate([np.asarray(g0["burned_cells"]), np.asarray(g1["burned_cells"])])
    counts = np.asarray(g0["burn_count"]).view(np.uint32).astype(np.int64) + \
        np.asarray(g1["burn_count"]).view(np.uint32)
    assert int(counts.sum()) == int(burned.sum())
    for k in (0, 4, 7):
        r = 2040 + k
        scen = int(np.asarray(g1["scenario"])[k])
        ref0 = oracle_run(w.fuel, w.elev, w.weather, **oracle_kwargs(w, reps=1, rep_offset=r))
        assert scen == int(ref0["scenario"][0])
        burnt = (np.asarray(g1["scar"][k]) | ref0["scar"][0]).reshape(w.rows, w.cols).astype(bool)
        cells = np.nonzero(dilate(burnt, 1).ravel())[0]
        _say(f"[fullsize] replication {r}: auditing {cells.size} cells x {w.n_periods} periods")
        keys, qs, n = fp32_overrides(sim, land, wx, w.fuel, w.elev, w.weather, reps=1, rep_ids=[r],
                                     n_periods=w.n_periods, seed=w.seed, sigma=w.sigma, rounding=w.rounding,
                                     scenarios=[scen], cells=cells)
        _say(f"[fullsize] replication {r}: {len(keys)} boundary cases in {n} audited integer rates")
        ref = oracle_run(w.fuel, w.elev, w.weather, overrides=(keys, qs),
                         **oracle_kwargs(w, reps=1, rep_offset=r))
        got = {"scar": np.asarray(g1["scar"][k:k + 1]), "burned_cells": np.asarray(g1["burned_cells"][k:k + 1])}
        assert_same_outputs(got, ref, ("scar", "burned_cells"), where=f"fp32 replication {r} in the launch")
    sim.unload_landscape(land)
    sim.unset_weather(wx)
