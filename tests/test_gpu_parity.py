"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Rates: FBP fields within 1e-5 relative (FP64 mode agrees to ~1e-12);
integer axis rates equal except where the oracle's floored value is within
rounding distance of an integer (audited; FP64 mode expects none).
Propagation: scars, arrival minutes and periods, burn counts and per-rep
areas bit-exact.  FP32 mode replays the FP32 integer rates of audited
boundary cases in the oracle (data only) and is then bit-exact too.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1905_09317_amd import Request, Simulator, inputs

from _helpers import (assert_same_outputs, boundary_case, fp32_overrides, oracle_kwargs,
                      oracle_run, request_kwargs)

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim():
    s = Simulator(0)
    yield s
    s.close()


# ------------------------------------------------------------- FBP field

def _wx_random(n_scen, n_periods, seed):
    rng = np.random.default_rng(seed)
    w = np.zeros((n_scen, n_periods, 4), np.float32)
    w[..., 0] = rng.uniform(70, 101, (n_scen, n_periods))
    w[..., 1] = rng.uniform(0, 200, (n_scen, n_periods))
    w[..., 2] = rng.uniform(0, 80, (n_scen, n_periods))
    w[..., 3] = rng.uniform(0, 360, (n_scen, n_periods))
    w[0, 0] = (90.0, 80.0, 0.0, 0.0)        # no wind
    w[0, 1] = (90.0, 64.0, 40.0, 270.0)     # the f(W) branch point
    return w


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("sigma,rounding", [(0.0, 0), (0.15, 1), (0.5, 1)])
def test_rate_field_parity(sim, precision, sigma, rounding):
    _say(f"rate field precision={precision} sigma={sigma}")
    fuel = inputs.fuel_grid(96, 80, 21)
    elev = inputs.elevation_grid(96, 80, 22, elev_max=1500.0)
    wx = _wx_random(2, 6, 23)
    land = sim.load_landscape(fuel, elev, cell_m=100, pc=35.0, curing=70.0)
    w = sim.set_weather(wx)
    tol = 1e-5 if precision == 1 else 1e-11
    qtol = 1e-5 if precision == 1 else 1e-12
    n_audit = 0
    for s in range(2):
        for p in range(6):
            g = sim.eval_ros(land, w, scenario=s, period=p, rep=3, seed=99, sigma=sigma,
                             rounding=rounding, precision=precision)
            o = oracle.eval_ros(fuel, elev, wx, scenario=s, period=p, rep=3, seed=99,
                                sigma=np.float32(sigma).item(), rounding=rounding,
                                pc=35.0, curing=70.0)
            for k in ("hros", "bros", "fros", "lb"):
                np.testing.assert_allclose(g[k], o[k], rtol=tol, atol=1e-9, err_msg=k)
            burn = fuel.ravel() != 0
            d = np.abs((g["raz"] - o["raz"] + 180.0) % 360.0 - 180.0)
            # The spread azimuth is the angle of the effective wind vector:
            # 1e-5 rad wherever the ellipse is elongated (LB > 1.001).  As the
            # vector shrinks by cancellation of wind against slope, LB -> 1,
            # the direction stops mattering and its FP32 angle loses digits;
            # there the axis rates above carry the 1e-5 bar.
            shaped = burn & (o["lb"] > 1.001)
            assert np.all(np.radians(d[shaped]) <= (1e-5 if precision else 1e-9)), d[shaped].max()
            assert np.all(d[burn] <= (0.01 if precision else 1e-7)), d[burn].max()
            np.testing.assert_allclose(g["x8"], o["x8"], rtol=tol, atol=1e-9)
            diff = g["q8"] != o["q8"]
            if diff.any():
                assert np.all(boundary_case(o["xu8"][diff], o["x8"][diff], qtol))
                assert np.all(np.abs(g["q8"][diff] - o["q8"][diff]) == 1)
                n_audit += int(diff.sum())
    if precision == 0:
        assert n_audit == 0
    sim.unload_landscape(land)
    sim.unset_weather(w)


def test_fuel_table_matches_oracle_rates(sim):
    """Every fuel type on flat ground at one weather row (catches a coefficient typo)."""
    fuel = np.arange(16, dtype=np.uint8).reshape(4, 4)
    wx = np.array([[[91.0, 77.0, 17.0, 200.0]]], np.float32)
    land = sim.load_landscape(fuel, None)
    w = sim.set_weather(wx)
    g = sim.eval_ros(land, w)
    o = oracle.eval_ros(fuel, None, wx)
    np.testing.assert_allclose(g["hros"], o["hros"], rtol=1e-12)
    np.testing.assert_allclose(g["bros"], o["bros"], rtol=1e-12)
    np.testing.assert_allclose(g["lb"], o["lb"], rtol=1e-12)


# ------------------------------------------------------------ propagation

def _run_both(sim, fuel, elev, wx, period_min=60, pc=50.0, curing=80.0, block=0, cap=0, **kw):
    land = sim.load_landscape(fuel, elev, cell_m=kw.get("cell_m", 100), pc=pc, curing=curing)
    w = sim.set_weather(wx, period_min=period_min)
    sim.set_tuning(block, cap)
    rk = {k: v for k, v in kw.items() if k != "cell_m"}
    g = sim.simulate(Request(landscape=land, weather=w, **rk))
    sim.set_tuning(0, 0)
    okw = {k: v for k, v in kw.items() if k != "precision"}
    r = oracle_run(fuel, elev, wx, period_min=period_min, pc=pc, curing=curing, **okw)
    sim.unload_landscape(land)
    sim.unset_weather(w)
    return g, r


def test_tiny_c2_grid(sim):
    """20x20 C-2, flat, centre ignition, FFMC 90, BUI 80, 20 km/h from 270 deg, 10 h."""
    _say("tiny c2")
    w = inputs.tiny_c2()
    g, r = _run_both(sim, w.fuel, w.elev, w.weather, **request_kwargs(w))
    assert_same_outputs(g, r, where="tiny")
    assert g["burned_cells"][0] == 226


def _random_case(seed, rows, cols, n_periods, nonfuel=0.1):
    rng = np.random.default_rng(seed)
    fuel = rng.integers(1, 16, size=(rows, cols)).astype(np.uint8)
    fuel[rng.random((rows, cols)) < 0.5] = rng.integers(1, 16)
    fuel[rng.random((rows, cols)) < nonfuel] = 0
    elev = rng.integers(0, 200, size=(rows, cols)).astype(np.int16)
    wx = np.zeros((3, n_periods, 4), np.float32)
    wx[..., 0] = rng.uniform(84, 97, (3, n_periods))
    wx[..., 1] = rng.uniform(0, 150, (3, n_periods))
    wx[..., 2] = rng.uniform(0, 50, (3, n_periods))
    wx[..., 3] = rng.uniform(0, 360, (3, n_periods))
    return fuel, elev, wx


@pytest.mark.parametrize("seed", range(8))
def test_random_heterogeneous_grids(sim, seed):
    """Short periods, noise, stochastic rounding, thresholds, all ignition modes."""
    P = [7, 13, 60, 30, 5, 60, 17, 1][seed]
    _say(f"random grid seed={seed} P={P}")
    fuel, elev, wx = _random_case(seed, 37, 29, n_periods=12)
    kw = dict(n_periods=12, reps=6, seed=1000 + seed, sigma=[0.0, 0.15, 0.3][seed % 3],
              rounding=seed % 2, threshold=[0.0, 0.0, 2.0, 6.0][seed % 4],
              ignition_mode=seed % 3, ignition_cell=37 * 29 // 2, scenario_mode=1,
              precision=0)
    g, r = _run_both(sim, fuel, elev, wx, period_min=P, **kw)
    assert_same_outputs(g, r, where=f"seed {seed}")


@pytest.mark.parametrize("block", [64, 128, 256, 512, 768, 1024])
def test_block_size_does_not_change_results(sim, block):
    _say(f"block {block}")
    w = inputs.batched_monte_carlo(side=64, reps=24, n_scenarios=5, n_periods=12)
    g, r = _run_both(sim, w.fuel, w.elev, w.weather, block=block, **request_kwargs(w))
    assert_same_outputs(g, r, where=f"block {block}")


def test_forced_list_overflow_relaunches_identically(sim):
    _say("overflow relaunch")
    w = inputs.batched_monte_carlo(side=96, reps=16, n_scenarios=4, n_periods=10)
    g, r = _run_both(sim, w.fuel, w.elev, w.weather, cap=1, **request_kwargs(w))
    assert sim.stats()["relaunches"] >= 1
    assert_same_outputs(g, r, where="overflow")


def test_edge_cases(sim):
    _say("edge cases")
    wx = inputs.constant_weather(3, 92.0, 90.0, 30.0, 250.0)
    cases = [
        (np.full((1, 1), 3, np.uint8), dict(ignition_mode=2)),                      # one cell
        (np.zeros((5, 7), np.uint8), dict(ignition_mode=1, reps=3)),                # no fuel
        (np.full((1, 300), 2, np.uint8), dict(ignition_mode=2)),                    # strip
        (np.full((300, 1), 14, np.uint8), dict(ignition_mode=2)),
        (np.pad(np.full((5, 5), 2, np.uint8), 2), dict(ignition_cell=0)),           # non-fuel ignition
    ]
    for fuel, extra in cases:
        kw = dict(n_periods=3, seed=5, precision=0)
        kw.update(extra)
        g, r = _run_both(sim, fuel, None, wx, **kw)
        assert_same_outputs(g, r, where=f"edge {fuel.shape}")


def test_long_periods_and_grass(sim):
    """Fast grass fires (rates above one cell per minute) and 3 h periods."""
    fuel = np.full((120, 120), 15, np.uint8)
    fuel[60:, :] = 14
    wx = inputs.constant_weather(4, 96.0, 60.0, 45.0, 300.0)
    g, r = _run_both(sim, fuel, None, wx, period_min=180, n_periods=4, ignition_mode=2,
                     sigma=0.2, rounding=1, seed=3, curing=95.0)
    assert_same_outputs(g, r, where="grass")


def test_batch_equals_separate_requests(sim):
    """Requests on different landscapes fused into one launch give the same
    results as each request alone."""
    _say("batch vs separate")
    w1 = inputs.batched_monte_carlo(side=48, reps=10, n_scenarios=3, n_periods=8, land_seed=31)
    w2 = inputs.batched_monte_carlo(side=80, reps=7, n_scenarios=2, n_periods=8, land_seed=32)
    l1 = sim.load_landscape(w1.fuel, w1.elev)
    l2 = sim.load_landscape(w2.fuel, w2.elev)
    x1 = sim.set_weather(w1.weather)
    x2 = sim.set_weather(w2.weather)
    r1 = Request(landscape=l1, weather=x1, **request_kwargs(w1))
    r2 = Request(landscape=l2, weather=x2, **request_kwargs(w2, seed=77))
    r3 = Request(landscape=l1, weather=x1, **request_kwargs(w1, seed=78, precision=1))
    batch = sim.simulate_batch([r1, r2, r3])
    for req, got in zip([r1, r2, r3], batch):
        alone = sim.simulate(req)
        assert_same_outputs(got, alone, where="batch")
    ref1 = oracle_run(w1.fuel, w1.elev, w1.weather, **oracle_kwargs(w1))
    assert_same_outputs(batch[0], ref1, where="batch vs oracle")
    for x in (l1, l2):
        sim.unload_landscape(x)
    for x in (x1, x2):
        sim.unset_weather(x)


def test_rep_offset_splits_add_up(sim):
    w = inputs.batched_monte_carlo(side=64, reps=20, n_scenarios=4, n_periods=10)
    land = sim.load_landscape(w.fuel, w.elev)
    x = sim.set_weather(w.weather)
    full = sim.simulate(Request(landscape=land, weather=x, **request_kwargs(w)))
    a = sim.simulate(Request(landscape=land, weather=x, **request_kwargs(w, reps=8)))
    b = sim.simulate(Request(landscape=land, weather=x, **request_kwargs(w, reps=12, rep_offset=8)))
    assert np.array_equal(full["burn_count"], a["burn_count"] + b["burn_count"])
    assert np.array_equal(full["arrival_minute"], np.concatenate([a["arrival_minute"], b["arrival_minute"]]))
    sim.unload_landscape(land)
    sim.unset_weather(x)


def test_repeated_calls_reuse_slots(sim):
    """Many calls on one context (arrival planes reused under fresh tags)."""
    w = inputs.batched_monte_carlo(side=40, reps=8, n_scenarios=2, n_periods=6)
    land = sim.load_landscape(w.fuel, w.elev)
    x = sim.set_weather(w.weather)
    ref = oracle_run(w.fuel, w.elev, w.weather, **oracle_kwargs(w))
    for it in range(40):
        g = sim.simulate(Request(landscape=land, weather=x, **request_kwargs(w)))
        assert_same_outputs(g, ref, where=f"call {it}")
    sim.unload_landscape(land)
    sim.unset_weather(x)


def test_device_outputs(sim):
    import torch
    w = inputs.batched_monte_carlo(side=32, reps=5, n_scenarios=2, n_periods=6)
    land = sim.load_landscape(w.fuel, w.elev)
    x = sim.set_weather(w.weather)
    g = sim.simulate(Request(landscape=land, weather=x, device_out=True, **request_kwargs(w)))
    host = {k: v.cpu().numpy() for k, v in g.items()}
    host["burn_count"] = host["burn_count"].view(np.uint32)
    ref = oracle_run(w.fuel, w.elev, w.weather, **oracle_kwargs(w))
    assert_same_outputs(host, ref, where="device out")
    torch.cuda.synchronize()
    sim.set_stream(None)
    sim.unload_landscape(land)
    sim.unset_weather(x)


def test_device_outputs_accumulate_on_default_stream(sim):
    """Device outputs of consecutive calls, summed by torch on its default
    stream without synchronising: the library's writes stay ordered with the
    pending additions that still read reused buffers."""
    import dataclasses

    import torch
    _say("device outputs, default stream")
    w = inputs.batched_monte_carlo(side=1024, reps=16, n_scenarios=2, n_periods=8)
    land = sim.load_landscape(w.fuel, w.elev)
    x = sim.set_weather(w.weather)
    req = Request(landscape=land, weather=x, device_out=True,
                  outputs=("burn_count", "burned_cells"), **request_kwargs(w))
    whole = sim.simulate(req)
    counts = None
    for r in range(w.reps):
        o = sim.simulate(dataclasses.replace(req, reps=1, rep_offset=r))
        counts = o["burn_count"].clone() if counts is None else counts + o["burn_count"]
    torch.cuda.synchronize()
    assert torch.equal(counts, whole["burn_count"])
    assert int(counts.sum().item()) == int(whole["burned_cells"].sum().item())
    sim.set_stream(None)
    sim.unload_landscape(land)
    sim.unset_weather(x)


def test_graph_replays_match_eager_runs(sim):
    """Synchronous calls replay one captured hipGraph (fills, propagation,
    dense outputs).  Replays interleaved with eager library work (rate
    fields, another request) each equal an eager run of the same request
    through a serving lane, which launches without graphs."""
    _say("graph replays")
    w = inputs.batched_monte_carlo(side=96, reps=12, n_scenarios=3, n_periods=8)
    land = sim.load_landscape(w.fuel, w.elev)
    x = sim.set_weather(w.weather)
    req = Request(landscape=land, weather=x, **request_kwargs(w))
    other = Request(landscape=land, weather=x, **request_kwargs(w, reps=3, seed=99))
    with Simulator(0) as eager_sim:
        land2 = eager_sim.load_landscape(w.fuel, w.elev)
        x2 = eager_sim.set_weather(w.weather)
        t, _ = eager_sim.submit(Request(landscape=land2, weather=x2, **request_kwargs(w)))
        eager = eager_sim.wait(t)
    for k in range(6):
        g = sim.simulate(req)
        assert_same_outputs(g, eager, where=f"replay {k}")
        sim.eval_ros(land, x, scenario=k % 3, period=k, rep=k)   # eager work between replays
        if k == 2:
            sim.simulate(other)      # another launch sequence: the next call captures anew
    sim.unload_landscape(land)
    sim.unset_weather(x)


def test_autotune_keeps_results(sim):
    _say("autotune")
    w = inputs.batched_monte_carlo(side=128, reps=40, n_scenarios=4, n_periods=8)
    land = sim.load_landscape(w.fuel, w.elev)
    x = sim.set_weather(w.weather)
    req = Request(landscape=land, weather=x, **request_kwargs(w))
    before = sim.simulate(req)
    sim.autotune(req)
    after = sim.simulate(req)
    st = sim.stats()
    assert st["block_threads"] in (64, 128, 256, 512, 768, 1024)
    assert_same_outputs(after, {k: np.asarray(v) for k, v in before.items()}, where="after autotune")
    sim.unload_landscape(land)
    sim.unset_weather(x)


def test_rep_order_keeps_results(sim):
    """More replications than resident groups: groups take the longest
    predicted replications first, which changes only the schedule."""
    _say("replication order")
    w = inputs.batched_monte_carlo(side=64, reps=700, n_scenarios=5, n_periods=6)
    land = sim.load_landscape(w.fuel, w.elev)
    x = sim.set_weather(w.weather)
    outs = ("burn_count", "burned_cells", "ignition_cell", "scenario")
    req = Request(landscape=land, weather=x, outputs=outs, **request_kwargs(w))
    sim.set_rep_order(0)
    plain = sim.simulate(req)
    st0 = sim.stats()
    sim.set_rep_order(1)
    ordered = sim.simulate(req)
    st1 = sim.stats()
    assert st0["rep_order"] == 0 and st1["rep_order"] == 1, (st0, st1)
    assert st1["grid_blocks"] < w.reps
    assert_same_outputs(ordered, plain, outs, where="ordered vs index order")
    ref = oracle_run(w.fuel, w.elev, w.weather, **oracle_kwargs(w, reps=4))
    for k in ("burned_cells", "ignition_cell", "scenario"):
        np.testing.assert_array_equal(np.asarray(ordered[k])[:4], ref[k], err_msg=k)
    sim.unload_landscape(land)
    sim.unset_weather(x)


# ------------------------------------------------------- medium workloads

def test_single_fire_512_fp64(sim):
    _say("single fire 512 fp64")
    w = inputs.single_large_fire(side=512, n_periods=48, precision=0)
    g, r = _run_both(sim, w.fuel, w.elev, w.weather, **request_kwargs(w))
    assert_same_outputs(g, r, where="single 512")
    assert g["burned_cells"][0] > 1000


def test_single_fire_256_fp32_with_audited_rates(sim):
    """FP32 rates: audit every (period, cell) integer rate against the FP64
    oracle, replay the audited boundary cases in the oracle, then demand
    bit-exact propagation."""
    _say("single fire 256 fp32")
    w = inputs.single_large_fire(side=256, n_periods=24, precision=1)
    land = sim.load_landscape(w.fuel, w.elev)
    x = sim.set_weather(w.weather)
    g = sim.simulate(Request(landscape=land, weather=x, **request_kwargs(w)))
    keys, q, n = fp32_overrides(sim, land, x, w.fuel, w.elev, w.weather, reps=1,
                                n_periods=w.n_periods, seed=w.seed, sigma=w.sigma,
                                rounding=w.rounding, scenarios=g["scenario"])
    _say(f"  audited {len(keys)} boundary cells of {n} rates")
    r = oracle_run(w.fuel, w.elev, w.weather, overrides=(keys, q), **oracle_kwargs(w))
    assert_same_outputs(g, r, where="fp32 256")
    sim.unload_landscape(land)
    sim.unset_weather(x)


def test_batched_mc_128_many_reps(sim):
    _say("batched mc 128 x 96 reps")
    w = inputs.batched_monte_carlo(side=128, reps=96, n_scenarios=10, n_periods=24)
    g, r = _run_both(sim, w.fuel, w.elev, w.weather, **request_kwargs(w))
    assert_same_outputs(g, r, where="mc 128")
