"""The tuning cache on disk: a choice made by the autotuner in one context is
written with c2f_save_tuning and read back by another context with
c2f_load_tuning, which then launches the same request with the same block
size and list capacity and gets the same results; files from another kind
of device, malformed files and missing files are refused and change
nothing."""
import sys

import numpy as np
import pytest

from paper_1905_09317_amd import C2FError, Request, Simulator, inputs

from _helpers import assert_same_outputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _setup(sim):
    rng = np.random.default_rng(41)
    fuel = rng.integers(1, 16, (160, 144)).astype(np.uint8)
    elev = inputs.elevation_grid(160, 144, 42, elev_max=300.0)
    wx = rng.uniform([86, 40, 5, 0], [94, 110, 35, 360], (3, 12, 4)).astype(np.float32)
    land = sim.load_landscape(fuel, elev)
    w = sim.set_weather(wx)
    return Request(landscape=land, weather=w, n_periods=12, reps=24, seed=5, sigma=0.15, rounding=1,
                   ignition_mode=1, scenario_mode=1, precision=0,
                   outputs=("burn_count", "burned_cells"))


def _run(sim, req):
    out = sim.simulate(req)
    st = sim.stats()
    return {k: np.asarray(v) for k, v in out.items()}, (st["block_threads"], st["list_capacity"])


def test_saved_tuning_carries_over_to_a_new_context(tmp_path):
    path = str(tmp_path / "tuning.txt")
    a = Simulator(0)
    try:
        req = _setup(a)
        _say("tuning: default launch")
        base, plan0 = _run(a, req)
        _say("tuning: autotune")
        a.autotune(req)
        tuned, plan_a = _run(a, req)
        assert_same_outputs(tuned, base, where="after autotune")
        a.save_tuning(path)
    finally:
        a.close()
    lines = open(path).read().splitlines()
    assert lines[0].split()[:2] == ["c2f-tuning", "1"]
    assert f"{160 * 144} 24 0 {plan_a[0]} {plan_a[1]}" in lines[1:]

    b = Simulator(0)
    try:
        req = _setup(b)
        _say("tuning: loaded")
        b.load_tuning(path)
        got, plan_b = _run(b, req)
        assert plan_b == plan_a
        assert_same_outputs(got, base, where="loaded tuning")
        # saving again reproduces the entry
        b.save_tuning(path + "2")
        assert f"{160 * 144} 24 0 {plan_a[0]} {plan_a[1]}" in open(path + "2").read().splitlines()[1:]
    finally:
        b.close()


def test_bad_tuning_files_are_refused_and_change_nothing(tmp_path):
    sim = Simulator(0)
    try:
        req = _setup(sim)
        _, plan0 = _run(sim, req)
        good = tmp_path / "good.txt"
        sim.save_tuning(str(good))
        header = open(good).read().splitlines()[0]
        arch, n_cu = header.split()[2], int(header.split()[3])
        other_block = 64 if plan0[0] != 64 else 128
        entry = f"{160 * 144} 24 0 {other_block} 4096"
        cases = {
            "missing": None,
            "empty": "",
            "bad_header": f"tuning 1 {arch} {n_cu}\n{entry}\n",
            "bad_version": f"c2f-tuning 2 {arch} {n_cu}\n{entry}\n",
            "other_arch": f"c2f-tuning 1 gfx942 {n_cu}\n{entry}\n",
            "other_cus": f"c2f-tuning 1 {arch} {n_cu + 1}\n{entry}\n",
            "bad_block": f"{header}\n{160 * 144} 24 0 100 4096\n",
            "bad_capacity": f"{header}\n{160 * 144} 24 0 256 0\n",
            "bad_precision": f"{header}\n{160 * 144} 24 2 256 4096\n",
            "trailing": f"{header}\n{entry} 7\n",
            "short": f"{header}\n{160 * 144} 24 0 256\n",
            # a good entry before a bad one is not applied either
            "partly_bad": f"{header}\n{entry}\n{160 * 144} 24 0 100 4096\n",
        }
        for name, text in cases.items():
            p = tmp_path / f"{name}.txt"
            if text is not None:
                p.write_text(text)
            with pytest.raises(C2FError) as e:
                sim.load_tuning(str(p))
            assert e.value.status == (-7 if name == "missing" else -1), name
            _, plan = _run(sim, req)
            assert plan == plan0, name
        # the same entry in a well-formed file is applied
        ok = tmp_path / "ok.txt"
        ok.write_text(f"{header}\n{entry}\n")
        sim.load_tuning(str(ok))
        _, plan = _run(sim, req)
        assert plan == (other_block, 4096)
    finally:
        sim.close()
