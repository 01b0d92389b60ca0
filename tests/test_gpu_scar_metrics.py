"""GPU scar comparison (Section 4 metrics) against the FP64 oracle: the
counts are exact on the device, so MSE and the Frobenius norm are equal;
SSIM agrees to 1e-9 relative (the oracle sums N <= 2^22 FP64 terms
directly, an error below N 2^-53)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1905_09317_amd import C2FError, Request, Simulator, inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim():
    s = Simulator(0)
    yield s
    s.close()


def _check(g, o):
    np.testing.assert_array_equal(g["mse"], o["mse"])
    np.testing.assert_allclose(g["ssim"], o["ssim"], rtol=1e-9, atol=1e-12)
    assert g["delta_norm"] == o["delta_norm"]


# Paths of the count kernel: n % 16 == 0 streams 16 cells per lane (4096,
# 300_000, 1024), n % 4 == 0 four (4_194_308 also takes two strides per
# block, 20_004 with T = 300 three windows of periods), other n and T >
# 4096 count one period per block.  T = 11 leaves a partial batch of periods.
@pytest.mark.parametrize("n,T", [(2, 1), (2047, 3), (4097, 5), (300_001, 2), (4096, 5), (300_000, 11),
                                 (4_194_308, 3), (20_004, 300), (1024, 1024), (1024, 4097)])
def test_random_scars_equal_oracle(sim, n, T):
    _say(f"scar comparison n={n} T={T}")
    rng = np.random.default_rng(n + T)
    arr = np.where(rng.random(n) < 0.4, rng.integers(0, T * 60 + 30, n), -1).astype(np.int32)
    ref = (rng.random((T, n)) < rng.random((T, 1))).astype(np.uint8)
    _check(sim.compare_scars(arr, ref), oracle.scar_metrics(arr, ref))


@pytest.mark.parametrize("offset", [1, 4])
def test_unaligned_device_reference(sim, offset):
    """A reference that starts 1 byte (read byte by byte) or 4 bytes (read
    word by word) into its allocation gives the same result."""
    import torch
    n, T = 8192, 6
    rng = np.random.default_rng(17)
    arr = np.where(rng.random(n) < 0.5, rng.integers(0, T * 60, n), -1).astype(np.int32)
    ref = (rng.random((T, n)) < 0.45).astype(np.uint8)
    buf = torch.zeros(T * n + offset, dtype=torch.uint8, device="cuda:0")
    buf[offset:] = torch.from_numpy(ref.reshape(-1)).to("cuda:0")
    view = buf[offset:].view(T, n)
    assert view.data_ptr() % 16 == offset
    _check(sim.compare_scars(torch.from_numpy(arr).to("cuda:0"), view), oracle.scar_metrics(arr, ref))


def test_identical_scars_give_exact_values(sim):
    rng = np.random.default_rng(5)
    arr = np.where(rng.random(5000) < 0.3, 10, -1).astype(np.int32)
    ref = (arr >= 0)[None].astype(np.uint8)
    g = sim.compare_scars(arr, ref)
    assert g["mse"][0] == 0.0 and g["ssim"][0] == 1.0 and g["delta_norm"] == 0.0


def test_fp32_against_fp64_fire_on_the_device(sim):
    """The 512^2 single fire in FP32 compared period by period with the
    same fire in FP64 (device tensors in, as a user would pass them)."""
    import torch
    _say("scar comparison fp32 vs fp64")
    w = inputs.single_large_fire(side=512, n_periods=24, precision=0)
    land = sim.load_landscape(w.fuel, w.elev)
    x = sim.set_weather(w.weather)
    kw = dict(n_periods=24, ignition_mode=2, outputs=("arrival_minute",), device_out=True)
    a64 = sim.simulate(Request(landscape=land, weather=x, precision=0, **kw))["arrival_minute"][0]
    a32 = sim.simulate(Request(landscape=land, weather=x, precision=1, **kw))["arrival_minute"][0]
    t = torch.arange(1, 25, device=a64.device, dtype=torch.int32)[:, None] * 60
    ref = ((a64[None] >= 0) & (a64[None] <= t)).to(torch.uint8)
    g = sim.compare_scars(a32, ref)
    o = oracle.scar_metrics(a32.cpu().numpy(), ref.cpu().numpy())
    _check(g, o)
    assert (g["ssim"] > 0.99).all()
    sim.unload_landscape(land)
    sim.unset_weather(x)


def test_compare_scars_checks_its_arguments(sim):
    with pytest.raises(C2FError) as e:
        sim.compare_scars(np.zeros(1, np.int32), np.zeros((1, 1), np.uint8))
    assert e.value.status == -1
    with pytest.raises(ValueError):
        sim.compare_scars(np.zeros(10, np.int32), np.zeros((2, 9), np.uint8))


def test_async_results_stay_on_the_device(sim):
    """Back-to-back stream-ordered calls (the third one grows the context's
    count buffer) give the synchronous call's values."""
    import torch
    _say("scar comparison async")
    rng = np.random.default_rng(23)
    cases = []
    for n, T in [(65_536, 9), (4099, 2), (20_000, 300)]:
        arr = np.where(rng.random(n) < 0.5, rng.integers(0, T * 60, n), -1).astype(np.int32)
        ref = (rng.random((T, n)) < 0.4).astype(np.uint8)
        cases.append((arr, ref))
    outs = []
    for arr, ref in cases:
        T = ref.shape[0]
        res = torch.full((2 * T + 1,), float("nan"), dtype=torch.float64, device="cuda:0")
        sim.compare_scars_async(torch.from_numpy(arr).to("cuda:0"), torch.from_numpy(ref).to("cuda:0"), res)
        outs.append(res)
    torch.cuda.synchronize()
    for (arr, ref), res in zip(cases, outs):
        T = ref.shape[0]
        r = res.cpu().numpy()
        g = {"mse": r[:T], "ssim": r[T:2 * T], "delta_norm": float(r[2 * T])}
        s = sim.compare_scars(arr, ref)
        np.testing.assert_array_equal(g["mse"], s["mse"])
        np.testing.assert_array_equal(g["ssim"], s["ssim"])
        assert g["delta_norm"] == s["delta_norm"]
        _check(g, oracle.scar_metrics(arr, ref))


def test_small_then_large_period_counts_stay_clean():
    """A comparison with few periods between two with many: the first fixes
    the context buffer's capacity, the second's results must not land on
    counts the third expects to find cleared."""
    s = Simulator(0)
    try:
        rng = np.random.default_rng(31)
        for T in (50, 2, 50, 7, 50):
            n = 4096
            arr = np.where(rng.random(n) < 0.5, rng.integers(0, T * 60, n), -1).astype(np.int32)
            ref = (rng.random((T, n)) < 0.5).astype(np.uint8)
            _check(s.compare_scars(arr, ref), oracle.scar_metrics(arr, ref))
    finally:
        s.close()


def test_full_size_comparison_equals_oracle(sim):
    """The measured shape: 48 reference scars of 2048^2 cells (16 cells per
    lane, one group per compute unit), random scars that grow period by
    period, against the oracle."""
    import torch
    _say("scar comparison 2048^2 x 48")
    n, T = 2048 * 2048, 48
    rng = np.random.default_rng(2048)
    arr = np.where(rng.random(n) < 0.6, rng.integers(0, T * 60 + 60, n), -1).astype(np.int32)
    start = rng.integers(0, T + 8, n)
    ref = (np.arange(T)[:, None] >= start[None, :]).astype(np.uint8)
    g = sim.compare_scars(torch.from_numpy(arr).to("cuda:0"), torch.from_numpy(ref).to("cuda:0"))
    _check(g, oracle.scar_metrics(arr, ref))
