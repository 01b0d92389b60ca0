"""Pins of the oracle's scar comparison (Section 4: MSE, SSIM of Wang et
al. 2004 over the whole grid, Frobenius norm of the difference)."""
from fractions import Fraction as F

import numpy as np

import oracle


def _arrivals_from(scar):
    """Arrival minutes whose scar at the end of period 1 (60 min) is `scar`."""
    return np.where(np.asarray(scar, bool), 30, -1).astype(np.int32)


def test_identical_scars():
    rng = np.random.default_rng(1)
    y = rng.random(500) < 0.3
    m = oracle.scar_metrics(_arrivals_from(y), y[None].astype(np.uint8))
    assert m["mse"][0] == 0.0 and m["ssim"][0] == 1.0 and m["delta_norm"] == 0.0


def test_complementary_scars():
    rng = np.random.default_rng(2)
    y = rng.random(400) < 0.4
    m = oracle.scar_metrics(_arrivals_from(y), (~y)[None].astype(np.uint8))
    assert m["mse"][0] == 1.0
    assert abs(m["delta_norm"] - np.sqrt(400)) < 1e-12
    assert m["ssim"][0] < 0.0          # perfectly anti-correlated


def test_worked_example():
    """N = 4, X = (1, 1, 0, 0), Y = (1, 0, 0, 0): by hand mu_x = 1/2,
    mu_y = 1/4, sigma_x^2 = 1/3, sigma_y^2 = 1/4, sigma_xy = 1/6 (N - 1
    normalisation), MSE = 1/4, delta = 1."""
    c1, c2 = F(1, 10**4), F(9, 10**4)
    mx, my, vx, vy, cxy = F(1, 2), F(1, 4), F(1, 3), F(1, 4), F(1, 6)
    expect = ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))
    m = oracle.scar_metrics(_arrivals_from([1, 0, 0, 0]), np.array([[1, 1, 0, 0]], np.uint8))
    assert m["mse"][0] == 0.25 and m["delta_norm"] == 1.0
    assert abs(m["ssim"][0] - float(expect)) < 1e-15


def test_properties_on_random_scars():
    rng = np.random.default_rng(3)
    for _ in range(20):
        n = int(rng.integers(10, 3000))
        x = rng.random(n) < rng.random()
        y = rng.random(n) < rng.random()
        a = oracle.scar_metrics(_arrivals_from(y), x[None].astype(np.uint8))
        b = oracle.scar_metrics(_arrivals_from(x), y[None].astype(np.uint8))
        p = rng.permutation(n)
        c = oracle.scar_metrics(_arrivals_from(y[p]), x[p][None].astype(np.uint8))
        hamming = int((x != y).sum())
        assert a["mse"][0] == hamming / n
        assert abs(a["delta_norm"] ** 2 - n * a["mse"][0]) < 1e-9
        assert abs(a["ssim"][0] - b["ssim"][0]) < 1e-12            # symmetric
        assert abs(a["ssim"][0] - c["ssim"][0]) < 1e-12            # whole-grid statistics
        assert a["ssim"][0] <= 1.0 + 1e-15


def test_periods_use_the_scar_at_each_period_end():
    """The oracle's own fire, compared with its own per-period scars, is
    identical at every period; against the final scar it differs until the
    last period."""
    fuel = np.full((30, 30), 2, np.uint8)
    elev = np.zeros((30, 30), np.int16)
    wx = np.tile(np.array([[90.0, 80.0, 20.0, 270.0]], np.float32), (6, 1))[None]
    o = oracle.simulate(fuel, elev, wx, n_periods=6, ignition_cell=15 * 30 + 5)
    m = o["arrival_minute"][0]
    own = np.stack([(m >= 0) & (m <= 60 * t) for t in range(1, 7)]).astype(np.uint8)
    r = oracle.scar_metrics(m, own)
    assert (r["mse"] == 0).all() and (r["ssim"] == 1).all()
    final = np.repeat(own[-1:], 6, axis=0)
    r2 = oracle.scar_metrics(m, final)
    assert (r2["mse"][:-1] > 0).all() and r2["mse"][-1] == 0
    assert (np.diff(r2["mse"]) <= 0).all()       # the growing fire approaches its final scar
