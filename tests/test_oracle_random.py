"""Pins for the oracle's random parts (Section 3.1, sources of uncertainty (2)
and (3)): the lognormal rate multiplier, the stochastic rounding of axis
rates, and the weather-scenario draw.

Each part is checked two ways.  A hand value for one counter, formed here
from the Philox words (themselves pinned to Random123's published known
answers in test_oracle_philox.py) with Python's math module, catches a
swapped word, a wrong tag or a dropped term.  A distribution test over many
independent counters, against a stated confidence bound, catches a wrong
sign or scale that one value could hide.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle

SEED = 0x1234_5678_9ABC_DEF0


def _words(seed, cell, period, rep, tag):
    key = [seed & 0xFFFFFFFF, seed >> 32]
    return [int(v) for v in oracle.philox4x32_10([cell, period, rep, tag], key)]


def _flat(rows, cols, fuel=2):
    return np.full((rows, cols), fuel, np.uint8), None


def _weather(ffmc=90.0, bui=80.0, ws=20.0, wd=270.0, periods=3):
    return np.tile(np.array([ffmc, bui, ws, wd], np.float32), (periods, 1))[None]


def _mu_field(sigma, rows=320, cols=320, period=1, rep=5, seed=SEED):
    """Per-cell multiplier mu as the oracle applies it: H(sigma) / H(0) on a
    uniform flat landscape (every cell has the same unperturbed rate)."""
    fuel, elev = _flat(rows, cols)
    wx = _weather()
    a = oracle.eval_ros(fuel, elev, wx, period=period, rep=rep, seed=seed, sigma=sigma)
    b = oracle.eval_ros(fuel, elev, wx, period=period, rep=rep, seed=seed, sigma=0.0)
    return a["hros"] / b["hros"], a, b


def test_noise_multiplier_hand_value():
    """mu = exp(sigma Z - sigma^2/2), Z = sqrt(-2 ln u1) cos(2 pi u2) with
    u1 = ((x0 >> 8) + 1) 2^-24 and u2 = (x1 >> 8) 2^-24 from the tag-0 words
    of counter (cell, period, rep)."""
    sigma = 0.15
    mu, a, b = _mu_field(sigma, rows=9, cols=11, period=2, rep=7)
    for cell in (0, 17, 98):
        x = _words(SEED, cell, 2, 7, 0)
        u1 = ((x[0] >> 8) + 1) / 2.0 ** 24
        u2 = (x[1] >> 8) / 2.0 ** 24
        z = math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)
        want = math.exp(sigma * z - 0.5 * sigma * sigma)
        assert mu[cell] == pytest.approx(want, rel=1e-13), cell
        # the same multiplier scales back and flank rates; LB is unchanged
        assert a["bros"][cell] == pytest.approx(want * b["bros"][cell], rel=1e-13)
        assert a["fros"][cell] == pytest.approx(want * b["fros"][cell], rel=1e-13)
        assert a["lb"][cell] == b["lb"][cell]
        np.testing.assert_allclose(a["x8"][cell], want * b["x8"][cell], rtol=1e-13)


def test_noise_multiplier_distribution():
    """Over 102400 independent counters: ln mu is normal with mean
    -sigma^2/2 and deviation sigma, so mu has mean 1 and coefficient of
    variation sqrt(exp(sigma^2) - 1).  Bounds are 5 standard errors."""
    sigma = 0.15
    mu, _, _ = _mu_field(sigma)
    n = mu.size
    lm = np.log(mu)
    # mean of ln mu: a flipped sign of sigma^2/2 moves it by sigma^2 = 0.0225
    assert abs(lm.mean() + 0.5 * sigma ** 2) < 5 * sigma / math.sqrt(n)
    # deviation of ln mu (standard error of a normal sample's deviation)
    assert abs(lm.std(ddof=1) - sigma) < 5 * sigma / math.sqrt(2 * n)
    # mean 1 and CV of mu itself
    cv = math.sqrt(math.expm1(sigma ** 2))
    assert abs(mu.mean() - 1.0) < 5 * cv / math.sqrt(n)
    assert abs(mu.std(ddof=1) / mu.mean() - cv) < 0.02 * cv
    # shape: the standardised logs are N(0, 1)
    z = (lm + 0.5 * sigma ** 2) / sigma
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_noise_multiplier_independent_across_period_and_rep():
    mu_a, _, _ = _mu_field(0.3, rows=200, cols=200, period=0, rep=3)
    mu_b, _, _ = _mu_field(0.3, rows=200, cols=200, period=1, rep=3)
    mu_c, _, _ = _mu_field(0.3, rows=200, cols=200, period=0, rep=4)
    n = mu_a.size
    for other in (mu_b, mu_c):
        r = np.corrcoef(np.log(mu_a), np.log(other))[0, 1]
        assert abs(r) < 5 / math.sqrt(n)


def test_zero_sigma_draws_nothing():
    mu, _, _ = _mu_field(0.0, rows=5, cols=5)
    assert np.all(mu == 1.0)


def test_stochastic_rounding_hand_value():
    """q_k = floor(x_k + u_k) with u_k = (w >> 8) 2^-24, w the k-th word of
    tag 1 (axes E, NE, N, NW) or tag 2 (axes W, SW, S, SE)."""
    fuel, elev = _flat(7, 9)
    wx = _weather()
    r = oracle.eval_ros(fuel, elev, wx, period=1, rep=3, seed=SEED, sigma=0.2, rounding=1)
    for cell in (0, 30, 62):
        w1 = _words(SEED, cell, 1, 3, 1)
        w2 = _words(SEED, cell, 1, 3, 2)
        u = [(w >> 8) / 2.0 ** 24 for w in w1 + w2]
        for k in range(8):
            assert r["xu8"][cell, k] == r["x8"][cell, k] + u[k]
            assert r["q8"][cell, k] == math.floor(r["x8"][cell, k] + u[k])
    # nearest rounding adds one half
    n = oracle.eval_ros(fuel, elev, wx, period=1, rep=3, seed=SEED, sigma=0.2, rounding=0)
    np.testing.assert_array_equal(n["xu8"], n["x8"] + 0.5)
    np.testing.assert_array_equal(n["q8"], np.floor(n["x8"] + 0.5).astype(np.int32))


def test_stochastic_rounding_is_unbiased_per_axis():
    """With no noise every cell of a uniform flat landscape has the same
    axis rates x_k; the stochastic integer rates then average x_k (E floor(x
    + U) = x for U uniform on [0, 1)).  Bound: 5 standard errors of a
    Bernoulli(frac x) mean over 102400 cells.  Nearest rounding would give
    round(x) on every cell, off by up to 1/2."""
    fuel, elev = _flat(320, 320)
    wx = _weather()
    r = oracle.eval_ros(fuel, elev, wx, period=0, rep=1, seed=SEED, sigma=0.0, rounding=1)
    x = r["x8"][0]
    assert np.all(r["x8"] == x)
    n = r["q8"].shape[0]
    for k in range(8):
        f = x[k] - math.floor(x[k])
        se = math.sqrt(max(f * (1 - f), 1e-12) / n)
        assert abs(r["q8"][:, k].mean() - x[k]) < 5 * se + 1e-12, k
        assert set(np.unique(r["q8"][:, k])) <= {math.floor(x[k]), math.floor(x[k]) + 1}


def test_scenario_draw_hand_value_and_uniformity():
    """scenario = (x S) >> 32 with x the first word of counter (~0, ~0, rep,
    4); over 14000 replications the counts of S = 7 scenarios fit the
    uniform law (chi-square, p > 1e-3)."""
    fuel = np.zeros((1, 1), np.uint8)           # nothing burns: only the draws run
    S, reps, seed = 7, 14000, 99
    wx = np.tile(np.array([90, 80, 10, 0], np.float32), (S, 2, 1))
    res = oracle.simulate(fuel, None, wx, n_periods=1, reps=reps, seed=seed, scenario_mode=1,
                          ignition_mode=0, ignition_cell=0, want_rep_outputs=False)
    sc = res["scenario"]
    for rep in (0, 1, 4097, reps - 1):
        x = _words(seed, 0xFFFFFFFF, 0xFFFFFFFF, rep, 4)[0]
        assert sc[rep] == (x * S) >> 32
    counts = np.bincount(sc, minlength=S)
    assert counts.size == S
    assert stats.chisquare(counts).pvalue > 1e-3
    # a draw that ignored rep would give one scenario only
    assert (counts > 0).all()
