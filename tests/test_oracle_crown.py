"""Pins for the oracle's FBP crown fire, fuel consumption and head fire
intensity (Section 2.3 and assumption A5 (iv)), and fuels D-2, M-3, M-4.

The FBP System's equations and constants are not printed in the paper and
the published tables are not available here, so agreement with them is
parity unpinned.  What is pinned: limits and special cases of the model
(crown fraction 0 below the critical surface rate and 1/2 at a stated
excess, fuel consumption at zero build-up and its asymptotes, the C-6
rate's surface and crown limits, the mixedwood limits), identities (head
fire intensity linear in the rate at fixed consumption, D-2 a fifth of D-1),
and the cutoff's effect on a simulation.
"""
import math

import numpy as np
import pytest

import oracle

CROWNING = [1, 2, 3, 4, 5, 6, 7, 9, 10, 17, 18]
NON_CROWNING = [8, 11, 12, 13, 14, 15, 16]


def _pt(fuel, ffmc=90.0, bui=80.0, ws=10.0, **kw):
    return oracle.fbp_point(fuel, ffmc, bui, ws, 270.0, **kw)


@pytest.mark.parametrize("fuel", NON_CROWNING)
def test_non_crowning_fuels_burn_no_crown(fuel):
    for ws in (0.0, 20.0, 60.0):
        r = _pt(fuel, ws=ws)
        assert r["cfb"] == 0.0 and r["tfc"] == r["sfc"]
    assert oracle.crown_coefficients(fuel)[1] == 0.0


@pytest.mark.parametrize("fuel", NON_CROWNING + [2, 3, 5, 7, 9, 17])
def test_intensity_is_linear_in_rate_at_fixed_consumption(fuel):
    """I = 300 TFC ROS: at fixed FFMC and BUI the wind changes the rate only,
    so I / ROS is 300 x consumption (and the consumption does not depend
    on the wind except through the crown fraction)."""
    for ws in (0.0, 7.0, 25.0):
        r = _pt(fuel, ws=ws)
        assert r["hfi"] == pytest.approx(300.0 * r["tfc"] * r["hros"], rel=1e-14)
        assert r["sfc"] == _pt(fuel, ws=0.0)["sfc"]


def _wind_where(fuel, ffmc, bui, pred, fmc=97.0):
    """Least wind speed (bisection) at which pred(point) holds."""
    lo, hi = 0.0, 300.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if pred(_pt(fuel, ffmc=ffmc, bui=bui, ws=mid, fmc=fmc)):
            hi = mid
        else:
            lo = mid
    return _pt(fuel, ffmc=ffmc, bui=bui, ws=hi, fmc=fmc)


@pytest.mark.parametrize("fuel", CROWNING)
def test_crown_fraction_onset_and_half_point(fuel):
    """CFB = 0 while the head rate (the surface rate for C-6) stays below the
    critical surface rate; above it CFB = 1 - exp(-0.23 excess).  At fixed
    FFMC and BUI (so fixed consumption and critical rate) the rate at which
    CFB reaches 1/2 exceeds the onset rate by ln 2 / 0.23."""
    cbh, cfl = oracle.crown_coefficients(fuel)
    assert cbh > 0 and cfl > 0
    for ffmc, bui, fmc in ((70.0, 60.0, 97.0), (75.0, 60.0, 97.0), (80.0, 60.0, 97.0),
                           (85.0, 60.0, 97.0), (88.0, 60.0, 97.0), (96.0, 200.0, 60.0)):
        if _pt(fuel, ffmc=ffmc, bui=bui, ws=0.0, fmc=fmc)["cfb"] == 0.0 and \
                _pt(fuel, ffmc=ffmc, bui=bui, ws=120.0, fmc=fmc)["cfb"] > 0.6:
            break
    else:
        raise AssertionError("no bracket for this fuel")
    surface = "isi" if fuel == 6 else None
    onset = _wind_where(fuel, ffmc, bui, lambda r: r["cfb"] > 0.0, fmc=fmc)
    half = _wind_where(fuel, ffmc, bui, lambda r: r["cfb"] >= 0.5, fmc=fmc)
    assert half["cfb"] == pytest.approx(0.5, abs=1e-9)
    assert half["tfc"] == pytest.approx(half["sfc"] + 0.5 * cfl, abs=1e-8)
    if surface is None:
        assert half["hros"] - onset["hros"] == pytest.approx(math.log(2.0) / 0.23, rel=1e-6)
    else:
        # C-6: the fraction follows the surface rate 30 (1 - exp(-0.08 ISI))^3 BE
        be = math.exp(50 * math.log(0.8) * (1 / bui - 1 / 62.0))
        rss = [30 * (1 - math.exp(-0.08 * r["isi"])) ** 3 * be for r in (onset, half)]
        assert rss[1] - rss[0] == pytest.approx(math.log(2.0) / 0.23, rel=1e-6)
    hot = _pt(fuel, ffmc=98.0, bui=150.0, ws=80.0, fmc=85.0)
    assert hot["cfb"] > 0.9


def test_critical_rate_scales_with_moisture_and_crown_base_height():
    """The critical surface rate is 0.001 CBH^1.5 (460 + 25.9 FMC)^1.5 / (300
    SFC).  At fixed FFMC and BUI the onset rates of crowning compare as
    ((460 + 25.9 FMC2) / (460 + 25.9 FMC1))^1.5 for one fuel, and as
    (CBH2 / CBH1)^1.5 for M-1 at 100 % conifer (the C-2 rate, C-2 consumption
    and crown load, but a 6 m crown base) against C-2 (3 m)."""
    def onset(fuel, fmc, pc=50.0):
        lo, hi = 0.0, 300.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if _pt(fuel, ffmc=80.0, bui=60.0, ws=mid, fmc=fmc, pc=pc)["cfb"] > 0.0:
                hi = mid
            else:
                lo = mid
        assert lo > 0.0
        return _pt(fuel, ffmc=80.0, bui=60.0, ws=hi, fmc=fmc, pc=pc)["hros"]
    r1, r2 = onset(2, 85.0), onset(2, 120.0)
    assert r2 / r1 == pytest.approx(((460 + 25.9 * 120.0) / (460 + 25.9 * 85.0)) ** 1.5, rel=1e-6)
    assert onset(9, 97.0, pc=100.0) / onset(2, 97.0) == pytest.approx(2.0 ** 1.5, rel=1e-6)


@pytest.mark.parametrize("fuel", [2, 8, 16, 11, 12, 13, 9, 17, 18])
def test_surface_consumption_vanishes_without_buildup(fuel):
    assert _pt(fuel, bui=0.0)["sfc"] == 0.0


@pytest.mark.parametrize("fuel,limit", [(2, 5.0), (3, 5.0), (4, 5.0), (5, 5.0), (6, 5.0), (8, 1.5),
                                        (16, 1.5), (11, 8.0), (12, 16.0), (13, 32.0), (17, 5.0),
                                        (18, 5.0)])
def test_surface_consumption_asymptotes_and_increases(fuel, limit):
    s = [_pt(fuel, bui=b)["sfc"] for b in (10.0, 40.0, 120.0, 400.0, 5000.0)]
    assert all(a < b for a, b in zip(s, s[1:]))
    assert s[-1] == pytest.approx(limit, rel=1e-6)


def test_c1_and_c7_and_grass_consumption_special_values():
    # C-1 depends on FFMC only: 0.75 kg/m^2 at 84, symmetric branches about it
    assert _pt(1, ffmc=84.0)["sfc"] == 0.75
    hi, lo = _pt(1, ffmc=90.0)["sfc"], _pt(1, ffmc=78.0)["sfc"]
    assert hi - 0.75 == pytest.approx(0.75 - lo, rel=1e-14)
    assert _pt(1, ffmc=90.0, bui=10.0)["sfc"] == _pt(1, ffmc=90.0, bui=150.0)["sfc"]
    # C-7: forest floor (FFMC above 70) plus woody fuel (BUI); both vanish
    assert _pt(7, ffmc=70.0, bui=0.0)["sfc"] == 0.0
    assert _pt(7, ffmc=101.0, bui=1e5)["sfc"] == pytest.approx(2.0 * (1 - math.exp(-0.104 * 31)) + 1.5,
                                                               rel=1e-9)
    # grass: the fuel load
    for f in (14, 15):
        assert _pt(f, bui=10.0)["sfc"] == 0.35 == _pt(f, bui=200.0)["sfc"]


def test_c6_surface_and_crown_limits():
    """C-6: the surface curve 30 (1 - exp(-0.08 ISI))^3 BE while no crowning;
    with crowning the rate lies between the surface rate and the crown rate
    60 (1 - exp(-0.0497 ISI)) FME / 0.778 and equals RSS + CFB (RSC - RSS);
    at FMC 97 the moisture effect is 0.778 itself."""
    r = _pt(6, ffmc=85.0, bui=60.0, ws=0.0, fmc=120.0)
    be = math.exp(50 * math.log(0.8) * (1 / 60.0 - 1 / 62.0))
    assert r["cfb"] == 0.0
    assert r["hros"] == pytest.approx(30 * (1 - math.exp(-0.08 * r["isi"])) ** 3 * be, rel=1e-13)
    r = _pt(6, ffmc=95.0, bui=100.0, ws=35.0, fmc=97.0)
    be = math.exp(50 * math.log(0.8) * (1 / 100.0 - 1 / 62.0))
    rss = 30 * (1 - math.exp(-0.08 * r["isi"])) ** 3 * be
    fme = 1000 * (1.5 - 0.00275 * 97.0) ** 4 / (460 + 25.9 * 97.0)
    assert fme / 0.778 == pytest.approx(1.0, abs=5e-4)
    rsc = 60 * (1 - math.exp(-0.0497 * r["isi"])) * fme / 0.778
    assert 0.0 < r["cfb"] < 1.0
    assert r["hros"] == pytest.approx(rss + r["cfb"] * (rsc - rss), rel=1e-13)
    assert min(rss, rsc) < r["hros"] < max(rss, rsc)
    # fuel consumption adds the crown's share of 1.8 kg/m^2
    assert r["tfc"] == pytest.approx(r["sfc"] + 1.8 * r["cfb"], rel=1e-14)


@pytest.mark.parametrize("slope", [0.0, 30.0])
def test_d2_is_a_fifth_of_d1(slope):
    for ws in (0.0, 15.0, 50.0):
        d1 = _pt(8, ws=ws, slope_pct=slope, upslope_az=45.0)
        d2 = _pt(16, ws=ws, slope_pct=slope, upslope_az=45.0)
        assert d2["hros"] == pytest.approx(0.2 * d1["hros"], rel=1e-13)
        assert d2["bros"] == pytest.approx(0.2 * d1["bros"], rel=1e-13)
        assert d2["lb"] == d1["lb"] and d2["sfc"] == d1["sfc"]


def test_dead_fir_mixedwood_limits():
    kw = dict(ffmc=91.0, bui=0.0, ws=12.0)
    d1 = _pt(8, **kw)["hros"]
    m3_pure = 120 * (1 - math.exp(-0.0572 * _pt(8, **kw)["isi"])) ** 1.4
    m4_pure = 100 * (1 - math.exp(-0.0404 * _pt(8, **kw)["isi"])) ** 1.48
    assert _pt(17, pdf=100.0, **kw)["hros"] == pytest.approx(m3_pure, rel=1e-13)
    assert _pt(18, pdf=100.0, **kw)["hros"] == pytest.approx(m4_pure, rel=1e-13)
    assert _pt(17, pdf=0.0, **kw)["hros"] == pytest.approx(d1, rel=1e-14)
    assert _pt(18, pdf=0.0, **kw)["hros"] == pytest.approx(0.2 * d1, rel=1e-14)
    assert _pt(17, pdf=30.0, **kw)["hros"] == pytest.approx(0.3 * m3_pure + 0.7 * d1, rel=1e-13)
    # on a slope, an all-dead-fir M-3 takes its own curve's slope effect
    s = dict(slope_pct=40.0, upslope_az=0.0, ws=0.0)
    flat = _pt(17, pdf=100.0, ffmc=91.0, bui=0.0, ws=0.0)["hros"]
    sf = math.exp(3.533 * 0.4 ** 1.2)
    assert _pt(17, pdf=100.0, ffmc=91.0, bui=0.0, **s)["hros"] == pytest.approx(sf * flat, rel=1e-11)


# ----------------------------------------------- the A5 (iv) cutoff, simulated

def _grid(seed, rows=30, cols=30):
    rng = np.random.default_rng(seed)
    fuel = rng.choice([1, 2, 3, 6, 8, 16, 17, 18, 11], size=(rows, cols)).astype(np.uint8)
    elev = rng.integers(0, 200, (rows, cols)).astype(np.int16)
    wx = rng.uniform([86, 40, 5, 0], [95, 110, 35, 360], (1, 10, 4)).astype(np.float32)
    return fuel, elev, wx


def test_intensity_cutoff_zero_changes_nothing_and_huge_stops_at_ignition():
    fuel, elev, wx = _grid(3)
    kw = dict(n_periods=10, reps=4, seed=5, sigma=0.2, rounding=1, ignition_mode=1)
    base = oracle.simulate(fuel, elev, wx, **kw)
    same = oracle.simulate(fuel, elev, wx, hfi_min=0.0, **kw)
    assert np.array_equal(base["arrival_minute"], same["arrival_minute"])
    none = oracle.simulate(fuel, elev, wx, hfi_min=1e12, **kw)
    assert np.all(none["burned_cells"] == 1)


def test_intensity_cutoff_only_shrinks_scars():
    """Under constant weather and no noise every cell's intensity is the same
    in every period, so a cell either burns out at its first evaluation or
    never, and a higher cutoff only removes spreading cells: the scars
    shrink.  (Under changing weather the cutoff is not monotone: a cell held
    back into a more intense period can spread where it would have burned
    out.)"""
    fuel, elev, _ = _grid(4)
    wx = np.tile(np.array([92.0, 90.0, 20.0, 250.0], np.float32), (1, 10, 1))
    kw = dict(n_periods=10, reps=3, seed=9, sigma=0.0, rounding=1, ignition_mode=1)
    prev = oracle.simulate(fuel, elev, wx, **kw)["scar"]
    for cut in (500.0, 2000.0, 8000.0, 30000.0):
        cur = oracle.simulate(fuel, elev, wx, hfi_min=cut, **kw)["scar"]
        assert np.all(cur <= prev)
        prev = cur


def test_cell_intensity_follows_the_noisy_rate():
    fuel, elev, wx = _grid(5, 12, 12)
    a = oracle.eval_ros(fuel, elev, wx, seed=3, sigma=0.3, rep=2)
    b = oracle.eval_ros(fuel, elev, wx, seed=3, sigma=0.0, rep=2)
    burn = fuel.ravel() != 0
    mu = a["hros"][burn] / b["hros"][burn]
    np.testing.assert_allclose(a["hfi"][burn], mu * b["hfi"][burn], rtol=1e-13)
    np.testing.assert_array_equal(a["cfb"], b["cfb"])
