"""Pins for the oracle's FBP System rates, ellipse fit and eq. (1).

The paper cites the FBP System without printing it, so the pins here are
closed forms, special cases and identities that a dropped term, a wrong sign
or a swapped coefficient would break, plus one hand evaluation.
"""
import math

import numpy as np
import pytest

import oracle

FUELS = list(range(1, 16))
SINGLE = [1, 2, 3, 4, 5, 6, 7, 8, 11, 12, 13]   # unmixed, non-grass fuels


def test_hand_evaluation_c2_ffmc90_bui80_ws20():
    """Independent hand evaluation of the closed forms for C-2, FFMC 90,
    BUI 80, wind 20 km/h from 270 deg, flat ground (six decimals)."""
    r = oracle.fbp_point(2, 90.0, 80.0, 20.0, 270.0)
    hand = dict(isi=11.745219, be=1.057313, hros=17.412164, bros=1.043263, lb=2.570745,
                fros=3.589509)
    for k, v in hand.items():
        assert r[k] == pytest.approx(v, abs=2e-6), k
    assert r["raz"] == pytest.approx(90.0, abs=1e-9)       # heads east, downwind
    axes = oracle.axis_ros(r["hros"], r["bros"], r["fros"], r["raz"])
    assert axes[0] == pytest.approx(17.728662, abs=2e-6)   # E (head)
    assert axes[1] == pytest.approx(4.005607, abs=2e-6)    # NE
    assert axes[7] == pytest.approx(4.005607, abs=2e-6)    # SE
    for k in (2, 3, 4, 5, 6):
        assert axes[k] == pytest.approx(1.396291, abs=2e-6)


@pytest.mark.parametrize("fuel", FUELS)
def test_no_wind_no_slope_is_circular(fuel):
    r = oracle.fbp_point(fuel, 91.0, 60.0, 0.0, 123.0)
    assert r["bros"] == r["hros"]           # back spread index equals ISI at zero wind
    assert r["lb"] == 1.0
    assert r["fros"] == pytest.approx(r["hros"], rel=1e-15)
    axes = oracle.axis_ros(r["hros"], r["bros"], r["fros"], r["raz"])
    np.testing.assert_allclose(axes, r["hros"], rtol=1e-14)


@pytest.mark.parametrize("fuel", FUELS)
def test_flank_identity(fuel):
    """a = LB * b with a = (H+B)/2 and b = FROS (Section 3.7)."""
    r = oracle.fbp_point(fuel, 88.0, 70.0, 17.0, 45.0, slope_pct=12.0, upslope_az=300.0)
    assert r["fros"] * r["lb"] == pytest.approx((r["hros"] + r["bros"]) / 2, rel=1e-14)


@pytest.mark.parametrize("fuel", [1, 2, 3, 4, 7, 8, 11, 12, 13])
def test_bui_at_reference_value_has_no_effect(fuel):
    bui0 = {1: 72, 2: 64, 3: 62, 4: 66, 7: 106, 8: 32, 11: 38, 12: 63, 13: 31}[fuel]
    r = oracle.fbp_point(fuel, 90.0, bui0, 10.0, 0.0)
    assert r["be"] == pytest.approx(1.0, abs=1e-15)
    assert oracle.fbp_point(fuel, 90.0, 0.0, 10.0, 0.0)["be"] == 1.0


@pytest.mark.parametrize("fuel", [14, 15])
def test_grass_has_no_bui_effect_and_curing_scales(fuel):
    a = oracle.fbp_point(fuel, 92.0, 10.0, 15.0, 180.0, curing=80.0)
    b = oracle.fbp_point(fuel, 92.0, 150.0, 15.0, 180.0, curing=80.0)
    assert a["be"] == 1.0 and b["be"] == 1.0
    assert a["hros"] == b["hros"]
    full = oracle.fbp_point(fuel, 92.0, 10.0, 15.0, 180.0, curing=100.0)
    # curing factor: 0.176 + 0.02 (C - 58.8) above 58.8 %: CF(100) = 1, CF(80) = 0.6
    assert a["hros"] / full["hros"] == pytest.approx(0.6, rel=1e-13)
    low = oracle.fbp_point(fuel, 92.0, 10.0, 15.0, 180.0, curing=50.0)
    # below 58.8 %: 0.005 (exp(0.061 C) - 1)
    assert low["hros"] / full["hros"] == pytest.approx(0.005 * math.expm1(0.061 * 50.0), rel=1e-13)
    # grass length-to-breadth: 1.1 WSV^0.464, independent of curing
    assert a["lb"] == pytest.approx(1.1 * 15.0 ** 0.464, rel=1e-14)
    assert oracle.fbp_point(fuel, 92.0, 10.0, 0.5, 180.0)["lb"] == 1.0


def test_mixedwood_limits():
    kw = dict(ffmc=90.0, bui=0.0, ws=12.0, wd=200.0)
    c2 = oracle.fbp_point(2, **kw)
    d1 = oracle.fbp_point(8, **kw)
    assert oracle.fbp_point(9, pc=100.0, **kw)["hros"] == pytest.approx(c2["hros"], rel=1e-15)
    assert oracle.fbp_point(9, pc=0.0, **kw)["hros"] == pytest.approx(d1["hros"], rel=1e-15)
    assert oracle.fbp_point(10, pc=0.0, **kw)["hros"] == pytest.approx(0.2 * d1["hros"], rel=1e-14)
    m1 = oracle.fbp_point(9, pc=30.0, **kw)
    assert m1["hros"] == pytest.approx(0.3 * c2["hros"] + 0.7 * d1["hros"], rel=1e-14)
    # on a slope, a pure-conifer M-1 takes exactly the C-2 slope effect
    s = dict(slope_pct=35.0, upslope_az=10.0)
    assert oracle.fbp_point(9, pc=100.0, **kw, **s)["hros"] == pytest.approx(
        oracle.fbp_point(2, **kw, **s)["hros"], rel=1e-13)


@pytest.mark.parametrize("fuel", SINGLE + [14, 15])
@pytest.mark.parametrize("gs", [5.0, 20.0, 45.0])
def test_slope_alone_multiplies_zero_wind_rate_by_slope_factor(fuel, gs):
    """With no wind, the slope-equivalent wind speed is built so that the
    head rate equals SF x (zero-wind rate), SF = exp(3.533 (GS/100)^1.2),
    and the fire heads straight upslope."""
    flat = oracle.fbp_point(fuel, 89.0, 55.0, 0.0, 0.0)
    r = oracle.fbp_point(fuel, 89.0, 55.0, 0.0, 0.0, slope_pct=gs, upslope_az=137.0)
    sf = math.exp(3.533 * (gs / 100.0) ** 1.2)
    if r["wse"] <= 40.0 and sf * flat["hros"] < 0.5 * 190:
        assert r["hros"] == pytest.approx(sf * flat["hros"], rel=1e-11)
    assert r["raz"] == pytest.approx(137.0, abs=1e-9)
    assert r["wsv"] == pytest.approx(r["wse"], rel=1e-14)


def test_steep_slope_factor_caps_at_ten():
    flat = oracle.fbp_point(8, 86.0, 40.0, 0.0, 0.0)
    r = oracle.fbp_point(8, 86.0, 40.0, 0.0, 0.0, slope_pct=85.0, upslope_az=0.0)
    assert r["hros"] == pytest.approx(10.0 * flat["hros"], rel=1e-11)


def test_wind_and_slope_aligned_add_as_speeds():
    w = oracle.fbp_point(3, 90.0, 70.0, 12.0, 180.0)          # wind from S -> heads N
    s = oracle.fbp_point(3, 90.0, 70.0, 0.0, 0.0, slope_pct=25.0, upslope_az=0.0)
    ws = oracle.fbp_point(3, 90.0, 70.0, 12.0, 180.0, slope_pct=25.0, upslope_az=0.0)
    assert ws["wsv"] == pytest.approx(12.0 + s["wse"], rel=1e-14)
    assert ws["raz"] == pytest.approx(0.0, abs=1e-6) or ws["raz"] == pytest.approx(360.0, abs=1e-6)
    assert ws["hros"] > w["hros"]


@pytest.mark.parametrize("wd,raz", [(270.0, 90.0), (0.0, 180.0), (90.0, 270.0), (180.0, 0.0),
                                    (225.0, 45.0)])
def test_fire_heads_downwind(wd, raz):
    r = oracle.fbp_point(2, 90.0, 80.0, 10.0, wd)
    d = abs((r["raz"] - raz + 180.0) % 360.0 - 180.0)
    assert d < 1e-9


@pytest.mark.parametrize("fuel", FUELS)
def test_wind_function_continuous_at_40(fuel):
    """The two branches of f(W) meet at 40 km/h up to the rounding of their
    published constants: exp(0.05039*40) = 7.5054, 12(1-exp(-0.0818*12)) = 7.5035."""
    lo = oracle.fbp_point(fuel, 90.0, 60.0, 40.0 - 1e-9, 0.0)
    hi = oracle.fbp_point(fuel, 90.0, 60.0, 40.0 + 1e-9, 0.0)
    assert hi["isi"] / lo["isi"] == pytest.approx(12 * -math.expm1(-0.0818 * 12) / math.exp(0.05039 * 40),
                                                  rel=1e-8)
    assert hi["hros"] == pytest.approx(lo["hros"], rel=2e-3)


@pytest.mark.parametrize("fuel", FUELS)
def test_rates_monotone_in_wind_and_ffmc(fuel):
    ws = np.linspace(0.0, 60.0, 61)
    h = [oracle.fbp_point(fuel, 90.0, 60.0, w, 270.0)["hros"] for w in ws]
    assert np.all(np.diff(h) > 0)
    ff = np.linspace(70.0, 99.0, 30)
    h2 = [oracle.fbp_point(fuel, f, 60.0, 10.0, 270.0)["hros"] for f in ff]
    assert np.all(np.diff(h2) > 0)
    # the head-axis rate of eq. (1) never falls as wind rises
    head = []
    for w in ws:
        r = oracle.fbp_point(fuel, 90.0, 60.0, w, 270.0)
        head.append(oracle.axis_ros(r["hros"], r["bros"], r["fros"], r["raz"])[0])
    assert np.all(np.diff(head) >= -1e-12)


@pytest.mark.parametrize("h,b,lb,raz", [(17.0, 1.0, 2.5, 90.0), (5.0, 0.5, 1.7, 10.0),
                                       (40.0, 3.0, 4.9, 250.0)])
def test_eq1_special_angles(h, b, lb, raz):
    """eq. (1) gives a(1+e) along the head direction and a(1-e^2) = a/LB^2
    across and behind it, with a from eq. (2) and e from eq. (4)."""
    a = (h + b) / 2.0
    f = a / lb
    e = math.sqrt(1.0 - 1.0 / lb**2)
    out = oracle.axis_ros(h, b, f, raz)
    theta_head = 90.0 - raz
    for k in range(8):
        phi = (45.0 * k - theta_head) % 360.0
        if abs(phi) < 1e-9 or abs(phi - 360.0) < 1e-9:
            assert out[k] == pytest.approx(a * (1 + e), rel=1e-13)
        if 90.0 <= phi <= 270.0:
            assert out[k] == pytest.approx(a / lb**2, rel=1e-13)
    assert max(out) <= a * (1 + e) * (1 + 1e-14)
    assert min(out) >= a / lb**2 * (1 - 1e-14)


def test_eq1_mirror_symmetry_about_head():
    r = oracle.fbp_point(4, 91.0, 90.0, 25.0, 225.0)      # heads NE (azimuth 45)
    out = oracle.axis_ros(r["hros"], r["bros"], r["fros"], r["raz"])
    # axes at +-45 deg from NE are N and E; +-90: NW and SE; +-135: W and S
    assert out[2] == pytest.approx(out[0], rel=1e-12)
    assert out[3] == pytest.approx(out[7], rel=1e-12)
    assert out[4] == pytest.approx(out[6], rel=1e-12)
    assert out[1] == max(out)


def test_horn_on_a_plane():
    """z = A*col - B*row rises A m per cell eastward and B m per cell
    northward; Horn's numerators are 8A and 8B inside, 4A/4B on the
    replicated edges."""
    A, B = 3, 5
    rr, cc = np.mgrid[0:9, 0:11]
    z = (A * cc - B * rr + 400).astype(np.int16)
    gx, gn = oracle.horn(z)
    assert np.all(gx[:, 1:-1] == 8 * A) and np.all(gx[:, [0, -1]] == 4 * A)
    assert np.all(gn[1:-1, :] == 8 * B) and np.all(gn[[0, -1], :] == 4 * B)


def test_slope_field_through_eval_ros():
    """On a plane the FBP evaluation sees slope 100*sqrt(A^2+B^2)/cs percent
    uphill towards azimuth atan2(A, B); with no wind, the head azimuth equals
    that upslope direction and the head rate equals SF x the flat rate."""
    A, B = 6, -4
    rr, cc = np.mgrid[0:7, 0:7]
    z = (A * cc - B * rr + 300).astype(np.int16)
    fuel = np.full(z.shape, 3, np.uint8)
    wx = np.array([[[90.0, 70.0, 0.0, 0.0]]], np.float32)
    r = oracle.eval_ros(fuel, z, wx)
    flat = oracle.eval_ros(fuel, None, wx)
    centre = 3 * 7 + 3
    gs = 100.0 * math.hypot(A, B) / 100.0
    az = math.degrees(math.atan2(A, B)) % 360.0
    assert r["raz"][centre] == pytest.approx(az, abs=1e-9)
    sf = math.exp(3.533 * (gs / 100.0) ** 1.2)
    assert r["hros"][centre] == pytest.approx(sf * flat["hros"][centre], rel=1e-11)


def test_eval_ros_cell_subset_equals_full_grid():
    """Selecting cells only changes which cells are evaluated, not the values."""
    from paper_1905_09317_amd import inputs
    w = inputs.batched_monte_carlo(side=48, reps=2, n_scenarios=3, n_periods=4)
    full = oracle.eval_ros(w.fuel, w.elev, w.weather, scenario=2, period=3, rep=1, seed=9, sigma=0.2,
                           rounding=1)
    cells = np.array([0, 47, 48 * 48 - 1, 1000, 1000, 5], np.int32)
    sub = oracle.eval_ros(w.fuel, w.elev, w.weather, scenario=2, period=3, rep=1, seed=9, sigma=0.2,
                          rounding=1, cells=cells)
    for k in full:
        assert np.array_equal(full[k][cells], sub[k]), k
    with pytest.raises(ValueError):
        oracle.eval_ros(w.fuel, w.elev, w.weather, cells=np.array([48 * 48], np.int32))


# ------------------------------------------------ steep slopes, fast fuels
# Published curve constants (a, b, c, q, BUI0) typed here for the closed
# forms below: C-2 and S-3.
_C2 = (110.0, 0.0282, 1.5, 0.70, 64.0)
_S3 = (55.0, 0.0829, 3.2, 0.75, 31.0)


def _ff(ffmc):
    m = 147.2 * (101.0 - ffmc) / (59.5 + ffmc)
    return 91.9 * math.exp(-0.1386 * m) * (1.0 + m ** 5.31 / 4.93e7)


def _be(k, bui):
    return math.exp(50.0 * math.log(k[3]) * (1.0 / bui - 1.0 / k[4]))


def test_slope_wind_above_40_kmh_keeps_the_slope_identity():
    """C-2, FFMC 94, 80 % slope, no wind: the slope-equivalent wind exceeds 40
    km/h, where f(W) = 12 (1 - exp(-0.0818 (W - 28))) and WSE = 28 -
    ln(1 - ISF / (2.496 f(F))) / 0.0818.  Because 0.208 x 12 = 2.496, the
    spread index at that wind is ISF again, so H = SF x H_flat still holds
    and the fire heads upslope at WSV = WSE."""
    flat = oracle.fbp_point(2, 94.0, 80.0, 0.0, 0.0)
    r = oracle.fbp_point(2, 94.0, 80.0, 0.0, 0.0, slope_pct=80.0, upslope_az=30.0)
    assert 40.0 < r["wse"] < 112.45
    assert r["wsv"] == pytest.approx(r["wse"], rel=1e-14)
    assert r["hros"] == pytest.approx(10.0 * flat["hros"], rel=1e-11)
    assert r["raz"] == pytest.approx(30.0, abs=1e-9)
    # the branch's own closed form, from the zero-wind rate inverted by hand
    a, b, c, _, _ = _C2
    ff = _ff(94.0)
    rsz = a * (-math.expm1(-b * 0.208 * ff)) ** c
    isf = math.log(1.0 - (10.0 * rsz / a) ** (1.0 / c)) / -b
    assert r["isi"] == pytest.approx(isf, rel=1e-11)
    assert r["wse"] == pytest.approx(28.0 - math.log(1.0 - isf / (2.496 * ff)) / 0.0818, rel=1e-11)


def test_slope_wind_cap_at_112_45_kmh():
    """C-2, FFMC 96, 80 % slope: ISF reaches 0.999 x 2.496 f(F), so WSE is
    capped at 112.45 km/h and H follows from that wind, below SF x H_flat."""
    a, b, c, _, _ = _C2
    ff = _ff(96.0)
    r = oracle.fbp_point(2, 96.0, 80.0, 0.0, 0.0, slope_pct=80.0, upslope_az=200.0)
    assert r["wse"] == 112.45 and r["wsv"] == pytest.approx(112.45, rel=1e-14)
    isi = 0.208 * 12.0 * (-math.expm1(-0.0818 * (112.45 - 28.0))) * ff
    assert r["isi"] == pytest.approx(isi, rel=1e-12)
    h = a * (-math.expm1(-b * isi)) ** c * _be(_C2, 80.0)
    assert r["hros"] == pytest.approx(h, rel=1e-12)
    assert r["hros"] < 10.0 * oracle.fbp_point(2, 96.0, 80.0, 0.0, 0.0)["hros"]


def test_isf_floor_inside_the_logarithm():
    """S-3, FFMC 96, 80 % slope: 1 - (RSF/a)^(1/c) falls below 0.01, so ISF
    = ln(0.01) / -b and the head rate is a (1 - 0.01)^c BE; WSE stays below
    40 km/h, on the ordinary branch."""
    a, b, c, _, _ = _S3
    ff = _ff(96.0)
    rsz = a * (-math.expm1(-b * 0.208 * ff)) ** c
    assert 1.0 - (10.0 * rsz / a) ** (1.0 / c) < 0.01
    r = oracle.fbp_point(13, 96.0, 80.0, 0.0, 0.0, slope_pct=80.0, upslope_az=90.0)
    isf = math.log(0.01) / -b
    assert r["isi"] == pytest.approx(isf, rel=1e-12)
    assert r["wse"] == pytest.approx(math.log(isf / (0.208 * ff)) / 0.05039, rel=1e-12)
    assert r["wse"] < 40.0
    assert r["hros"] == pytest.approx(a * 0.99 ** c * _be(_S3, 80.0), rel=1e-12)
