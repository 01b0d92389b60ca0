"""Seeded synthetic input generators: determinism, ranges, class balance."""
import numpy as np

from paper_1905_09317_amd import inputs


def test_fuel_grid_deterministic_and_balanced():
    a = inputs.fuel_grid(256, 256, 2)
    b = inputs.fuel_grid(256, 256, 2)
    assert a.dtype == np.uint8 and np.array_equal(a, b)
    assert not np.array_equal(a, inputs.fuel_grid(256, 256, 3))
    freq = np.bincount(a.ravel(), minlength=16) / a.size
    assert a.max() <= 15 and np.all(freq > 0.02) and np.all(freq < 0.12)
    # spatially correlated: neighbours mostly share a class
    assert (a[:, 1:] == a[:, :-1]).mean() > 0.7


def test_elevation_range():
    z = inputs.elevation_grid(128, 96, 3)
    assert z.dtype == np.int16 and z.shape == (128, 96)
    assert z.min() == 0 and z.max() == 800
    assert np.array_equal(z, inputs.elevation_grid(128, 96, 3))


def test_weather_ranges():
    w = inputs.weather_scenarios(5, 48, 6)
    assert w.shape == (5, 48, 4) and w.dtype == np.float32
    assert w[..., 0].min() >= 85 and w[..., 0].max() <= 94
    assert w[..., 1].min() >= 40 and w[..., 1].max() <= 120
    assert w[..., 2].min() >= 5 and w[..., 2].max() <= 40
    assert w[..., 3].min() >= 0 and w[..., 3].max() < 360
    # BUI holds for a day
    assert np.all(w[:, 1:24, 1] == w[:, :1, 1])


def test_query_stream():
    q = inputs.query_stream(200, 50.0, 8)
    t = np.array([x[0] for x in q])
    assert np.all(np.diff(t) >= 0)
    assert all(128 <= s <= 4096 and 1 <= r <= 256 for _, s, r in q)
