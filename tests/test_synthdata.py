"""The seeded generators: determinism, ranges and the grid ordering."""
import numpy as np

import synthdata as sd


def test_same_seed_same_bytes():
    a = sd.make_problem("terrain2d", scale=1 / 256)
    b = sd.make_problem("terrain2d", scale=1 / 256)
    for x, y in [(a.points, b.points), (a.values, b.values), (a.test_points, b.test_points)]:
        assert x.tobytes() == y.tobytes()
    c = sd.make_problem("terrain2d", scale=1 / 256, seed=99)
    assert c.points.tobytes() != a.points.tobytes()


def test_ranges_and_split():
    p = sd.make_problem("terrain2d", scale=1 / 64)
    assert p.points.min() >= 0 and p.points.max() <= 1
    n = p.points.shape[1] + p.test_points.shape[1]
    assert p.test_points.shape[1] == round(0.01 * n)
    assert np.isfinite(p.values).all()


def test_grid_centres_first_coordinate_fastest():
    c = sd.grid_centers(4, 2)
    assert c.shape == (2, 16)
    assert np.allclose(c[:, 1], [1 / 3, 0.0]) and np.allclose(c[:, 4], [0.0, 1 / 3])
    c3 = sd.grid_centers(3, 3)
    assert np.allclose(c3[:, 1], [0.5, 0, 0]) and np.allclose(c3[:, 3], [0, 0.5, 0])
    assert np.allclose(c3[:, 9], [0, 0, 0.5])


def test_radius_covers_k_centres():
    for dim, g in ((2, 256), (3, 64)):
        rho = sd.support_radius_for_k(g, dim, 40.0)
        delta = 1 / (g - 1)
        vol = np.pi * rho ** 2 if dim == 2 else 4 / 3 * np.pi * rho ** 3
        assert abs(vol / delta ** dim - 40.0) < 1e-9


def test_franke_config_uses_printed_radius():
    p = sd.make_problem("franke2d")
    assert p.rho == 0.12 and p.points.shape == (2, 10_000) and p.centers.shape == (2, 1024)


def test_halton_points_radical_inverse():
    # radical inverses of 1..6 in bases 2 and 3, written out
    p = sd.halton_points(6, 2)
    np.testing.assert_array_equal(p[0], [1 / 2, 1 / 4, 3 / 4, 1 / 8, 5 / 8, 3 / 8])
    np.testing.assert_allclose(p[1], [1 / 3, 2 / 3, 1 / 9, 4 / 9, 7 / 9, 2 / 9], rtol=1e-15)
    q = sd.halton_points(1089, 2)
    assert q.shape == (2, 1089) and np.all((q > 0) & (q < 1))
    assert len(np.unique(q[0])) == 1089
