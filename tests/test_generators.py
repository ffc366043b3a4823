"""The seeded input generators reproduce the stated recipes."""
import numpy as np

import microstructures as ms


def test_circle32_voxel_count():
    m = ms.circle(32, 8.0, (16.0, 16.0))
    assert int(m.phase.sum()) == 208
    assert m.E.max() == 10.0 and m.E.min() == 1.0


def test_voronoi_deterministic_and_two_phase():
    a = ms.voronoi((64, 48), 10, 5)
    b = ms.voronoi((64, 48), 10, 5)
    assert np.array_equal(a.phase, b.phase)
    assert set(np.unique(a.E)) <= {1.0, 100.0}
    assert set(np.unique(a.nu)) <= {0.3, 0.2}


def test_rsa_spheres_non_overlapping_and_fraction():
    m = ms.rsa_spheres(40, 3, (2.0, 4.0), 0.2)
    assert m.phase.mean() >= 0.2
    c, r = m.extra["centres"], m.extra["radii"]
    for i in range(len(r)):
        d = c[i] - c
        d -= 40 * np.round(d / 40)
        dist = np.sqrt((d * d).sum(1))
        dist[i] = np.inf
        assert np.all(dist >= r[i] + r - 1e-12)


def test_grf_normalised():
    g = ms.gaussian_random_field((32, 32, 32), 4.0, 1)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1) < 1e-12
    m = ms.grf_modulus((16, 16, 16), 4.0, 2)
    assert np.all(m.E > 0) and np.all(m.nu == 0.3)


def test_uneven_batch_recipe():
    maps = ms.uneven_batch()
    assert len(maps) == 48
    for m in maps:
        n = m.shape[0]
        assert m.shape == (n, n) and n in (64, 128, 256, 512)
        c = m.extra["contrast"]
        assert 2.0 <= c <= 1000.0
        assert set(np.unique(m.E)) == {1.0, c}
    again = ms.uneven_batch()
    assert all(np.array_equal(a.E, b.E) for a, b in zip(maps, again))
