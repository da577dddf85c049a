"""Seeded input generators: determinism and recipe invariants (CPU only)."""
import numpy as np

import fa_inputs as fi


def test_knots_clamped_uniform():
    for p in (1, 2, 3):
        for n in (p + 1, 8, 32):
            t = fi.clamped_uniform_knots(n, p)
            assert t.dtype == np.float32 and len(t) == n + p + 1
            assert np.all(t[:p + 1] == 0) and np.all(t[n:] == 1)
            assert np.all(np.diff(t) >= 0)
            assert np.allclose(np.diff(t[p:n + 1]), 1.0 / (n - p), atol=1e-7)


def test_seeded_determinism():
    a = fi.config_c2(nblocks=16)
    b = fi.config_c2(nblocks=16)
    for f in ("ncp", "deg", "knot_off", "ctrl_off", "knots", "ctrl"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    c = fi.config_c2(seed=7, nblocks=16)
    assert not np.array_equal(a.ctrl, c.ctrl)
    assert set(np.unique(a.ncp)) <= set(fi.NCP_CHOICES_C2)
    assert set(np.unique(a.deg)) <= {2, 3}
    assert np.all(a.ctrl_off % fi.CTRL_ALIGN == 0)


def test_c1_recipe():
    b = fi.config_c1()
    assert b.nblocks == 1 and tuple(b.ncp[0]) == (16, 16, 16) and tuple(b.deg[0]) == (3, 3, 3)
    assert b.ctrl64 is not None
    assert np.array_equal(b.ctrl, b.ctrl64.astype(np.float32))


def test_turbulence_normalised():
    g = fi.rng(9)
    f = fi.turbulence_cube(g, 16, 3)
    assert f.shape == (3, 16, 16, 16) and f.dtype == np.float32
    assert np.allclose(f.mean(axis=(1, 2, 3)), 0, atol=1e-5)
    assert np.allclose(f.std(axis=(1, 2, 3)), 1, atol=1e-4)


def test_rays_hit_cube():
    xyz = fi.ray_samples_np(3, 32, 18, 16)
    assert xyz.shape == (32 * 18 * 16, 3)
    assert np.all(xyz > -1e-5) and np.all(xyz < 1 + 1e-5)
    o, d, t0, t1, j = fi.camera_rays(3, 32, 18)
    assert np.all(t1 > t0)


def test_voxel_subset_is_a_seeded_sample_without_replacement():
    s = fi.voxel_subset(7, (5, 6, 9), frac=0.1, seed=3)
    total = 7 * 5 * 6 * 9
    assert s.shape == (int(total * 0.1), 4) and s.dtype == np.int32
    flat = ((s[:, 0] * 5 + s[:, 1]) * 6 + s[:, 2]) * 9 + s[:, 3]
    assert np.all(np.diff(flat) > 0)  # distinct, increasing
    assert s[:, 0].max() < 7 and s[:, 1].max() < 5 and s[:, 2].max() < 6 and s[:, 3].max() < 9
    assert s.min() >= 0
    assert np.array_equal(s, fi.voxel_subset(7, (5, 6, 9), frac=0.1, seed=3))
    # 1% of C5's 4096 x 64^3 pairs
    assert int(4096 * 64 ** 3 * 0.01) == 10_737_418


def test_jittered_knots_nonuniform_and_increasing():
    g = fi.rng(5)
    for n, p in ((8, 3), (32, 3), (12, 2), (4, 3)):
        t = fi.jittered_knots(g, n, p)
        assert t.dtype == np.float32 and len(t) == n + p + 1
        assert np.all(t[:p + 1] == 0) and np.all(t[n:] == 1)
        assert np.all(np.diff(t[p:n + 1]) > 0)
        if n - p > 1:
            assert not np.array_equal(t, fi.clamped_uniform_knots(n, p))
    a, b = fi.config_c3_blocks(nb=2), fi.config_c3_blocks(nb=2, nonuniform=True)
    assert np.array_equal(a.ncp, b.ncp) and not np.array_equal(a.knots, b.knots)
