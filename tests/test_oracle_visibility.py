"""The visibility oracle (the cells a ray caster's samples fall in, Alg. 2)
against hand-derived cell sets (CPU)."""
import numpy as np

from oracle import visibility as vis


def _flags(cells, nb):
    f = np.zeros(int(np.prod(nb)), np.int32)
    for (i, j, k) in cells:
        f[(i * nb[1] + j) * nb[2] + k] = 1
    return f


def test_axis_aligned_rays():
    nb = (4, 5, 6)
    S = 16
    # along +x at y = 0.3, z = 0.7: samples x = (s + 1/2) / S cross every x cell
    r1 = [0.0, 0.3, 0.7, 1.0, 0.0, 0.0, 0.0, 1.0]
    want = _flags([(i, 1, 4) for i in range(4)], nb)
    assert np.array_equal(vis.visible_cells(np.array([r1], np.float32), S, nb, (0, 0, 0),
                                            (1, 1, 1)), want)
    # along -z over the first half of the segment only (t1 = 0.5): z in (0.5, 1)
    r2 = [0.55, 0.95, 1.0, 0.0, 0.0, -1.0, 0.0, 0.5]
    want2 = _flags([(2, 4, k) for k in (3, 4, 5)], nb)
    got2 = vis.visible_cells(np.array([r2], np.float32), S, nb, (0, 0, 0), (1, 1, 1))
    assert np.array_equal(got2, want2)
    # a miss (t1 <= t0) flags nothing; both rays together give the union
    r3 = [0.5, 0.5, 0.5, 1.0, 0.0, 0.0, 0.3, 0.3]
    got = vis.visible_cells(np.array([r1, r2, r3], np.float32), S, nb, (0, 0, 0), (1, 1, 1))
    assert np.array_equal(got, np.maximum(want, want2))


def test_positions_outside_are_clamped_and_origin_extent():
    nb = (2, 2, 2)
    # a ray outside the domain on y < origin is clamped onto the y = 0 cells
    r = [-1.0, -5.0, 0.25, 1.0, 0.0, 0.0, 0.0, 4.0]  # x from -1 to 3, y = -5, z = 0.25
    origin, extent = (-1.0, -1.0, 0.0), (4.0, 2.0, 1.0)
    # x cells: floor((x + 1) * 2 / 4) over x in (-1, 3): both; y clamped -> 0; z: floor(0.5) = 0
    want = _flags([(0, 0, 0), (1, 0, 0)], nb)
    got = vis.visible_cells(np.array([r], np.float32), 8, nb, origin, extent)
    assert np.array_equal(got, want)


def test_one_sample_lands_on_the_segment_midpoint():
    nb = (8, 8, 8)
    # S = 1: the only sample is at t = (t0 + t1) / 2
    r = [0.0, 0.0, 0.0, 0.6, 0.8, 0.0, 0.2, 0.6]  # midpoint t = 0.4: (0.24, 0.32, 0)
    got = vis.visible_cells(np.array([r], np.float32), 1, nb, (0, 0, 0), (1, 1, 1))
    assert np.array_equal(got, _flags([(1, 2, 0)], nb))
