"""The Marschner-Lobb field (Eq. 5) and its analytic gradient (CPU)."""
import numpy as np

import fa_inputs as fi


def test_ml_gradient_matches_central_differences():
    g = fi.rng(70)
    p = g.uniform(0, 7, (2000, 3))
    p[:5, :2] = 0.0  # on the axis r = 0
    h = 1e-6
    gx, gy, gz = fi.ml_gradient(p[:, 0], p[:, 1], p[:, 2])
    G = np.stack([gx, gy, gz], 1)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (fi.ml_value(*(p + e).T) - fi.ml_value(*(p - e).T)) / (2 * h)
        if a < 2:
            fd[:5] = 0.0  # one-sided kink-free: symmetric in x, y at r = 0
        assert np.abs(fd - G[:, a]).max() < 2e-6 * (1 + np.abs(G[:, a]).max())


def test_ml_known_values():
    # z = 0, r = 0: rho = cos(2 pi f_M) = 1 -> F = (1 + 2 alpha) / (2 (1 + alpha))
    a = fi.ML_ALPHA
    assert abs(fi.ml_value(0.0, 0.0, 0.0) - (1 + 2 * a) / (2 * (1 + a))) < 1e-15
    # z = 1: sin(pi/2) = 1; r = 1: cos(pi/2) = 0 -> rho = 1
    assert abs(fi.ml_value(1.0, 0.0, 1.0) - 2 * a / (2 * (1 + a))) < 1e-15
    x = fi.rng(71).uniform(0, 7, (10000, 3))
    v = fi.ml_value(*x.T)
    assert v.min() >= 0.0 and v.max() <= 1.0


def test_ml_blocks_share_boundaries():
    R = 9
    Y = fi.ml_blocks(1, R)
    assert Y.shape == (8, R, R, R)
    # block (0,0,0) last x plane == block (1,0,0) first x plane
    assert np.array_equal(Y[0][-1], Y[4][0])
    assert np.array_equal(Y[0][:, :, -1], Y[1][:, :, 0])
    x, y, z = fi.block_grid(2, 63, R)
    assert x[-1] == 7.0 and z[-1] == 7.0 and abs(x[0] - 5.25) < 1e-15
