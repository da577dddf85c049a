"""Pins of the adaptive-encoding oracle (Sec. 4.2, Eq. 4, Alg. 1) against
facts fixed by the mathematics, not by re-running its own formulas (CPU)."""
import numpy as np
import pytest

import fa_inputs as fi
import oracle
from oracle import adaptive as ad


def _decode(P, ncp, deg, knots, R):
    kn = np.concatenate([np.asarray(k, np.float64) for k in knots])
    b = oracle.Blocks(np.array([ncp]), np.array([deg]), np.zeros(1), np.zeros(1), kn,
                      np.asarray(P, np.float64).reshape(-1))
    return oracle.decode_blocks(b, R, mask=1)[0, 0]


def test_knots_and_grid_match_the_stored_fp32_values():
    for n, p in ((5, 3), (9, 2), (33, 3), (64, 3)):
        assert np.array_equal(ad.uniform_knots(n, p), fi.clamped_uniform_knots(n, p))
    assert ad.grid_params(64)[-1] == 1.0 and ad.grid_params(64)[0] == 0.0


def test_fit_recovers_a_spline_exactly():
    """y = decode of P_true (full column rank: R >= n per axis) -> the least
    squares fit returns P_true and both error metrics vanish."""
    g = fi.rng(40)
    ncp, deg, R = (5, 7, 6), (2, 3, 3), (12, 10, 11)
    kn = [ad.uniform_knots(ncp[a], deg[a]) for a in range(3)]
    P = g.normal(size=ncp)
    y = _decode(P, ncp, deg, kn, R)
    Pf = ad.fit_block(y, ncp, deg, kn)
    assert np.abs(Pf - P).max() < 1e-10
    emax, erms = ad.model_errors(y, Pf, ncp, deg, kn)
    assert emax < 1e-12 and erms < 1e-12


def test_fit_equals_full_kronecker_least_squares():
    """Brute force: the design matrix assembled column by column from decodes
    of unit control lattices (no collocation matrices, no Kronecker
    factorisation), solved as one R^3 x n^3 least-squares problem."""
    g = fi.rng(41)
    ncp, deg, R = (4, 3, 5), (2, 1, 3), (6, 5, 7)
    kn = [ad.uniform_knots(ncp[a], deg[a]) for a in range(3)]
    cols = []
    for j in range(int(np.prod(ncp))):
        e = np.zeros(int(np.prod(ncp)))
        e[j] = 1.0
        cols.append(_decode(e.reshape(ncp), ncp, deg, kn, R).reshape(-1))
    A = np.stack(cols, 1)
    y = g.normal(size=R)
    want = np.linalg.lstsq(A, y.reshape(-1), rcond=None)[0].reshape(ncp)
    assert np.abs(ad.fit_block(y, ncp, deg, kn) - want).max() < 1e-10


def test_fit_residual_is_orthogonal_to_the_model_space():
    """Normal equations: B^T (y - B P) = 0, with B^T applied by the oracle's
    adjoint (a scatter code independent of the least-squares solve)."""
    g = fi.rng(42)
    ncp, deg, R = (8, 6, 9), (3, 2, 3), (16, 13, 20)
    kn = [ad.uniform_knots(ncp[a], deg[a]) for a in range(3)]
    y = g.normal(size=R)
    P = ad.fit_block(y, ncp, deg, kn)
    r = y - _decode(P, ncp, deg, kn, R)
    knc = np.concatenate(kn)
    b = oracle.Blocks(np.array([ncp]), np.array([deg]), np.zeros(1), np.zeros(1), knc,
                      np.zeros(int(np.prod(ncp))))
    G = oracle.decode_adjoint(b, R, r[None, None])
    assert np.abs(G).max() < 1e-11 * np.abs(y).sum()
    # and the fit is strictly better than a perturbed lattice (minimiser)
    e0 = ad.model_errors(y, P, ncp, deg, kn)[1]
    for _ in range(5):
        e1 = ad.model_errors(y, P + 1e-3 * g.normal(size=ncp), ncp, deg, kn)[1]
        assert e1 > e0


def test_linear_fields_have_zero_error_for_every_ncp():
    """Linear precision of clamped B-splines: a trilinear-free linear field
    lies in every model space, so Error(NCP) = 0 for all candidates."""
    R, p = 12, 3
    u = ad.grid_params(R)
    y = 0.3 + 1.5 * u[:, None, None] - 0.7 * u[None, :, None] + 2.0 * u[None, None, :]
    errs = ad.error_map(y, p, p + 2, R)
    assert np.abs(errs).max() < 1e-12


def test_error_metrics_are_max_and_rms():
    g = fi.rng(43)
    y = g.normal(size=(5, 6, 7))
    kn = [ad.uniform_knots(4, 2)] * 3
    emax, erms = ad.model_errors(y, np.zeros((4, 4, 4)), (4, 4, 4), (2, 2, 2), kn)
    assert emax == np.abs(y).max()
    assert abs(erms - np.sqrt((y * y).mean())) < 1e-15


def test_error_falls_to_zero_at_full_resolution():
    """NCP = R makes B square and invertible (Schoenberg-Whitney holds on the
    uniform grid): the fit interpolates, Error(R) = 0; fewer control points
    than samples leave a non-zero residual for a generic field."""
    g = fi.rng(44)
    R, p = 9, 3
    y = g.normal(size=(R, R, R))
    errs = ad.error_map(y, p, p + 2, R)
    assert errs[-1].max() < 1e-11
    assert np.all(errs[:-1, 1] > 1e-3)


def test_select_ncp_rule():
    """Eq. 4: the smallest NCP with Error < e; complex iff some Error > e."""
    errs = np.array([[9, 0.9], [5, 0.5], [2, 0.2], [0.5, 0.05], [0.1, 0.01]])  # NCP 5..9
    assert ad.select_ncp(errs, 5, 0.3) == (7, True)
    assert ad.select_ncp(errs, 5, 0.06) == (8, True)
    assert ad.select_ncp(errs, 5, 1.0) == (5, False)
    assert ad.select_ncp(errs, 5, 0.001) == (9, True)  # none below e: the largest
    assert ad.select_ncp(errs, 5, 3.0, ad.METRIC_MAX) == (7, True)
    assert ad.select_ncp(errs, 5, 0.9) == (6, False)  # Error == e is neither below nor over


def test_cross_level_searches_only_children_of_complex_blocks():
    """Level 0: one block with a sharp bump near one corner (complex);
    level 1: only the child holding the bump stays complex, the flat
    children get NCP* = degree + 2 (searched: their parent is complex);
    level 2: only the 8 children of that child are searched, every other
    block takes degree + 1 without a search."""
    R, p = 8, 2
    c = np.array([0.1, 0.12, 0.15])

    def field(x, y, z):
        return np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2 * 0.03 ** 2))

    levels = []
    for k in range(3):
        m = 1 << k
        Y = np.empty((m ** 3, R, R, R))
        u = ad.grid_params(R)
        for b in range(m ** 3):
            bx, by, bz = b // (m * m), (b // m) % m, b % m
            X = (bx + u) / m
            Yc = (by + u) / m
            Z = (bz + u) / m
            Y[b] = field(X[:, None, None], Yc[None, :, None], Z[None, None, :])
        levels.append(Y)
    res = ad.cross_level(levels, p, 1e-4, ncp_lo=p + 2, ncp_hi=R)
    n0, c0, s0, _ = res[0]
    assert s0.all() and c0[0]
    n1, c1, s1, _ = res[1]
    assert s1.all()
    assert c1[0] and not c1[1:].any()
    assert np.all(n1[1:] == p + 2)
    n2, c2, s2, _ = res[2]
    kids = [((bx * 4) + by) * 4 + bz for bx in (0, 1) for by in (0, 1) for bz in (0, 1)]
    assert set(np.nonzero(s2)[0]) == set(kids)
    others = np.setdiff1d(np.arange(64), kids)
    assert np.all(n2[others] == p + 1)

