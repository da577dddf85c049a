"""Planted mistakes in the adaptive-encoding oracle: every one must make at
least one of its pins fail (CPU)."""
import numpy as np
import pytest

import test_oracle_adaptive as pins
from oracle import adaptive as ad

PINS = [pins.test_knots_and_grid_match_the_stored_fp32_values,
        pins.test_fit_recovers_a_spline_exactly,
        pins.test_fit_equals_full_kronecker_least_squares,
        pins.test_fit_residual_is_orthogonal_to_the_model_space,
        pins.test_linear_fields_have_zero_error_for_every_ncp,
        pins.test_error_metrics_are_max_and_rms,
        pins.test_error_falls_to_zero_at_full_resolution,
        pins.test_select_ncp_rule,
        pins.test_cross_level_searches_only_children_of_complex_blocks]

_orig = {k: getattr(ad, k) for k in ("grid_params", "uniform_knots", "collocation", "fit_block",
                                     "model_errors", "select_ncp", "cross_level")}


def _cell_grid(R):  # cell-centred grid instead of end points included
    return (np.arange(R) + 0.5) / R


def _knots_off(n, p):
    t = _orig["uniform_knots"](n, p)
    if n - p > 1:
        t[p + 1] = t[p + 1] * 0.9
    return t


def _fit_swapped(y, ncp, deg, knots):  # contracts the axes with each other's matrices
    y = np.asarray(y, np.float64)
    P = y
    for a in range(3):
        b = 2 - a
        B = ad.collocation(ncp[b], deg[b], knots[b], y.shape[a])
        Pa = np.moveaxis(P, a, 0)
        X = np.linalg.lstsq(B, Pa.reshape(Pa.shape[0], -1), rcond=None)[0]
        P = np.moveaxis(X.reshape((ncp[b],) + Pa.shape[1:]), 0, a)
    return P


def _fit_transpose(y, ncp, deg, knots):  # B^T instead of the pseudo-inverse
    y = np.asarray(y, np.float64)
    P = y
    for a in range(3):
        B = ad.collocation(ncp[a], deg[a], knots[a], y.shape[a])
        Pa = np.moveaxis(P, a, 0)
        X = B.T @ Pa.reshape(Pa.shape[0], -1)
        P = np.moveaxis(X.reshape((ncp[a],) + Pa.shape[1:]), 0, a)
    return P


def _errors_no_sqrt(y, P, ncp, deg, knots):
    m, r = _orig["model_errors"](y, P, ncp, deg, knots)
    return m, r * r


def _select_largest(errs, ncp_lo, e, metric=ad.METRIC_RMS):
    err = np.asarray(errs)[:, metric]
    below = np.nonzero(err < e)[0]
    nstar = ncp_lo + (int(below[-1]) if below.size else err.shape[0] - 1)
    return nstar, bool((err > e).any())


def _select_ge(errs, ncp_lo, e, metric=ad.METRIC_RMS):
    nstar, _ = _orig["select_ncp"](errs, ncp_lo, e, metric)
    return nstar, bool((np.asarray(errs)[:, metric] >= e).any())


def _cross_inverted(levels, p, e, metric=ad.METRIC_RMS, ncp_lo=None, ncp_hi=None):
    out = _orig["cross_level"](levels[:1], p, e, metric, ncp_lo, ncp_hi)
    R = levels[0].shape[1]
    lo = p + 2 if ncp_lo is None else ncp_lo
    hi = R if ncp_hi is None else ncp_hi
    prev = out[0][1]
    for k, Y in enumerate(levels[1:], start=1):
        m = 1 << k
        nb = Y.shape[0]
        nstar = np.full(nb, p + 1, np.int32)
        cplx = np.zeros(nb, bool)
        searched = np.zeros(nb, bool)
        for b in range(nb):
            bx, by, bz = b // (m * m), (b // m) % m, b % m
            parent = ((bx // 2) * (m // 2) + by // 2) * (m // 2) + bz // 2
            if prev[parent]:  # mistake: searches the children of simple blocks
                continue
            searched[b] = True
            nstar[b], cplx[b] = ad.select_ncp(ad.error_map(Y[b], p, lo, hi), lo, e, metric)
        out.append((nstar, cplx, searched, {}))
        prev = cplx
    return out


MUTANTS = {
    "cell_centred_grid": ("grid_params", _cell_grid),
    "perturbed_knot": ("uniform_knots", _knots_off),
    "swapped_axes_fit": ("fit_block", _fit_swapped),
    "transpose_not_pinv": ("fit_block", _fit_transpose),
    "rms_without_sqrt": ("model_errors", _errors_no_sqrt),
    "largest_ncp_below_bound": ("select_ncp", _select_largest),
    "complex_on_equality": ("select_ncp", _select_ge),
    "children_of_simple_blocks": ("cross_level", _cross_inverted),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(monkeypatch, name):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(ad, attr, fn)
    failures = 0
    for pin in PINS:
        try:
            pin()
        except Exception:  # an assertion or a shape error: the pin fails
            failures += 1
    assert failures > 0, f"no pin catches {name}"
