"""FP64 oracle of the adaptive encoding -- TEST INFRASTRUCTURE.

Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
import this module; the product path never does.

What it computes (Sec. 4.2.1, Eq. 4; Sec. 4.2.2, Alg. 1):
  model(NCP, degree): the least-squares fit of a tensor-product clamped
    B-spline with NCP control points per axis (clamped uniform knots) to the
    R^3 samples of a micro-block on its grid u_i = fl32(i / (R - 1)).  The
    design matrix is the Kronecker product B_x (x) B_y (x) B_z of the
    per-axis collocation matrices B_a[i, j] = N_j(u_i), so the minimiser is
    P = y x_1 pinv(B_x) x_2 pinv(B_y) x_3 pinv(B_z) (the pseudo-inverse of a
    Kronecker product is the product of the pseudo-inverses).  pinv is the
    library least-squares solve, in FP64.
  Error(NCP): of the fitted model decoded back on the grid: the maximum
    absolute residual and the root-mean-square residual over the R^3
    samples.
  In-level selection (Eq. 4): NCP* = the smallest NCP whose error is below
    the bound e; a block is complex when some candidate's error exceeds e.
    No candidate below e: NCP* = the largest candidate.
  Cross-level (Alg. 1): the coarsest level is searched in full; a block of
    a finer level is searched only if its parent (the coarser block holding
    it) is complex, otherwise NCP* = degree + 1.
"""
import numpy as np

from . import Blocks, axis_basis, decode_blocks

METRIC_MAX, METRIC_RMS = 0, 1


def grid_params(R):
    """The decode grid of one axis: fl32(i / (R - 1)), i = 0..R-1."""
    return (np.arange(R, dtype=np.float32) / np.float32(R - 1)).astype(np.float64)


def uniform_knots(n, p):
    """Clamped uniform knots t_{p+j} = fl32(j / (n - p)) as FP64 values."""
    t = np.zeros(n + p + 1)
    t[n:] = 1.0
    for j in range(1, n - p):
        t[p + j] = float(np.float32(j) / np.float32(n - p))
    return t


def collocation(n, p, t, R):
    """B[i, j] = N_{j,p}(u_i) on the decode grid (R x n, FP64)."""
    s, N, _ = axis_basis(n, p, t, grid_params(R))
    B = np.zeros((R, n))
    for i in range(R):
        B[i, s[i] - p:s[i] + 1] = N[i]
    return B


def fit_block(y, ncp, deg, knots):
    """Kronecker least squares of one block: y [Rx, Ry, Rz] -> P [nx, ny, nz]."""
    y = np.asarray(y, np.float64)
    P = y
    for a in range(3):
        B = collocation(ncp[a], deg[a], knots[a], y.shape[a])
        # contract axis a of P with pinv(B) (n x R): solve B X = (axis-a fibres)
        Pa = np.moveaxis(P, a, 0)
        X = np.linalg.lstsq(B, Pa.reshape(Pa.shape[0], -1), rcond=None)[0]
        P = np.moveaxis(X.reshape((ncp[a],) + Pa.shape[1:]), 0, a)
    return P


def model_errors(y, P, ncp, deg, knots):
    """(max |y - f|, rms(y - f)) of the model P decoded on y's grid."""
    y = np.asarray(y, np.float64)
    kn = np.concatenate([np.asarray(k, np.float64) for k in knots])
    b = Blocks(np.array([ncp]), np.array([deg]), np.zeros(1), np.zeros(1), kn,
               np.asarray(P, np.float64).reshape(-1))
    f = decode_blocks(b, y.shape, mask=1)[0, 0]
    r = y - f
    return float(np.abs(r).max()), float(np.sqrt(np.mean(r * r)))


def error_map(y, p, ncp_lo, ncp_hi):
    """errs[n - ncp_lo] = (max, rms) of model(n, p) for n = ncp_lo..ncp_hi,
    the same n on every axis (Alg. 1 searches one NCP per block)."""
    out = np.zeros((ncp_hi - ncp_lo + 1, 2))
    for n in range(ncp_hi, ncp_lo - 1, -1):  # from the largest NCP down (Sec. 4.2.1)
        kn = [uniform_knots(n, p)] * 3
        P = fit_block(y, (n, n, n), (p, p, p), kn)
        out[n - ncp_lo] = model_errors(y, P, (n, n, n), (p, p, p), kn)
    return out


def select_ncp(errs, ncp_lo, e, metric=METRIC_RMS):
    """Eq. 4 over one block's error map: (NCP*, complex)."""
    err = np.asarray(errs)[:, metric]
    below = np.nonzero(err < e)[0]
    nstar = ncp_lo + (int(below[0]) if below.size else err.shape[0] - 1)
    return nstar, bool((err > e).any())


def cross_level(levels, p, e, metric=METRIC_RMS, ncp_lo=None, ncp_hi=None):
    """Alg. 1 over a pyramid.  levels[k]: samples [(2^k)^3, R, R, R] of
    level k (block (bx, by, bz) at index (bx * 2^k + by) * 2^k + bz), k = 0
    the coarsest.  Returns per level (ncp_star [nb], complex [nb], searched
    [nb]) and the error maps of the searched blocks."""
    R = levels[0].shape[1]
    lo = p + 2 if ncp_lo is None else ncp_lo
    hi = R if ncp_hi is None else ncp_hi
    out = []
    prev_complex = None
    for k, Y in enumerate(levels):
        m = 1 << k
        nb = Y.shape[0]
        nstar = np.full(nb, p + 1, np.int32)
        cplx = np.zeros(nb, bool)
        searched = np.zeros(nb, bool)
        maps = {}
        for b in range(nb):
            if k > 0:
                bx, by, bz = b // (m * m), (b // m) % m, b % m
                parent = ((bx // 2) * (m // 2) + by // 2) * (m // 2) + bz // 2
                if not prev_complex[parent]:
                    continue
            searched[b] = True
            maps[b] = error_map(Y[b], p, lo, hi)
            nstar[b], cplx[b] = select_ncp(maps[b], lo, e, metric)
        out.append((nstar, cplx, searched, maps))
        prev_complex = cplx
    return out
