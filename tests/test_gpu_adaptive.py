"""Adaptive encoding on the GPU (Sec. 4.2: least-squares fit, error map,
NCP* of Eq. 4, cross-level search of Alg. 1) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import fa_inputs as fi
import oracle
from gpu_util import say
from oracle import adaptive as ad

pytestmark = pytest.mark.gpu

# Tolerance of the fit (a first-order error estimate, derived step by step
# in the design doc's conditioning paragraph).  Per axis a the GPU solves
# G_a X_a = B_a^T in FP64 (G_a = B_a^T B_a formed in FP64, band Cholesky of
# half-bandwidth p, two band triangular solves) and applies the three X_a to
# the samples as FP64 contractions of length R_a; the lattice is rounded to
# FP32 once.  The solve is backward stable with a perturbation of G_a of
# relative size
#   eps_a = gamma(R_a)                  Gram sums (B >= 0: no cancellation)
#         + (2p+1) gamma(3(p+1)+1)      band Cholesky and solves; the
#                                       factor bounds || |R^T||R| || / ||G||
#         + 4 gamma(5p)                 FP64 basis of the GPU and of the
#                                       oracle (5 roundings per recursion
#                                       level, non-negative terms)
# which moves the solution by kappa(G_a) eps_a = kappa(B_a)^2 eps_a
# relative to max |P|; the oracle's library solve moves it by at most as
# much (factor 2), and the three contractions add gamma(R_x + R_y + R_z):
#   |P_gpu - P| <= u32 |P| + (2 sum_a kappa(B_a)^2 eps_a + gamma(3R)) max|P|.
# The error map entries move by at most the decoded model's change,
# |f_gpu - f|_inf <= |P_gpu - P|_inf (rows of B are convex weights), plus the
# FP32 decode's own rounding (64 u32 max |P|): c32 = 80 covers both FP32
# terms there.  kappa(B_a) grows quickly as NCP approaches R (about 4e4 at
# NCP = R = 64 for cubics), and with it the error any FP32 model can have.
U32 = 2.0 ** -24
U64 = 2.0 ** -53


def gamma(k):
    return k * U64 / (1.0 - k * U64)


def kappas2(ncp, deg, R):
    """kappa(B_a)^2 of the oracle's FP64 collocation matrices, per axis."""
    out = []
    for a in range(3):
        B = ad.collocation(ncp[a], deg[a], ad.uniform_knots(ncp[a], deg[a]), R[a])
        sv = np.linalg.svd(B, compute_uv=False)
        out.append((sv[0] / sv[-1]) ** 2)
    return out


def svals(ncp, deg, R):
    """Product of the axes' smallest singular values."""
    lo = 1.0
    for a in range(3):
        B = ad.collocation(ncp[a], deg[a], ad.uniform_knots(ncp[a], deg[a]), R[a])
        lo *= np.linalg.svd(B, compute_uv=False)[-1]
    return lo


def fit_rel(ncp, deg, R):
    """Multiplier of max |P| in the fit's error estimate (FP64 part)."""
    k2 = kappas2(ncp, deg, R)
    eps = [gamma(R[a]) + (2 * deg[a] + 1) * gamma(3 * (deg[a] + 1) + 1) + 4 * gamma(5 * deg[a])
           for a in range(3)]
    return 2.0 * sum(k * e for k, e in zip(k2, eps)) + gamma(sum(R))


def tol_from(P, ncp, deg, R, c32=80.0):
    return (c32 * U32 + fit_rel(ncp, deg, R)) * np.abs(P).max()


@pytest.fixture(scope="module")
def fa():
    import paper_2409_00184_amd as fa
    assert torch.cuda.is_available()
    return fa


def _smooth_blocks(seed, nb, R, noise=0.0):
    """Sum-of-sinusoid samples on each block's grid, FP32, per-block offset."""
    g = fi.rng(seed)
    k, phi = fi.sinusoid_params(g, nterms=6, kmax=2.0)
    u = ad.grid_params(R)
    Y = np.empty((nb, R, R, R), np.float32)
    for b in range(nb):
        o = g.uniform(0, 4, 3)
        Y[b] = fi.sinusoid_field(k, phi, o[0] + u[:, None, None], o[1] + u[None, :, None],
                                 o[2] + u[None, None, :])
        if noise:
            Y[b] += noise * g.normal(size=(R, R, R)).astype(np.float32)
    return Y


def _oracle_fit(m, Y):
    desc = m.host_desc
    kn = m.knots.cpu().numpy().astype(np.float64)
    out = []
    for b in range(len(desc)):
        n = tuple(int(v) for v in desc["ncp"][b])
        p = tuple(int(v) for v in desc["degree"][b])
        o = int(desc["knot_off"][b])
        ks = [kn[o:o + n[0] + p[0] + 1], kn[o + n[0] + p[0] + 1:o + n[0] + n[1] + p[0] + p[1] + 2],
              kn[o + n[0] + n[1] + p[0] + p[1] + 2:o + sum(n) + sum(p) + 3]]
        out.append((n, p, ks, ad.fit_block(Y[b].astype(np.float64), n, p, ks)))
    return out


def test_fit_matches_oracle_uneven_batch(fa):
    """Blocks of uneven NCP per axis and degree 1..3, non-cubic grid."""
    say("fit uneven")
    g = fi.rng(60)
    R = (24, 20, 28)
    nb = 9
    ncp = np.stack([g.integers(2 + 2, 20, nb), g.integers(4, 20, nb), g.integers(4, 28, nb)], 1)
    deg = g.integers(1, 4, nb)
    ncp = np.maximum(ncp, deg[:, None] + 1)
    m = fa.uniform_models(ncp, deg)
    Y = np.stack([_smooth_blocks(61 + b, 1, 28)[0][:R[0], :R[1], :R[2]] for b in range(nb)])
    Y = np.ascontiguousarray(Y + 0.05 * g.normal(size=Y.shape).astype(np.float32))
    fa.fit(m, R, torch.as_tensor(Y).cuda())
    got = m.ctrl.cpu().numpy().astype(np.float64)
    for b, (n, p, ks, P) in enumerate(_oracle_fit(m, Y)):
        o = int(m.host_desc["ctrl_off"][b])
        Pg = got[o:o + int(np.prod(n))].reshape(n)
        err = np.abs(Pg - P)
        tol = U32 * np.abs(P) + tol_from(P, n, p, R, c32=0.0)
        say("  block", b, n, p, "err / tol", (err / tol).max())
        assert np.all(err <= tol)


def test_fit_recovers_spline(fa):
    """y = decode of a random lattice (rounded to FP32): the GPU fit returns
    the lattice to FP32 accuracy and the model errors are at rounding level."""
    say("fit recovers")
    g = fi.rng(62)
    R, nb = 32, 4
    ncp = np.array([[12, 9, 17], [5, 5, 5], [32, 20, 8], [7, 30, 16]])
    m = fa.uniform_models(ncp, [3, 2, 3, 3])
    P = g.normal(size=m.ctrl.numel())
    kn = m.knots.cpu().numpy().astype(np.float64)
    ob = oracle.Blocks(m.host_desc["ncp"], m.host_desc["degree"], m.host_desc["knot_off"],
                       m.host_desc["ctrl_off"], kn, P)
    Y = oracle.decode_blocks(ob, (R, R, R), mask=1)[:, 0].astype(np.float32)
    fa.fit(m, (R, R, R), torch.as_tensor(Y).cuda())
    got = m.ctrl.cpu().numpy()
    degs = [3, 2, 3, 3]
    errs = fa.model_errors(m, (R, R, R), torch.as_tensor(Y).cuda()).cpu().numpy()
    for b in range(nb):
        o, n = int(m.host_desc["ctrl_off"][b]), int(np.prod(ncp[b]))
        dg, RR = (degs[b],) * 3, (R,) * 3
        # y is the FP32 rounding of the exact decode of P, so P is the exact
        # fit of data within u32 |y|_2 of y: |P - fit(y)|_2 <= u32 |y|_2 / s_min
        lo = svals(ncp[b], dg, RR)
        tol = U32 * np.linalg.norm(Y[b]) / lo + tol_from(P[o:o + n], ncp[b], dg, RR, c32=1.0)
        d = np.abs(got[o:o + n] - P[o:o + n]).max()
        say("  block", b, ncp[b], "err", d, "tol", tol)
        assert d <= tol
        assert errs[b, 0] <= tol + tol_from(P[o:o + n], ncp[b], dg, RR)


def test_ncp_search_matches_oracle_error_map(fa):
    """Every (block, NCP) error of the in-level search against the oracle's
    error map; NCP* and the complex flag valid for the oracle's errors."""
    say("ncp search")
    R, p, nb = 16, 3, 5
    Y = _smooth_blocks(63, nb, R, noise=1e-3)
    errs = fa.ncp_search(torch.as_tensor(Y).cuda(), p).cpu().numpy()
    lo = p + 2
    assert errs.shape == (nb, R - lo + 1, 2)
    tols = np.zeros((nb, R - lo + 1, 2))
    for b in range(nb):
        for n in range(lo, R + 1):
            kn = [ad.uniform_knots(n, p)] * 3
            P = ad.fit_block(Y[b].astype(np.float64), (n,) * 3, (p,) * 3, kn)
            tols[b, n - lo] = tol_from(P, (n,) * 3, (p,) * 3, (R,) * 3)
    for b in range(nb):
        ref = ad.error_map(Y[b].astype(np.float64), p, lo, R)
        d = np.abs(errs[b] - ref)
        say("  block", b, "max |err_gpu - err_oracle| / tol", (d / tols[b]).max(0))
        assert np.all(d <= tols[b])
    bound = 0.02
    nstar, cplx = fa.ncp_select(errs, lo, bound)
    for b in range(nb):
        tol = tols[b, :, 1]
        ref = ad.error_map(Y[b].astype(np.float64), p, lo, R)[:, 1]
        k = nstar[b] - lo
        # valid choice: below the bound (within tol), every smaller NCP not clearly below
        assert ref[k] < bound + tol[k] or k == ref.shape[0] - 1
        assert np.all(ref[:k] >= bound - tol[:k])
        want_c = bool((ref > bound).any())
        assert cplx[b] == want_c or np.any(np.abs(ref - bound) <= tol)


def test_ncp_search_full_size_sampled(fa):
    """64^3 micro-blocks (the paper's micro-block size), candidates 5..64:
    sampled NCPs against the oracle fit."""
    say("ncp search 64^3")
    R, p, nb = 64, 3, 2
    Y = _smooth_blocks(64, nb, R, noise=1e-2)
    errs = fa.ncp_search(torch.as_tensor(Y).cuda(), p).cpu().numpy()
    assert errs.shape == (nb, R - p - 1, 2)
    for n in (5, 18, 41, 56, 64):
        kn = [ad.uniform_knots(n, p)] * 3
        for b in range(nb):
            P = ad.fit_block(Y[b].astype(np.float64), (n, n, n), (p, p, p), kn)
            tol = tol_from(P, (n,) * 3, (p,) * 3, (R,) * 3)
            ref = ad.model_errors(Y[b].astype(np.float64), P, (n, n, n), (p, p, p), kn)
            d = np.abs(errs[b, n - p - 2] - ref)
            say("  n", n, "block", b, errs[b, n - p - 2], ref, "d / tol", d / tol)
            assert np.all(d <= tol)


def test_adaptive_encode_cross_level(fa):
    """Alg. 1 over a 3-level pyramid of a field with one sharp feature:
    the same blocks are searched and complex as in the oracle, NCP* agree
    (the bound is chosen away from every error, checked), and the encoded
    models meet the bound."""
    say("adaptive cross-level")
    R, p = 12, 2
    c = np.array([0.3, 0.35, 0.7])

    def field(x, y, z):
        return np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2 * 0.05 ** 2))

    levels = []
    u = ad.grid_params(R)
    for k in range(3):
        m = 1 << k
        Y = np.empty((m ** 3, R, R, R), np.float32)
        for b in range(m ** 3):
            bx, by, bz = b // (m * m), (b // m) % m, b % m
            Y[b] = field(((bx + u) / m)[:, None, None], ((by + u) / m)[None, :, None],
                         ((bz + u) / m)[None, None, :])
        levels.append(Y)
    bound = 2e-3
    ref = ad.cross_level([L.astype(np.float64) for L in levels], p, bound)
    for k, lvl in enumerate(ref):
        for b, e in lvl[3].items():
            tol = np.array([tol_from(ad.fit_block(levels[k][b].astype(np.float64), (n,) * 3,
                                                  (p,) * 3, [ad.uniform_knots(n, p)] * 3),
                                     (n,) * 3, (p,) * 3, (R,) * 3)
                            for n in range(p + 2, R + 1)])
            assert np.all(np.abs(e[:, 1] - bound) > tol)  # no ambiguous decision
    got = fa.adaptive_encode([torch.as_tensor(L).cuda() for L in levels], p, bound)
    for k in range(3):
        say("  level", k, "searched", got[k]["searched"].sum(), "complex", got[k]["complex"].sum(),
            "ncp*", np.bincount(got[k]["ncp_star"]).nonzero()[0])
        assert np.array_equal(got[k]["searched"], ref[k][2])
        assert np.array_equal(got[k]["complex"], ref[k][1])
        assert np.array_equal(got[k]["ncp_star"], ref[k][0])
        errs = fa.model_errors(got[k]["models"], (R, R, R), torch.as_tensor(levels[k]).cuda())
        rms = errs[:, 1].cpu().numpy()
        s = got[k]["searched"]
        assert np.all(rms[s] < bound + 1e-5)
