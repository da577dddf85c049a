"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each pin is a plain function that raises AssertionError on failure, so the
same checks run against the oracle (tests/test_oracle_pins.py) and against
copies of it with planted mistakes (tests/test_oracle_mutants.py).

What pins what (B-spline facts, de Boor's recursion -- the spline basis the
paper cites in Sec. 1 -- and the micro-model content of Sec. 4.2 / Eq. 2):
  span        invariant t_s <= u < t_{s+1} with a non-empty span
  unity       sum_i N_{i,p} = 1, N >= 0, sum_i N'_{i,p} = 0
  bernstein   n = p+1 gives Bernstein polynomials and their derivatives
  cardinal    uniform cubic at interior knots: 1/6, 4/6, 1/6, 0 and
              derivatives -(n-p)/2, 0, (n-p)/2, 0; golden fixture values
  linear      Greville control points reproduce a + bu + cv + dw exactly
  quadratic   Marsden's identity reproduces u^2 (and tensor products)
  corners     clamped knots interpolate the corner control points, and the
              end derivative is p/(t_{p+1}) (P_1 - P_0)
  fd          central differences of the value match the gradient
  one_sided   at a knot of multiplicity p the derivative is the one from
              the right; at a double knot of a cubic both sides agree
  brute       local evaluation equals the all-basis brute force
  adjoint     <B P, g> = <P, B^T g>
  query       block lookup + chain rule on a tiled domain of linear blocks
  render      compositing, termination and shading closed forms
"""
import math
import os

import numpy as np

import fa_inputs as fi
import oracle
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def random_clamped_knots(g, n, p, repeat=False):
    """Clamped knots on [0,1] with random (optionally repeated) interior."""
    m = n - p - 1
    inner = np.sort(g.uniform(0.02, 0.98, size=m))
    if repeat and m >= 2 and p >= 2:
        inner[1] = inner[0]  # a double knot (continuity drops to C^{p-2})
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)]).astype(np.float32).astype(np.float64)


def single(ncp, deg, knots, P):
    t = np.concatenate(knots)
    return oracle.Blocks(np.array([ncp]), np.array([deg]), np.array([0]), np.array([0]), t,
                         np.asarray(P, np.float64).reshape(-1))


# ------------------------------------------------------------------- pins

def pin_span():
    g = fi.rng(101)
    for p in (1, 2, 3):
        for n in (p + 1, p + 2, 7, 12):
            for rep in (False, True):
                t = random_clamped_knots(g, n, p, rep)
                us = np.concatenate([g.uniform(0, 1, 200), t, [0.0, 1.0]])
                for u in us:
                    s = oracle.find_span(n, p, t, u)
                    assert p <= s <= n - 1, (n, p, u, s)
                    assert t[s] < t[s + 1], "span must be non-empty"
                    if u >= 1.0:
                        assert s == n - 1
                    else:
                        assert t[s] <= u < t[s + 1], (t, u, s)


def pin_unity():
    g = fi.rng(102)
    for p in (1, 2, 3):
        for n in (p + 1, p + 3, 10):
            t = random_clamped_knots(g, n, p, repeat=True)
            u = np.concatenate([g.uniform(0, 1, 300), t])
            s, N, dN = oracle.axis_basis(n, p, t, u)
            assert np.all(N >= -1e-15)
            assert np.allclose(N.sum(1), 1.0, atol=1e-13, rtol=0)
            scale = np.abs(dN).sum(1).max() + 1
            assert np.allclose(dN.sum(1), 0.0, atol=1e-12 * scale, rtol=0)


def pin_bernstein():
    g = fi.rng(103)
    for p in (1, 2, 3):
        n = p + 1
        t = np.concatenate([np.zeros(p + 1), np.ones(p + 1)])
        u = np.concatenate([g.uniform(0, 1, 50), [0.0, 0.5, 1.0]])
        s, N, dN = oracle.axis_basis(n, p, t, u)
        for q, x in enumerate(u):
            assert s[q] == p
            for i in range(p + 1):
                b = math.comb(p, i) * x ** i * (1 - x) ** (p - i)
                # d/dx C(p,i) x^i (1-x)^(p-i) = p (B_{i-1,p-1} - B_{i,p-1})
                lo = math.comb(p - 1, i - 1) * x ** (i - 1) * (1 - x) ** (p - i) if i >= 1 else 0.0
                hi = math.comb(p - 1, i) * x ** i * (1 - x) ** (p - 1 - i) if i <= p - 1 else 0.0
                db = p * (lo - hi)
                assert abs(N[q, i] - b) < 1e-14, (p, i, x)
                assert abs(dN[q, i] - db) < 1e-13, (p, i, x, dN[q, i], db)


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


def _frac(s):
    if "/" in s:
        a, b = s.split("/")
        return float(a) / float(b)
    return float(s)


def pin_cardinal():
    # uniform cubic at interior knots away from the clamped ends
    for n in (10, 16, 32):
        p = 3
        t = fi.clamped_uniform_knots(n, p).astype(np.float64)
        h = n - p
        for s_k in range(p + 3, n - 3 + 1):
            u = t[s_k]
            s, N, dN = oracle.axis_basis(n, p, t, [u])
            assert s[0] == s_k
            assert np.allclose(N[0], [1 / 6, 4 / 6, 1 / 6, 0.0], atol=1e-6)
            assert np.allclose(dN[0], [-h / 2, 0.0, h / 2, 0.0], atol=1e-5 * h)
    # golden closed-form values (tests/golden/bspline_closed_forms.txt)
    for row in _golden_rows("bspline_closed_forms.txt"):
        kind, p, n, span, frac_in_span = row[0], int(row[1]), int(row[2]), int(row[3]), _frac(row[4])
        vals = [_frac(v) for v in row[5:5 + p + 1]]
        ders = [_frac(v) for v in row[5 + p + 1:5 + 2 * (p + 1)]]
        t = np.zeros(n + p + 1)
        for j in range(n + p + 1):  # exact uniform clamped knots in FP64
            t[j] = min(max(j - p, 0), n - p) / (n - p)
        u = t[span] + frac_in_span * (t[span + 1] - t[span])
        s, N, dN = oracle.axis_basis(n, p, t, [u])
        assert s[0] == span, (kind, s[0], span)
        assert np.allclose(N[0], vals, atol=1e-14), (kind, N[0], vals)
        assert np.allclose(dN[0], np.array(ders) * (n - p), atol=1e-12), (kind, dN[0])


def _greville(t, n, p):
    return np.array([np.mean(t[i + 1:i + p + 1]) for i in range(n)])


def _marsden2(t, n, p):
    """Control coefficients reproducing u^2 (p >= 2): the degree-2
    elementary symmetric function of t_{i+1..i+p}, divided by C(p, 2)."""
    c = np.zeros(n)
    for i in range(n):
        kn = t[i + 1:i + p + 1]
        acc = 0.0
        for a in range(p):
            for b in range(a + 1, p):
                acc += kn[a] * kn[b]
        c[i] = acc / math.comb(p, 2)
    return c


def pin_linear():
    g = fi.rng(104)
    for trial in range(12):
        deg = [int(v) for v in g.integers(1, 4, size=3)]
        ncp = [int(deg[a] + 1 + g.integers(0, 9)) for a in range(3)]
        kn = [random_clamped_knots(g, ncp[a], deg[a], repeat=bool(trial % 2)) for a in range(3)]
        xi = [_greville(kn[a], ncp[a], deg[a]) for a in range(3)]
        a0, bx, by, bz = g.normal(size=4)
        P = a0 + bx * xi[0][:, None, None] + by * xi[1][None, :, None] + bz * xi[2][None, None, :]
        blk = single(ncp, deg, kn, P)
        uvw = np.concatenate([g.uniform(0, 1, (300, 3)), [[0, 0, 0], [1, 1, 1], [1, 0, 0.5]]])
        out = oracle.eval_params(blk, np.zeros(len(uvw), np.int32), uvw)
        want = a0 + bx * uvw[:, 0] + by * uvw[:, 1] + bz * uvw[:, 2]
        assert np.allclose(out[:, 0], want, atol=1e-12)
        assert np.allclose(out[:, 1], bx, atol=1e-10)
        assert np.allclose(out[:, 2], by, atol=1e-10)
        assert np.allclose(out[:, 3], bz, atol=1e-10)


def pin_quadratic():
    g = fi.rng(105)
    for trial in range(8):
        deg = [int(v) for v in g.integers(2, 4, size=3)]
        ncp = [int(deg[a] + 1 + g.integers(0, 8)) for a in range(3)]
        kn = [random_clamped_knots(g, ncp[a], deg[a]) for a in range(3)]
        xi = [_greville(kn[a], ncp[a], deg[a]) for a in range(3)]
        m2 = [_marsden2(kn[a], ncp[a], deg[a]) for a in range(3)]
        # f = u^2 + 2 v^2 - w^2 + u v w
        P = (m2[0][:, None, None] + 2 * m2[1][None, :, None] - m2[2][None, None, :]
             + xi[0][:, None, None] * xi[1][None, :, None] * xi[2][None, None, :])
        blk = single(ncp, deg, kn, P)
        uvw = g.uniform(0, 1, (300, 3))
        u, v, w = uvw.T
        out = oracle.eval_params(blk, np.zeros(len(uvw), np.int32), uvw)
        assert np.allclose(out[:, 0], u * u + 2 * v * v - w * w + u * v * w, atol=1e-12)
        assert np.allclose(out[:, 1], 2 * u + v * w, atol=1e-10)
        assert np.allclose(out[:, 2], 4 * v + u * w, atol=1e-10)
        assert np.allclose(out[:, 3], -2 * w + u * v, atol=1e-10)


def pin_corners():
    g = fi.rng(106)
    for trial in range(10):
        deg = [int(v) for v in g.integers(1, 4, size=3)]
        ncp = [int(deg[a] + 1 + g.integers(0, 7)) for a in range(3)]
        kn = [random_clamped_knots(g, ncp[a], deg[a]) for a in range(3)]
        P = g.normal(size=ncp)
        blk = single(ncp, deg, kn, P)
        for cx in (0, 1):
            for cy in (0, 1):
                for cz in (0, 1):
                    out = oracle.eval_params(blk, [0], [[cx, cy, cz]])[0]
                    i = cx * (ncp[0] - 1)
                    j = cy * (ncp[1] - 1)
                    k = cz * (ncp[2] - 1)
                    assert abs(out[0] - P[i, j, k]) < 1e-12
        # end derivatives along x at the (0, 0, 0) and (1, 0, 0) corners
        p, tx = deg[0], kn[0]
        out0 = oracle.eval_params(blk, [0], [[0, 0, 0]])[0]
        assert abs(out0[1] - p / tx[p + 1] * (P[1, 0, 0] - P[0, 0, 0])) < 1e-9
        n = ncp[0]
        out1 = oracle.eval_params(blk, [0], [[1, 0, 0]])[0]
        want = p / (1.0 - tx[n - 1]) * (P[n - 1, 0, 0] - P[n - 2, 0, 0])
        assert abs(out1[1] - want) < 1e-9 * max(1.0, abs(want))


def pin_fd():
    g = fi.rng(107)
    h = 1e-5
    for trial in range(6):
        deg = [int(v) for v in g.integers(2, 4, size=3)]
        ncp = [int(deg[a] + 1 + g.integers(0, 10)) for a in range(3)]
        kn = [fi.clamped_uniform_knots(ncp[a], deg[a]).astype(np.float64) for a in range(3)]
        P = g.normal(size=ncp)
        blk = single(ncp, deg, kn, P)
        uvw = g.uniform(0.05, 0.95, (100, 3))
        out = oracle.eval_params(blk, np.zeros(100, np.int32), uvw)
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            fp = oracle.eval_params(blk, np.zeros(100, np.int32), uvw + e)[:, 0]
            fm = oracle.eval_params(blk, np.zeros(100, np.int32), uvw - e)[:, 0]
            fd = (fp - fm) / (2 * h)
            scale = np.abs(out[:, 1 + a]).max() + 1.0
            assert np.abs(fd - out[:, 1 + a]).max() < 1e-5 * scale, (a, np.abs(fd - out[:, 1 + a]).max())


def pin_one_sided():
    """At an interior knot of multiplicity m the spline is C^{p-m}.  At a
    knot of multiplicity p the derivative jumps, and the right-continuous
    span rule makes the value at the knot the derivative from the right: it
    equals a second-order one-sided difference from the right and not the
    one from the left.  At a double knot of a cubic (C^1) both one-sided
    differences give it."""
    g = fi.rng(113)
    h = 1e-5

    def right(f, t):
        return (-3 * f(t) + 4 * f(t + h) - f(t + 2 * h)) / (2 * h)

    def left(f, t):
        return (3 * f(t) - 4 * f(t - h) + f(t - 2 * h)) / (2 * h)

    for p, mult, jumps in ((2, 2, True), (3, 3, True), (3, 2, False), (1, 1, True)):
        n = p + 1 + mult + 2
        k = 0.375  # exact in FP32 and FP64
        inner = np.sort(np.concatenate([[0.125], [k] * mult, [0.8125]]))
        assert len(inner) == n - p - 1
        t = np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])
        P = g.normal(size=(n, 2, 2))
        blk = single([n, 2, 2], [p, 1, 1], [t, [0, 0, 1, 1], [0, 0, 1, 1]], P)

        def f(u):
            return oracle.eval_params(blk, [0], [[u, 0.3, 0.6]])[0, 0]

        d = oracle.eval_params(blk, [0], [[k, 0.3, 0.6]])[0, 1]
        dr, dl = right(f, k), left(f, k)
        scale = 1.0 + abs(dr) + abs(dl)
        assert abs(d - dr) < 1e-6 * scale, (p, mult, d, dr)
        if jumps:
            assert abs(dl - dr) > 1e-3 * scale, (p, mult, dl, dr)
        else:
            assert abs(d - dl) < 1e-6 * scale, (p, mult, d, dl)


def pin_brute():
    g = fi.rng(108)
    for trial in range(12):
        deg = [int(v) for v in g.integers(1, 4, size=3)]
        ncp = [int(deg[a] + 1 + g.integers(0, 4)) for a in range(3)]
        kn = [random_clamped_knots(g, ncp[a], deg[a], repeat=bool(trial % 3 == 0)) for a in range(3)]
        P = g.normal(size=ncp)
        blk = single(ncp, deg, kn, P)
        pts = np.concatenate([g.uniform(0, 1, (20, 3)),
                              [[0, 0, 0], [1, 1, 1], [kn[0][deg[0] + 1], 1, 0]]])
        out = oracle.eval_params(blk, np.zeros(len(pts), np.int32), pts)
        Pl = P.tolist()
        for q, (u, v, w) in enumerate(pts):
            want = brute.eval_block(ncp, deg, list(kn[0]), list(kn[1]), list(kn[2]), Pl, u, v, w)
            scale = 1.0 + max(abs(x) for x in want)
            assert np.allclose(out[q], want, atol=1e-12 * scale, rtol=0), (q, out[q], want)


def pin_decode_layout():
    """Grid decode, sampled decode and parameter evaluation agree; the grid
    position of voxel i is the FP32 value i/(R-1)."""
    g = fi.rng(109)
    ncp = [[5, 7, 6], [4, 4, 9]]
    deg = [[2, 3, 1], [3, 1, 2]]
    kl, lat = [], []
    for b in range(2):
        kl.append([random_clamped_knots(g, ncp[b][a], deg[b][a]) for a in range(3)])
        lat.append(g.normal(size=ncp[b]))
    bt = fi.pack(ncp, deg, kl, lat)
    blk = oracle.Blocks(bt.ncp, bt.deg, bt.knot_off, bt.ctrl_off, bt.knots, bt.ctrl)
    res = (5, 6, 7)
    full = oracle.decode_blocks(blk, res, 15)
    part = oracle.decode_blocks(blk, res, 0b1010)
    assert np.array_equal(part[:, 0], full[:, 1]) and np.array_equal(part[:, 1], full[:, 3])
    idx = np.array([[b, x, y, z] for b in range(2) for x in range(5) for y in range(6)
                    for z in range(7)], np.int32)
    smp = oracle.decode_samples(blk, res, idx)
    assert np.array_equal(smp.reshape(2, 5, 6, 7, 4).transpose(0, 4, 1, 2, 3), full)
    uvw = np.stack([np.float32(idx[:, 1]) / np.float32(res[0] - 1),
                    np.float32(idx[:, 2]) / np.float32(res[1] - 1),
                    np.float32(idx[:, 3]) / np.float32(res[2] - 1)], 1).astype(np.float64)
    ev = oracle.eval_params(blk, idx[:, 0], uvw)
    assert np.array_equal(ev, smp)


def pin_adjoint():
    g = fi.rng(110)
    ncp = [[5, 7, 6], [4, 4, 9], [6, 5, 4]]
    deg = [[2, 3, 1], [3, 1, 2], [3, 3, 3]]
    kl, lat = [], []
    for b in range(3):
        kl.append([random_clamped_knots(g, ncp[b][a], deg[b][a]) for a in range(3)])
        lat.append(g.normal(size=ncp[b]))
    bt = fi.pack(ncp, deg, kl, lat)
    blk = oracle.Blocks(bt.ncp, bt.deg, bt.knot_off, bt.ctrl_off, bt.knots, bt.ctrl)
    res = (9, 7, 8)
    valid = np.zeros_like(blk.ctrl, bool)
    for b in range(3):
        o = int(blk.ctrl_off[b])
        valid[o:o + int(np.prod(ncp[b]))] = True
    for mask in (1, 2, 4, 8, 15, 0b0110):
        BP = oracle.decode_blocks(blk, res, mask)
        gg = g.normal(size=BP.shape)
        G = oracle.decode_adjoint(blk, res, gg, mask)
        lhs = float((BP * gg).sum())
        rhs = float((blk.ctrl * G).sum())
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.abs(BP).sum()), (mask, lhs, rhs)
        assert np.all(G[~valid] == 0.0)


def pin_query():
    """Tiled domain, each block a different linear field in global
    coordinates: value and global gradient are known in closed form."""
    g = fi.rng(111)
    nb = (2, 3, 2)
    origin = np.array([-0.5, 0.25, 1.0], np.float32)
    extent = np.array([2.0, 3.0, 0.5], np.float32)
    ncells = int(np.prod(nb))
    ncp, deg, kl, lat, coef = [], [], [], [], []
    r = (np.array(nb, np.float32) / extent).astype(np.float64)
    for c in range(ncells):
        d = [int(v) for v in g.integers(1, 4, size=3)]
        n = [d[a] + 1 + int(g.integers(0, 5)) for a in range(3)]
        kn = [random_clamped_knots(g, n[a], d[a]) for a in range(3)]
        a0, b1, b2, b3 = g.normal(size=4)
        xi = [_greville(kn[a], n[a], d[a]) for a in range(3)]
        P = a0 + b1 * xi[0][:, None, None] + b2 * xi[1][None, :, None] + b3 * xi[2][None, None, :]
        ncp.append(n), deg.append(d), kl.append(kn), lat.append(P), coef.append((a0, b1, b2, b3))
    # cell -> block map is a permutation with one empty cell
    perm = g.permutation(ncells).astype(np.int32)
    boc = np.empty(ncells, np.int32)
    boc[perm] = np.arange(ncells, dtype=np.int32)
    empty_cell = int(perm[3])
    boc[empty_cell] = -1
    bt = fi.pack(ncp, deg, kl, lat)
    blk = oracle.Blocks(bt.ncp, bt.deg, bt.knot_off, bt.ctrl_off, bt.knots, bt.ctrl)
    xyz = (origin + g.uniform(-0.1, 1.1, (2000, 3)) * extent).astype(np.float32)
    out = oracle.query_points(blk, xyz, nb, origin, extent, boc)
    for q in range(len(xyz)):
        gq = ((xyz[q].astype(np.float32) - origin) * (np.array(nb, np.float32) / extent)).astype(np.float64)
        gq = np.clip(gq, 0, np.array(nb, np.float64))
        bidx = np.minimum(np.floor(gq).astype(int), np.array(nb) - 1)
        cell = (bidx[0] * nb[1] + bidx[1]) * nb[2] + bidx[2]
        if cell == empty_cell:
            assert np.all(out[q] == 0.0)
            continue
        a0, b1, b2, b3 = coef[boc[cell]]
        u = gq - bidx
        assert abs(out[q, 0] - (a0 + b1 * u[0] + b2 * u[1] + b3 * u[2])) < 1e-6
        assert np.allclose(out[q, 1:], np.array([b1, b2, b3]) * r, atol=1e-8)


def _one_block_linear(a0, bx, by, bz, n=6, p=3):
    t = fi.clamped_uniform_knots(n, p).astype(np.float64)
    xi = _greville(t, n, p)
    P = a0 + bx * xi[:, None, None] + by * xi[None, :, None] + bz * xi[None, None, :]
    bt = fi.pack([(n, n, n)], [(p, p, p)], [[t, t, t]], [P])
    return oracle.Blocks(bt.ncp, bt.deg, bt.knot_off, bt.ctrl_off, bt.knots, bt.ctrl)


def pin_render():
    """Closed forms of front-to-back compositing over one block:
    constant field -> A = 1 - (1 - a)^S and C = rgb * ka * A (gradient 0);
    early termination stops at the first S' with 1 - (1 - a)^S' > O_max;
    linear field of gradient g -> every sample shaded by
    ka + kd |n.L| + ks |n.H|^m with n = g/|g|."""
    nb, origin, extent = (1, 1, 1), (0, 0, 0), (1, 1, 1)
    boc = np.zeros(1, np.int32)
    rays = np.array([[0.1, 0.5, 0.5, 1, 0, 0, 0.0, 0.8],
                     [0.5, 0.2, 0.3, 0, 0.8, 0.6, 0.0, 0.5],
                     [0.5, 0.5, 0.5, 1, 0, 0, 0.4, 0.1]], np.float32)  # last one misses
    light = np.array([0.0, 0.6, 0.8], np.float32)
    alpha, rgb = float(np.float32(0.05)), (0.9, 0.5, 0.2)  # the TF holds FP32 values
    tf = np.array([[*rgb, alpha], [*rgb, alpha]], np.float32)
    # constant field (a linear field with zero slope)
    blk = _one_block_linear(0.3, 0.0, 0.0, 0.0)
    S = 37
    img = oracle.render(blk, rays, S, 2.0, -1.0, 1.0, tf, light, 0.4, 0.5, 0.3, 16.0, nb,
                        origin, extent, boc)
    A = 1 - (1 - alpha) ** S
    for q in range(2):
        assert abs(img[q, 3] - A) < 1e-12
        assert np.allclose(img[q, :3], np.array(rgb, np.float64).astype(np.float32) * 0.4 * A,
                           atol=1e-7)
    assert np.all(img[2] == 0.0)
    # early termination
    omax = 0.5
    img = oracle.render(blk, rays, S, omax, -1.0, 1.0, tf, light, 0.4, 0.5, 0.3, 16.0, nb,
                        origin, extent, boc)
    Sp = next(k for k in range(1, S + 1) if 1 - (1 - alpha) ** k > omax)
    assert abs(img[0, 3] - (1 - (1 - alpha) ** Sp)) < 1e-12
    # linear field: constant gradient (world units = block units here)
    g = np.array([0.3, -1.2, 0.7])
    blk = _one_block_linear(0.1, *g)
    img = oracle.render(blk, rays[:2], S, 2.0, -10.0, 10.0, tf, light, 0.4, 0.5, 0.3, 16.0, nb,
                        origin, extent, boc)
    nrm = g / np.linalg.norm(g)
    L = light.astype(np.float64)
    for q in range(2):
        d = rays[q, 3:6].astype(np.float64)
        H = L - d
        H /= np.linalg.norm(H)
        shade = 0.4 + 0.5 * abs(nrm @ L) + 0.3 * abs(nrm @ H) ** 16.0
        assert abs(img[q, 3] - A) < 1e-12
        want = np.array(rgb, np.float32).astype(np.float64) * shade * A
        assert np.allclose(img[q, :3], want, atol=1e-9), (img[q], want)


ALL_PINS = [pin_span, pin_unity, pin_bernstein, pin_cardinal, pin_linear, pin_quadratic,
            pin_corners, pin_fd, pin_one_sided, pin_brute, pin_decode_layout, pin_adjoint, pin_query,
            pin_render]
