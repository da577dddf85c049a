"""Repeated interior knots (multiplicity 2..p, continuity C^{p-m} there) on
the GPU against the FP64 oracle: grid decode (VALU, plain and matrix-core
forms), point query and the adjoint, with samples exactly on the repeated
knots.  At a knot of multiplicity p the first derivative jumps; both sides
take the span right-continuously (t_s <= u < t_{s+1}) from the same FP32
knot and position values, so both return the derivative from the right and
the comparison stays element by element."""
import numpy as np
import pytest
import torch

import fa_inputs as fi
import oracle
from gpu_util import check_elementwise_bound, check_normwise, models, oracle_blocks, say

pytestmark = pytest.mark.gpu

# interior knots, all multiples of 1/32 (so they are voxel positions i/(R-1)
# of R = 33 and R = 65, and exact in FP32)
_INTERIOR = {
    # p = 3: multiplicity 2 (C^1) and 3 (C^0)
    (3, 10): [4, 8, 8, 16, 16, 16],
    (3, 9): [6, 6, 12, 20, 20],
    (3, 12): [2, 8, 8, 8, 12, 18, 24, 24],
    (3, 5): [16],
    # p = 2: multiplicity 2 (C^0)
    (2, 9): [4, 8, 8, 16, 24, 24],
    (2, 7): [10, 10, 20, 20],
    (2, 11): [3, 6, 9, 9, 16, 16, 22, 26],
}


def _knots(n, p):
    inner = np.array(_INTERIOR[(p, n)], np.float64) / 32.0
    assert len(inner) == n - p - 1
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)]).astype(np.float32)


def repeated_batch(seed):
    g = fi.rng(seed)
    shapes = [((10, 9, 12), 3), ((12, 10, 5), 3), ((9, 12, 10), 3), ((9, 7, 11), 2),
              ((11, 9, 7), 2), ((7, 11, 9), 2)]
    ncp, deg, kl, lat = [], [], [], []
    for n, p in shapes:
        ncp.append(n)
        deg.append((p, p, p))
        kl.append([_knots(n[a], p) for a in range(3)])
        lat.append(g.normal(size=n))
    return fi.pack(ncp, deg, kl, lat)


@pytest.fixture(scope="module")
def fa():
    import paper_2409_00184_amd as fa
    assert torch.cuda.is_available()
    return fa


def _all_voxels(b, res):
    return np.array([[k, x, y, z] for k in range(b.nblocks) for x in range(res[0])
                     for y in range(res[1]) for z in range(res[2])], np.int32)


@pytest.mark.parametrize("form", ["default", "plan", "plain"])
def test_decode_repeated_knots(fa, form):
    say("repeated knots decode", form)
    b = repeated_batch(91)
    m = models(b)
    res = (33, 65, 33)
    if form == "default":
        out = fa.decode(m, res, 15)
    elif form == "plan":
        out = fa.decode(m, res, 15, plan=fa.Plan(m, res, rows=4, waves=2, grid=5))
    else:
        out = fa.decode_plain(m, res, 15)
    out = out.cpu().numpy()
    ob = oracle_blocks(b)
    ref = oracle.decode_blocks(ob, res, 15)
    check_normwise(out, ref, 1e-5, f"repeated knots decode {form}")
    _, S = oracle.decode_samples(ob, res, _all_voxels(b, res), with_abs=True)
    S = S.reshape(b.nblocks, *res, 4).transpose(0, 4, 1, 2, 3)
    check_elementwise_bound(out, ref, S, 64.0, f"repeated knots decode {form}")


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_decode_repeated_knots_matrix_cores(fa, dtype):
    """The BF16/FP16 matrix-core decode on the same blocks, under the bound
    of its roundings (P, z basis, z-stage result, y basis: 6 u allowed)."""
    say("repeated knots mfma", dtype)
    b = repeated_batch(92)
    m = models(b)
    res = (33, 65, 33)
    out = fa.decode(m, res, 15, dtype=dtype, plan=fa.Plan(m, res, kernel=1)).cpu().numpy()
    ob = oracle_blocks(b)
    ref, S = oracle.decode_samples(ob, res, _all_voxels(b, res), with_abs=True)
    got = out.transpose(0, 2, 3, 4, 1).reshape(-1, 4).astype(np.float64)
    u = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}[dtype]
    lim = (6 * u + 64 * 2.0 ** -24) * S + 1e-30
    assert (np.abs(got - ref) <= lim).all(), float((np.abs(got - ref) / lim).max())


def test_query_on_repeated_knots(fa):
    """Each block alone on the unit cube (block coordinate = position,
    exactly): positions on its repeated knots, one FP32 ulp either side of
    them, and uniform ones, on every axis."""
    say("repeated knots query")
    b = repeated_batch(93)
    m = models(b)
    g = fi.rng(94)
    for k in range(b.nblocks):
        p = int(b.deg[k, 0])
        per_axis = []
        for a in range(3):
            kv = np.array(sorted(set(_INTERIOR[(p, int(b.ncp[k, a]))])), np.float32) / 32
            per_axis.append(np.concatenate([kv, np.nextafter(kv, np.float32(0)),
                                            np.nextafter(kv, np.float32(1))]))
        on = np.stack([v[g.integers(0, v.size, 6000)] for v in per_axis], 1)
        xyz = np.concatenate([on, g.uniform(0, 1, (2000, 3))]).astype(np.float32)
        boc = np.array([k], np.int32)
        for mask in (15, 0b1010):
            q = fa.query(m, torch.as_tensor(xyz).cuda(), (1, 1, 1), (0, 0, 0), (1, 1, 1),
                         torch.as_tensor(boc).cuda(), mask).cpu().numpy()
            r, S = oracle.query_points(oracle_blocks(b), xyz, (1, 1, 1), (0, 0, 0), (1, 1, 1),
                                       boc, with_abs=True)
            for c in range(4):
                if not (mask >> c) & 1:
                    r[:, c] = 0.0
                    S[:, c] = 0.0
            check_elementwise_bound(q, r, S, 64.0, f"repeated knots query block {k} mask {mask}")


@pytest.mark.parametrize("res", [(65, 33, 33), (33, 33, 64)])
@pytest.mark.parametrize("mask", [1, 15])
def test_adjoint_repeated_knots(fa, mask, res):
    """res[2] = 64: the value adjoint on the matrix cores (16-byte rows);
    33: the VALU adjoint.  The adjoint takes y and z resolutions up to 64."""
    say("repeated knots adjoint", mask, res)
    b = repeated_batch(95)
    m = models(b)
    nchan = bin(mask).count("1")
    g = torch.randn((b.nblocks, nchan) + res, generator=torch.Generator().manual_seed(96))
    G = fa.decode_backward(m, res, g.cuda().contiguous(), mask).cpu().numpy()
    Gr = oracle.decode_adjoint(oracle_blocks(b), res, g.numpy().astype(np.float64), mask)
    for k in range(b.nblocks):
        o, n = int(b.ctrl_off[k]), int(np.prod(b.ncp[k]))
        err = np.abs(G[o:o + n] - Gr[o:o + n]).max()
        assert err <= 1e-5 * np.abs(Gr[o:o + n]).max(), (k, err)
