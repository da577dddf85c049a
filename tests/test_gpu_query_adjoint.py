"""Point query and the decode adjoint on the GPU against the FP64 oracle."""
import numpy as np
import pytest
import torch

import fa_inputs as fi
import oracle
from gpu_util import (check_elementwise_bound, check_normwise, dequant, host_quantize,
                      mixed_batch, models, oracle_blocks, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fa():
    import paper_2409_00184_amd as fa
    assert torch.cuda.is_available()
    return fa


def _query_case(fa, b, nb, origin, extent, boc, xyz, what, mask=15):
    m = models(b)
    q = fa.query(m, torch.as_tensor(xyz).cuda().contiguous(), nb, origin, extent,
                 torch.as_tensor(boc, dtype=torch.int32).cuda(), mask).cpu().numpy()
    r, S = oracle.query_points(oracle_blocks(b), xyz, nb, origin, extent, boc, with_abs=True)
    for c in range(4):
        if not (mask >> c) & 1:
            r[:, c] = 0.0
            S[:, c] = 0.0
    check_elementwise_bound(q, r, S, 64.0, what)
    return q, r


def test_query_mixed_domain(fa):
    """2x3x2 cells, permuted cell map with an empty cell, non-unit
    origin/extent, points inside, outside (clamped), on faces and knots."""
    say("query mixed")
    nb = (2, 3, 2)
    b = mixed_batch(31, 12)
    g = fi.rng(32)
    boc = g.permutation(12).astype(np.int32)
    boc[5] = -1
    origin = np.array([-0.5, 0.25, 1.0], np.float32)
    extent = np.array([2.0, 3.0, 0.5], np.float32)
    u = g.uniform(-0.1, 1.1, (20000, 3))
    faces = (g.integers(0, 7, (2000, 3)) / 6.0)  # multiples of 1/6: cell faces for nb 2,3
    u = np.concatenate([u, faces, [[0, 0, 0], [1, 1, 1]]])
    xyz = (origin + u * extent).astype(np.float32)
    for mask in (15, 1, 0b1010):
        _query_case(fa, b, nb, origin, extent, boc, xyz, f"query mixed mask {mask}", mask)


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_query_low_precision_lattices(fa, dtype):
    """BF16/FP16 lattices (P / s_b, per-block scale): the query equals the
    oracle on the dequantised lattice to FP32 accuracy.  Lattices with an odd
    number of values end on a half dword; points next to each cell's far
    corner give the last lattice value the largest weight."""
    say("query low precision", dtype)
    nb = (2, 2, 3)
    g = fi.rng(33)
    ncp = [(5, 7, 9), (6, 3, 11), (9, 9, 9), (4, 5, 7), (8, 6, 5), (3, 3, 3),
           (7, 7, 6), (5, 9, 4), (11, 3, 5), (5, 5, 5), (13, 5, 7), (2, 3, 5)]
    deg = [(p, p, p) for p in (3, 2, 3, 1, 2, 2, 3, 3, 2, 3, 3, 1)]
    kl = [[fi.clamped_uniform_knots(n[a], p[0]) for a in range(3)] for n, p in zip(ncp, deg)]
    b = fi.pack(ncp, deg, kl, [g.normal(size=n) for n in ncp])
    assert sum(int(np.prod(n)) % 2 for n in ncp) >= 6
    boc = np.arange(12, dtype=np.int32)
    u = g.uniform(0, 1, (30000, 3))
    corner = 1.0 - g.uniform(0, 1e-3, (4000, 3))  # just inside the far corners
    cells = g.integers(0, 12, 4000)
    cidx = np.stack([cells // 6, (cells // 3) % 2, cells % 3], 1)
    pts = np.concatenate([u * np.array(nb), cidx + corner]) / np.array(nb)
    xyz = pts.astype(np.float32)
    m = models(b)
    q = fa.query(m, torch.as_tensor(xyz).cuda(), nb, (0, 0, 0), (1, 1, 1),
                 torch.as_tensor(boc).cuda(), 15, dtype).cpu().numpy()
    codes, scales = host_quantize(b, dtype)
    ob = oracle_blocks(b, ctrl=dequant(b, codes, scales, dtype))
    r, S = oracle.query_points(ob, xyz, nb, (0, 0, 0), (1, 1, 1), boc, with_abs=True)
    check_elementwise_bound(q, r, S, 64.0, f"query {dtype}")


def test_query_c3_blocks_rays(fa):
    """Config C3 micro-models (16^3 blocks, NCP* in 8..32, cubic) queried by
    seeded camera rays (reduced image: 160 x 90 rays, 512 samples each)."""
    say("query C3 reduced rays")
    b = fi.config_c3_blocks()
    xyz = fi.ray_samples_np(3, 160, 90, 512)
    q, r = _query_case(fa, b, (16, 16, 16), (0, 0, 0), (1, 1, 1), fi.identity_cells(16 ** 3),
                       xyz, "C3 rays")
    scale = np.abs(r).max(0)
    assert np.all(np.abs(q - r).max(0) <= 1e-5 * scale)


@pytest.mark.parametrize("w,h,k", [(160, 90, 512), (37, 11, 70), (8, 8, 64), (3, 1, 5)])
def test_query_rays_matches_flat(fa, w, h, k):
    """The ray-structured order computes exactly the flat query's values
    (ragged tiles and sample chunks included), and both match the oracle."""
    say("query rays", w, h, k)
    b = fi.config_c3_blocks()
    m = models(b)
    xyz = torch.as_tensor(fi.ray_samples_np(3, w, h, k)).cuda().contiguous()
    boc = torch.as_tensor(fi.identity_cells(4096), device="cuda")
    flat = fa.query(m, xyz, (16, 16, 16), (0, 0, 0), (1, 1, 1), boc)
    rays = fa.query_rays(m, xyz, w, h, k, (16, 16, 16), (0, 0, 0), (1, 1, 1), boc)
    assert torch.equal(flat, rays)
    if w * h * k <= 200000:
        r, S = oracle.query_points(oracle_blocks(b), xyz.cpu().numpy(), (16, 16, 16), (0, 0, 0),
                                   (1, 1, 1), fi.identity_cells(4096), with_abs=True)
        check_elementwise_bound(rays.cpu().numpy(), r, S, 64.0, "rays")


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_query_rays_low_precision_and_nonuniform(fa, dtype):
    """The ray order on 2-byte lattices (rows read from the LDS slots as
    dword pairs) and on blocks with non-uniform knots (binary span search on
    the knots in LDS), including blocks larger than one LDS slot (the
    per-lane fallback) in every lattice type: bit for bit the flat query,
    which the oracle checks."""
    say("query rays lowp / nonuniform", dtype)
    g = fi.rng(47)
    nb = (4, 4, 4)
    ncp, deg, kl, lat = [], [], [], []
    for k in range(64):
        p = int(g.choice([2, 3]))
        n = [int(v) for v in g.integers(p + 1, 33, 3)]
        if k == 5:
            n = [40, 30, 20]  # 24000 values: above one LDS slot in FP32
        if k == 9:
            n = [64, 40, 20]  # 51200 values: above one LDS slot in 2 bytes too
        ks = []
        for a in range(3):
            if k % 3 == 0 and n[a] > p + 1:
                inner = np.sort(g.uniform(0.02, 0.98, n[a] - p - 1))
                ks.append(np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)]).astype(np.float32))
            else:
                ks.append(fi.clamped_uniform_knots(n[a], p))
        ncp.append(n)
        deg.append((p, p, p))
        kl.append(ks)
        lat.append(g.normal(size=n))
    b = fi.pack(ncp, deg, kl, lat)
    m = models(b)
    w, h, k = 96, 40, 48
    o, d, t0, t1, j = fi.camera_rays(48, w, h)
    s = np.arange(k)
    t = t0[:, None] + (s[None] + j[:, None]) / k * (t1 - t0)[:, None]
    xyz = torch.as_tensor((o[:, None] + d[:, None] * t[..., None]).reshape(-1, 3)
                          .astype(np.float32)).cuda()
    boc = torch.as_tensor(np.arange(64, dtype=np.int32), device="cuda")
    for dt in ("f32", dtype):
        flat = fa.query(m, xyz, nb, (0, 0, 0), (1, 1, 1), boc, dtype=dt)
        rays = fa.query_rays(m, xyz, w, h, k, nb, (0, 0, 0), (1, 1, 1), boc, dtype=dt)
        assert torch.equal(flat, rays), dt
    r, S = oracle.query_points(oracle_blocks(b), xyz.cpu().numpy(), nb, (0, 0, 0), (1, 1, 1),
                               np.arange(64, dtype=np.int32), with_abs=True)
    check_elementwise_bound(fa.query_rays(m, xyz, w, h, k, nb, (0, 0, 0), (1, 1, 1), boc)
                            .cpu().numpy(), r, S, 64.0, "rays nonuniform f32")


def test_query_c3_full_sampled(fa):
    """C3 at full size: 1920x1080 rays x 512 samples generated on the GPU
    (1.06e9 samples); 300k sampled outputs checked against the oracle."""
    say("query C3 full")
    b = fi.config_c3_blocks()
    m = models(b)
    o, d, t0, t1, j = fi.camera_rays(3, 1920, 1080)
    nray, ns = o.shape[0], 512
    dev = "cuda"
    O = torch.as_tensor(o, dtype=torch.float64, device=dev)
    D = torch.as_tensor(d, dtype=torch.float64, device=dev)
    T0 = torch.as_tensor(t0, dtype=torch.float64, device=dev)
    T1 = torch.as_tensor(t1, dtype=torch.float64, device=dev)
    J = torch.as_tensor(j, dtype=torch.float64, device=dev)
    xyz = torch.empty((nray, ns, 3), dtype=torch.float32, device=dev)
    s = torch.arange(ns, dtype=torch.float64, device=dev)
    for r0 in range(0, nray, 1 << 18):
        r1 = min(nray, r0 + (1 << 18))
        t = T0[r0:r1, None] + (s[None] + J[r0:r1, None]) / ns * (T1 - T0)[r0:r1, None]
        xyz[r0:r1] = (O[r0:r1, None] + D[r0:r1, None] * t[..., None]).float()
    xyz = xyz.reshape(-1, 3)
    boc = torch.as_tensor(fi.identity_cells(4096), device=dev)
    out = fa.query_rays(m, xyz, 1920, 1080, 512, (16, 16, 16), (0, 0, 0), (1, 1, 1), boc)
    torch.cuda.synchronize()
    g = fi.rng(33)
    idx = torch.as_tensor(g.integers(0, xyz.shape[0], 300000), device=dev)
    xs = xyz[idx].cpu().numpy()
    got = out[idx].cpu().numpy()
    del out, xyz
    r, S = oracle.query_points(oracle_blocks(b), xs, (16, 16, 16), (0, 0, 0), (1, 1, 1),
                               fi.identity_cells(4096), with_abs=True)
    check_elementwise_bound(got, r, S, 64.0, "C3 full sampled")


@pytest.mark.parametrize("mask", [1, 15, 0b0110, 8])
@pytest.mark.parametrize("res", [(17, 23, 29), (64, 64, 64), (40, 3, 64)])
def test_adjoint_vs_oracle(fa, mask, res):
    say("adjoint", mask, res)
    b = mixed_batch(41, 10, ncp_hi=24)
    m = models(b)
    nchan = bin(mask).count("1")
    g = torch.randn((b.nblocks, nchan) + res, generator=torch.Generator().manual_seed(42))
    G = fa.decode_backward(m, res, g.cuda().contiguous(), mask).cpu().numpy()
    Gr = oracle.decode_adjoint(oracle_blocks(b), res, g.numpy().astype(np.float64), mask)
    for bb in range(b.nblocks):
        o = int(b.ctrl_off[bb])
        k = int(np.prod(b.ncp[bb]))
        err = np.abs(G[o:o + k] - Gr[o:o + k]).max()
        assert err <= 1e-5 * np.abs(Gr[o:o + k]).max(), (bb, err)


@pytest.mark.parametrize("res", [(19, 64, 64), (33, 37, 50), (65, 33, 36), (19, 8, 8)])
def test_adjoint_wide_lattices_vs_oracle(fa, res):
    """Value cotangents of lattices with NCP_y or NCP_z above 32 (several
    j and k tiles per micro-model) next to narrow ones in one batch, NCP_x
    above the x resolution (several control planes complete per x slice,
    and planes between the x chunks of two waves that no slice touches),
    y and z resolutions that are not multiples of 16 (partial row bands and
    column groups), and z resolutions that are not multiples of 4 (rows
    that the matrix-core kernel cannot read as 16-byte vectors: the VALU
    adjoint)."""
    say("adjoint wide", res)
    g = fi.rng(45)
    ncp = [(8, 40, 36), (6, 33, 20), (5, 10, 64), (12, 24, 24), (40, 12, 8), (7, 64, 33)]
    deg = [(3, 3, 3), (2, 2, 2), (1, 1, 1), (3, 3, 3), (2, 2, 2), (3, 3, 3)]
    kl = [[fi.clamped_uniform_knots(n[a], p[0]) for a in range(3)] for n, p in zip(ncp, deg)]
    b = fi.pack(ncp, deg, kl, [g.normal(size=n) for n in ncp])
    m = models(b)
    gt = torch.randn((b.nblocks, 1) + res, generator=torch.Generator().manual_seed(46))
    G = fa.decode_backward(m, res, gt.cuda().contiguous(), 1).cpu().numpy()
    Gr = oracle.decode_adjoint(oracle_blocks(b), res, gt.numpy().astype(np.float64), 1)
    for bb in range(b.nblocks):
        o = int(b.ctrl_off[bb])
        k = int(np.prod(b.ncp[bb]))
        err = np.abs(G[o:o + k] - Gr[o:o + k]).max()
        say("  block", ncp[bb], "err / scale", err / np.abs(Gr[o:o + k]).max())
        assert err <= 1e-5 * np.abs(Gr[o:o + k]).max(), (bb, err)


def test_adjoint_dot_product(fa):
    """<B P, g> = <P, B^T g> with the GPU forward and the GPU adjoint."""
    say("adjoint dot")
    b = mixed_batch(43, 16, ncp_hi=32)
    m = models(b)
    res = (64, 64, 64)
    for mask in (1, 15):
        BP = fa.decode(m, res, mask).double()
        g = torch.randn_like(BP)
        G = fa.decode_backward(m, res, g.float().contiguous(), mask).double()
        lhs = (BP * g.double()).sum().item()
        rhs = (m.ctrl.double() * G).sum().item()
        assert abs(lhs - rhs) <= 1e-5 * (BP.abs() * g.abs()).sum().item(), (mask, lhs, rhs)


def test_adjoint_leaves_padding(fa):
    """Elements between lattices are not touched by the adjoint."""
    b = mixed_batch(44, 5)
    m = models(b)
    res = (8, 8, 8)
    g = torch.randn((5, 1) + res, device="cuda")
    G = torch.full_like(m.ctrl, 7.0)
    fa.decode_backward(m, res, g, 1, grad_ctrl=G)
    G = G.cpu().numpy()
    inside = np.zeros(G.size, bool)
    for bb in range(5):
        o = int(b.ctrl_off[bb])
        inside[o:o + int(np.prod(b.ncp[bb]))] = True
    assert np.all(G[~inside] == 7.0)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_query_lattice_beyond_4gb(fa, dtype):
    """Blocks whose lattice lies past the first 4 GB of the lattice array
    (element offsets beyond 32-bit byte range) give bit for bit the values
    of the same blocks near its start, for points spread over several
    blocks per wave, in the flat and the ray order."""
    import copy
    say("query far lattice", dtype)
    nb = (2, 2, 2)
    b = mixed_batch(35, 8, ncp_lo=4, ncp_hi=24)
    near = models(b)
    far = copy.copy(near)
    F = 1 << 30  # elements: 4 GB of FP32 before the first block
    hd = near.host_desc.copy()
    hd["ctrl_off"] += F
    far.host_desc = hd
    far.desc = torch.from_numpy(hd.view(np.uint8).copy()).cuda()
    big = torch.zeros(F + near.ctrl.numel(), dtype=torch.float32, device="cuda")
    big[F:] = near.ctrl
    far.ctrl, far.ctrl_lp, far.desc_lp = big, {}, {}
    boc = np.arange(8, dtype=np.int32)
    bocd = torch.as_tensor(boc, device="cuda")
    g = fi.rng(36)
    xyz = torch.as_tensor(g.uniform(0, 1, (200000, 3)).astype(np.float32), device="cuda")
    o, e = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    rn = fa.query(near, xyz, nb, o, e, bocd, dtype=dtype)
    rf = fa.query(far, xyz, nb, o, e, bocd, dtype=dtype)
    assert torch.equal(rn, rf)
    # the ray order on the same positions (50 x 40 rays x 100 samples):
    # waves with samples outside the LDS slots read the far blocks one block
    # at a time (FP32: past 4 GB) or through 32-bit offsets (2-byte lattices)
    rr = fa.query_rays(far, xyz, 50, 40, 100, nb, o, e, bocd, dtype=dtype)
    assert torch.equal(rn, rr)
    del big, far
    torch.cuda.empty_cache()
