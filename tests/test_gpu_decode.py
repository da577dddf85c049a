"""Grid decode on the GPU against the FP64 oracle (FP32 path)."""
import numpy as np
import pytest
import torch

import fa_inputs as fi
import oracle
from gpu_util import (check_elementwise_bound, check_normwise, mixed_batch, models,
                      oracle_blocks, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fa():
    import paper_2409_00184_amd as fa
    assert torch.cuda.is_available()
    return fa


@pytest.mark.parametrize("res", [(17, 23, 29), (9, 5, 70), (2, 2, 2), (33, 64, 64)])
@pytest.mark.parametrize("form", ["default", "plan", "plain"])
def test_decode_mixed_small(fa, res, form):
    say("decode mixed", res, form)
    b = mixed_batch(21, 24)
    m = models(b)
    if form == "default":
        out = fa.decode(m, res, 15)
    elif form == "plan":
        out = fa.decode(m, res, 15, plan=fa.Plan(m, res, rows=4, waves=2, grid=5))
    else:
        out = fa.decode_plain(m, res, 15)
    out = out.cpu().numpy()
    ob = oracle_blocks(b)
    ref = oracle.decode_blocks(ob, res, 15)
    check_normwise(out, ref, 1e-5, f"decode {form} {res}")
    idx = np.array([[bb, x, y, z] for bb in range(b.nblocks) for x in range(res[0])
                    for y in range(res[1]) for z in range(res[2])], np.int32)
    _, S = oracle.decode_samples(ob, res, idx, with_abs=True)
    S = S.reshape(b.nblocks, *res, 4).transpose(0, 4, 1, 2, 3)
    check_elementwise_bound(out, ref, S, 64.0, f"decode {form} {res}")


@pytest.mark.parametrize("mask", [1, 2, 4, 8, 0b0101, 0b1110])
def test_decode_masks(fa, mask):
    say("decode mask", mask)
    b = mixed_batch(22, 8)
    m = models(b)
    res = (12, 13, 14)
    out = fa.decode(m, res, mask).cpu().numpy()
    ref = oracle.decode_blocks(oracle_blocks(b), res, mask)
    assert out.shape == ref.shape
    check_normwise(out, ref, 1e-5, f"mask {mask}")


@pytest.mark.parametrize("rows,waves,grid", [(1, 1, 3), (4, 4, 64), (8, 4, 0), (16, 8, 7),
                                             (3, 2, 1)])
def test_decode_tunings_agree(fa, rows, waves, grid):
    say("decode tuning", rows, waves, grid)
    b = mixed_batch(23, 12, ncp_hi=40)
    m = models(b)
    res = (21, 19, 66)
    ref = fa.decode(m, res, 15).cpu().numpy()
    out = fa.decode(m, res, 15, plan=fa.Plan(m, res, rows=rows, waves=waves, grid=grid))
    out2 = fa.decode(m, res, 15, tune=fa.FATune(rows, waves, grid, 0, 4096, 1))
    assert np.array_equal(out.cpu().numpy(), ref), "schedule must not change results"
    assert np.array_equal(out2.cpu().numpy(), ref)


def test_decode_edge_cases(fa):
    """Bezier blocks (n = p+1), n = 64 (slab chunking), degree 1."""
    say("decode edge")
    ncp = [(2, 2, 2), (4, 4, 4), (64, 64, 64), (64, 5, 64), (3, 64, 2)]
    deg = [(1, 1, 1), (3, 3, 3), (3, 3, 3), (2, 2, 2), (1, 1, 1)]
    g = fi.rng(24)
    kl = [[fi.clamped_uniform_knots(n[a], p[0]) for a in range(3)] for n, p in zip(ncp, deg)]
    b = fi.pack(ncp, deg, kl, [g.normal(size=n) for n in ncp])
    m = models(b)
    for res in [(64, 64, 64), (7, 130, 3)]:
        out = fa.decode(m, res, 15).cpu().numpy()
        ref = oracle.decode_blocks(oracle_blocks(b), res, 15)
        check_normwise(out, ref, 1e-5, f"edge {res}")


def test_decode_c1(fa):
    """Config C1: one 16^3 cubic block, 64^3 voxels, whole grid."""
    say("decode C1")
    b = fi.config_c1()
    m = models(b)
    out = fa.decode(m, (64, 64, 64), 15).cpu().numpy()
    ref = oracle.decode_blocks(oracle_blocks(b), (64, 64, 64), 15)
    w = check_normwise(out, ref, 1e-5, "C1")
    # against the FP64 source lattice the FP32 rounding of P is included
    ref64 = oracle.decode_blocks(oracle_blocks(b, b.ctrl64), (64, 64, 64), 15)
    check_normwise(out, ref64, 1e-5, "C1 vs FP64 source")
    say("C1 worst normwise", w)


def test_decode_c2_full(fa):
    """Config C2 at full size (512 blocks, 64^3, planned persistent launch):
    16 blocks compared whole, 200k sampled voxels of all blocks."""
    say("decode C2 full")
    b = fi.config_c2()
    m = models(b)
    res = (64, 64, 64)
    plan = fa.Plan(m, res)
    out = torch.full((b.nblocks, 4) + res, float("nan"), device="cuda")
    fa.decode(m, res, 15, plan=plan, out=out)
    assert not torch.isnan(out).any(), "every voxel written exactly by the plan"
    ob = oracle_blocks(b)
    g = fi.rng(25)
    pick = g.choice(b.nblocks, 16, replace=False)
    sub = oracle.Blocks(ob.ncp[pick], ob.deg[pick], ob.knot_off[pick], ob.ctrl_off[pick],
                        ob.knots, ob.ctrl)
    ref = oracle.decode_blocks(sub, res, 15)
    check_normwise(out[torch.as_tensor(pick, device="cuda")].cpu().numpy(), ref, 1e-5, "C2 whole")
    idx = np.stack([g.integers(0, b.nblocks, 200000)] + [g.integers(0, 64, 200000)] * 1 +
                   [g.integers(0, 64, 200000), g.integers(0, 64, 200000)], 1).astype(np.int32)
    r, S = oracle.decode_samples(ob, res, idx, with_abs=True)
    ti = torch.as_tensor(idx, device="cuda").long()
    got = out[ti[:, 0], :, ti[:, 1], ti[:, 2], ti[:, 3]].cpu().numpy()
    check_elementwise_bound(got, r, S, 64.0, "C2 sampled")


@pytest.mark.parametrize("res", [(17, 23, 29), (64, 64, 64), (2, 2, 2)])
@pytest.mark.parametrize("sched", [None, (4, 2, 5), (16, 8, 0)])
def test_decode_interleaved_matches_planar(fa, res, sched):
    """mask 15 | OUT_INTERLEAVED stores the planar decode's values as one
    (value, d/du, d/dv, d/dw) record per voxel, bit for bit."""
    say("decode interleaved", res, sched)
    b = mixed_batch(26, 19, ncp_hi=40)
    m = models(b)
    plan = None if sched is None else fa.Plan(m, res, rows=sched[0], waves=sched[1],
                                              grid=sched[2])
    planar = fa.decode(m, res, 15, plan=plan)
    inter = torch.full((b.nblocks,) + res + (4,), float("nan"), device="cuda")
    fa.decode(m, res, 15 | fa.OUT_INTERLEAVED, plan=plan, out=inter)
    assert torch.equal(inter, planar.permute(0, 2, 3, 4, 1)), "same values, other layout"
    ref = oracle.decode_blocks(oracle_blocks(b), res, 15)
    check_normwise(inter.permute(0, 4, 1, 2, 3).cpu().numpy(), ref, 1e-5, f"interleaved {res}")


def test_decode_interleaved_c2_sampled(fa):
    """C2 at full size in the interleaved layout (the bench's form):
    sampled voxels within the FP32 elementwise bound of the oracle."""
    say("decode interleaved C2")
    b = fi.config_c2()
    m = models(b)
    res = (64, 64, 64)
    out = torch.full((b.nblocks,) + res + (4,), float("nan"), device="cuda")
    fa.decode(m, res, 15 | fa.OUT_INTERLEAVED, plan=fa.Plan(m, res), out=out)
    assert not torch.isnan(out).any()
    g = fi.rng(27)
    n = 100000
    idx = np.stack([g.integers(0, b.nblocks, n), g.integers(0, 64, n), g.integers(0, 64, n),
                    g.integers(0, 64, n)], 1).astype(np.int32)
    r, S = oracle.decode_samples(oracle_blocks(b), res, idx, with_abs=True)
    ti = torch.as_tensor(idx, device="cuda").long()
    got = out[ti[:, 0], ti[:, 1], ti[:, 2], ti[:, 3]].cpu().numpy()
    check_elementwise_bound(got, r, S, 64.0, "C2 interleaved sampled")



@pytest.mark.parametrize("layout", ["planar", "interleaved"])
def test_decode_maximum_resolution(fa, layout):
    """Grids of FA_MAX_RES = 256 per axis and lattices of FA_MAX_NCP = 64 per
    axis: every voxel written (NaN fill), sampled voxels within the FP32
    elementwise bound of the oracle."""
    say("decode max res", layout)
    g = fi.rng(29)
    ncp = [(64, 64, 64), (2, 2, 2), (33, 64, 5)]
    deg = [(3, 3, 3), (1, 1, 1), (2, 2, 2)]
    kl = [[fi.clamped_uniform_knots(n[a], p[0]) for a in range(3)] for n, p in zip(ncp, deg)]
    b = fi.pack(ncp, deg, kl, [g.normal(size=n) for n in ncp])
    m = models(b)
    res = (256, 256, 256)
    if layout == "planar":
        out = torch.full((b.nblocks, 4) + res, float("nan"), device="cuda")
        fa.decode(m, res, 15, plan=fa.Plan(m, res), out=out)
    else:
        out = torch.full((b.nblocks,) + res + (4,), float("nan"), device="cuda")
        fa.decode(m, res, 15 | fa.OUT_INTERLEAVED, plan=fa.Plan(m, res), out=out)
    assert not torch.isnan(out).any()
    n = 60000
    idx = np.stack([g.integers(0, b.nblocks, n), g.integers(0, 256, n), g.integers(0, 256, n),
                    g.integers(0, 256, n)], 1).astype(np.int32)
    idx[:8, 1:] = [[0, 0, 0], [255, 255, 255], [0, 255, 0], [255, 0, 255],
                   [128, 1, 254], [1, 128, 0], [255, 255, 0], [0, 0, 255]]
    r, S = oracle.decode_samples(oracle_blocks(b), res, idx, with_abs=True)
    ti = torch.as_tensor(idx, device="cuda").long()
    if layout == "planar":
        got = out[ti[:, 0], :, ti[:, 1], ti[:, 2], ti[:, 3]].cpu().numpy()
    else:
        got = out[ti[:, 0], ti[:, 1], ti[:, 2], ti[:, 3]].cpu().numpy()
    check_elementwise_bound(got, r, S, 64.0, f"max res {layout}")
    del out
    torch.cuda.empty_cache()


def test_query_empty_input(fa):
    """Zero points: the call returns without a launch and leaves the output
    untouched."""
    say("query empty")
    b = mixed_batch(30, 2)
    m = models(b)
    xyz = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    out = torch.full((1, 4), 7.0, device="cuda")
    fa.query(m, xyz, (1, 1, 2), (0, 0, 0), (1, 1, 1),
             torch.as_tensor(np.arange(2, dtype=np.int32), device="cuda"), out=out)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
