"""BF16/FP16 lattices: per-block max-abs quantisation (bit-exact against a
host reference) and the low-precision decodes (VALU kernel with 2-byte
storage, MFMA kernel) against the FP64 oracle under an a-priori bound.

Bound used (u = 2^-8 for BF16, 2^-11 for FP16, S = the oracle's
sum |basis product| |P| of each output, which is the same for P and P/s
up to the factor s that the kernels apply in FP32):
  VALU, 2-byte storage: only P is rounded        -> |err| <= (u + 64 u32) S
  MFMA: P, the z basis, the z-stage result Q and the y basis are rounded
        (4 roundings; 6 allowed for second-order terms) -> (6 u + 64 u32) S
"""
import numpy as np
import pytest
import torch

import fa_inputs as fi
import oracle
from gpu_util import U32, dequant, host_quantize, mixed_batch, models, oracle_blocks, say

pytestmark = pytest.mark.gpu
ULP = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}


@pytest.fixture(scope="module")
def fa():
    import paper_2409_00184_amd as fa
    assert torch.cuda.is_available()
    return fa


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_quantize_bit_exact(fa, dtype):
    say("quantize", dtype)
    b = mixed_batch(51, 20, ncp_hi=16)
    b.ctrl[int(b.ctrl_off[3]):int(b.ctrl_off[3]) + int(np.prod(b.ncp[3]))] = 0.0  # zero block
    m = models(b)
    desc, lp = m.lattice(dtype)
    codes, scales = host_quantize(b, dtype)
    got = lp.cpu().numpy().view(np.uint16)
    for k in range(b.nblocks):
        o, n = int(b.ctrl_off[k]), int(np.prod(b.ncp[k]))
        assert np.array_equal(got[o:o + n], codes[o:o + n]), k
    d = desc.cpu().numpy().view(fa.BLOCK_DTYPE)
    assert np.array_equal(d["scale"], scales)
    assert d["scale"][3] == 1.0


def _bound_check(out, ref, S, c, u, what):
    err = np.abs(out.astype(np.float64) - ref)
    lim = (c * u + 64 * U32) * S + 1e-30
    worst = float((err / lim).max())
    assert worst <= 1.0, f"{what}: error {worst:.3f} x bound"
    return worst


def _decode_case(fa, b, res, dtype, kernel):
    m = models(b)
    if kernel == 1:
        plan = fa.Plan(m, res, kernel=1)
    else:
        plan = fa.Plan(m, res)
    out = fa.decode(m, res, 15, dtype=dtype, plan=plan).cpu().numpy()
    ob = oracle_blocks(b)
    idx = np.array([[k, x, y, z] for k in range(b.nblocks) for x in range(res[0])
                    for y in range(res[1]) for z in range(res[2])], np.int32)
    ref, S = oracle.decode_samples(ob, res, idx, with_abs=True)
    got = out.transpose(0, 2, 3, 4, 1).reshape(-1, 4)
    c = 6.0 if kernel == 1 else 1.0
    return _bound_check(got, ref, S, c, ULP[dtype], f"{dtype} kernel {kernel} {res}")


@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("dtype", ["bf16", "f16"])
@pytest.mark.parametrize("res", [(64, 64, 64), (23, 17, 41), (16, 5, 64)])
def test_lowp_decode_bound(fa, kernel, dtype, res):
    say("lowp decode", kernel, dtype, res)
    b = mixed_batch(52, 10, ncp_lo=4, ncp_hi=32, nonuniform=0.3)
    w = _decode_case(fa, b, res, dtype, kernel)
    say("  worst / bound", w)


def test_mfma_fallback_items(fa):
    """Blocks the MFMA tile does not take (NCP > 32, wide y windows at a
    small y resolution) go through the voxel-by-voxel path of the same
    kernel and stay within the storage-rounding bound."""
    say("mfma fallback")
    g = fi.rng(53)
    ncp = [(40, 8, 8), (8, 48, 12), (6, 6, 33), (32, 32, 32)]
    deg = [(3, 3, 3), (2, 2, 2), (1, 1, 1), (3, 3, 3)]
    kl = [[fi.clamped_uniform_knots(n[a], p[0]) for a in range(3)] for n, p in zip(ncp, deg)]
    b = fi.pack(ncp, deg, kl, [g.normal(size=n) for n in ncp])
    for res in [(20, 6, 33), (64, 64, 64)]:
        _decode_case(fa, b, res, "bf16", 1)


def test_mfma_rejects_f32_and_bad_tiles(fa):
    b = mixed_batch(54, 3)
    m = models(b)
    with pytest.raises(fa.FAError) as e:
        fa.decode(m, (16, 16, 16), 15, dtype="f32", plan=fa.Plan(m, (16, 16, 16), kernel=1))
    assert e.value.status == 2
    for rows, waves in ((4, 4), (16, 8)):  # the tile is 16 rows x 4 waves
        with pytest.raises(fa.FAError) as e:
            fa.Plan(m, (16, 16, 16), rows, waves, 0, 1)
        assert e.value.status == 2


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_mfma_wide_z_and_channel_masks(fa, dtype):
    """z resolutions above one 64-column tile (several column items per
    row band), odd NCP_z (lattice rows starting on half dwords) and partial
    channel masks, against the oracle under the MFMA bound; every mask's
    channels equal the full decode's."""
    say("mfma wide z", dtype)
    g = fi.rng(56)
    ncp = [(9, 7, 31), (12, 17, 5), (5, 6, 32), (7, 9, 13)]
    deg = [(3, 3, 3), (2, 2, 2), (1, 1, 1), (3, 3, 3)]
    kl = [[fi.clamped_uniform_knots(n[a], p[0]) for a in range(3)] for n, p in zip(ncp, deg)]
    b = fi.pack(ncp, deg, kl, [g.normal(size=n) for n in ncp])
    res = (9, 21, 150)
    _decode_case(fa, b, res, dtype, 1)
    m = models(b)
    plan = fa.Plan(m, res, kernel=1)
    full = fa.decode(m, res, 15, dtype=dtype, plan=plan)
    for mask in (1, 6, 8, 13):
        part = fa.decode(m, res, mask, dtype=dtype, plan=fa.Plan(m, res, kernel=1))
        chans = [c for c in range(4) if (mask >> c) & 1]
        assert torch.equal(part, full[:, chans]), mask


def test_c5_sampled(fa):
    """Config C5 (4096 blocks of 32^3 control points, k^-5/3 lattices, 64^3
    voxels each, 1.07e9 voxels) on its 1% seeded uniform subset (10,737,418
    (block, voxel) pairs, without replacement): FP32 on the VALU, BF16 and
    FP16 on the matrix cores and BF16 and FP16 storage on the VALU, each
    against the FP64 oracle under its a-priori bound and against the FP32
    path under the sum of the two bounds."""
    say("C5 1% subset")
    b = fi.config_c5()
    m = models(b)
    res = (64, 64, 64)
    idx = fi.voxel_subset(b.nblocks, res, 0.01, seed=55)
    assert idx.shape[0] == 10_737_418
    ref, S = oracle.decode_samples(oracle_blocks(b), res, idx, with_abs=True)
    ti = torch.as_tensor(idx, device="cuda").long()
    out = torch.empty((b.nblocks, 4) + res, dtype=torch.float32, device="cuda")
    f32 = None
    for dtype, kernel in (("f32", 0), ("bf16", 1), ("f16", 1), ("bf16", 0), ("f16", 0)):
        say("  ", dtype, "kernel", kernel)
        out.fill_(float("nan"))
        plan = fa.Plan(m, res, kernel=kernel) if kernel else fa.Plan(m, res)
        fa.decode(m, res, 15, dtype=dtype, plan=plan, out=out)
        got = out[ti[:, 0], :, ti[:, 1], ti[:, 2], ti[:, 3]].cpu().numpy()
        assert np.isfinite(got).all()
        if dtype == "f32":
            _bound_check(got, ref, S, 0.0, 0.0, "C5 f32")
            f32 = got.astype(np.float64)
        else:
            c = 6.0 if kernel == 1 else 1.0
            w = _bound_check(got, ref, S, c, ULP[dtype], f"C5 {dtype} kernel {kernel}")
            # against the FP32 path: both errors against the exact value
            err = np.abs(got - f32)
            lim = (c * ULP[dtype] + 2 * 64 * U32) * S + 1e-30
            assert (err <= lim).all(), f"C5 {dtype} kernel {kernel} vs f32: {(err / lim).max()}"
            say("    worst / bound", w)
    del out


def _fallback_batch():
    g = fi.rng(57)
    ncp = [(40, 8, 8), (8, 48, 12), (6, 6, 33), (9, 7, 31), (12, 17, 5), (5, 6, 32)]
    deg = [(3, 3, 3), (2, 2, 2), (1, 1, 1), (3, 3, 3), (2, 2, 2), (1, 1, 1)]
    kl = [[fi.clamped_uniform_knots(n[a], p[0]) for a in range(3)] for n, p in zip(ncp, deg)]
    return fi.pack(ncp, deg, kl, [g.normal(size=n) for n in ncp])


@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("dtype", ["bf16", "f16"])
@pytest.mark.parametrize("batch", ["mixed", "fallback"])
def test_lowp_interleaved_matches_planar(fa, kernel, dtype, batch):
    """Interleaved records (mask 15 | OUT_INTERLEAVED) hold the planar
    decode's values bit for bit, on the matrix-core kernel (tile and
    voxel-by-voxel items, partial row bands and column tiles) and on the
    VALU kernel with 2-byte lattices."""
    say("lowp interleaved", kernel, dtype, batch)
    b = (mixed_batch(58, 9, ncp_lo=4, ncp_hi=32, nonuniform=0.3) if batch == "mixed"
         else _fallback_batch())
    m = models(b)
    for res in [(64, 64, 64), (23, 17, 41), (9, 21, 150)]:
        plan = fa.Plan(m, res, kernel=kernel) if kernel else fa.Plan(m, res)
        planar = fa.decode(m, res, 15, dtype=dtype, plan=plan)
        inter = torch.full((b.nblocks,) + res + (4,), float("nan"), device="cuda")
        fa.decode(m, res, 15 | fa.OUT_INTERLEAVED, dtype=dtype, plan=plan, out=inter)
        assert torch.equal(inter, planar.permute(0, 2, 3, 4, 1)), res
