"""Helpers shared by the GPU parity tests (inputs -> both sides, checks)."""
import sys

import numpy as np

import oracle

U32 = 2.0 ** -24


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_blocks(b, ctrl=None):
    return oracle.Blocks(b.ncp, b.deg, b.knot_off, b.ctrl_off, b.knots,
                         b.ctrl if ctrl is None else ctrl)


def models(b):
    import paper_2409_00184_amd as fa
    return fa.MicroModels.from_batch(b)


def check_normwise(gpu, ref, rel=1e-5, what=""):
    """Per block and channel: max |gpu - ref| <= rel * max |ref|."""
    gpu = np.asarray(gpu, np.float64)
    nb, nc = ref.shape[:2]
    worst = 0.0
    for b in range(nb):
        for c in range(nc):
            r = ref[b, c]
            scale = np.abs(r).max()
            err = np.abs(gpu[b, c] - r).max()
            ratio = err / scale if scale > 0 else err
            worst = max(worst, ratio)
            assert err <= rel * scale + 1e-30, f"{what} block {b} ch {c}: err {err} scale {scale}"
    return worst


def check_elementwise_bound(gpu, ref, S, c=32.0, what=""):
    """|gpu - ref| <= c * 2^-24 * S elementwise (S: oracle's abs sum)."""
    err = np.abs(np.asarray(gpu, np.float64) - ref)
    lim = c * U32 * S + 1e-30
    bad = err > lim
    assert not bad.any(), f"{what}: {bad.sum()} elements over {c}*u*S, worst ratio {(err / lim).max()}"
    return float((err / lim).max())


def mixed_batch(seed, nblocks, ncp_lo=2, ncp_hi=20, degs=(1, 2, 3), nonuniform=0.3):
    """Blocks of random NCP per axis and degree, some with non-uniform knots,
    lattices ~ N(0, 1)."""
    import fa_inputs as fi
    g = fi.rng(seed)
    ncp, deg, kl, lat = [], [], [], []
    for b in range(nblocks):
        p = int(g.choice(degs))
        n = [int(g.integers(max(ncp_lo, p + 1), ncp_hi + 1)) for _ in range(3)]
        ks = []
        for a in range(3):
            if g.uniform() < nonuniform and n[a] > p + 1:
                inner = np.sort(g.uniform(0.01, 0.99, n[a] - p - 1))
                ks.append(np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)]).astype(np.float32))
            else:
                ks.append(fi.clamped_uniform_knots(n[a], p))
        ncp.append(n)
        deg.append([p, p, p])
        kl.append(ks)
        lat.append(g.normal(size=n))
    return fi.pack(ncp, deg, kl, lat)


def host_quantize(b, dtype):
    """Reference of fa_quantize_blocks: s = max|P| (1 if zero), q =
    clamp(P * fl(1/s), -1, 1) in FP32, then RNE to the 2-byte type."""
    codes = np.zeros(b.ctrl.size, np.uint16)
    scales = np.zeros(b.nblocks, np.float32)
    for k in range(b.nblocks):
        o, n = int(b.ctrl_off[k]), int(np.prod(b.ncp[k]))
        P = b.ctrl[o:o + n].astype(np.float32)
        s = np.float32(np.abs(P).max()) if np.abs(P).max() > 0 else np.float32(1.0)
        inv = np.float32(1.0) / s
        q = np.clip(P * inv, np.float32(-1), np.float32(1)).astype(np.float32)
        if dtype == "bf16":
            u = q.view(np.uint32).astype(np.uint64)
            u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
            codes[o:o + n] = u.astype(np.uint16)
        else:
            codes[o:o + n] = q.astype(np.float16).view(np.uint16)
        scales[k] = s
    return codes, scales


def dequant(b, codes, scales, dtype):
    out = np.zeros(b.ctrl.size, np.float64)
    if dtype == "bf16":
        vals = (codes.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    else:
        vals = codes.view(np.float16).astype(np.float64)
    for k in range(b.nblocks):
        o, n = int(b.ctrl_off[k]), int(np.prod(b.ncp[k]))
        out[o:o + n] = vals[o:o + n] * float(scales[k])
    return out
