"""fa_decode_residual_noalloc (partial sums in the library's fixed device
array, no allocation) against fa_decode_residual (caller workspace): the
same kernels, so the cotangent and the per-block sums of squares must be
equal bit for bit, on consecutive calls of shrinking size (the second call
reuses the array the first one filled) and at the array's maximum size."""
import ctypes

import numpy as np
import pytest
import torch

import fa_inputs as fi
from gpu_util import mixed_batch, models, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fa():
    import paper_2409_00184_amd as fa
    assert torch.cuda.is_available()
    return fa


def _both(fa, b, res, seed, tune=None, use_plan=True):
    m = models(b)
    g = fi.rng(seed)
    y = torch.as_tensor(g.normal(size=(b.nblocks,) + res).astype(np.float32)).cuda()
    scale = 2.0 / (b.nblocks * int(np.prod(res)))
    plan = (fa.Plan(m, res, *tune) if tune else fa.Plan(m, res)) if use_plan else None
    kw = dict(plan=plan) if plan is not None else dict(tune=fa.FATune(*tune) if tune else None)
    ref_g, ref_s = fa.decode_residual(m, res, y, scale, **kw)
    # outputs pre-filled with NaN: every element must be written
    got_g = torch.full_like(ref_g, float("nan"))
    got_s = torch.full_like(ref_s, float("nan"))
    fa.decode_residual_noalloc(m, res, y, scale, grad=got_g, sumsq=got_s, **kw)
    torch.cuda.synchronize()
    assert torch.equal(got_g, ref_g), res
    assert torch.equal(got_s, ref_s), res
    return m, y, scale


def test_noalloc_matches_workspace_form_shrinking_calls(fa):
    say("noalloc: large then small call")
    b1 = mixed_batch(81, 12, ncp_lo=4, ncp_hi=32)
    _both(fa, b1, (40, 48, 70), 82, tune=(16, 8, 1 << 20, 0, 4096, 0))
    b2 = mixed_batch(83, 3, ncp_lo=3, ncp_hi=12)
    _both(fa, b2, (17, 9, 23), 84)
    # and once more without a plan (default item order, default tune)
    _both(fa, b2, (17, 9, 23), 85, use_plan=False)


def test_noalloc_at_scratch_limit_and_beyond(fa):
    """131072 work items (1024 blocks x 32 row tiles x 4 column tiles at
    res (2, 256, 256) and 8 rows per item) fill the array exactly; one block
    more is refused before any launch."""
    say("noalloc: scratch limit")
    res = (2, 256, 256)
    b = mixed_batch(86, 1024, ncp_lo=2, ncp_hi=6)
    m, y, scale = _both(fa, b, res, 87, use_plan=False)
    t = fa.FATune(0, 0, 0, 0, 0, 0)
    need = fa.lib.fa_decode_residual_workspace(1024, fa._i32x3(res), ctypes.byref(t))
    assert need == fa.NOALLOC_SCRATCH_BYTES
    vp = ctypes.c_void_p(16)  # never dereferenced: the size check fails first
    st = fa.lib.fa_decode_residual_noalloc(vp, 1025, vp, vp, fa._i32x3(res), None, None, None,
                                           0, vp, 1.0, vp, vp, None)
    assert st == fa.FA_ERR_UNSUPPORTED
    # a smaller call after the largest one still matches
    b2 = mixed_batch(88, 5, ncp_lo=4, ncp_hi=20)
    _both(fa, b2, (64, 64, 64), 89)
