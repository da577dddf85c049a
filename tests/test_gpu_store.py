"""Visible cells, storage and staging on the GPU (Alg. 2): the visible set of
a view equals the oracle's, and rendering from micro-models staged through
the file + host LRU cache equals rendering from the resident batch."""
import numpy as np
import pytest
import torch

import fa_inputs as fi
from gpu_util import say
from oracle import visibility

pytestmark = pytest.mark.gpu

SHADE = dict(light=(0.0, 0.6, 0.8), ka=0.3, kd=0.6, ks=0.3, shininess=16.0)


@pytest.fixture(scope="module")
def fa():
    import paper_2409_00184_amd as fa
    assert torch.cuda.is_available()
    return fa


@pytest.mark.parametrize("nb,origin,extent,w,h,S,fov", [
    ((16, 16, 16), (0, 0, 0), (1, 1, 1), 64, 48, 128, 24.0),
    ((5, 3, 7), (-0.1, 0.2, 0.05), (1.3, 0.7, 0.9), 37, 11, 61, 40.0)])
def test_visible_cells_match_oracle(fa, nb, origin, extent, w, h, S, fov):
    say("visible", nb, w, h, S)
    rays = fi.render_rays(21, w, h, fov_v_deg=fov)
    flags = fa.visible_cells(torch.as_tensor(rays).cuda(), w, h, S, nb, origin, extent)
    ref = visibility.visible_cells(rays, S, nb, origin, extent)
    got = flags.cpu().numpy()
    say("  visible", int(got.sum()), "of", got.size)
    assert np.array_equal(got, ref)
    assert 0 < ref.sum() < ref.size


def _cubic_domain(seed, nb=4, p=3):
    g = fi.rng(seed)
    k, phi = fi.sinusoid_params(g)
    ncp = g.integers(5, 21, nb ** 3)
    kl, lat = [], []
    for b in range(nb ** 3):
        bx, by, bz = b // (nb * nb), (b // nb) % nb, b % nb
        n = int(ncp[b])
        ts = [fi.clamped_uniform_knots(n, p)] * 3
        kl.append(ts)
        lat.append(fi.sinusoid_lattice(k, phi, ts[0], ts[1], ts[2], (n,) * 3, (p,) * 3,
                                       offset=(bx, by, bz)))
    return fi.pack(np.repeat(ncp[:, None], 3, 1), np.full((nb ** 3, 3), p), kl, lat)


def test_stage_then_render_equals_resident_render(fa, tmp_path):
    say("stage + render")
    nb = 4
    b = _cubic_domain(22, nb)
    full = fa.MicroModels.from_batch(b)
    path = tmp_path / "dom.fam"
    fa.store_write(path, full.host_desc, b.knots, b.ctrl)
    store = fa.Store(path, cache_blocks=9, pinned=True)
    tf = torch.as_tensor(fi.transfer_function(23)).cuda()
    w, h, S = 48, 40, 160
    all_cells = torch.as_tensor(fi.identity_cells(nb ** 3)).cuda()
    frames = [fi.render_rays(s, w, h, fov_v_deg=20.0) for s in (24, 24, 25)]
    prev = None
    for f, rays_np in enumerate(frames):
        rays = torch.as_tensor(rays_np).cuda()
        flags = fa.visible_cells(rays, w, h, S, (nb,) * 3, (0, 0, 0), (1, 1, 1))
        ids = np.nonzero(flags.cpu().numpy())[0].astype(np.int32)
        staged, st = store.stage(ids)
        boc = np.full(nb ** 3, -1, np.int32)
        boc[ids] = np.arange(ids.size, dtype=np.int32)
        args = (w, h, tf, (nb,) * 3, (0, 0, 0), (1, 1, 1))
        img_s = fa.render(staged, rays, *args, torch.as_tensor(boc).cuda(), S, opacity_max=0.95,
                          tf_range=(-4.0, 4.0), **SHADE)
        img_f = fa.render(full, rays, *args, all_cells, S, opacity_max=0.95,
                          tf_range=(-4.0, 4.0), **SHADE)
        torch.cuda.synchronize()
        say("  frame", f, "visible", ids.size, st)
        assert torch.equal(img_s, img_f)
        assert ids.size > 9  # more visible blocks than cache slots: evictions while staging
        assert st["evictions"] > 0
        if f == 1:  # the same view again: only the blocks evicted meanwhile are re-read
            assert st["misses"] - prev["misses"] <= ids.size
            assert st["bytes_h2d"] - prev["bytes_h2d"] > 0
        prev = st
    store.close()


def test_fetch_after_stage_keeps_the_staged_batch(fa, tmp_path):
    """A fetch right after a stage refills the cache slots the stage's gather
    reads; it waits for that gather, so the staged batch holds the lattices
    and knots of the staged blocks."""
    say("stage then fetch")
    nb = 3
    b = _cubic_domain(26, nb)
    full = fa.MicroModels.from_batch(b)
    path = tmp_path / "dom.fam"
    fa.store_write(path, full.host_desc, b.knots, b.ctrl)
    store = fa.Store(path, cache_blocks=6, pinned=True)
    ids = np.array([4, 0, 13, 7, 21, 2], np.int32)
    staged, _ = store.stage(ids)
    # every slot refilled with other blocks, no synchronisation in between
    store.fetch(np.array([k for k in range(nb ** 3) if k not in set(ids)][:12], np.int32))
    torch.cuda.synchronize()
    desc = staged.desc.cpu().numpy().view(fa.BLOCK_DTYPE)[:ids.size]
    kn = staged.knots.cpu().numpy()
    P = staged.ctrl.cpu().numpy()
    for i, k in enumerate(ids):
        n, p = int(b.ncp[k, 0]), int(b.deg[k, 0])
        d = desc[i]
        assert int(d["ncp"][0]) == n
        assert np.array_equal(P[d["ctrl_off"]:d["ctrl_off"] + n ** 3],
                              b.ctrl[b.ctrl_off[k]:b.ctrl_off[k] + n ** 3])
        kl = 3 * (n + p + 1)
        assert np.array_equal(kn[d["knot_off"]:d["knot_off"] + kl],
                              b.knots[b.knot_off[k]:b.knot_off[k] + kl])
    store.close()
