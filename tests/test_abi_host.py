"""The C-ABI library loads, exports every symbol include/fa.h declares, and
its host-only calls (validation, batch plan) behave as documented (CPU)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import fa_inputs as fi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fa.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fa_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def fa():
    import paper_2409_00184_amd as fa
    return fa


def test_exports_every_declared_symbol(fa):
    names = declared_functions()
    assert {"fa_decode_blocks", "fa_query_points", "fa_decode_backward"} <= set(names)
    raw = ctypes.CDLL(fa.library_path())
    for n in names:
        assert hasattr(raw, n), n
    assert fa.lib.fa_version() >= 10000


def test_struct_layouts(fa):
    assert fa.BLOCK_DTYPE.itemsize == 64
    assert fa.BLOCK_DTYPE.fields["knot_off"][1] == 24
    assert fa.BLOCK_DTYPE.fields["ctrl_off"][1] == 32
    assert fa.BLOCK_DTYPE.fields["scale"][1] == 40
    assert fa.WORK_DTYPE.itemsize == 12


def test_struct_layouts_match_header(fa, tmp_path):
    """sizeof/offsetof as a C compiler sees include/fa.h == the binding's."""
    src = tmp_path / "sz.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "fa.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n",'
        ' sizeof(fa_block), sizeof(fa_work), sizeof(fa_tune), sizeof(fa_ray),'
        ' sizeof(fa_render_params), offsetof(fa_render_params, light),'
        ' offsetof(fa_render_params, grad_min), offsetof(fa_tune, store),'
        ' offsetof(fa_block, scale)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = [fa.BLOCK_DTYPE.itemsize, fa.WORK_DTYPE.itemsize, ctypes.sizeof(fa.FATune), 32,
            ctypes.sizeof(fa.FARenderParams), fa.FARenderParams.light.offset,
            fa.FARenderParams.grad_min.offset, fa.FATune.store.offset,
            fa.BLOCK_DTYPE.fields["scale"][1]]
    assert got == want


def _desc(fa, b):
    return fa.host_descriptors(b.ncp, b.deg, b.knot_off, b.ctrl_off)


def test_validate_sets_uniform_flags(fa):
    b = fi.config_c2(nblocks=8)
    d = fa.fa_validate_blocks(_desc(fa, b), b.knots, b.ctrl.size)
    assert np.all(d["flags"] == 7)
    # a non-uniform interior knot clears that axis' flag only
    k = b.knots.copy()
    n, p = b.ncp[0], b.deg[0]
    k[int(b.knot_off[0]) + p[0] + 1] *= 0.5
    d = fa.fa_validate_blocks(_desc(fa, b), k, b.ctrl.size)
    assert d["flags"][0] == 6 and np.all(d["flags"][1:] == 7)


@pytest.mark.parametrize("case", ["ncp_small", "deg_mixed", "knot_oob", "ctrl_oob",
                                  "unclamped", "decreasing", "nan_knot", "misaligned"])
def test_validate_rejects(fa, case):
    b = fi.config_c2(nblocks=4)
    d = _desc(fa, b)
    k = b.knots.copy()
    nctrl = b.ctrl.size
    if case == "ncp_small":
        d["ncp"][1, 2] = d["degree"][1, 2]
    elif case == "deg_mixed":
        d["degree"][2, 1] = 1 if d["degree"][2, 0] != 1 else 2
    elif case == "knot_oob":
        d["knot_off"][3] = len(k)
    elif case == "ctrl_oob":
        nctrl = int(b.ctrl_off[3]) + 10
    elif case == "unclamped":
        k[int(b.knot_off[2])] = 0.01
    elif case == "decreasing":
        o = int(b.knot_off[1]) + int(b.deg[1, 0]) + 2
        k[o] = k[o - 1] - 0.01
    elif case == "nan_knot":
        k[int(b.knot_off[0]) + int(b.deg[0, 0]) + 1] = np.nan
    elif case == "misaligned":
        d["ctrl_off"][1] += 1
    before = d.copy()
    with pytest.raises(fa.FAError) as e:
        fa.fa_validate_blocks(d, k, nctrl)
    assert e.value.status == 1
    assert np.array_equal(d, before), "nothing is written on error"


def test_validate_unsupported(fa):
    b = fi.pack([(70, 8, 8)], [(3, 3, 3)],
                [[fi.clamped_uniform_knots(70, 3), fi.clamped_uniform_knots(8, 3),
                  fi.clamped_uniform_knots(8, 3)]], [np.zeros((70, 8, 8))])
    with pytest.raises(fa.FAError) as e:
        fa.fa_validate_blocks(_desc(fa, b), b.knots, b.ctrl.size)
    assert e.value.status == 2


def _plan(fa, d, res, rows, waves, grid):
    cap = len(d) * res[1] * ((res[2] + 63) // 64)
    work = np.zeros(cap, fa.WORK_DTYPE)
    off = np.zeros(cap + 1, np.int32)
    nw, ng = ctypes.c_int64(), ctypes.c_int32()
    t = fa.FATune(rows, waves, grid, 0, 0, 0)
    st = fa.lib.fa_plan_decode(d.ctypes.data, len(d), fa._i32x3(res), ctypes.byref(t),
                               work.ctypes.data, off.ctypes.data, cap, ctypes.byref(nw),
                               ctypes.byref(ng))
    return st, work[:nw.value], off[:ng.value + 1]


@pytest.mark.parametrize("res,rows,grid", [((64, 64, 64), 8, 768), ((17, 23, 70), 4, 7),
                                           ((5, 3, 2), 8, 1000)])
def test_plan_covers_every_item_once(fa, res, rows, grid):
    b = fi.config_c2(nblocks=37)
    d = fa.fa_validate_blocks(_desc(fa, b), b.knots, b.ctrl.size)
    st, work, off = _plan(fa, d, res, rows, 4, grid)
    assert st == 0
    nrowt = -(-res[1] // rows)
    ncolt = -(-res[2] // 64)
    assert len(work) == 37 * nrowt * ncolt
    assert off[0] == 0 and off[-1] == len(work) and np.all(np.diff(off) >= 0)
    assert len(off) - 1 == min(grid, len(work))
    # every voxel row of every block appears exactly once
    cover = np.zeros((37, res[1], ncolt), np.int32)
    for w in work:
        assert 0 < w["nrows"] <= rows and w["row0"] % rows == 0 and w["col0"] % 64 == 0
        cover[w["block"], w["row0"]:w["row0"] + w["nrows"], w["col0"] // 64] += 1
    assert np.all(cover == 1)


def test_plan_balances_uneven_blocks(fa):
    """LPT on the cost model: the heaviest workgroup carries at most the
    mean load plus one item (the classic LPT guarantee is 4/3 of optimal)."""
    b = fi.config_c2(nblocks=512)
    d = fa.fa_validate_blocks(_desc(fa, b), b.knots, b.ctrl.size)
    st, work, off = _plan(fa, d, (64, 64, 64), 8, 4, 768)
    assert st == 0
    counts = np.diff(off)
    assert counts.max() - counts.min() <= 2


def test_plan_rejects_small_capacity(fa):
    b = fi.config_c2(nblocks=4)
    d = fa.fa_validate_blocks(_desc(fa, b), b.knots, b.ctrl.size)
    work = np.zeros(3, fa.WORK_DTYPE)
    off = np.zeros(4, np.int32)
    nw, ng = ctypes.c_int64(), ctypes.c_int32()
    st = fa.lib.fa_plan_decode(d.ctypes.data, 4, fa._i32x3((64, 64, 64)), None,
                               work.ctypes.data, off.ctypes.data, 3, ctypes.byref(nw),
                               ctypes.byref(ng))
    assert st == 1


def test_hot_calls_reject_bad_arguments_without_launch(fa):
    """Argument errors return before any launch (no GPU is touched here)."""
    L = fa.lib
    vp = ctypes.c_void_p(16)  # never dereferenced: the checks fail first
    r = fa._i32x3((64, 64, 64))
    assert L.fa_decode_blocks(None, 1, vp, vp, 0, r, 15, None, None, None, 0, vp, None) == 1
    assert L.fa_decode_blocks(vp, 0, vp, vp, 0, r, 15, None, None, None, 0, vp, None) == 1
    assert L.fa_decode_blocks(vp, 1, vp, vp, 0, r, 0, None, None, None, 0, vp, None) == 1
    assert L.fa_decode_blocks(vp, 1, vp, vp, 7, r, 15, None, None, None, 0, vp, None) == 1
    assert L.fa_decode_blocks(vp, 1, vp, vp, 0, fa._i32x3((1, 4, 4)), 15, None, None, None, 0,
                              vp, None) == 1
    assert L.fa_decode_blocks(vp, 1, vp, vp, 0, fa._i32x3((300, 4, 4)), 15, None, None, None,
                              0, vp, None) == 2
    assert L.fa_decode_blocks(vp, 1, vp, vp, 0, r, 15, None, vp, None, 0, vp, None) == 1
    # interleaved records need all four channels; unknown mask bits are rejected
    assert L.fa_decode_blocks(vp, 1, vp, vp, 0, r, 1 | fa.OUT_INTERLEAVED, None, None, None, 0,
                              vp, None) == 1
    assert L.fa_decode_blocks(vp, 1, vp, vp, 0, r, 15 | 0x200, None, None, None, 0, vp,
                              None) == 1
    assert L.fa_query_points(vp, 1, vp, fa._i32x3((1, 1, 1)), fa._f32x3((0, 0, 0)),
                             fa._f32x3((1, 0, 1)), vp, vp, 0, vp, 5, 15, vp, None) == 1
    assert L.fa_query_rays(vp, 1, vp, fa._i32x3((1, 1, 1)), fa._f32x3((0, 0, 0)),
                           fa._f32x3((1, 1, 1)), vp, vp, 0, vp, 0, 4, 4, 15, vp, None) == 1
    assert L.fa_query_rays(vp, 1, vp, fa._i32x3((1, 1, 1)), fa._f32x3((0, 0, 0)),
                           fa._f32x3((1, 1, 1)), vp, vp, 0, vp, 4, 4, 4, 0, vp, None) == 1
    rp = fa.FARenderParams(16, 0.98, -1.0, 1.0, 2, (ctypes.c_float * 3)(0, 0, 1), 0.3, 0.6,
                           0.3, 32.0, 1e-6)
    args = lambda w, h, p: (vp, 1, vp, fa._i32x3((1, 1, 1)), fa._f32x3((0, 0, 0)),
                            fa._f32x3((1, 1, 1)), vp, vp, 0, vp, w, h, ctypes.byref(p), vp, vp,
                            None)
    for bad in (dict(samples=0), dict(tf_size=1), dict(tf_hi=-1.0), dict(grad_min=-1.0),
                dict(tf_lo=float("nan"))):
        q = fa.FARenderParams.from_buffer_copy(rp)
        for k, v in bad.items():
            setattr(q, k, v)
        assert L.fa_render_rays(*args(4, 4, q)) == 1, bad
    assert L.fa_render_rays(*args(0, 4, rp)) == 1
    assert L.fa_render_rays(*args(4, -1, rp)) == 1
    a = list(args(4, 4, rp))
    a[13] = None  # no transfer function
    assert L.fa_render_rays(*a) == 1
    assert L.fa_decode_backward(vp, 1, vp, fa._i32x3((64, 65, 64)), 1, vp, vp, None) == 2
    assert L.fa_decode_backward(vp, 1, vp, r, 16, vp, vp, None) == 1
    assert L.fa_quantize_blocks(vp, 1, vp, 0, vp, None) == 1
    # Adam step: every argument error returns before the device is touched
    ok = dict(lr=0.05, b1=0.9, b2=0.999, eps=1e-8, wd=0.0)
    adam = lambda p, n, **kw: L.fa_adam_step(p, vp, vp, vp, n, kw["lr"], kw["b1"], kw["b2"],
                                             kw["eps"], kw["wd"], vp, None)
    assert adam(None, 8, **ok) == 1
    assert L.fa_adam_step(vp, vp, vp, vp, 8, 0.05, 0.9, 0.999, 1e-8, 0.0, None, None) == 1
    assert adam(vp, -1, **ok) == 1
    for k, v in (("b1", 1.0), ("b1", -0.1), ("b2", 1.0), ("eps", 0.0), ("eps", float("inf")),
                 ("lr", float("nan")), ("wd", float("inf"))):
        assert adam(vp, 8, **dict(ok, **{k: v})) == 1, (k, v)
    # the loss from per-block sums: null pointers, no blocks, a count that is
    # not positive and finite
    assert L.fa_mse_loss(None, 4, 8.0, vp, None) == 1
    assert L.fa_mse_loss(vp, 4, 8.0, None, None) == 1
    assert L.fa_mse_loss(vp, 0, 8.0, vp, None) == 1
    for c in (0.0, -1.0, float("inf"), float("nan")):
        assert L.fa_mse_loss(vp, 4, c, vp, None) == 1, c
    # the allocation-free residual: bad arguments, then a batch whose work
    # items exceed its fixed scratch array, both before any device call
    assert L.fa_decode_residual_noalloc(None, 1, vp, vp, r, None, None, None, 0, vp, 1.0, vp,
                                        vp, None) == 1
    assert L.fa_decode_residual_noalloc(vp, 1, vp, vp, r, None, None, None, 0, vp,
                                        float("inf"), vp, vp, None) == 1
    assert L.fa_decode_residual_noalloc(vp, 20000, vp, vp, r, None, None, None, 0, vp, 1.0, vp,
                                        vp, None) == 2
    assert L.fa_decode_blocks_plain(vp, 1, vp, None, r, 15, vp, None) == 1


def test_uniform_layout_matches_input_packing(fa):
    """fa_uniform_layout: knots equal the clamped uniform knots of the input
    generator, lattices at 64-element offsets, descriptors validate."""
    ncp = np.array([[5, 7, 9], [4, 4, 4], [33, 12, 64]], np.int32)
    deg = np.array([[3, 3, 3], [2, 2, 2], [3, 3, 3]], np.int32)
    nk, nc = ctypes.c_int64(0), ctypes.c_int64(0)
    desc = np.zeros(3, fa.BLOCK_DTYPE)
    knots = np.zeros(1000, np.float32)
    assert fa.lib.fa_uniform_layout(3, ncp.ctypes.data, deg.ctypes.data, desc.ctypes.data,
                                    knots.ctypes.data, knots.size, ctypes.byref(nk),
                                    ctypes.byref(nc)) == 0
    b = fi.pack(ncp, deg, [[fi.clamped_uniform_knots(n, d[0]) for n in c]
                           for c, d in zip(ncp, deg)], [np.zeros(c) for c in ncp])
    assert nk.value == b.knots.size
    assert np.array_equal(knots[:nk.value], b.knots)
    assert np.array_equal(desc["ctrl_off"], b.ctrl_off)
    assert np.array_equal(desc["knot_off"], b.knot_off)
    assert nc.value >= b.ctrl_off[-1] + np.prod(ncp[-1])
    fa.fa_validate_blocks(desc.copy(), knots[:nk.value], nc.value)
    # capacity and shape errors
    assert fa.lib.fa_uniform_layout(3, ncp.ctypes.data, deg.ctypes.data, None,
                                    knots.ctypes.data, 10, ctypes.byref(nk),
                                    ctypes.byref(nc)) == 1
    bad = ncp.copy()
    bad[1, 0] = 2
    assert fa.lib.fa_uniform_layout(3, bad.ctypes.data, deg.ctypes.data, None, None, 0,
                                    ctypes.byref(nk), ctypes.byref(nc)) == 1


def test_ncp_select_agrees_with_oracle_rule(fa):
    """fa_ncp_select on seeded error maps == the oracle's Eq. 4 rule."""
    from oracle import adaptive as ad
    g = np.random.Generator(np.random.PCG64(5))
    errs = np.sort(g.uniform(0, 1, (50, 12, 2)), axis=1)[:, ::-1].astype(np.float32)
    errs[7] = 0.5  # ties with the bound
    for metric in (0, 1):
        for bound in (0.05, 0.3, 0.5, 0.99, 2.0):
            ns, cx = fa.ncp_select(errs, 5, bound, metric)
            for b in range(50):
                assert (ns[b], cx[b]) == ad.select_ncp(errs[b].astype(np.float64), 5,
                                                       np.float32(bound), metric)


def test_search_arguments_rejected_without_launch(fa):
    r = fa._i32x3((16, 16, 16))
    vp = ctypes.c_void_p(16)
    assert fa.lib.fa_ncp_search_workspace(4, r, 3, 16) > 4 * 16 ** 3 * 4
    assert fa.lib.fa_ncp_search_workspace(0, r, 3, 16) == -1
    ws = fa.lib.fa_ncp_search_workspace(4, r, 3, 16)
    assert fa.lib.fa_ncp_search(vp, 4, r, 3, 5, 17, vp, ctypes.c_void_p(256), ws, None) == 1
    assert fa.lib.fa_ncp_search(vp, 4, r, 3, 3, 16, vp, ctypes.c_void_p(256), ws, None) == 1
    assert fa.lib.fa_ncp_search(vp, 4, r, 3, 5, 16, vp, ctypes.c_void_p(256), ws - 1, None) == 1
    assert fa.lib.fa_ncp_search(vp, 4, r, 3, 5, 16, vp, ctypes.c_void_p(257), ws, None) == 1
    assert fa.lib.fa_ncp_search(vp, 4, r, 4, 5, 16, vp, ctypes.c_void_p(256), ws, None) == 2
    big = fa._i32x3((80, 80, 80))
    assert fa.lib.fa_ncp_search(vp, 4, big, 3, 5, 70, vp, ctypes.c_void_p(256),
                                fa.lib.fa_ncp_search_workspace(4, big, 3, 70), None) == 2
    wide = fa._i32x3((80, 16, 16))
    assert fa.lib.fa_ncp_search(vp, 4, wide, 3, 5, 16, vp, ctypes.c_void_p(256),
                                fa.lib.fa_ncp_search_workspace(4, wide, 3, 16), None) == 2
    fws = fa.lib.fa_fit_workspace(4, r, 16)
    assert fws == (4 * 16 * 16 * 16 + 4 * 3 * 64 * 64) * 8  # T slices + per-axis pseudo-inverses
    assert fa.lib.fa_fit_blocks(vp, 1, vp, fa._i32x3((64, 65, 64)), vp, vp, 16,
                                ctypes.c_void_p(256), 1 << 30, None) == 2
    assert fa.lib.fa_fit_blocks(vp, 1, vp, r, vp, vp, 65, ctypes.c_void_p(256), 1 << 30,
                                None) == 2
    assert fa.lib.fa_fit_blocks(None, 1, vp, r, vp, vp, 16, ctypes.c_void_p(256), fws,
                                None) == 1
    assert fa.lib.fa_fit_blocks(vp, 4, vp, r, vp, vp, 16, ctypes.c_void_p(256), fws - 1,
                                None) == 1
    assert fa.lib.fa_fit_blocks(vp, 4, vp, r, vp, vp, 16, ctypes.c_void_p(264), fws,
                                None) == 1
    assert fa.lib.fa_model_errors(vp, 1, vp, vp, 0, r, vp, vp, vp, 1, None) == 1
