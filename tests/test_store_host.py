"""Micro-model file format (Eq. 2) and the host LRU cache of Alg. 2 (CPU)."""
import collections
import ctypes
import struct

import numpy as np
import pytest

import fa_inputs as fi


@pytest.fixture(scope="module")
def fa():
    import paper_2409_00184_amd as fa
    return fa


def _batch(fa, seed, nb, degs=(2, 3), ncps=(4, 6, 9, 17, 32)):
    g = fi.rng(seed)
    ncp = g.choice(ncps, nb)
    deg = g.choice(degs, nb)
    ncp = np.maximum(ncp, deg + 1)
    b = fi.pack(np.repeat(ncp[:, None], 3, 1), np.repeat(deg[:, None], 3, 1),
                [[fi.clamped_uniform_knots(n, p)] * 3 for n, p in zip(ncp, deg)],
                [g.normal(size=(n, n, n)) for n in ncp])
    desc = fa.host_descriptors(b.ncp, b.deg, b.knot_off, b.ctrl_off)
    return b, desc


def test_record_sizes_follow_eq2(fa, tmp_path):
    b, desc = _batch(fa, 80, 12)
    path = tmp_path / "m.fam"
    fa.store_write(path, desc, b.knots, b.ctrl)
    raw = path.read_bytes()
    assert raw[:4] == b"FAM1"
    version, nblocks, zero = struct.unpack("<iii", raw[4:16])
    assert (version, nblocks, zero) == (1, 12, 0)
    idx = np.frombuffer(raw[16:16 + 16 * 12], np.int64).reshape(12, 2)
    for k in range(12):
        n, p = int(b.ncp[k, 0]), int(b.deg[k, 0])
        off, size = idx[k]
        assert size == 1 + ((n + p) * 3 + n ** 3) * 4  # Eq. 2
        rec = raw[off:off + size]
        assert rec[0] == p
        kn = np.frombuffer(rec[1:1 + 12 * (n + p)], np.float32).reshape(3, n + p)
        full = b.knots[b.knot_off[k]:b.knot_off[k] + 3 * (n + p + 1)].reshape(3, n + p + 1)
        assert np.array_equal(kn, full[:, :-1]) and np.all(full[:, -1] == 1.0)
        P = np.frombuffer(rec[1 + 12 * (n + p):], np.float32)
        assert np.array_equal(P, b.ctrl[b.ctrl_off[k]:b.ctrl_off[k] + n ** 3])
    assert len(raw) == idx[-1].sum()


def test_roundtrip_and_lru_against_reference(fa, tmp_path):
    """Random access sequences: hits, misses, evictions and slot contents
    equal those of a reference LRU (hit refreshes recency)."""
    b, desc = _batch(fa, 81, 40)
    path = tmp_path / "m.fam"
    fa.store_write(path, desc, b.knots, b.ctrl)
    cap = 7
    s = fa.Store(path, cache_blocks=cap, pinned=False)
    assert s.nblocks == 40 and np.array_equal(s.ncp, b.ncp[:, 0])
    ref = collections.OrderedDict()
    hits = misses = ev = 0
    g = fi.rng(82)
    for frame in range(30):
        ids = g.choice(40, g.integers(1, 12), replace=False) if frame % 3 else \
            g.integers(0, 10, 5)  # repeats inside a frame too
        slots, st = s.fetch(ids)
        for i, k in zip(ids, slots):
            if i in ref:
                hits += 1
                ref.move_to_end(i)
            else:
                misses += 1
                if len(ref) == cap:
                    ref.popitem(last=False)
                    ev += 1
                ref[i] = True
        assert (st["hits"], st["misses"], st["evictions"]) == (hits, misses, ev)
        # the last id of the frame is resident and its slot holds its data
        blk, kn, P = s.slot(slots[-1])
        assert blk == ids[-1]
        n, p = int(b.ncp[blk, 0]), int(b.deg[blk, 0])
        assert np.array_equal(P.reshape(-1), b.ctrl[b.ctrl_off[blk]:b.ctrl_off[blk] + n ** 3])
        assert np.array_equal(kn.reshape(-1),
                              b.knots[b.knot_off[blk]:b.knot_off[blk] + 3 * (n + p + 1)])
    s.close()


def test_store_rejects_bad_input(fa, tmp_path):
    b, desc = _batch(fa, 83, 3)
    bad = desc.copy()
    bad["ncp"][1] = [5, 6, 5]  # Eq. 2 has one NCP per block
    with pytest.raises(fa.FAError):
        fa.store_write(tmp_path / "x.fam", bad, b.knots, b.ctrl)
    (tmp_path / "junk.fam").write_bytes(b"FAM2" + bytes(40))
    with pytest.raises(fa.FAError):
        fa.Store(tmp_path / "junk.fam", pinned=False)
    with pytest.raises(fa.FAError):
        fa.Store(tmp_path / "missing.fam", pinned=False)
    path = tmp_path / "m.fam"
    fa.store_write(path, desc, b.knots, b.ctrl)
    raw = bytearray(path.read_bytes())
    raw[16 + 8:16 + 16] = struct.pack("<q", 12345)  # a record size no NCP gives
    (tmp_path / "t.fam").write_bytes(bytes(raw))
    with pytest.raises(fa.FAError):
        fa.Store(tmp_path / "t.fam", pinned=False)
    s = fa.Store(path, pinned=False, cache_blocks=2)
    with pytest.raises(fa.FAError):
        s.fetch([0, 3])
    # staging needs page-locked slots: refused before any copy
    ids = np.zeros(1, np.int32)
    vp = ctypes.c_void_p(256)
    assert fa.lib.fa_store_stage(s.h, ids.ctypes.data, 1, vp, vp, 1 << 20, vp, 1 << 20, None,
                                 None) == 1
    s.close()


def test_truncated_file_is_refused_at_open(fa, tmp_path):
    """A record that reaches past the end of the file is refused by
    fa_store_open (before any fetch can read it into the cache)."""
    b, desc = _batch(fa, 84, 6)
    path = tmp_path / "m.fam"
    fa.store_write(path, desc, b.knots, b.ctrl)
    raw = path.read_bytes()
    (tmp_path / "cut.fam").write_bytes(raw[:-7])
    with pytest.raises(fa.FAError) as e:
        fa.Store(tmp_path / "cut.fam", pinned=False)
    assert e.value.status == fa.FA_ERR_INVALID_ARG
    # an index entry pointing into the header is refused as well
    bad = bytearray(raw)
    bad[16:24] = struct.pack("<q", 4)
    (tmp_path / "hdr.fam").write_bytes(bytes(bad))
    with pytest.raises(fa.FAError):
        fa.Store(tmp_path / "hdr.fam", pinned=False)


def test_failed_fetch_leaves_cache_unchanged(fa, tmp_path):
    """A record with malformed knots fails its fetch without touching the
    LRU: later fetches (with evictions) behave as if it was never asked for."""
    b, desc = _batch(fa, 85, 8)
    path = tmp_path / "m.fam"
    fa.store_write(path, desc, b.knots, b.ctrl)
    raw = bytearray(path.read_bytes())
    idx = np.frombuffer(bytes(raw[16:16 + 16 * 8]), np.int64).reshape(8, 2)
    bad_id = 5
    off = int(idx[bad_id, 0])
    # first x knot of block 5 set to 0.5: no longer clamped at 0
    raw[off + 1:off + 5] = struct.pack("<f", 0.5)
    (tmp_path / "k.fam").write_bytes(bytes(raw))
    s = fa.Store(tmp_path / "k.fam", cache_blocks=2, pinned=False)
    s.fetch([0])
    with pytest.raises(fa.FAError) as e:
        s.fetch([bad_id])
    assert e.value.status == fa.FA_ERR_INVALID_ARG
    # the failed fetch counted nothing and took no slot: 0 is still cached
    slots, st = s.fetch([0, 1, 2, 3])
    assert (st["hits"], st["misses"], st["evictions"]) == (1, 4, 2)
    for k, sl in zip([2, 3], slots[2:]):
        blk, kn, P = s.slot(sl)
        n = int(b.ncp[k, 0])
        assert blk == k
        assert np.array_equal(P.reshape(-1), b.ctrl[b.ctrl_off[k]:b.ctrl_off[k] + n ** 3])
    s.close()


def test_degree_above_kernel_limit_is_unsupported(fa, tmp_path):
    """Degrees the kernels do not take are refused when written and when a
    file holding one is opened."""
    n, p = 6, 4
    kn = np.concatenate([np.zeros(p + 1), np.arange(1, n - p) / (n - p), np.ones(p + 1)])
    knots = np.tile(kn.astype(np.float32), 3)
    ctrl = np.zeros(n ** 3, np.float32)
    desc = np.zeros(1, fa.BLOCK_DTYPE)
    desc["ncp"][0] = n
    desc["degree"][0] = p
    with pytest.raises(fa.FAError) as e:
        fa.store_write(tmp_path / "p4.fam", desc, knots, ctrl)
    assert e.value.status == fa.FA_ERR_UNSUPPORTED
    # the same record written by hand (Eq. 2 bytes) is refused at open
    rec = bytes([p]) + b"".join(kn[:-1].astype(np.float32).tobytes() for _ in range(3)) + \
        ctrl.tobytes()
    head = b"FAM1" + struct.pack("<iii", 1, 1, 0) + struct.pack("<qq", 32, len(rec))
    (tmp_path / "p4h.fam").write_bytes(head + rec)
    with pytest.raises(fa.FAError) as e:
        fa.Store(tmp_path / "p4h.fam", pinned=False)
    assert e.value.status == fa.FA_ERR_UNSUPPORTED


def test_write_refuses_unclamped_or_decreasing_knots(fa, tmp_path):
    b, desc = _batch(fa, 86, 2, degs=(3,), ncps=(9,))
    for pos, val in ((1, 0.25), (6, 0.1)):  # a leading zero moved; a decreasing interior knot
        kn = b.knots.copy()
        kn[b.knot_off[1] + pos] = val
        with pytest.raises(fa.FAError) as e:
            fa.store_write(tmp_path / "bad.fam", desc, kn, b.ctrl)
        assert e.value.status == fa.FA_ERR_INVALID_ARG
