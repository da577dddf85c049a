"""Autotuner of the batched decode (row a0): tile and schedule search.

For a batch of micro-models, a grid resolution, a channel mask and a
lattice dtype it times every candidate (rows per work item, waves per
workgroup, persistent grid size, kernel) through fa_plan_decode and
fa_decode_blocks with HIP events, and keeps the fastest.  Results are
cached in a JSON file keyed by a signature of the batch (histogram of NCP*
and degree), so a later process with the same kind of batch skips the
search.  Timing only chooses among schedules; every candidate computes the
same result (the GPU tests check that schedules agree bit for bit).
"""
import hashlib
import json
import os

import numpy as np
import torch

from . import Plan, decode, nch

CACHE = os.environ.get("FA_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "fa_tune.json"))
# Results of this search on MI355X for the standard workloads, shipped with
# the package (the same format as the cache): a process whose batch matches
# one of them takes that schedule without searching, so every run of such a
# workload executes the same schedule.
TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json")

def _candidates():
    out = []
    for rows in (4, 8, 16):
        for waves in (2, 4, 8):
            if waves > rows:
                continue
            for grid in (512, 768, 1024, 1536, 2048, 1 << 20):
                for slab in (4096, 6144, 8192):
                    for store in (0, 1):
                        out.append((rows, waves, grid, 0, slab, store))
    return out


# (rows per item, waves, persistent grid, kernel, LDS slab floats, store kind)
CANDIDATES = _candidates()


def signature(models, res, mask, dtype):
    """Hash of the multiset of (NCP_x, NCP_y, NCP_z, degree) rows of the
    batch, the resolution, mask, dtype and the device's architecture and
    compute-unit count (the marketing name differs between otherwise equal
    boards)."""
    d = models.host_desc
    rows = np.concatenate([d["ncp"], d["degree"][:, :1]], axis=1).astype(np.int32)
    uniq, cnt = np.unique(rows, axis=0, return_counts=True)
    h = hashlib.sha1()
    h.update(uniq.tobytes())
    h.update(cnt.astype(np.int64).tobytes())
    props = torch.cuda.get_device_properties(models.device)
    arch = getattr(props, "gcnArchName", "").split(":")[0]
    h.update(repr((tuple(int(r) for r in res), int(mask), dtype, arch,
                   int(props.multi_processor_count))).encode())
    return h.hexdigest()[:20]


def _load_json(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _load_cache():
    return _load_json(CACHE)


def _save_cache(c):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def _median_launch_ms(fn, reps, warmup=2):
    for _ in range(warmup):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = sorted(a.elapsed_time(b) for a, b in ev)
    return t[len(t) // 2]


def time_plan(models, res, mask, dtype, plan, out, reps=9):
    """Median duration of single launches (each bracketed by its own events)."""
    return _median_launch_ms(lambda: decode(models, res, mask, dtype, plan=plan, out=out), reps)


def time_graph(models, res, mask, dtype, plan, out, reps=15):
    """Median duration of replays of a captured graph of one launch (the way
    a caller that captures the decode runs it)."""
    from . import capture
    g, _ = capture(lambda: decode(models, res, mask, dtype, plan=plan, out=out))
    ms = _median_launch_ms(g.replay, reps)
    del g
    return ms


def tune(models, res, mask=15, dtype="f32", candidates=None, use_cache=True, kernels=(0,),
         verbose=False, top=4):
    """Return (best Plan, report list of (candidate, ms)).  With use_cache,
    a schedule found earlier for the same kind of batch (the user cache,
    then the table shipped with the package) is returned without searching;
    a search that runs stores its result in the user cache."""
    sig = signature(models, res, mask, dtype)
    if use_cache:
        for known in (_load_cache(), _load_json(TABLE)):
            if sig in known:
                c = known[sig]["best"]
                return Plan(models, res, *c), [(tuple(c), known[sig]["ms"])]
    cands = [c for c in (candidates or CANDIDATES) if c[3] in kernels]
    # planar [nb][nch][res] or interleaved [nb][res][4]: the same number of floats
    out = torch.empty((models.nblocks, nch(mask)) + tuple(res), dtype=torch.float32,
                      device=models.device)
    report = []
    best = None
    for c in cands:
        try:
            plan = Plan(models, res, *c)
            ms = time_plan(models, res, mask, dtype, plan, out)
        except RuntimeError as e:  # unsupported combination for this kernel
            if verbose:
                print("skip", c, e)
            continue
        report.append((c, ms))
        if verbose:
            print("tune", c, f"{ms:.4f} ms")
        if best is None or ms < best[1]:
            best = (c, ms, plan)
    if best is None:
        raise RuntimeError("no decode schedule candidate ran")
    # re-time the leaders as graph replays and keep the fastest of those
    leaders = sorted(report, key=lambda r: r[1])[:top]
    best = None
    for c, _ in leaders:
        plan = Plan(models, res, *c)
        ms = time_graph(models, res, mask, dtype, plan, out)
        if best is None or ms < best[1]:
            best = (c, ms, plan)
    cache = _load_cache()
    cache[sig] = {"best": list(best[0]), "ms": best[1]}
    _save_cache(cache)
    return best[2], report
