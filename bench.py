#!/usr/bin/env python3
"""Throughput of the micro-model decode/query path on one MI355X.

Headline workload (C2): batched decode of 512 micro-models with NCP* per axis
drawn from {8,12,16,24,32} and degree from {2,3}, each decoded to a 64^3
voxel grid (value + 3 gradient channels, FP32), as one launch replayed from a
captured HIP graph, schedule picked by the autotuner.  The default run
prints the C2 line with the ray-sample query (C3), the fit iteration (C4)
and the BF16/FP16 precision configuration (C5) as sub-records.

One step = one decode of the whole batch with inputs resident in HBM.
Prints one JSON line (rank 0) with the throughput, the roofline of the
dominant kernel (HIP events on the launch stream), the plain
one-launch-per-block baseline, the error against the FP64 oracle on a seeded
sample, and the FP64 oracle's own rate on a bounded sample of the workload
(host cores).  Other workloads (--workload c1|c3|c4|c5) print the same kind
of line for the other configurations.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "decoded voxels/sec (value+grad), batched vs plain, % HBM/MFMA roofline"
KERNEL_SOURCES = {
    "decode_sep": ["paper_2409_00184_amd/csrc/fa_decode.hip",
                   "paper_2409_00184_amd/csrc/fa_device.hpp"],
    "query": ["paper_2409_00184_amd/csrc/fa_query.hip", "paper_2409_00184_amd/csrc/fa_eval.hpp",
              "paper_2409_00184_amd/csrc/fa_device.hpp"],
    "decode_mfma": ["paper_2409_00184_amd/csrc/fa_mfma.hip",
                    "paper_2409_00184_amd/csrc/fa_device.hpp"],
    "adjoint": ["paper_2409_00184_amd/csrc/fa_adjoint.hip",
                "paper_2409_00184_amd/csrc/fa_adjoint_mfma.hip",
                "paper_2409_00184_amd/csrc/fa_device.hpp"],
    "ncp_search": ["paper_2409_00184_amd/csrc/fa_fit.hip",
                   "paper_2409_00184_amd/csrc/fa_decode.hip",
                   "paper_2409_00184_amd/csrc/fa_device.hpp"],
    "fit": ["paper_2409_00184_amd/csrc/fa_fit.hip", "paper_2409_00184_amd/csrc/fa_device.hpp"],
    "fit_decode": ["paper_2409_00184_amd/csrc/fa_fit.hip",
                   "paper_2409_00184_amd/csrc/fa_adjoint.hip",
                   "paper_2409_00184_amd/csrc/fa_decode.hip",
                   "paper_2409_00184_amd/csrc/fa_device.hpp"],
    "render": ["paper_2409_00184_amd/csrc/fa_render.hip", "paper_2409_00184_amd/csrc/fa_eval.hpp",
               "paper_2409_00184_amd/csrc/fa_device.hpp"],
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(kernel):
    h = hashlib.sha1()
    for p in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def traffic_from_profiles(kernel, workload, profiles=None):
    """HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE and
    WRITE_SIZE (scaled by the copy-kernel calibration), from
    profiles/<kernel>_<workload>_traffic.json, if taken on this exact kernel
    source; else None."""
    p = os.path.join(profiles or os.path.join(ROOT, "profiles"),
                     f"{kernel}_{workload}_traffic.json")
    try:
        with open(p) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash(kernel):
        return None
    return t.get("hbm_bytes_per_launch")


def timed_steps(fn, steps, warmup, stream):
    """W untimed steps, then K timed steps between synchronisations; HIP
    events on `stream` around every step give the per-launch duration."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = [a.elapsed_time(b) for a, b in evs]
    return wall * 1e3 / steps, sum(ev_ms) / len(ev_ms), min(ev_ms)


def timed_launches(fn, reps, steps, warmup, stream):
    """Average duration of one launch of fn when launched back to back: a
    HIP graph of reps calls, replayed W + K times with HIP events around each
    of the K replays (no host latency inside the timed region)."""
    import torch

    import paper_2409_00184_amd as fa

    def many():
        for _ in range(reps):
            fn()

    g, _ = fa.capture(many)
    ms, ev_ms, mn = timed_steps(g.replay, steps, warmup, stream)
    del g
    return ms / reps, ev_ms / reps, mn / reps


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rate(run, kmax, target_s, unit, scale, what):
    """Time the FP64 oracle as it stands: run(k, threads) evaluates the
    first k units of a seeded order.  Calibrated on one unit, then sized for
    about target_s on every host thread the oracle uses, and for a quarter of
    that on one thread; value = units * scale / s."""
    import oracle
    th = oracle.nthreads_default()
    t0 = time.perf_counter()
    run(1, th)
    t1 = max(time.perf_counter() - t0, 1e-4)
    k = int(max(1, min(kmax, target_s / t1)))
    t0 = time.perf_counter()
    run(k, th)
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    run(1, 1)
    s1 = max(time.perf_counter() - t0, 1e-4)
    k1 = int(max(1, min(kmax, 0.25 * target_s / s1)))
    t0 = time.perf_counter()
    run(k1, 1)
    d1 = time.perf_counter() - t0
    return {"value": k * scale / dt, "unit": unit, "cores": th, "kind": "oracle",
            "sample": f"{k} {what}, {dt:.1f} s", "cpu_model": cpu_model(),
            "single_core": {"value": k1 * scale / d1, "sample": f"{k1} {what}, {d1:.1f} s"}}


def cpu_baseline_decode(batch, res, target_s=15.0):
    """The FP64 oracle (as it stands) on a seeded sample of whole blocks."""
    import numpy as np

    import oracle
    ob = oracle.Blocks(batch.ncp, batch.deg, batch.knot_off, batch.ctrl_off, batch.knots,
                       batch.ctrl)
    order = np.random.Generator(np.random.PCG64(99)).permutation(batch.nblocks)

    def run(k, th):
        sel = order[:k]
        oracle.decode_blocks(oracle.Blocks(ob.ncp[sel], ob.deg[sel], ob.knot_off[sel],
                                           ob.ctrl_off[sel], ob.knots, ob.ctrl), res, 15,
                             nthreads=th)

    return oracle_rate(run, batch.nblocks, target_s, "voxels/s", int(np.prod(res)),
                       f"of {batch.nblocks} blocks (seeded), full {res[0]}x{res[1]}x{res[2]} "
                       "grids, value+grad, FP64")


def cpu_baseline_fit(batch, y, res, target_s=15.0):
    """The FP64 oracle's fit iteration (decode, residual, adjoint B^T r) on a
    seeded sample of whole blocks, as iterations/s of the whole batch."""
    import numpy as np

    import oracle
    order = np.random.Generator(np.random.PCG64(98)).permutation(batch.nblocks)
    ob = oracle.Blocks(batch.ncp, batch.deg, batch.knot_off, batch.ctrl_off, batch.knots,
                       batch.ctrl)
    y64 = np.asarray(y, np.float64).reshape(batch.nblocks, 1, *res)

    def run(k, th):
        sel = order[:k]
        sub = oracle.Blocks(ob.ncp[sel], ob.deg[sel], ob.knot_off[sel], ob.ctrl_off[sel],
                            ob.knots, ob.ctrl)
        f = oracle.decode_blocks(sub, res, 1, nthreads=th)
        oracle.decode_adjoint(sub, res, f - y64[sel], 1, nthreads=th)

    return oracle_rate(run, batch.nblocks, target_s, "iterations/s", 1.0 / batch.nblocks,
                       f"of {batch.nblocks} blocks (seeded): FP64 value decode, residual and "
                       "adjoint, scaled to the whole batch (optimizer step excluded)")


def err_vs_oracle_decode(batch, out, res, nsample=20000, src=None, interleaved=False):
    """Max |gpu - FP64| / max |FP64| per channel on seeded voxels (out planar
    [nb][4][res] or interleaved [nb][res][4])."""
    import numpy as np
    import torch

    import oracle
    g = np.random.Generator(np.random.PCG64(7))
    idx = np.stack([g.integers(0, batch.nblocks, nsample), g.integers(0, res[0], nsample),
                    g.integers(0, res[1], nsample), g.integers(0, res[2], nsample)], 1)
    idx = idx.astype(np.int32)
    ob = oracle.Blocks(batch.ncp, batch.deg, batch.knot_off, batch.ctrl_off, batch.knots,
                       batch.ctrl if src is None else src)
    ref = oracle.decode_samples(ob, res, idx)
    ti = torch.as_tensor(idx, device=out.device).long()
    if interleaved:
        got = out[ti[:, 0], ti[:, 1], ti[:, 2], ti[:, 3]].double().cpu().numpy()
    else:
        got = out[ti[:, 0], :, ti[:, 1], ti[:, 2], ti[:, 3]].double().cpu().numpy()
    names = ["value", "d/du", "d/dv", "d/dw"]
    return {names[c]: float(np.abs(got[:, c] - ref[:, c]).max() / np.abs(ref[:, c]).max())
            for c in range(4)}


# ------------------------------------------------------------------ C2

def bench_c2(args):
    import torch

    import fa_inputs as fi
    import paper_2409_00184_amd as fa
    from paper_2409_00184_amd import autotune

    res = (64, 64, 64)
    batch = fi.config_c2()
    m = fa.MicroModels.from_batch(batch)
    stream = torch.cuda.current_stream()
    # the timed form stores one (value, d/du, d/dv, d/dw) record per voxel;
    # the planar [nb][4][res] form is timed beside it
    mask = 15 | fa.OUT_INTERLEAVED

    def schedule(mk):
        if args.tune:
            return fa.Plan(m, res, *args.tune), [(tuple(args.tune), None)]
        return autotune.tune(m, res, mk, "f32", use_cache=not args.retune)

    plan, report = schedule(mask)
    log("schedule", [plan.tune.rows_per_item, plan.tune.waves, plan.ngroups,
                     plan.tune.slab_floats, plan.tune.store],
        "fastest candidates", sorted(report, key=lambda r: r[1] or 0)[:6])
    out = torch.empty((batch.nblocks,) + res + (4,), dtype=torch.float32, device="cuda")
    graph, _ = fa.capture(lambda: fa.decode(m, res, mask, plan=plan, out=out))
    ms, ev_ms, ev_min = timed_steps(graph.replay, args.steps, args.warmup, stream)
    err = err_vs_oracle_decode(batch, out, res, interleaved=True)
    del graph, out
    pplan, _ = schedule(15)
    out = torch.empty((batch.nblocks, 4) + res, dtype=torch.float32, device="cuda")
    pgraph, _ = fa.capture(lambda: fa.decode(m, res, 15, plan=pplan, out=out))
    planar_ms, planar_ev, _ = timed_steps(pgraph.replay, args.steps, args.warmup, stream)
    del pgraph
    nvox = batch.nblocks * res[0] * res[1] * res[2]
    value = nvox / (ms * 1e-3)
    lattice_bytes = 4 * int(sum(int(n.prod()) for n in batch.ncp))
    alg_bytes = nvox * 16 + lattice_bytes + 4 * batch.knots.size + 64 * batch.nblocks
    achieved = alg_bytes / (ev_ms * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": value, "unit": "voxels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C2 batched decode: 512 micro-models, NCP* per axis in "
                               "{8,12,16,24,32}, degree in {2,3}, 64^3 voxels each, value + 3 "
                               "gradients, FP32, one launch over the batch plan's work items "
                               "in longest-first order at the autotuner's schedule (one "
                               "workgroup per item), replayed from a HIP graph, one 16-byte "
                               "record per voxel",
                   "nblocks": batch.nblocks, "res": list(res), "channels": 4,
                   "layout": "[block][x][y][z][value, d/du, d/dv, d/dw]",
                   "schedule": {"rows_per_item": plan.tune.rows_per_item,
                                "waves": plan.tune.waves, "workgroups": plan.ngroups,
                                "items": plan.nwork, "slab_floats": plan.tune.slab_floats,
                                "store": ["non-temporal", "ordinary"][plan.tune.store]}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_from_profiles("decode_sep", "c2"),
                     "kernel": "decode_sep_kernel", "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": ev_ms, "min_launch_ms": ev_min},
        "err_vs_fp64": err,
        "planar": {"value": nvox / (planar_ms * 1e-3), "ms_per_step": planar_ms,
                   "avg_launch_ms": planar_ev,
                   "layout": "[block][channel][x][y][z]",
                   "schedule": [pplan.tune.rows_per_item, pplan.tune.waves, pplan.ngroups,
                                pplan.tune.slab_floats, pplan.tune.store]},
    }
    # the persistent form of the plan (a fixed number of workgroups, each
    # running its longest-first share of the items) beside the timed one
    pers = []
    t = plan.tune
    for grid in (512, 768, 1024, 1536, 2048):
        pp = fa.Plan(m, res, t.rows_per_item, t.waves, grid, 0, t.slab_floats, t.store)
        o3 = torch.empty((batch.nblocks,) + res + (4,), dtype=torch.float32, device="cuda")
        g3, _ = fa.capture(lambda: fa.decode(m, res, mask, plan=pp, out=o3))
        pms3 = timed_steps(g3.replay, args.steps, args.warmup, stream)[0]
        pers.append((pms3, grid))
        del g3, o3
    pms3, pgrid = min(pers)
    line["persistent"] = {"value": nvox / (pms3 * 1e-3), "ms_per_step": pms3,
                          "workgroups": pgrid, "vs_timed": ms / pms3,
                          "grids_tried": {str(g): v for v, g in pers}}
    if not args.no_plain:
        pms, pev, _ = timed_steps(lambda: fa.decode_plain(m, res, 15, out=out),
                                  max(2, args.steps // 10), 1, stream)
        line["plain"] = {"value": nvox / (pms * 1e-3), "ms_per_step": pms,
                         "form": "one launch per block, one thread per voxel, no graph"}
        line["speedup_vs_plain"] = pms / ms
    if not args.no_lowp:
        lp = {}
        for dt in ("bf16", "f16"):
            m.lattice(dt)
            for kern, pl in (("valu", plan), ("mfma", fa.Plan(m, res, kernel=1))):
                o2 = torch.empty_like(out)
                g2, _ = fa.capture(lambda: fa.decode(m, res, 15, dtype=dt, plan=pl, out=o2))
                lms, lev, _ = timed_steps(g2.replay, args.steps, args.warmup, stream)
                lp[f"{dt}_{kern}"] = {"value": nvox / (lms * 1e-3), "ms_per_step": lms,
                                      "speedup_vs_f32_planar": planar_ms / lms,
                                      "err_vs_fp64": err_vs_oracle_decode(batch, o2, res)}
                del o2, g2
        line["lowp"] = lp
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_decode(batch, res, args.cpu_seconds)
    return line


def _common(args, metric, value, unit, ms, dtype, workload, extra):
    line = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": {"workload": workload}}
    line.update(extra)
    return line


def _roof(alg_bytes, ev_ms, kernel, workload, bound="hbm"):
    achieved = alg_bytes / (ev_ms * 1e-3) / 1e9
    return {"bound": bound, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profiles(kernel, workload),
            "kernel": kernel, "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": ev_ms}


# ------------------------------------------------------------------ C1

def bench_c1(args):
    import torch

    import fa_inputs as fi
    import paper_2409_00184_amd as fa
    from paper_2409_00184_amd import autotune
    res = (64, 64, 64)
    batch = fi.config_c1()
    m = fa.MicroModels.from_batch(batch)
    # one block: items of one or two y rows give more workgroups than the
    # batch schedules do
    cands = list(autotune.CANDIDATES) + [(r, w, 1 << 20, 0, 8192, st) for r in (1, 2)
                                         for w in (1, 2) if w <= r for st in (0, 1)]
    plan, _ = autotune.tune(m, res, 15, "f32", candidates=cands, use_cache=not args.retune)
    out = torch.empty((1, 4) + res, device="cuda")
    graph, _ = fa.capture(lambda: fa.decode(m, res, 15, plan=plan, out=out))
    ms, ev_ms, _ = timed_steps(graph.replay, args.steps, args.warmup,
                               torch.cuda.current_stream())
    nvox = 64 ** 3
    line = _common(args, METRIC, nvox / (ms * 1e-3), "voxels/s", ms, "f32",
                   "C1 single micro-model: 16^3 control points, cubic, decoded to 64^3 voxels "
                   "(value + 3 gradients, FP32); latency-bound (one block)",
                   {"roofline": _roof(nvox * 16 + 4 * 4096, ev_ms, "decode_sep", "c1"),
                    "latency_us": ev_ms * 1e3,
                    "err_vs_fp64": err_vs_oracle_decode(batch, out, res, src=batch.ctrl64)})
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_decode(batch, res, args.cpu_seconds)
    return line


# ------------------------------------------------------------------ C3

def c3_samples(nx=1920, ny=1080, ns=512, seed=3):
    """Ray-major FP32 sample positions of the seeded camera, built on the GPU
    in chunks of rays (the same recipe as fa_inputs.ray_samples_np)."""
    import torch

    import fa_inputs as fi
    o, d, t0, t1, j = fi.camera_rays(seed, nx, ny)
    nray = o.shape[0]
    f64 = dict(dtype=torch.float64, device="cuda")
    O, D = torch.as_tensor(o, **f64), torch.as_tensor(d, **f64)
    T0, T1, J = torch.as_tensor(t0, **f64), torch.as_tensor(t1, **f64), torch.as_tensor(j, **f64)
    xyz = torch.empty((nray, ns, 3), dtype=torch.float32, device="cuda")
    s = torch.arange(ns, **f64)
    for r0 in range(0, nray, 1 << 18):
        r1 = min(nray, r0 + (1 << 18))
        t = T0[r0:r1, None] + (s[None] + J[r0:r1, None]) / ns * (T1 - T0)[r0:r1, None]
        xyz[r0:r1] = (O[r0:r1, None] + D[r0:r1, None] * t[..., None]).float()
    return xyz.reshape(-1, 3)


def bench_c3(args):
    import numpy as np
    import torch

    import fa_inputs as fi
    import oracle
    import paper_2409_00184_amd as fa
    b = fi.config_c3_blocks()
    m = fa.MicroModels.from_batch(b)
    xyz = c3_samples()
    n = xyz.shape[0]
    boc = torch.as_tensor(fi.identity_cells(4096), device="cuda")
    out = torch.empty((n, 4), device="cuda")
    flat = lambda: fa.query(m, xyz, (16, 16, 16), (0, 0, 0), (1, 1, 1), boc, out=out)
    rays = lambda: fa.query_rays(m, xyz, 1920, 1080, 512, (16, 16, 16), (0, 0, 0), (1, 1, 1),
                                 boc, out=out)
    stream = torch.cuda.current_stream()
    orders = {}
    for name, fn in (("flat", flat), ("rays", rays)):
        graph, _ = fa.capture(fn)
        orders[name] = timed_steps(graph.replay, args.steps, args.warmup, stream)
        del graph
    best = min(orders, key=lambda k: orders[k][1])
    ms, ev_ms, _ = orders[best]
    (flat if best == "flat" else rays)()
    torch.cuda.synchronize()
    g = np.random.Generator(np.random.PCG64(8))
    idx = torch.as_tensor(g.integers(0, n, 200000), device="cuda")
    xs = xyz[idx].cpu().numpy()
    got = out[idx].double().cpu().numpy()
    ob = oracle.Blocks(b.ncp, b.deg, b.knot_off, b.ctrl_off, b.knots, b.ctrl)
    ref = oracle.query_points(ob, xs, (16, 16, 16), (0, 0, 0), (1, 1, 1), fi.identity_cells(4096))
    err = {k: float(np.abs(got[:, c] - ref[:, c]).max() / np.abs(ref[:, c]).max())
           for c, k in enumerate(["value", "d/dx", "d/dy", "d/dz"])}
    flops = 2 * 192 + 3 * 45  # contraction FMAs + basis/span work per sample (p = 3)
    tflops = n * flops / (ev_ms * 1e-3) / 1e12
    hbm = _roof(n * 28 + 4 * b.ctrl.size, ev_ms, "query", "c3")
    line = _common(args, "queried samples/sec (value+grad)", n / (ms * 1e-3), "samples/s", ms,
                   "f32",
                   "C3 ray-sample query: 1024^3 domain as 16^3 micro-models (NCP* per axis in "
                   "8..32, cubic), 1920x1080 rays x 512 samples (1.06e9 non-grid positions), "
                   "block lookup + span search + value + gradient, FP32",
                   {"roofline": {"bound": "alu", "achieved": tflops, "peak": VALU_PEAK_TFLOPS,
                                 "unit": "TFLOP/s", "frac": tflops / VALU_PEAK_TFLOPS,
                                 "frac_of_unpacked_fp32": tflops / VALU_UNPACKED_TFLOPS,
                                 "traffic": hbm["traffic"], "kernel": "query",
                                 "flops_per_sample": flops, "avg_launch_ms": ev_ms,
                                 "hbm": {"achieved": hbm["achieved"], "unit": "GB/s",
                                         "frac": hbm["frac"],
                                         "alg_bytes_per_launch": hbm["alg_bytes_per_launch"]}},
                    "order": {k: {"ms_per_step": v[0], "avg_launch_ms": v[1]}
                              for k, v in orders.items()},
                    "timed_order": best,
                    "err_vs_fp64": err})
    if not args.no_lowp:
        # 2-byte lattices (P / s_b with the per-block max-abs scale), the
        # ray-tile order; errors against the FP64 oracle of the FP32 lattice
        lp = {}
        for dt in ("bf16", "f16"):
            m.lattice(dt)
            fn = lambda: fa.query_rays(m, xyz, 1920, 1080, 512, (16, 16, 16), (0, 0, 0),
                                       (1, 1, 1), boc, dtype=dt, out=out)
            graph, _ = fa.capture(fn)
            lms, lev, _ = timed_steps(graph.replay, args.steps, args.warmup, stream)
            del graph
            fn()
            torch.cuda.synchronize()
            g2 = out[idx].double().cpu().numpy()
            lp[dt] = {"value": n / (lms * 1e-3), "ms_per_step": lms, "avg_launch_ms": lev,
                      "speedup_vs_f32": ms / lms,
                      "err_vs_fp64": {k: float(np.abs(g2[:, c] - ref[:, c]).max() /
                                               np.abs(ref[:, c]).max())
                                      for c, k in enumerate(["value", "d/dx", "d/dy", "d/dz"])}}
        line["lowp"] = lp
    # the same tiling and camera with every interior knot jittered (binary
    # span search instead of the uniform-knot guess)
    bn = fi.config_c3_blocks(nonuniform=True)
    mn = fa.MicroModels.from_batch(bn)
    fnu = lambda: fa.query_rays(mn, xyz, 1920, 1080, 512, (16, 16, 16), (0, 0, 0), (1, 1, 1),
                                boc, out=out)
    graph, _ = fa.capture(fnu)
    nms, nev, _ = timed_steps(graph.replay, args.steps, args.warmup, stream)
    del graph
    fnu()
    torch.cuda.synchronize()
    gn = out[idx].double().cpu().numpy()
    obn = oracle.Blocks(bn.ncp, bn.deg, bn.knot_off, bn.ctrl_off, bn.knots, bn.ctrl)
    refn = oracle.query_points(obn, xs, (16, 16, 16), (0, 0, 0), (1, 1, 1),
                               fi.identity_cells(4096))
    line["nonuniform_knots"] = {
        "value": n / (nms * 1e-3), "ms_per_step": nms, "avg_launch_ms": nev,
        "vs_uniform": ms / nms,
        "err_vs_fp64": {k: float(np.abs(gn[:, c] - refn[:, c]).max() / np.abs(refn[:, c]).max())
                        for c, k in enumerate(["value", "d/dx", "d/dy", "d/dz"])}}
    del mn
    if not args.no_cpu_baseline:
        k_max = 20_000_000
        sidx = torch.as_tensor(g.integers(0, n, k_max), device="cuda")
        xk = xyz[sidx].cpu().numpy()
        del sidx
        cells = fi.identity_cells(4096)
        line["cpu_baseline"] = oracle_rate(
            lambda k, th: oracle.query_points(ob, xk[:20000 * k], (16, 16, 16), (0, 0, 0),
                                              (1, 1, 1), cells, nthreads=th),
            k_max // 20000, args.cpu_seconds, "samples/s", 20000,
            "x 20000 seeded samples of the 1.06e9 (ray-major positions), FP64")
    del xyz, out
    return line


# ------------------------------------------------------------------ F1

VALU_PEAK_TFLOPS = 157.3
# the same vector ALUs without packed FP32 (one FMA per lane per clock):
# 256 CUs x 64 lanes x 2 FLOP x 2.4 GHz; the kernels here are built without
# packed FP32 instructions, so this is the rate their FMAs can reach
VALU_UNPACKED_TFLOPS = 78.6


def bench_f1(args):
    """Direct volume rendering of the C3 micro-models: 1920x1080 rays of the
    seeded camera, 512 samples each (early termination off, so every sample
    is evaluated; the terminating variant is reported beside it)."""
    import numpy as np
    import torch

    import fa_inputs as fi
    import oracle
    import paper_2409_00184_amd as fa
    W, H, S = 1920, 1080, 512
    b = fi.config_c3_blocks()
    m = fa.MicroModels.from_batch(b)
    rays_np = fi.render_rays(3, W, H)
    rays = torch.as_tensor(rays_np, device="cuda")
    tf_np = fi.transfer_function(4)
    tf = torch.as_tensor(tf_np, device="cuda")
    boc = torch.as_tensor(fi.identity_cells(4096), device="cuda")
    img = torch.empty((H, W, 4), device="cuda")
    shade = dict(light=(0.0, 0.6, 0.8), ka=0.3, kd=0.6, ks=0.3, shininess=16.0)
    run = lambda omax: (lambda: fa.render(m, rays, W, H, tf, (16, 16, 16), (0, 0, 0), (1, 1, 1),
                                          boc, S, opacity_max=omax, tf_range=(-4.0, 4.0),
                                          out=img, **shade))
    stream = torch.cuda.current_stream()
    graph, _ = fa.capture(run(0.98))
    ms_t, ev_t, _ = timed_steps(graph.replay, args.steps, args.warmup, stream)
    del graph
    graph, _ = fa.capture(run(2.0))
    ms, ev_ms, _ = timed_steps(graph.replay, args.steps, args.warmup, stream)
    del graph
    run(2.0)()
    torch.cuda.synchronize()
    n = W * H * S
    g = np.random.Generator(np.random.PCG64(11))
    pix = g.integers(0, W * H, 2000)
    got = img.reshape(-1, 4)[torch.as_tensor(pix, device="cuda")].double().cpu().numpy()
    ob = oracle.Blocks(b.ncp, b.deg, b.knot_off, b.ctrl_off, b.knots, b.ctrl)
    oargs = lambda r: (ob, r, S, 2.0, -4.0, 4.0, tf_np, shade["light"], shade["ka"], shade["kd"],
                       shade["ks"], shade["shininess"], (16, 16, 16), (0, 0, 0), (1, 1, 1),
                       fi.identity_cells(4096))
    ref = oracle.render(*oargs(rays_np[pix]))
    scale = np.abs(ref).max(0)
    err = {k: float(np.abs(got[:, c] - ref[:, c]).max() / scale[c])
           for c, k in enumerate(["R", "G", "B", "A"])}
    # the same view of the micro-models with every interior knot jittered
    # (span search by bisection with cross-lane knot reads in block-uniform
    # waves, per lane otherwise)
    bn = fi.config_c3_blocks(nonuniform=True)
    mn = fa.MicroModels.from_batch(bn)
    rnu = lambda: fa.render(mn, rays, W, H, tf, (16, 16, 16), (0, 0, 0), (1, 1, 1), boc, S,
                            opacity_max=2.0, tf_range=(-4.0, 4.0), out=img, **shade)
    graph, _ = fa.capture(rnu)
    ms_n, ev_n, _ = timed_steps(graph.replay, args.steps, args.warmup, stream)
    del graph, mn
    run(2.0)()
    torch.cuda.synchronize()
    flops = 2 * 192 + 3 * 45 + 40  # contraction + basis/span + TF/shading/compositing
    tflops = n * flops / (ev_ms * 1e-3) / 1e12
    line = _common(args, "rendered samples/sec (DVR ray casting)", n / (ms * 1e-3), "samples/s",
                   ms, "f32",
                   "F1 direct volume rendering of the C3 micro-models (16^3 blocks, NCP* per "
                   "axis in 8..32, cubic): 1920x1080 rays x 512 samples, value + gradient, "
                   "RGBA transfer function, Blinn-Phong shading, front-to-back compositing, "
                   "FP32; early termination off",
                   {"roofline": {"bound": "alu", "achieved": tflops, "peak": VALU_PEAK_TFLOPS,
                                 "unit": "TFLOP/s", "frac": tflops / VALU_PEAK_TFLOPS,
                                 "frac_of_unpacked_fp32": tflops / VALU_UNPACKED_TFLOPS,
                                 "traffic": traffic_from_profiles("render", "f1"),
                                 "kernel": "render", "flops_per_sample": flops,
                                 "avg_launch_ms": ev_ms},
                    "frames_per_s": 1e3 / ms,
                    "early_termination": {"opacity_max": 0.98, "ms_per_step": ms_t,
                                          "avg_launch_ms": ev_t, "frames_per_s": 1e3 / ms_t},
                    "nonuniform_knots": {"ms_per_step": ms_n, "avg_launch_ms": ev_n,
                                         "vs_uniform": ms / ms_n},
                    "err_vs_fp64": err})
    if not args.no_cpu_baseline:
        th = oracle.nthreads_default()
        t0 = time.perf_counter()
        oracle.render(*oargs(rays_np[pix[:200]]), nthreads=th)
        rate = 200 / (time.perf_counter() - t0)
        k = int(min(W * H, max(200, rate * args.cpu_seconds)))
        sel = g.integers(0, W * H, k)
        t0 = time.perf_counter()
        oracle.render(*oargs(rays_np[sel]), nthreads=th)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": k * S / dt, "unit": "samples/s", "cores": th,
                                "kind": "oracle",
                                "sample": f"{k} seeded pixels of 1920x1080, {S} samples each, "
                                          f"no early termination, FP64, {dt:.1f} s"}
    return line


# ------------------------------------------------------------------ F2

def bench_f2(args):
    """In-level adaptive NCP search (Sec. 4.2.1, the inner loop of Alg. 1):
    64 micro-blocks of 64^3 FP32 samples, degree 3, every NCP from 64 down
    to 5 fitted (least squares), decoded and scored; one step = the whole
    search (60 candidate fits per block)."""
    import numpy as np
    import torch

    import fa_inputs as fi
    import paper_2409_00184_amd as fa
    R, p, nb = 64, 3, 64
    lo, hi = p + 2, R
    ncand = hi - lo + 1
    Y = torch.as_tensor(fi.turbulence_cube(fi.rng(12), R, nb)).cuda().contiguous()
    ws = torch.empty(fa.lib.fa_ncp_search_workspace(nb, fa._i32x3((R, R, R)), p, hi),
                     dtype=torch.uint8, device="cuda")
    errs = torch.empty((nb, ncand, 2), device="cuda")
    st = lambda: fa.lib.fa_ncp_search(fa._ptr(Y), nb, fa._i32x3((R, R, R)), p, lo, hi,
                                      fa._ptr(errs), fa._ptr(ws), ws.numel(), fa._stream())
    run = lambda: fa._check("fa_ncp_search", st())
    stream = torch.cuda.current_stream()
    graph, _ = fa.capture(run)
    ms, ev_ms, _ = timed_steps(graph.replay, args.steps, args.warmup, stream)
    del graph
    # per-stage breakdown at a few NCPs: the fit alone (per-block
    # pseudo-inverses and the two products) and the search over that one
    # candidate (its shared pseudo-inverses, descriptors, the products, the
    # value decode reduced to the error-map entry), HIP events on the launch
    # stream
    stages = {}
    for n in (8, 32, 64):
        m = fa.uniform_models(np.full((nb, 3), n), np.full(nb, p))
        fws = torch.empty(fa.lib.fa_fit_workspace(nb, fa._i32x3((R, R, R)), n),
                          dtype=torch.uint8, device="cuda")
        f_ms = timed_steps(lambda: fa.fit(m, (R, R, R), Y, workspace=fws), 5, 2, stream)[1]
        one = lambda: fa._check("fa_ncp_search", fa.lib.fa_ncp_search(
            fa._ptr(Y), nb, fa._i32x3((R, R, R)), p, n, n, fa._ptr(errs), fa._ptr(ws),
            ws.numel(), fa._stream()))
        c_ms = timed_steps(one, 5, 2, stream)[1]
        stages[str(n)] = {"fit_ms": f_ms, "candidate_ms": c_ms}
        del m, fws
    vox = nb * R ** 3
    # HBM floor of the two passes over the voxels per candidate: the fit
    # reads y, the error-map decode reads y (8 B/voxel)
    alg = ncand * vox * 8
    line = _common(args, "micro-blocks searched/sec (adaptive NCP, Eq. 4)", nb / (ms * 1e-3),
                   "blocks/s", ms, "f32",
                   "F2 in-level adaptive NCP search: 64 micro-blocks of 64^3 FP32 samples "
                   "(k^-5/3 turbulence), degree 3, NCP 64..5 (60 least-squares fits, decodes "
                   "and error reductions per block)",
                   {"roofline": _roof(alg, ev_ms, "ncp_search", "f2"),
                    "fits_per_s": nb * ncand / (ms * 1e-3),
                    "stages_at_ncp": stages})
    if not args.no_cpu_baseline:
        import oracle
        from oracle import adaptive as ad
        y0 = Y[0].double().cpu().numpy()
        t0 = time.perf_counter()
        k = 0
        for n in range(hi, lo - 1, -1):
            kn = [ad.uniform_knots(n, p)] * 3
            P = ad.fit_block(y0, (n, n, n), (p, p, p), kn)
            ad.model_errors(y0, P, (n, n, n), (p, p, p), kn)
            k += 1
            if time.perf_counter() - t0 > args.cpu_seconds:
                break
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": k / ncand / dt, "unit": "blocks/s",
                                "cores": oracle.nthreads_default(), "kind": "oracle",
                                "sample": f"{k} of the {ncand} candidate fits of one 64^3 block "
                                          f"(from NCP 64 down), FP64 least squares + decode, "
                                          f"{dt:.1f} s"}
    return line


# ------------------------------------------------------------------ F3

PCIE_PEAK_GBS = 64.0  # PCIe 5.0 x16, one direction


def bench_f3(args):
    """Caching and memory copy of Alg. 2 for the C3 camera: the visible
    micro-models of the view (fa_visible_cells), fetched through the host
    LRU cache from an Eq. 2 file and staged to the GPU with page-locked
    asynchronous copies.  Warm frames (the view fits the cache) measure the
    copy; cold frames and the paper's 200-block cache add file reads."""
    import tempfile

    import numpy as np
    import torch

    import fa_inputs as fi
    import paper_2409_00184_amd as fa
    nb, p = 16, 3
    g = fi.rng(13)
    k, phi = fi.sinusoid_params(g)
    ncp = g.integers(8, 33, nb ** 3)
    kl, lat = [], []
    for b in range(nb ** 3):
        n = int(ncp[b])
        ts = [fi.clamped_uniform_knots(n, p)] * 3
        kl.append(ts)
        lat.append(np.zeros((n, n, n)) if b % 7 else
                   fi.sinusoid_lattice(k, phi, ts[0], ts[1], ts[2], (n,) * 3, (p,) * 3))
    batch = fi.pack(np.repeat(ncp[:, None], 3, 1), np.full((nb ** 3, 3), p), kl, lat)
    desc = fa.host_descriptors(batch.ncp, batch.deg, batch.knot_off, batch.ctrl_off)
    tmp = tempfile.mkdtemp()
    path = os.path.join(tmp, "c3.fam")
    fa.store_write(path, desc, batch.knots, batch.ctrl)
    file_bytes = os.path.getsize(path)
    W, H, S = 1920, 1080, 512
    rays = torch.as_tensor(fi.render_rays(3, W, H), device="cuda")
    flags = fa.visible_cells(rays, W, H, S, (nb,) * 3, (0, 0, 0), (1, 1, 1))
    stream = torch.cuda.current_stream()
    vis_ms = timed_steps(lambda: fa.visible_cells(rays, W, H, S, (nb,) * 3, (0, 0, 0),
                                                  (1, 1, 1), out=flags), 5, 2, stream)[1]
    ids = np.nonzero(flags.cpu().numpy())[0].astype(np.int32)
    out = {}
    for name, cache in (("warm", len(ids)), ("paper_cache_200", 200)):
        store = fa.Store(path, cache_blocks=cache, pinned=True, max_stage=len(ids))
        store.stage(ids)  # first (cold) frame
        torch.cuda.synchronize()
        st0 = store.stage(ids)[1]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, st = store.stage(ids)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        h2d = (st["bytes_h2d"] - st0["bytes_h2d"]) / args.steps
        out[name] = {"ms_per_frame": dt * 1e3, "h2d_bytes_per_frame": h2d,
                     "h2d_gbs": h2d / dt / 1e9,
                     "misses_per_frame": (st["misses"] - st0["misses"]) / args.steps,
                     "read_bytes_per_frame": (st["bytes_read"] - st0["bytes_read"]) / args.steps}
        store.close()
    os.remove(path)
    os.rmdir(tmp)
    warm = out["warm"]
    line = _common(args, "staged micro-model bytes/sec (Alg. 2 caching + copy, warm cache)",
                   warm["h2d_bytes_per_frame"] / (warm["ms_per_frame"] * 1e-3), "B/s",
                   warm["ms_per_frame"], "f32",
                   "F3 caching + copy of the visible micro-models of the C3 view (16^3 "
                   "cubic micro-models, NCP 8..32, degree 3, Eq. 2 file; 1920x1080 rays x 512 "
                   "samples for visibility)",
                   {"roofline": {"bound": "pcie", "achieved": warm["h2d_gbs"],
                                 "peak": PCIE_PEAK_GBS, "unit": "GB/s",
                                 "frac": warm["h2d_gbs"] / PCIE_PEAK_GBS, "traffic": None,
                                 "kernel": "hipMemcpyAsync H2D"},
                    "visible_blocks": int(len(ids)), "file_bytes": file_bytes,
                    "visible_cells_ms": vis_ms, "frames": out})
    return line


# ------------------------------------------------------------------ F4

def ml_level_samples(level, R, blocks, torch, device="cuda"):
    """FP32 Marschner-Lobb samples [len(blocks), R, R, R] of one pyramid level,
    generated on the GPU in FP64 (same recipe as fa_inputs.ml_blocks)."""
    import fa_inputs as fi
    m = 1 << level
    b = torch.as_tensor(blocks, device=device)
    u = torch.arange(R, dtype=torch.float64, device=device) / (R - 1)
    h = fi.ML_EXTENT / m
    bx = (b // (m * m)).double()
    by = ((b // m) % m).double()
    bz = (b % m).double()
    x = (h * (bx[:, None] + u[None]))[:, :, None, None]
    y = (h * (by[:, None] + u[None]))[:, None, :, None]
    z = (h * (bz[:, None] + u[None]))[:, None, None, :]
    return fi.ml_value(x, y, z, xp=torch).float().contiguous()


def bench_f4(args):
    """Marschner-Lobb end to end (Eq. 5): level 4 of the pyramid (16^3
    micro-blocks of 64^3 samples with shared faces = a 1009^3 grid over
    [0,7]^3), FAM encode (least-squares fit at NCP 32) + decode of value and
    gradient; quality against the analytic field, and the adaptive encoding
    (in-level search, Eq. 4) beside it."""
    import numpy as np
    import torch

    import fa_inputs as fi
    import paper_2409_00184_amd as fa
    level, R, p, n_fam = 4, 64, 3, 32
    nb = (1 << level) ** 3
    Y = torch.empty((nb, R, R, R), device="cuda")
    for b0 in range(0, nb, 256):
        Y[b0:b0 + 256] = ml_level_samples(level, R, list(range(b0, min(nb, b0 + 256))), torch)
    m = fa.uniform_models(np.full((nb, 3), n_fam), np.full(nb, p))
    out = torch.empty((nb, 4, R, R, R), device="cuda")
    plan = fa.Plan(m, (R, R, R), rows=4, waves=4, grid=1 << 20, store=0)
    fws = torch.empty(fa.lib.fa_fit_workspace(nb, fa._i32x3((R, R, R)), n_fam),
                      dtype=torch.uint8, device="cuda")

    def step():
        fa.fit(m, (R, R, R), Y, workspace=fws)
        fa.decode(m, (R, R, R), 15, plan=plan, out=out)

    stream = torch.cuda.current_stream()
    graph, _ = fa.capture(step)
    ms, ev_ms, _ = timed_steps(graph.replay, args.steps, args.warmup, stream)
    del graph
    fit_ms = timed_steps(lambda: fa.fit(m, (R, R, R), Y, workspace=fws), 5, 2, stream)[1]
    dec_ms = timed_steps(lambda: fa.decode(m, (R, R, R), 15, plan=plan, out=out), 5, 2,
                         stream)[1]
    step()
    torch.cuda.synchronize()

    def quality(o):
        """value PSNR (range [0,1]) and gradient relative RMS against Eq. 5."""
        se_v = se_g = ng = 0.0
        dudx = (1 << level) / fi.ML_EXTENT
        u = torch.arange(R, dtype=torch.float64, device="cuda") / (R - 1)
        h = fi.ML_EXTENT / (1 << level)
        for b0 in range(0, nb, 256):
            b = torch.arange(b0, min(nb, b0 + 256), device="cuda")
            mm = 1 << level
            x = (h * ((b // (mm * mm)).double()[:, None] + u[None]))[:, :, None, None]
            y = (h * (((b // mm) % mm).double()[:, None] + u[None]))[:, None, :, None]
            z = (h * ((b % mm).double()[:, None] + u[None]))[:, None, None, :]
            v = fi.ml_value(x, y, z, xp=torch)
            g = fi.ml_gradient(x, y, z, xp=torch)
            ob = o[b0:b0 + 256].double()
            se_v += float(((ob[:, 0] - v) ** 2).sum())
            for a in range(3):
                se_g += float(((ob[:, 1 + a] * dudx - g[a]) ** 2).sum())
                ng += float((g[a] ** 2).sum())
        mse = se_v / (nb * R ** 3)
        return {"value_psnr_db": 10 * np.log10(1.0 / mse), "value_rmse": mse ** 0.5,
                "grad_rel_rms": (se_g / ng) ** 0.5}

    q_fam = quality(out)
    sizes = lambda ncp: float(np.sum(1 + (3 * (ncp + p) + ncp.astype(np.float64) ** 3) * 4))
    raw = nb * R ** 3 * 4
    fam = dict(q_fam, ncp=n_fam, bytes=sizes(np.full(nb, n_fam)),
               compression=raw / sizes(np.full(nb, n_fam)))
    # adaptive (Eq. 4): in-level search on every block of the level, RMS bounds
    t0 = time.perf_counter()
    errs = fa.ncp_search(Y, p, p + 2, 40)
    torch.cuda.synchronize()
    search_s = time.perf_counter() - t0
    adaptive = {}
    for bound in (1e-3, 1e-4):
        nstar, cplx = fa.ncp_select(errs, p + 2, bound)
        ma = fa.uniform_models(np.repeat(nstar[:, None], 3, 1), np.full(nb, p))
        fa.fit(ma, (R, R, R), Y)
        fa.decode(ma, (R, R, R), 15, out=out)
        torch.cuda.synchronize()
        adaptive[str(bound)] = dict(
            quality(out), rms_bound=bound, ncp_mean=float(nstar.mean()),
            ncp_hist={int(k): int(v) for k, v in zip(*np.unique(nstar, return_counts=True))},
            complex_blocks=int(cplx.sum()), bytes=sizes(nstar), compression=raw / sizes(nstar))
        del ma
    adaptive["search_s"] = search_s
    adaptive["search_candidates"] = "5..40"
    vox = nb * R ** 3
    line = _common(args, "encoded+decoded voxels/sec (Marschner-Lobb, FAM fit + value/grad "
                   "decode)", vox / (ms * 1e-3), "voxels/s", ms, "f32",
                   "F4 Marschner-Lobb (Eq. 5, f_M 6, alpha 0.05, [0,7]^3): 16^3 micro-blocks "
                   "of 64^3 samples (1009^3 grid), least-squares fit at NCP 32 + decode of "
                   "value and gradient, FP32; quality vs the analytic field",
                   {"roofline": _roof(vox * 4 + vox * 16 + 8 * m.ctrl.numel(), ev_ms,
                                      "fit_decode", "f4"),
                    "stages": {"fit_ms": fit_ms, "decode_ms": dec_ms},
                    "quality": {"fam": fam, "adaptive": adaptive}})
    if not args.no_cpu_baseline:
        import oracle
        from oracle import adaptive as ad
        y0 = Y[0].double().cpu().numpy()
        kn = [ad.uniform_knots(n_fam, p)] * 3
        t0 = time.perf_counter()
        k = 0
        while True:
            P = ad.fit_block(y0, (n_fam,) * 3, (p,) * 3, kn)
            ob = oracle.Blocks(np.array([[n_fam] * 3]), np.array([[p] * 3]), np.zeros(1),
                               np.zeros(1), np.concatenate(kn), P.reshape(-1))
            oracle.decode_blocks(ob, (R, R, R), 15)
            k += 1
            if time.perf_counter() - t0 > min(args.cpu_seconds, 10.0):
                break
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": k * R ** 3 / dt, "unit": "voxels/s",
                                "cores": oracle.nthreads_default(), "kind": "oracle",
                                "sample": f"{k} x block 0 (64^3): FP64 least-squares fit at "
                                          f"NCP 32 + value/gradient decode, {dt:.1f} s"}
    del Y, out
    return line


# ------------------------------------------------------------------ C4

def bench_c4(args):
    import numpy as np
    import torch

    import fa_inputs as fi
    import paper_2409_00184_amd as fa
    res = (64, 64, 64)
    b, y = fi.config_c4()
    m = fa.MicroModels.from_batch(b)
    plan = fa.Plan(m, res)
    yt = torch.as_tensor(y, device="cuda").reshape(b.nblocks, 1, *res)
    ctrl = torch.zeros(b.ctrl.size, device="cuda", requires_grad=True)
    # the library's Adam step (fa_adam_step: a counter launch and one update
    # launch); gradients are set, not accumulated into a zeroed buffer (the
    # adjoint writes every control point)
    opt = fa.Adam([ctrl], lr=0.05)
    losses = []

    yf = yt.reshape(b.nblocks, *res).contiguous()

    def it():  # fused loss: decode, residual + loss + cotangent, adjoint
        opt.zero_grad(set_to_none=True)
        loss = fa.FAFitMSE.apply(ctrl, m, res, yf, plan)
        loss.backward()
        opt.step()
        return loss

    def it_torch():  # the same step with the loss composed of torch operations
        opt.zero_grad(set_to_none=True)
        loss = ((fa.FADecode.apply(ctrl, m, res, 1, plan) - yt) ** 2).mean()
        loss.backward()
        opt.step()
        return loss

    stream = torch.cuda.current_stream()
    ms, ev_ms, _ = timed_steps(lambda: losses.append(it()), args.steps, args.warmup, stream)
    first, last = float(losses[0].detach()), float(losses[-1].detach())
    ms_t = timed_steps(it_torch, args.steps, args.warmup, stream)[0]
    # the same iteration captured into one HIP graph (the same Adam step,
    # its step count on the device); every replay does the whole iteration's work
    mg = fa.MicroModels.from_batch(b)
    ctrl_g = torch.zeros(b.ctrl.size, device="cuda", requires_grad=True)
    opt_g = fa.Adam([ctrl_g], lr=0.05)
    graph, loss_g = fa.capture_fit_step(ctrl_g, opt_g, mg, res, yf, fa.Plan(mg, res))
    ms_g = timed_steps(graph.replay, args.steps, args.warmup, stream)[0]
    loss_graph = float(loss_g.detach())
    # the two HIP kernels of an iteration, timed alone
    out = torch.empty((b.nblocks, 1) + res, device="cuda")
    # two cotangents (268 MB each) used in turn, so that no launch finds its
    # input still in the 256 MB Infinity Cache (one buffer: about 8% faster)
    gins = [torch.randn_like(out), torch.randn_like(out)]
    G = torch.empty_like(m.ctrl)
    turn = [0]

    def adjoint():
        fa.decode_backward(m, res, gins[turn[0] % 2], 1, grad_ctrl=G)
        turn[0] += 1

    # (ten launches per replayed graph: a launch's own duration, without the
    # host's launch latency that events around a single call would include)
    fms, fev, _ = timed_launches(lambda: fa.decode(m, res, 1, plan=plan, out=out), 10, 10, 2,
                                 stream)
    bms, bev, _ = timed_launches(adjoint, 10, 10, 2, stream)
    nvox = b.nblocks * 64 ** 3
    lat = 4 * int(sum(int(n.prod()) for n in b.ncp))
    # loss and gradient of the fitted lattice against the FP64 oracle:
    # L = sum (B P - y)^2 / M and (2/M) B^T (B P - y) on 8 seeded blocks
    import oracle
    opt.zero_grad(set_to_none=True)
    loss = fa.FAFitMSE.apply(ctrl, m, res, yf, plan)
    loss.backward()
    grad = ctrl.grad.detach().double().cpu().numpy()
    P = ctrl.detach().double().cpu().numpy()
    sel = np.random.Generator(np.random.PCG64(97)).permutation(b.nblocks)[:8]
    ob = oracle.Blocks(b.ncp, b.deg, b.knot_off, b.ctrl_off, b.knots, P)
    f = oracle.decode_blocks(ob, res, 1)
    r = f - np.asarray(y, np.float64).reshape(b.nblocks, 1, *res)
    loss64 = float((r * r).sum() / nvox)
    sub = oracle.Blocks(b.ncp[sel], b.deg[sel], b.knot_off[sel], b.ctrl_off[sel], b.knots, P)
    G = oracle.decode_adjoint(sub, res, r[sel] * (2.0 / nvox), 1)
    gerr = 0.0
    for k in sel:
        o, n = int(b.ctrl_off[k]), int(np.prod(b.ncp[k]))
        gerr = max(gerr, float(np.abs(grad[o:o + n] - G[o:o + n]).max() /
                               np.abs(G[o:o + n]).max()))
    err = {"loss": abs(float(loss.detach()) - loss64) / loss64, "gradient": gerr,
           "sample": "loss over all 256 blocks; gradient max |gpu - fp64| / max |fp64| per "
                     "block on 8 seeded blocks, at the lattice after the timed steps"}
    # the timed form: the eager iteration or its HIP-graph replay (the same
    # kernels, one graph launch per iteration), whichever is faster
    form = "graph" if ms_g < ms else "eager"
    ms_best = min(ms, ms_g)
    return _common(args, "fit iterations/sec (forward decode + MSE + HIP adjoint + Adam)",
                   1e3 / ms_best, "iterations/s", ms_best, "f32",
                   "C4 fit: 256 micro-models, NCP* per axis in {16,24,32}, cubic, 64^3 "
                   "k^-5/3 samples each (67M), MSE through torch.autograd (fused residual "
                   "kernel), Adam",
                   {"roofline": _roof(nvox * 4 + lat, bev, "adjoint", "c4"),
                    "forward_decode": {"ms": fev, "GB/s": (nvox * 4 + lat) / (fev * 1e-3) / 1e9},
                    "adjoint": {"ms": bev, "GB/s": (nvox * 4 + lat) / (bev * 1e-3) / 1e9},
                    "timed_form": form,
                    "eager_ms_per_step": ms,
                    "graph_ms_per_step": ms_g,
                    "graph_loss_after_warmup_and_timed_replays": loss_graph,
                    "torch_composed_loss_ms_per_step": ms_t,
                    "loss_first_last": [first, last],
                    "err_vs_fp64": err},
                   ) | ({} if args.no_cpu_baseline else
                        {"cpu_baseline": cpu_baseline_fit(b, y, res, args.cpu_seconds)})


# ------------------------------------------------------------------ C5

def bench_c5(args):
    import numpy as np
    import torch

    import fa_inputs as fi
    import oracle
    import paper_2409_00184_amd as fa
    res = (64, 64, 64)
    b = fi.config_c5()
    m = fa.MicroModels.from_batch(b)
    nvox = b.nblocks * 64 ** 3
    out = torch.empty((b.nblocks, 4) + res, device="cuda")
    stream = torch.cuda.current_stream()
    from paper_2409_00184_amd import autotune
    # the 1% seeded uniform subset of (block, voxel) pairs: every variant is
    # compared on it with the FP64 oracle and with the FP32 path
    idx = fi.voxel_subset(b.nblocks, res, 0.01, seed=55)
    ref = oracle.decode_samples(oracle.Blocks(b.ncp, b.deg, b.knot_off, b.ctrl_off, b.knots,
                                              b.ctrl), res, idx)
    ti = torch.as_tensor(idx, device="cuda").long()
    names = ["value", "d/du", "d/dv", "d/dw"]
    scale = np.abs(ref).max(0)

    def gather(inter):
        o = out.view((b.nblocks,) + res + (4,)) if inter else out
        if inter:
            return o[ti[:, 0], ti[:, 1], ti[:, 2], ti[:, 3]].double().cpu().numpy()
        return o[ti[:, 0], :, ti[:, 1], ti[:, 2], ti[:, 3]].double().cpu().numpy()

    def rel(a, r):
        return {names[c]: float(np.abs(a[:, c] - r[:, c]).max() / scale[c]) for c in range(4)}

    # schedules the VALU kernel is tuned over for this uniform batch
    cands = [(r, w, gr, 0, 8192, st) for r in (8, 16) for w in (4, 8) for gr in (768, 1 << 20)
             for st in (0, 1)]
    variants = {}
    f32 = {}
    # planar [block][channel][x][y][z] output, and one 16-byte record per voxel
    for name, dtype, kernel, inter in (("f32_valu", "f32", 0, 0), ("bf16_mfma", "bf16", 1, 0),
                                       ("f16_mfma", "f16", 1, 0), ("bf16_valu", "bf16", 0, 0),
                                       ("f16_valu", "f16", 0, 0),
                                       ("f32_valu_interleaved", "f32", 0, 1),
                                       ("bf16_valu_interleaved", "bf16", 0, 1),
                                       ("bf16_mfma_interleaved", "bf16", 1, 1),
                                       ("f16_mfma_interleaved", "f16", 1, 1)):
        m.lattice(dtype)
        mk = 15 | fa.OUT_INTERLEAVED if inter else 15
        if kernel:
            plan = fa.Plan(m, res, kernel=1)
        else:
            plan, _ = autotune.tune(m, res, mk, dtype, candidates=cands,
                                    use_cache=not args.retune)
        graph, _ = fa.capture(lambda: fa.decode(m, res, mk, dtype=dtype, plan=plan, out=out))
        ms, ev_ms, _ = timed_steps(graph.replay, max(5, args.steps // 5), 2, stream)
        del graph
        lat_b = (4 if dtype == "f32" else 2) * b.ctrl.size
        got = gather(inter)
        if dtype == "f32":
            f32[inter] = got
        v = {"value": nvox / (ms * 1e-3), "ms_per_step": ms,
             "roofline": _roof(nvox * 16 + lat_b, ev_ms,
                               "decode_mfma" if kernel else "decode_sep", "c5"),
             "schedule": [plan.tune.rows_per_item, plan.tune.waves, plan.ngroups,
                          plan.tune.slab_floats, plan.tune.store],
             "err_vs_fp64": rel(got, ref)}
        if dtype != "f32":
            v["diff_vs_f32_path"] = rel(got, f32[inter])
        variants[name] = v
    del ti
    base = variants["f32_valu"]["ms_per_step"]
    for v in variants.values():
        v["speedup_vs_f32"] = base / v["ms_per_step"]
    for k in ("bf16_valu_interleaved", "bf16_mfma_interleaved", "f16_mfma_interleaved"):
        variants[k]["speedup_vs_f32_interleaved"] = (
            variants["f32_valu_interleaved"]["ms_per_step"] / variants[k]["ms_per_step"])
    # the timed form: the faster BF16 decode (matrix cores or VALU, both FP32
    # accumulation, planar output); every variant is reported beside it
    bname = min(("bf16_mfma", "bf16_valu"), key=lambda k: variants[k]["ms_per_step"])
    best = variants[bname]
    line = _common(args, METRIC, best["value"], "voxels/s", best["ms_per_step"], "bf16",
                   "C5 precision: 4096 micro-models of 32^3 control points (k^-5/3), cubic, "
                   "64^3 voxels each (1.07e9), value + 3 gradients; BF16/FP16 lattices with "
                   "per-block max-abs scale (FP32 accumulation on the matrix cores or the "
                   "VALU) vs FP32",
                   {"timed_variant": bname,
                    "roofline": best["roofline"], "err_vs_fp64": best["err_vs_fp64"],
                    "diff_vs_f32_path": best["diff_vs_f32_path"], "variants": variants,
                    "err_sample": f"1% seeded uniform subset of (block, voxel) pairs "
                                  f"({idx.shape[0]}), max |x - ref| / max |ref| per channel"})
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_decode(b, res, args.cpu_seconds)
    del out
    return line


def probe(args):
    """Counter run: a few plain launches (no graph) of the workload's dominant
    kernel, then one device copy of exactly 1 GiB each way (the reference for
    scaling FETCH_SIZE / WRITE_SIZE).  Prints what it ran."""
    import torch

    import fa_inputs as fi
    import paper_2409_00184_amd as fa
    res = (64, 64, 64)
    w = args.workload
    if w == "c3":
        b = fi.config_c3_blocks()
        m = fa.MicroModels.from_batch(b)
        xyz = c3_samples()
        boc = torch.as_tensor(fi.identity_cells(4096), device="cuda")
        out = torch.empty((xyz.shape[0], 4), device="cuda")
        run = lambda: fa.query_rays(m, xyz, 1920, 1080, 512, (16, 16, 16), (0, 0, 0),
                                    (1, 1, 1), boc, out=out)
    elif w == "c4":
        b, _ = fi.config_c4()
        m = fa.MicroModels.from_batch(b)
        gins = [torch.randn((b.nblocks, 1) + res, device="cuda") for _ in range(2)]
        G = torch.empty_like(m.ctrl)
        turn = [0]

        def run():  # two cotangents in turn, as the C4 line times the adjoint
            fa.decode_backward(m, res, gins[turn[0] % 2], 1, grad_ctrl=G)
            turn[0] += 1
    elif w == "f1":
        b = fi.config_c3_blocks()
        m = fa.MicroModels.from_batch(b)
        rays = torch.as_tensor(fi.render_rays(3, 1920, 1080), device="cuda")
        tf = torch.as_tensor(fi.transfer_function(4), device="cuda")
        boc = torch.as_tensor(fi.identity_cells(4096), device="cuda")
        img = torch.empty((1080, 1920, 4), device="cuda")
        run = lambda: fa.render(m, rays, 1920, 1080, tf, (16, 16, 16), (0, 0, 0), (1, 1, 1), boc,
                                512, opacity_max=2.0, tf_range=(-4.0, 4.0), out=img,
                                light=(0.0, 0.6, 0.8), ka=0.3, kd=0.6, ks=0.3, shininess=16.0)
    elif w == "f2":
        import numpy as np
        Y = torch.as_tensor(fi.turbulence_cube(fi.rng(12), 64, 64)).cuda().contiguous()
        m = fa.uniform_models(np.full((64, 3), 32), np.full(64, 3))
        fws = torch.empty(fa.lib.fa_fit_workspace(64, fa._i32x3(res), 32), dtype=torch.uint8,
                          device="cuda")
        dec = torch.empty_like(Y)
        run = lambda: (fa.fit(m, res, Y, workspace=fws),
                       fa.model_errors(m, res, Y, decoded=dec))
    elif w == "c5":
        # the FP32 VALU decode at the schedule the bench times, then the
        # BF16 matrix-core decode
        from paper_2409_00184_amd import autotune
        b = fi.config_c5()
        m = fa.MicroModels.from_batch(b)
        cands = [(r, wv, gr, 0, 8192, st) for r in (8, 16) for wv in (4, 8)
                 for gr in (768, 1 << 20) for st in (0, 1)]
        fplan = (fa.Plan(m, res, *args.probe_tune) if args.probe_tune else
                 autotune.tune(m, res, 15, "f32", candidates=cands)[0])
        m.lattice("bf16")
        plan = fa.Plan(m, res, kernel=1)
        out = torch.empty((b.nblocks, 4) + res, device="cuda")
        run = lambda: (fa.decode(m, res, 15, dtype="f32", plan=fplan, out=out),
                       fa.decode(m, res, 15, dtype="bf16", plan=plan, out=out))
    else:
        from paper_2409_00184_amd import autotune
        b = fi.config_c2() if w == "c2" else fi.config_c1()
        m = fa.MicroModels.from_batch(b)
        # C2 is timed in the interleaved layout, C1 in the planar one; the
        # schedule is the one the bench times (the autotuner's table) unless
        # --probe-tune names one
        mk = 15 | fa.OUT_INTERLEAVED if w == "c2" else 15
        plan = (fa.Plan(m, res, *args.probe_tune) if args.probe_tune else
                autotune.tune(m, res, mk, "f32")[0])
        out = torch.empty((b.nblocks, 4) + res, device="cuda")
        run = lambda: fa.decode(m, res, mk, plan=plan, out=out)
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"probe": w, "launches": args.steps, "copy_bytes_each_way": 1 << 30,
                      "tune": list(args.probe_tune) if args.probe_tune else "autotuner"}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="all",
                    choices=["all", "c1", "c2", "c3", "c4", "c5", "f1", "f2", "f3", "f4"],
                    help="all (default): the C2 line with C3, C4 and C5 as sub-records")
    ap.add_argument("--retune", action="store_true", help="ignore the autotuner cache")
    ap.add_argument("--tune", type=int, nargs=6, default=None,
                    metavar=("ROWS", "WAVES", "GRID", "KERNEL", "SLAB", "STORE"),
                    help="fixed decode schedule instead of the autotuner's")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-lowp", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--probe", action="store_true",
                    help="counter calibration run (decode launches + a 1 GiB copy)")
    ap.add_argument("--probe-tune", type=int, nargs=6, default=None,
                    metavar=("ROWS", "WAVES", "GRID", "KERNEL", "SLAB", "STORE"))
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the decode "
              "shards by micro-block with no exchange, so N GPUs is N independent runs",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", "0")))
    if args.probe:
        probe(args)
        return
    runs = {"c1": bench_c1, "c2": bench_c2, "c3": bench_c3, "c4": bench_c4,
            "c5": bench_c5, "f1": bench_f1, "f2": bench_f2, "f3": bench_f3, "f4": bench_f4}
    if args.workload != "all":
        print(json.dumps(runs[args.workload](args)), flush=True)
        return
    # the headline C2 line, with the other configurations of the metric as
    # sub-records (each with its own roofline, error and oracle baseline)
    t0 = time.perf_counter()
    line = bench_c2(args)
    log(f"C2 done ({time.perf_counter() - t0:.0f} s)")
    line["workloads"] = {}
    for w in ("c3", "c4", "c5"):
        torch.cuda.empty_cache()
        sub = runs[w](args)
        for k in ("n_gpus", "steps", "warmup", "scaling", "vs_baseline", "data"):
            sub.pop(k, None)
        line["workloads"][w] = sub
        log(f"{w.upper()} done ({time.perf_counter() - t0:.0f} s)")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
