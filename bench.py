#!/usr/bin/env python3
"""Throughput of the micro-model decode/query path on one MI355X.

Default workload (C2): batched decode of 512 micro-models with NCP* per axis
drawn from {8,12,16,24,32} and degree from {2,3}, each decoded to a 64^3
voxel grid (value + 3 gradient channels, FP32), as one persistent launch
replayed from a captured HIP graph, schedule picked by the autotuner.

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
    "query": ["paper_2409_00184_amd/csrc/fa_query.hip", "paper_2409_00184_amd/csrc/fa_device.hpp"],
    "decode_mfma": ["paper_2409_00184_amd/csrc/fa_mfma.hip",
                    "paper_2409_00184_amd/csrc/fa_device.hpp"],
    "adjoint": ["paper_2409_00184_amd/csrc/fa_adjoint.hip",
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


def traffic_from_profiles(kernel, workload):
    """HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE and
    WRITE_SIZE (scaled by the copy-kernel calibration), from
    profiles/<kernel>_<workload>_traffic.json, if taken on this exact kernel
    source; else None."""
    p = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
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


def cpu_baseline_decode(batch, res, target_s=15.0):
    """The FP64 oracle (as it stands) on a seeded sample of whole blocks."""
    import numpy as np

    import oracle
    th = oracle.nthreads_default()
    ob = oracle.Blocks(batch.ncp, batch.deg, batch.knot_off, batch.ctrl_off, batch.knots,
                       batch.ctrl)
    g = np.random.Generator(np.random.PCG64(99))
    order = g.permutation(batch.nblocks)
    vox = int(np.prod(res))
    # calibrate on one block, then size the sample for ~target_s
    sub = lambda k: oracle.Blocks(ob.ncp[order[:k]], ob.deg[order[:k]], ob.knot_off[order[:k]],
                                  ob.ctrl_off[order[:k]], ob.knots, ob.ctrl)
    t0 = time.perf_counter()
    oracle.decode_blocks(sub(1), res, 15, nthreads=th)
    t1 = time.perf_counter() - t0
    k = int(max(1, min(batch.nblocks, target_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    oracle.decode_blocks(sub(k), res, 15, nthreads=th)
    dt = time.perf_counter() - t0
    return {"value": k * vox / dt, "unit": "voxels/s", "cores": th, "kind": "oracle",
            "sample": f"{k} of {batch.nblocks} blocks (seeded), full {res[0]}^3 grids, "
                      f"value+grad, FP64, {dt:.1f} s"}


def err_vs_oracle_decode(batch, out, res, nsample=20000, src=None):
    """Max |gpu - FP64| / max |FP64| per channel on seeded voxels."""
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
    plan, report = autotune.tune(m, res, 15, "f32", use_cache=not args.retune)
    log("schedule", [plan.tune.rows_per_item, plan.tune.waves, plan.ngroups,
                     plan.tune.slab_floats, plan.tune.store],
        "fastest candidates", sorted(report, key=lambda r: r[1])[:6])
    out = torch.empty((batch.nblocks, 4) + res, dtype=torch.float32, device="cuda")
    graph, _ = fa.capture(lambda: fa.decode(m, res, 15, plan=plan, out=out))
    ms, ev_ms, ev_min = timed_steps(graph.replay, args.steps, args.warmup, stream)
    nvox = batch.nblocks * res[0] * res[1] * res[2]
    value = nvox / (ms * 1e-3)
    lattice_bytes = 4 * int(sum(int(n.prod()) for n in batch.ncp))
    alg_bytes = nvox * 16 + lattice_bytes + 4 * batch.knots.size + 64 * batch.nblocks
    achieved = alg_bytes / (ev_ms * 1e-3) / 1e9
    err = err_vs_oracle_decode(batch, out, res)
    line = {
        "metric": METRIC, "value": value, "unit": "voxels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C2 batched decode: 512 micro-models, NCP* per axis in "
                               "{8,12,16,24,32}, degree in {2,3}, 64^3 voxels each, value + 3 "
                               "gradients, FP32, one persistent launch replayed from a HIP graph",
                   "nblocks": batch.nblocks, "res": list(res), "channels": 4,
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
    }
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
            o2 = torch.empty_like(out)
            g2, _ = fa.capture(lambda: fa.decode(m, res, 15, dtype=dt, plan=plan, out=o2))
            lms, lev, _ = timed_steps(g2.replay, args.steps, args.warmup, stream)
            lp[dt] = {"value": nvox / (lms * 1e-3), "ms_per_step": lms,
                      "speedup_vs_f32": ms / lms,
                      "err_vs_fp64": err_vs_oracle_decode(batch, o2, res)}
        line["lowp_storage"] = lp
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_decode(batch, res, args.cpu_seconds)
    return line


def probe(args):
    """Counter calibration run: a few plain launches of the workload's
    dominant kernel and one device copy of exactly 1 GiB (the reference for
    FETCH_SIZE / WRITE_SIZE scaling).  Prints what it ran."""
    import torch

    import fa_inputs as fi
    import paper_2409_00184_amd as fa
    res = (64, 64, 64)
    batch = fi.config_c2()
    m = fa.MicroModels.from_batch(batch)
    plan = fa.Plan(m, res, *args.probe_tune)
    out = torch.empty((batch.nblocks, 4) + res, dtype=torch.float32, device="cuda")
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        fa.decode(m, res, 15, plan=plan, out=out)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "c2", "decode_launches": args.steps,
                      "copy_bytes_each_way": 1 << 30, "tune": list(args.probe_tune)}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2", choices=["c2"])
    ap.add_argument("--retune", action="store_true", help="ignore the autotuner cache")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-lowp", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--probe", action="store_true",
                    help="counter calibration run (decode launches + a 1 GiB copy)")
    ap.add_argument("--probe-tune", type=int, nargs=4, default=[8, 4, 768, 0],
                    metavar=("ROWS", "WAVES", "GRID", "KERNEL"))
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
    line = {"c2": bench_c2}[args.workload](args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
