"""Host-side checks of bench.py (no GPU): the one-GPU contract, and that
the traffic figures it reports are used only when they were measured on the
current kernel sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in (r.stdout + r.stderr)


@pytest.mark.parametrize("kernel,workload", [("decode_sep", "c2"), ("query", "c3"),
                                             ("adjoint", "c4"), ("decode_mfma", "c5"),
                                             ("render", "f1"), ("fit", "f2")])
def test_traffic_files_match_sources(kernel, workload):
    """bench.py reports a committed traffic summary only when it was taken on
    the kernel sources in the tree, and null otherwise."""
    import bench
    with open(os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")) as f:
        t = json.load(f)
    if t["source_hash"] == bench.source_hash(kernel):
        assert bench.traffic_from_profiles(kernel, workload) == t["hbm_bytes_per_launch"]
    else:
        assert bench.traffic_from_profiles(kernel, workload) is None
    # the counters see at least the algorithmic bytes (the render re-fetches
    # lattice lines, about 4.7x; the others stay within 10%)
    ratio = t["hbm_bytes_per_launch"] / t["alg_bytes_per_launch"]
    assert 0.99 < ratio < (5.0 if kernel == "render" else 1.2)
