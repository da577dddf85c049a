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
                                             ("render", "f1"), ("fit", "f2"),
                                             ("decode_sep", "c5")])
def test_traffic_files_match_sources(kernel, workload):
    """Every committed traffic summary was taken on the kernel sources in the
    tree (a kernel changed since its counters were read must be profiled
    again), and bench.py reports its figure."""
    import bench
    with open(os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")) as f:
        t = json.load(f)
    assert t["source_hash"] == bench.source_hash(kernel), \
        f"profiles/{kernel}_{workload}_traffic.json is stale: profile the kernel again"
    assert bench.traffic_from_profiles(kernel, workload) == t["hbm_bytes_per_launch"]
    # the counters see at least the algorithmic bytes (the render re-fetches
    # lattice lines, the ray-ordered query copies each micro-model a ray tile
    # enters into LDS: about one copy per tile and micro-model, from L2 and
    # the Infinity Cache; the others stay within 20%)
    ratio = t["hbm_bytes_per_launch"] / t["alg_bytes_per_launch"]
    assert 0.99 < ratio < {"render": 5.0, "query": 2.0}.get(kernel, 1.2)


def test_stale_traffic_summary_reports_null(tmp_path):
    """A summary taken on other kernel sources is not reported."""
    import bench
    good = {"kernel": "decode_sep", "workload": "c2", "hbm_bytes_per_launch": 123.0,
            "alg_bytes_per_launch": 120.0, "source_hash": bench.source_hash("decode_sep")}
    (tmp_path / "decode_sep_c2_traffic.json").write_text(json.dumps(good))
    assert bench.traffic_from_profiles("decode_sep", "c2", str(tmp_path)) == 123.0
    stale = dict(good, source_hash="0" * 12)
    (tmp_path / "decode_sep_c2_traffic.json").write_text(json.dumps(stale))
    assert bench.traffic_from_profiles("decode_sep", "c2", str(tmp_path)) is None
    assert bench.traffic_from_profiles("decode_sep", "c9", str(tmp_path)) is None
