"""Host logic of bench.py that needs no GPU: the counter-traffic lookup (launch-weighted
over a kernel's template instances, only while the library sources are unchanged) and
the refusal to run on more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_traffic_is_launch_weighted_over_instances(tmp_path, monkeypatch):
    import bench
    doc = {"source_hash": "x", "kernels": {
        "fg::k_reduce_panel<double, 1>": {"launches": 3, "traffic_bytes": 100.0},
        "fg::k_reduce_panel<double, 2>": {"launches": 1, "traffic_bytes": 500.0},
        "fg::k_reduce_vec<double>": {"launches": 9, "traffic_bytes": 7.0}}}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "pmc_large_1d.md").write_text("# t\n\n```json\n" + json.dumps(doc) + "\n```\n")
    src = tmp_path / "paper_2006_06537_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "a.hip").write_text("kernel text")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    import hashlib
    h = hashlib.sha256(b"kernel text").hexdigest()[:16]
    assert bench.counter_traffic("k_reduce_panel") is None  # sources changed since
    doc["source_hash"] = h
    (prof / "pmc_large_1d.md").write_text("# t\n\n```json\n" + json.dumps(doc) + "\n```\n")
    assert bench.counter_traffic("k_reduce_panel") == pytest.approx((3 * 100 + 500) / 4)
    assert bench.counter_traffic("k_reduce_vec") == pytest.approx(7.0)
    assert bench.counter_traffic("k_leaf") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
