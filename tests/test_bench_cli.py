"""bench.py contract checks that need no GPU: the one-GPU guard and the rule
that counted HBM traffic is reported only for the pass and workload the
committed counter summary covers, taken on the current library sources."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_counted_traffic_only_for_its_pass_and_workload():
    import bench
    assert bench.counted_traffic("stencil_dots", "c2") is None
    assert bench.counted_traffic("fused", "c3") is None


def test_counted_traffic_needs_matching_sources(tmp_path, monkeypatch):
    import bench
    from paper_1012_5379_amd.trace_summary import source_hash
    f = tmp_path / "pmc.txt"
    f.write_text("traffic_bytes_per_launch: 123456\nsource_sha256: " + source_hash() + "\n")
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(f))
    assert bench.counted_traffic("fused", "c2") == pytest.approx(123456.0)
    f.write_text("traffic_bytes_per_launch: 123456\nsource_sha256: " + "0" * 64 + "\n")
    assert bench.counted_traffic("fused", "c2") is None
