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
    assert bench.counted_traffic("fused", "c3") is None          # no counter summary for this workload
    assert bench.counted_traffic("no_such_kind", "c4_fp64") is None


def test_counted_traffic_needs_matching_sources(tmp_path, monkeypatch):
    import bench
    from paper_1012_5379_amd.trace_summary import source_hash
    (tmp_path / "profiles").mkdir()
    f = tmp_path / "profiles" / "pmc.txt"
    monkeypatch.setattr(bench, "HERE", str(tmp_path))
    monkeypatch.setattr(bench, "PMC_SUMMARY", {"c4_fp64": "pmc.txt"})
    f.write_text("traffic_bytes_per_launch[fused]: 123456\nsource_sha256: " + source_hash() + "\n")
    assert bench.counted_traffic("fused", "c4_fp64") == pytest.approx(123456.0)
    assert bench.counted_traffic("outer_h", "c4_fp64") is None
    f.write_text("traffic_bytes_per_launch[fused]: 123456\nsource_sha256: " + "0" * 64 + "\n")
    assert bench.counted_traffic("fused", "c4_fp64") is None


def test_vcycle_working_set_labels():
    """The 1024^2 FP64 cycle's vectors fit the 256 MB Infinity Cache (an
    effective rate); the 16-RHS 128^3 cycle's do not (an HBM fraction)."""
    import bench
    c2 = [1087 ** 2, 543 ** 2, 271 ** 2, 135 ** 2, 67 ** 2, 33 ** 2, 16 ** 2, 8 ** 2]
    c4 = [159 ** 3, 79 ** 3, 39 ** 3, 19 ** 3, 9 ** 3, 4 ** 3]
    assert bench.vcycle_working_set(c2, 1, 16) < bench.MALL_BYTES
    assert bench.vcycle_working_set(c4, 16, 16) > bench.MALL_BYTES
