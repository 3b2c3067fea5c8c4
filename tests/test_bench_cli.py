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


def _trace_csv(path, launches):
    """A kernel-trace CSV of (name, workgroups, microseconds) launches in order."""
    import csv
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Grid_Size_X", "Workgroup_Size_X", "Start_Timestamp", "End_Timestamp"])
        t = 0
        for name, blocks, us in launches:
            w.writerow([f"void csg::{name}(int)", blocks * 512, 512, t, t + int(us * 1000)])
            t += int(us * 1000) + 1000


def test_trace_summary_kinds_and_working_launches(tmp_path, capsys):
    """The 3-D fused kind holds only the finest level's k_slab passes (not the
    slab transfer or w = H z passes of the same grid), pass 0 goes to
    stencil_dots, and the working averages leave out the no-op launches of
    columns queued after convergence."""
    from paper_1012_5379_amd import trace_summary as T
    launches = []
    for _ in range(10):
        launches += [("k_slab<double, 4, -1>", 152, 500.0), ("k_slab<double, 4, 0>", 152, 1000.0),
                     ("k_slab<double, 4, 1>", 152, 1200.0), ("k_slab_pr<double>", 152, 900.0),
                     ("k_slab_down<double, 4>", 152, 1100.0), ("k_slab<double, 4, 1>", 136, 200.0),
                     ("k_slab_hdot<double>", 152, 1800.0), ("k_proj0w<double, 4, 1, true>", 256, 5000.0)]
    # one column queued after convergence: every pass a no-op
    launches += [("k_slab<double, 4, -1>", 152, 4.0), ("k_slab<double, 4, 0>", 152, 4.0),
                 ("k_slab<double, 4, 1>", 152, 4.0), ("k_slab_hdot<double>", 152, 4.0)]
    p = tmp_path / "t.csv"
    _trace_csv(p, launches)
    names = [n for n, _, _ in launches]
    blocks = [b for _, b, _ in launches]
    kinds = T.kind_launches([T._short(f"void csg::{n}(int)") for n in names], blocks)
    assert {names[i] for i in kinds["fused"]} == {"k_slab<double, 4, 0>", "k_slab<double, 4, 1>"}
    assert all(blocks[i] == 152 for i in kinds["fused"])
    assert {names[i] for i in kinds["stencil_dots"]} == {"k_slab<double, 4, -1>"}
    assert {names[i] for i in kinds["outer_h"]} == {"k_slab_hdot<double>"}
    assert T.working([1000.0, 1200.0, 4.0, 1100.0]) == [1000.0, 1200.0, 1100.0]
    T.kernels(str(p))
    out = capsys.readouterr().out
    line = [l for l in out.splitlines() if l.startswith("fused:")][0]
    assert "n 22," in line and "working launches 20, avg 1100.00 us" in line
