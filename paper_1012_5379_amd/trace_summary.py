"""Summaries of rocprofv3 output for one benchmark run of libcsg.

    python -m paper_1012_5379_amd.trace_summary kernels TRACE_CSV
    python -m paper_1012_5379_amd.trace_summary counters FETCH_CSV WRITE_CSV --copy-bytes N
    python -m paper_1012_5379_amd.trace_summary occupancy SQ_CSV
    python -m paper_1012_5379_amd.trace_summary ranges KERNEL_CSV HIP_API_CSV MARKER_CSV

`kernels` reads a kernel trace (rocprofv3 --kernel-trace --output-format csv)
and prints, per kernel and grid size, the dispatch count and the average, min
and max duration (and over the launches that did work, see `working`), then
the pass kinds bench.py times on their own.  The 2-D
finest-level fused pass shares its kernel and grid size with the next level's,
so its launches are told apart by position: every FGMRES iteration is one
V-cycle followed by k_hdot, and the V-cycle opens and closes on the finest
level, so its first two and last two fused launches are the finest level's
(s = 3); 3-D slab passes of the finest level have the largest grid.

`counters` reads two counter collections of the same command (rocprofv3
--pmc FETCH_SIZE, then --pmc WRITE_SIZE; KiB per dispatch), scales each by
what the counter reads for the run's plain device-to-device copy of
--copy-bytes bytes (the largest __amd_rocclr_copyBuffer dispatch), and prints
the HBM bytes per dispatch of every kernel and per launch of each pass kind,
with the hash of the library sources the counters belong to.

`occupancy` reads one collection of SQ counters (SQ_WAVES, SQ_WAVE_CYCLES,
SQ_BUSY_CYCLES, SQ_WAIT_INST_ANY, SQ_INSTS_VALU, SQ_INSTS_VMEM_RD,
SQ_INSTS_VMEM_WR, SQ_INSTS_LDS) and prints per kernel and grid the mean
counts per dispatch, the wave-cycles per busy cycle (proportional to the mean
number of resident waves: compare across kernels) and the share of wave time
spent waiting on an outstanding instruction (mostly memory).

`ranges` attributes kernel time to the library's roctx ranges (CSG_ROCTX=1,
eager launches: CSG_GRAPHS=0; rocprofv3 --kernel-trace --hip-trace
--marker-trace): each dispatch is matched to its launch call by correlation
id, the call to the innermost range open on its thread at that time, and the
kernel time is summed per range (the outer column number dropped).
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os
import sys

FUSED = "k_os_tile"
CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def source_hash() -> str:
    """sha256 over the library's sources (kernel counters are stale once it changes)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").replace("csg::", "").strip()


def _rows(path):
    with open(path) as f:
        return list(csv.DictReader(f))


def finest_fused(names):
    """Indices (into the time-ordered dispatch list) of the finest-level fused
    passes: per V-cycle window (between the previous iteration's last pass and
    k_hdot) the first two and the last two fused launches."""
    out = []
    start = 0
    for i, nm in enumerate(names):
        if nm.startswith("k_hdot"):
            win = [k for k in range(start, i) if names[k].startswith(FUSED)]
            if len(win) >= 4:
                out += win[:2] + win[-2:]
            start = i + 1
    return out


def kernels(trace: str) -> None:
    rows = sorted(_rows(trace), key=lambda r: int(r["Start_Timestamp"]))
    dur = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows]
    names = [_short(r["Kernel_Name"]) for r in rows]
    by = collections.defaultdict(list)
    for r, nm, d in zip(rows, names, dur):
        g = int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"])
        by[(nm, g)].append(d)
    tot = sum(dur)
    print(f"{'kernel':44s} {'blocks':>6s} {'n':>7s} {'avg us':>9s} {'min us':>8s} {'max us':>8s} {'total %':>8s} "
          f"{'work n':>7s} {'work avg us':>11s}")
    for (nm, g), v in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        w = working(v)
        print(f"{nm[:44]:44s} {g:6d} {len(v):7d} {sum(v) / len(v):9.2f} {min(v):8.2f} {max(v):8.2f} "
              f"{100 * sum(v) / tot:8.2f} {len(w):7d} {sum(w) / max(1, len(w)):11.2f}")
    blocks = [_blocks(r) for r in rows]
    for kind, idx in kind_launches(names, blocks).items():
        d = [dur[i] for i in idx]
        w = working(d)
        print(f"\n{kind}: n {len(d)}, avg {sum(d) / len(d):.2f} us, min {min(d):.2f} us, max {max(d):.2f} us; "
              f"working launches {len(w)}, avg {sum(w) / max(1, len(w)):.2f} us")
    print(f"dispatches {len(rows)}, kernel time {tot / 1e3:.2f} ms")


def working(d):
    """The launches that did work: a solve queues FGMRES columns ahead of the
    convergence reports, and the columns queued after every right-hand side
    has stopped run as no-op launches of a few microseconds (all blocks return
    at once); bench.py drops them from its timings too.  Launches shorter than
    a third of the median of the same kernel and grid are taken for those."""
    if not d:
        return []
    m = sorted(d)[len(d) // 2]
    return [x for x in d if x >= m / 3]


def _blocks(r) -> int:
    """Workgroups of a dispatch (counter collections give the total grid)."""
    if "Grid_Size" in r:
        return int(r["Grid_Size"]) // int(r["Workgroup_Size"])
    return (int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"])) * int(r.get("Grid_Size_Y", 1))


def kind_launches(names, blocks):
    """Dispatch indices of the pass kinds bench.py times: the finest level's
    fused Arnoldi passes and pass 0 (2-D tiles: by position, see finest_fused;
    3-D slabs: the largest grid of k_slab), and the three outer FGMRES passes."""
    out = {}
    fused2 = finest_fused(names)
    if fused2:
        out["fused"] = fused2
        out["stencil_dots"] = [i for i, nm in enumerate(names) if nm.startswith("k_st0_tile")]
    slab = [i for i, nm in enumerate(names) if nm.startswith("k_slab<")]
    if slab:
        top = max(blocks[i] for i in slab)
        out["fused"] = [i for i in slab if blocks[i] == top and not names[i].endswith("-1>")]
        out["stencil_dots"] = [i for i in slab if blocks[i] == top and names[i].endswith("-1>")]
    # w = H z: one kernel per column, or (3-D slabs, columns of more than 8
    # vectors) k_slab_hdot followed by k_hdot_groups
    out["outer_h"] = [i for i, nm in enumerate(names) if nm.startswith(("k_hdot", "k_slab_hdot"))]
    out["outer_cgs1"] = [i for i, nm in enumerate(names) if nm.startswith("k_proj0")]
    out["outer_proj2"] = [i for i, nm in enumerate(names) if nm.startswith("k_proj1")]
    return {k: v for k, v in out.items() if v}


def counters(fetch_csv: str, write_csv: str, copy_bytes: int) -> None:
    per = {}
    scales = {}
    names = blocks = None
    for key, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = sorted(_rows(path), key=lambda r: int(r["Dispatch_Id"]))
        nm = [_short(r["Kernel_Name"]) for r in rows]
        vals = [float(r["Counter_Value"]) * 1024.0 for r in rows]
        copies = [v for n, v in zip(nm, vals) if n.startswith("__amd_rocclr_copyBuffer")]
        ref = max(copies) if copies else 0.0
        scale = copy_bytes / ref if ref > 0 else float("nan")
        scales[key] = (scale, ref)
        per[key] = [v * scale for v in vals]
        names, blocks = nm, [_blocks(r) for r in rows]
    f, w = scales["FETCH_SIZE"], scales["WRITE_SIZE"]
    print(f"calibration copy: {copy_bytes} bytes; FETCH_SIZE read {f[1]:.0f} bytes (scale {f[0]:.4f}), "
          f"WRITE_SIZE read {w[1]:.0f} bytes (scale {w[0]:.4f})")
    print("\nper kernel and grid (workgroups), scaled bytes per dispatch:")
    print(f"{'kernel':40s} {'blocks':>7s} {'n':>6s} {'fetch MB':>10s} {'write MB':>10s}")
    agg = collections.defaultdict(list)
    for i, (n, b) in enumerate(zip(names, blocks)):
        agg[(n, b)].append(i)
    tot = lambda ix, k: sum(per[k][i] for i in ix)
    for (n, b), ix in sorted(agg.items(), key=lambda kv: -(tot(kv[1], "FETCH_SIZE") + tot(kv[1], "WRITE_SIZE")))[:30]:
        print(f"{n[:40]:40s} {b:7d} {len(ix):6d} {tot(ix, 'FETCH_SIZE') / len(ix) / 1e6:10.1f} "
              f"{tot(ix, 'WRITE_SIZE') / len(ix) / 1e6:10.1f}")
    print("\nper pass kind (bench.py's names), bytes per launch that did work (see `working`):")
    for kind, ix in kind_launches(names, blocks).items():
        tb = [per["FETCH_SIZE"][i] + per["WRITE_SIZE"][i] for i in ix]
        m = sorted(tb)[len(tb) // 2]
        ix = [i for i, t in zip(ix, tb) if t >= m / 3]
        fe = tot(ix, "FETCH_SIZE") / len(ix)
        wr = tot(ix, "WRITE_SIZE") / len(ix)
        print(f"launches[{kind}]: {len(ix)}")
        print(f"fetch_bytes_per_launch[{kind}]: {fe:.0f}")
        print(f"write_bytes_per_launch[{kind}]: {wr:.0f}")
        print(f"traffic_bytes_per_launch[{kind}]: {fe + wr:.0f}")
    print(f"source_sha256: {source_hash()}")


def occupancy(sq_csv: str) -> None:
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for r in _rows(sq_csv):
        key = (_short(r["Kernel_Name"]), _blocks(r))
        agg[key][r["Counter_Name"]] += float(r["Counter_Value"])
        disp[key].add(r["Dispatch_Id"])
    print(f"{'kernel':36s} {'blocks':>6s} {'n':>5s} {'waves':>7s} {'VALU/wave':>10s} {'VMEM rd/wave':>12s} "
          f"{'LDS/wave':>9s} {'wave-cyc/busy':>13s} {'wait share':>10s}")
    for key in sorted(agg, key=lambda k: -agg[k]["SQ_BUSY_CYCLES"]):
        a, n = agg[key], len(disp[key])
        waves = a["SQ_WAVES"] / n
        per = lambda c: a[c] / max(1.0, a["SQ_WAVES"])
        occ = a["SQ_WAVE_CYCLES"] / a["SQ_BUSY_CYCLES"] if a["SQ_BUSY_CYCLES"] else 0.0
        wait = a["SQ_WAIT_INST_ANY"] / a["SQ_WAVE_CYCLES"] if a["SQ_WAVE_CYCLES"] else 0.0
        print(f"{key[0][:36]:36s} {key[1]:6d} {n:5d} {waves:7.0f} {per('SQ_INSTS_VALU'):10.0f} "
              f"{per('SQ_INSTS_VMEM_RD'):12.0f} {per('SQ_INSTS_LDS'):9.0f} {occ:13.2f} {wait:10.3f}")
    print(f"source_sha256: {source_hash()}")


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(names[0])


def ranges(kernel_csv: str, hip_csv: str, marker_csv: str) -> None:
    import bisect
    import re
    kern = {}
    for r in _rows(kernel_csv):
        kern[r["Correlation_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    calls = {}
    for r in _rows(hip_csv):
        if "Launch" in _col(r, "Function", "Operation"):
            calls[r["Correlation_Id"]] = (r["Thread_Id"], int(r["Start_Timestamp"]))
    by_thread = collections.defaultdict(list)
    for r in _rows(marker_csv):
        name = _col(r, "Function", "Message", "Operation")
        by_thread[r["Thread_Id"]].append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), name))
    for v in by_thread.values():
        v.sort()
    tot = collections.defaultdict(float)
    unmatched = 0.0
    for cid, us in kern.items():
        c = calls.get(cid)
        best = None
        if c:
            lst = by_thread.get(c[0], [])
            i = bisect.bisect_right(lst, (c[1], float("inf"), ""))
            # innermost open range: the latest-starting one that still covers the call
            for k in range(i - 1, max(-1, i - 64), -1):
                s0, e0, nm = lst[k]
                if s0 <= c[1] <= e0:
                    best = nm
                    break
        if best is None:
            unmatched += us
        else:
            tot[re.sub(r"FGMRES column \d+", "FGMRES column", best)] += us
    allt = sum(tot.values()) + unmatched
    print(f"{'range':40s} {'kernel ms':>10s} {'share %':>8s}")
    for nm, us in sorted(tot.items(), key=lambda kv: -kv[1]):
        print(f"{nm[:40]:40s} {us / 1e3:10.2f} {100 * us / allt:8.2f}")
    print(f"{'(outside any range)':40s} {unmatched / 1e3:10.2f} {100 * unmatched / allt:8.2f}")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("trace")
    c = sub.add_parser("counters")
    c.add_argument("fetch")
    c.add_argument("write")
    c.add_argument("--copy-bytes", type=int, required=True)
    o = sub.add_parser("occupancy")
    o.add_argument("sq")
    g = sub.add_parser("ranges")
    g.add_argument("kernel")
    g.add_argument("hip")
    g.add_argument("marker")
    a = ap.parse_args(argv)
    if a.cmd == "kernels":
        kernels(a.trace)
    elif a.cmd == "occupancy":
        occupancy(a.sq)
    elif a.cmd == "ranges":
        ranges(a.kernel, a.hip, a.marker)
    else:
        counters(a.fetch, a.write, a.copy_bytes)


if __name__ == "__main__":
    sys.exit(main())
