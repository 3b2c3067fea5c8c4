"""Autotuner of libcsg's execution knobs.

The knobs change how the passes are laid out on the GPU, never what they
compute (results move by rounding only): the z-marching slab workgroups per
right-hand side and the level size from which 3-D levels take the slab
passes, the LDS tiles per chunked-pass block of the 2-D fused passes, the
fused-pass size limit and the level size from which the one-workgroup coarse
tail takes over.  For one problem the tuner times a fixed number of FGMRES
iterations (tolerance unreachable, so every candidate does the same work) for
each candidate value of one knob at a time, keeps the fastest, and repeats the
sweep until no knob moves (coordinate descent from the library defaults).

The table is JSON keyed by (dimension, cycle precision, smoother, size class);
the size class is log2 of the finest-level unknowns times the right-hand sides
solved together, rounded, since that product sets how many workgroups a pass
has to fill the chip with.  ``Operator(..., tuned=True)`` looks the key up and
fills in every knob the caller left at 0 (library default).

    python -m paper_1012_5379_amd.tune --workload c4_fp64 --out tuned.json

writes (or merges into) the table; the package's own table is ``tuned.json``
beside this file.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

from . import binding as B

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")

# candidate values per knob (0 never appears: it means "library default")
CANDIDATES = {
    2: {"tile_mult": [1, 2, 4], "fuse_max": [-1, 300000, 4000000], "tail_max": [-1, 600, 1200, 5000]},
    3: {"slab_blocks": [32, 64, 128, 256, 512], "slab_min": [20000, 100000, 400000, -1],
        "tail_max": [-1, 600, 1200, 8000]},
}
# the library's defaults, the descent's starting point
DEFAULTS = {"tile_mult": 1, "fuse_max": 300000, "tail_max": 1200, "slab_blocks": 128, "slab_min": 100000}
KNOBS = ("slab_blocks", "tile_mult", "slab_min", "tail_max", "fuse_max")


def key(params: dict) -> str:
    """Table key of a parameter set: dimension, cycle precision, smoother and
    size class (log2 of finest unknowns x right-hand sides, rounded)."""
    p = B.make_params(**{k: v for k, v in params.items() if k not in KNOBS})
    _, dims = B.csg_plan_levels(p)
    n = 1
    for d in dims[0][: p.dim]:
        n *= int(d)
    cls = int(round(math.log2(max(1, n * max(1, p.max_rhs)))))
    prec = "c64" if p.cycle_prec else "c128"
    smo = "poly" if p.smoother else "gmres"
    return f"d{p.dim}-{prec}-{smo}-2^{cls}"


def load(path: str = TABLE) -> dict:
    if not os.path.exists(path):
        return {"entries": {}}
    with open(path) as f:
        t = json.load(f)
    t.setdefault("entries", {})
    return t


def knobs_for(params: dict, path: str = TABLE) -> dict:
    """The tuned knobs for these parameters (empty when the table has no entry)."""
    e = load(path)["entries"].get(key(params))
    return dict(e["knobs"]) if e else {}


def apply(params: dict, path: str = TABLE) -> dict:
    """params with every knob the caller left at 0 (or absent) taken from the table."""
    out = dict(params)
    for k, v in knobs_for(params, path).items():
        if not out.get(k):
            out[k] = v
    return out


def time_iterations(params: dict, phi, chi, iters: int = 8, repeats: int = 3) -> float:
    """Seconds per FGMRES iteration (minimum over repeats) of one operator
    built with these parameters: `iters` iterations of every right-hand side
    with an unreachable tolerance, after one untimed run that captures graphs."""
    import torch
    from . import Operator
    op = Operator(params, phi)
    try:
        c = torch.from_numpy(chi).to("cuda")
        u = torch.empty_like(c)
        stream = torch.cuda.current_stream().cuda_stream
        nrhs = c.shape[0]
        restart = int(params.get("restart", 30))

        def run():
            rc, infos = B.helm_solve(op.op, c.data_ptr(), u.data_ptr(), nrhs, 1e-300, restart, iters, 0, stream)
            if rc not in (0, B.CSG_ENOCONV):
                raise RuntimeError(f"tuning solve failed: {B.STATUS.get(rc, rc)}")
            return infos

        run()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(repeats):
            t0 = time.perf_counter()
            infos = run()
            torch.cuda.synchronize()
            best = min(best, (time.perf_counter() - t0) / max(1, infos[0]["iterations"]))
        return best
    finally:
        del op
        torch.cuda.empty_cache()


def tune(params: dict, phi, chi, iters: int = 8, repeats: int = 3, passes: int = 2, log=None) -> dict:
    """Coordinate descent over CANDIDATES[dim] from DEFAULTS; a move must gain
    more than 1% to count (timing noise).  Returns the table entry."""
    dim = int(params["dim"])
    cand = CANDIDATES[dim]
    cur = {k: DEFAULTS[k] for k in cand}
    trials = []
    seen = {}

    def measure(kn):
        t = tuple(sorted(kn.items()))
        if t not in seen:
            seen[t] = time_iterations(dict(params, **kn), phi, chi, iters, repeats)
            trials.append({"knobs": dict(kn), "ms_per_iteration": seen[t] * 1e3})
            if log:
                log(f"[tune] {kn}: {seen[t] * 1e3:.3f} ms/iteration")
        return seen[t]

    base = measure(cur)
    best = base
    for _ in range(passes):
        moved = False
        for k, vals in cand.items():
            for v in vals:
                if v == cur[k]:
                    continue
                kn = dict(cur, **{k: v})
                t = measure(kn)
                if t < best * 0.99:
                    best, cur, moved = t, kn, True
        if not moved:
            break
    return {"knobs": cur, "ms_per_iteration": best * 1e3, "default_ms_per_iteration": base * 1e3,
            "iterations_timed": iters, "trials": trials}


def merge(path: str, k: str, entry: dict, device: str) -> None:
    t = load(path)
    t["entries"][k] = dict(entry, device=device)
    with open(path, "w") as f:
        json.dump(t, f, indent=1, sort_keys=True)
        f.write("\n")


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", action="append", required=True,
                    help="synthetic workload to tune on (c2, c3, c3_fp64, c4, c4_fp64); repeatable")
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--iters", type=int, default=8)
    ap.add_argument("--repeats", type=int, default=3)
    a = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("tuning needs a HIP device", file=sys.stderr)
        return 2
    from synth import workloads as W
    named = {"c2": lambda: W.c2(), "c3": lambda: W.c3(), "c3_fp64": lambda: W.c3(cycle_prec=0),
             "c4": lambda: W.c4(), "c4_fp64": lambda: W.c4(cycle_prec=0)}
    dev = torch.cuda.get_device_name(0)
    for name in a.workload:
        w = named[name]()
        params = dict(w.params(), cycle_prec=w.cycle_prec, max_rhs=w.nrhs, restart=w.restart)
        k = key(params)
        print(f"[tune] {name} -> {k}", flush=True)
        e = tune(params, w.phi, w.chi, a.iters, a.repeats, log=lambda s: print(s, flush=True))
        e["workload"] = name
        merge(a.out, k, e, dev)
        print(f"[tune] {name}: {e['knobs']} {e['ms_per_iteration']:.3f} ms/iteration "
              f"(defaults {e['default_ms_per_iteration']:.3f})", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
