#!/usr/bin/env python3
"""Benchmark of the GMRES-smoothed CSG multigrid / FGMRES Helmholtz solve on one
MI355X.

Default workload (the largest single-GPU configuration, all in complex128):
the 3-D 128^3-interior problem with 16-cell ECS layers (phi = k^2 (1 + 0.3 g),
g a smooth random field with correlation length 8h, max kh = 0.5), 16
unit point sources solved together, beta = 0.4, 6 levels, V(1,1) with
GMRES(3), FGMRES(30) to true relative residual 1e-6.  One step = one complete
solve of all 16 right-hand sides (every pass of the hot path, setup excluded,
inputs resident in HBM); `value` counts right-hand sides solved per second.
The same inputs are then solved with the V-cycle in complex64 (outer FGMRES in
complex128), reported beside it as the mixed-precision gain.

Printed JSON (one line): solves/s as `value`, p50/p99 solve latency, V-cycle
GB/s, the roofline of the dominant pass (its algorithmic bytes per launch over
its average launch time, both measured with HIP events on the solve's stream
inside the timed region), a measured device-to-device copy ceiling, the CPU
oracle timed on a bounded sample, a second configuration (the 2-D 2048^2
three-layer model in complex128) and a bounded serving stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBPS = 8000.0
MALL_BYTES = 256 << 20
HERE = os.path.dirname(os.path.abspath(__file__))
PMC_SUMMARY = {"c2": "pmc_c2_1024sq_fp64.txt", "c4_fp64": "pmc_c4_128cube_16rhs_fp64.txt"}


def counted_traffic(kind: str, workload: str):
    """HBM bytes per launch of one pass kind from the committed rocprofv3
    counter summary of this workload, if it was taken on the current library
    sources (null otherwise)."""
    name = PMC_SUMMARY.get(workload)
    path = os.path.join(HERE, "profiles", name) if name else None
    if not path or not os.path.exists(path):
        return None
    from paper_1012_5379_amd.trace_summary import source_hash
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != source_hash():
        return None
    try:
        return float(vals[f"traffic_bytes_per_launch[{kind}]"])
    except (KeyError, ValueError):
        return None


def copy_ceiling(torch, mib=2048, reps=5):
    """Device-to-device copy rate (bytes read + written per second) of a plain
    torch copy of `mib` MiB, timed with events: the streaming ceiling the
    passes are compared with beside the nominal HBM peak."""
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2.0 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbps


METRIC = "solves/s & p99 latency at relres 1e-6; V-cycle GB/s vs HBM peak"


def _workload(name):
    from synth import workloads as W
    if name == "c2":
        return W.c2(), "2d_1024sq_ecs32_kh0.5_gauss_beta0.4_8lev_fp64"
    if name == "c3":
        return W.c3(), "2d_2048sq_ecs32_3layer_kh0.5_beta0.3_9lev_c64cycle"
    if name == "c3_fp64":
        return W.c3(cycle_prec=0), "2d_2048sq_ecs32_3layer_kh0.5_beta0.3_9lev_fp64"
    if name == "c1":
        return W.c1(), "2d_64sq_ecs8_k20_beta0.4_5lev_fp64"
    if name == "c4":
        return W.c4(), "3d_128cube_ecs16_16rhs_beta0.4_6lev_c64cycle"
    if name == "c4_fp64":
        return W.c4(cycle_prec=0), "3d_128cube_ecs16_16rhs_beta0.4_6lev_fp64"
    if name == "c2_mixed":
        return W.c2().with_(cycle_prec=1), "2d_1024sq_ecs32_kh0.5_gauss_beta0.4_8lev_c64cycle"
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(w, its_per_solve, sample_its):
    """Oracle (as it stands) on the same workload, per right-hand side like
    `value`: whole solves of the first right-hand sides, as many as fit in
    about 20 s (at least one) when a whole solve takes at most 30 s; otherwise
    the first `sample_its`-or-fewer FGMRES iterations of one right-hand side,
    scaled to the GPU solve's iteration count."""
    from oracle import oracle as O
    O.lib()
    p = O.Params(**w.params())
    t0 = time.perf_counter()
    o = O.Oracle(p, w.phi)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    o.fgmres(w.chi[0], tol=w.tol, restart=w.restart, maxit=2)
    probe = (time.perf_counter() - t0) / 2
    if probe * its_per_solve <= 30.0:
        nrhs = int(max(1, min(w.nrhs, 20.0 // max(probe * its_per_solve, 1e-6))))
        t0 = time.perf_counter()
        its = []
        for r in range(nrhs):
            _, info = o.fgmres(w.chi[r], tol=w.tol, restart=w.restart, maxit=w.maxit)
            its.append(info.iterations)
        dt = time.perf_counter() - t0
        return {
            "value": nrhs / dt,
            "unit": "solves/s",
            "cores": O.threads(),
            "kind": "oracle",
            "sample": (f"whole FGMRES solves of the first {nrhs} of {w.nrhs} right-hand sides of the same workload "
                       f"on the CPU oracle ({dt:.1f} s, iterations {its}; setup {t_setup:.2f} s excluded)"),
        }
    # a bounded sample: about 20 s of iterations, at most sample_its
    sample_its = int(max(3, min(sample_its, 20.0 / max(probe, 1e-6))))
    t0 = time.perf_counter()
    _, info = o.fgmres(w.chi[0], tol=w.tol, restart=w.restart, maxit=sample_its)
    dt = time.perf_counter() - t0
    per_it = dt / max(1, info.iterations)
    return {
        # one right-hand side timed: solves/s per right-hand side, the unit of `value`
        "value": 1.0 / (per_it * its_per_solve),
        "unit": "solves/s",
        "cores": O.threads(),
        "kind": "oracle",
        "sample": (f"first {info.iterations} FGMRES iterations of the same solve on the CPU oracle "
                   f"({dt:.1f} s, {per_it * 1e3:.1f} ms/iteration; setup {t_setup:.2f} s excluded), "
                   f"scaled to the {its_per_solve} iterations of a full solve of one right-hand side"),
    }


def vcycle_working_set(level_sizes, nrhs, csize, s=3):
    """Bytes the V-cycle touches: per non-coarsest level the cycle vectors
    (b, x twice, r, u_1..u_s, w twice) of every RHS, plus phi."""
    return sum(n * (nrhs * (s + 6) * csize + csize // 2) for n in level_sizes[:-1])


def second_workload(name, steps, tuned):
    """A second configuration beside the headline (default: the 2-D 2048^2
    three-layer model all in complex128): solves/s over `steps` timed solves
    after one warm-up solve, iteration count and true residual."""
    import torch
    from paper_1012_5379_amd import Operator
    from paper_1012_5379_amd import binding as B
    w, wname = _workload(name)
    params = dict(w.params(), cycle_prec=w.cycle_prec, max_rhs=w.nrhs, restart=w.restart)
    op = Operator(params, w.phi, tuned=tuned)
    chi = torch.from_numpy(w.chi).to("cuda")
    u = torch.empty_like(chi)
    stream = torch.cuda.current_stream().cuda_stream

    def solve():
        rc, infos = B.helm_solve(op.op, chi.data_ptr(), u.data_ptr(), w.nrhs, w.tol, w.restart, w.maxit, 0, stream)
        if rc != 0:
            raise RuntimeError(f"{wname}: solve did not converge: {B.STATUS.get(rc, rc)}")
        return infos

    solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infos = solve()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {"workload": wname, "value": steps * w.nrhs / el, "unit": "solves/s", "steps": steps,
           "ms_per_step": el / steps * 1e3, "iterations_per_solve": infos[0]["iterations"],
           "relres_true": max(i["relres_true"] for i in infos), "dtype": "f32" if w.cycle_prec else "f64"}
    print(f"[bench] second workload {wname}: {out['ms_per_step']:.1f} ms per solve, {out['iterations_per_solve']} its",
          file=sys.stderr, flush=True)
    del op
    torch.cuda.empty_cache()
    return out


def serving(count, streams, load, batch=4, graphs=False):
    """Serving stream: `count` seeded C5 requests (2-D 256^2..2048^2 and 3-D
    64^3..192^3, 1-8 point sources, complex64 cycle; requests of one size
    class queued together share one batched operator).  A closed-loop pass
    (every request queued at once) measures the saturated rate; an open-loop
    pass then replays Poisson arrivals at `load` times that rate.  Latency =
    arrival -> last RHS done, setup included."""
    import torch
    from synth import workloads as W
    from paper_1012_5379_amd.serve import Engine, report, request_from_workload

    t0 = time.perf_counter()
    base = [W.c5_request(i) for i in range(count)]
    print(f"[bench] c5: {count} requests generated in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)

    def reqs(arrivals):
        return [request_from_workload(w, rid=i, arrival=float(a)) for i, (w, a) in enumerate(zip(base, arrivals))]

    # warm-up (kernels loaded, allocator primed): two small requests
    eng = Engine(streams=streams, keep_solutions=False, cache=False, batch=batch, graphs=graphs)
    eng.run([request_from_workload(W.c5_request(10 ** 5 + i, dim=2, n=256), rid=i) for i in range(2)],
            realtime=False)
    eng.close()

    eng = Engine(streams=streams, keep_solutions=False, cache=False, batch=batch, graphs=graphs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = eng.run(reqs([0.0] * count), realtime=False)
    torch.cuda.synchronize()
    closed = report(done, time.perf_counter() - t0)
    closed["hbm_high_water_GB"] = eng.high_water / 1e9
    closed["batched_operators"] = eng.batches
    eng.close()
    print(f"[bench] c5 closed loop: {json.dumps(closed)}", file=sys.stderr, flush=True)

    rate = load * closed["requests_per_s"]
    arr, _ = W.c5_stream(count, rate)
    eng = Engine(streams=streams, keep_solutions=False, cache=False, batch=batch, graphs=graphs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = eng.run(reqs(arr), realtime=True)
    torch.cuda.synchronize()
    opened = report(done, time.perf_counter() - t0)
    opened["hbm_high_water_GB"] = eng.high_water / 1e9
    opened["batched_operators"] = eng.batches
    eng.close()
    print(f"[bench] c5 open loop: {json.dumps(opened)}", file=sys.stderr, flush=True)
    classes = {}
    for w in base:
        k = f"{w.dim}d_{w.n[0]}"
        classes[k] = classes.get(k, 0) + 1
    return {"workload": "c5_serving_stream_2d256-2048_3d64-192_1-8rhs_c64cycle", "requests": count,
            "classes": classes, "streams": streams, "max_batch": batch, "tol": 1e-6,
            "closed_loop": closed, "open_loop": dict(opened, offered_rate_rps=rate, load=load),
            "p50_latency_ms": opened["p50_latency_ms"], "p99_latency_ms": opened["p99_latency_ms"]}


def serve_bench(args):
    """--workload c5: the serving stream as the headline line."""
    sv = serving(args.requests, args.streams, args.load, args.batch)
    closed = sv["closed_loop"]
    out = {
        "metric": METRIC,
        "value": closed["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": sv["requests"],
        "warmup": 2,
        "ms_per_step": closed["seconds"] / sv["requests"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": sv["workload"], "requests": sv["requests"], "classes": sv["classes"],
                   "streams": sv["streams"], "max_batch": sv["max_batch"], "tol": 1e-6, "outer_dtype": "f64",
                   "parallelism": "single-gpu"},
        "closed_loop": closed,
        "open_loop": sv["open_loop"],
        "p50_latency_ms": sv["p50_latency_ms"],
        "p99_latency_ms": sv["p99_latency_ms"],
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4_fp64")
    ap.add_argument("--no-mixed", action="store_true", help="skip the complex64-cycle solve of the same inputs")
    ap.add_argument("--cpu-sample-its", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-survey", action="store_true", help="skip the per-pass time survey")
    ap.add_argument("--requests", type=int, default=24, help="c5: requests per pass")
    ap.add_argument("--streams", type=int, default=4, help="c5: concurrent solves")
    ap.add_argument("--load", type=float, default=0.75, help="c5: offered rate / saturated rate")
    ap.add_argument("--batch", type=int, default=4, help="c5: problems of one size class per batched operator")
    ap.add_argument("--serving-requests", type=int, default=12,
                    help="requests of the bounded serving stream reported beside the headline (0: skip)")
    ap.add_argument("--no-tuned", action="store_true", help="library default knobs instead of the tuned table")
    ap.add_argument("--second", default="c3_fp64",
                    help="a second workload timed beside the headline ('' to skip): solves/s of a few solves")
    ap.add_argument("--second-steps", type=int, default=2)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="one device-to-device copy of MIB MiB before the solves (a plain copy of known size "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the solver runs every solve on a single MI355X "
              "(requests and right-hand sides would shard across GPUs without exchange); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1012_5379_amd import Operator
    from paper_1012_5379_amd import binding as B

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c5":
        serve_bench(args)
        return

    w, wname = _workload(args.workload)
    params = dict(w.params(), cycle_prec=w.cycle_prec, max_rhs=w.nrhs, restart=w.restart)
    t0 = time.perf_counter()
    op = Operator(params, w.phi, tuned=not args.no_tuned)
    t_setup = time.perf_counter() - t0
    knobs = {k: op.params[k] for k in ("slab_blocks", "tile_mult", "slab_min", "tail_max", "fuse_max")
             if op.params.get(k)}
    chi = torch.from_numpy(w.chi).to("cuda")
    u = torch.empty_like(chi)
    if args.calibrate_copy > 0:
        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {n} bytes read, {n} bytes written", file=sys.stderr, flush=True)
        del src, dst
    stream = torch.cuda.current_stream().cuda_stream
    nrhs = w.nrhs

    def solve():
        rc, infos = B.helm_solve(op.op, chi.data_ptr(), u.data_ptr(), nrhs, w.tol, w.restart, w.maxit, 0, stream)
        if rc != 0:
            raise RuntimeError(f"solve did not converge: {B.STATUS.get(rc, rc)} {infos}")
        return infos

    print(f"[bench] workload {wname}: levels {op.levels} dims {op.dims[0]}; setup {t_setup:.2f}s", file=sys.stderr,
          flush=True)
    op_levels = [int(np.prod(d)) for d in op.dims[: op.levels]]
    n_levels = op.levels
    for i in range(args.warmup):
        infos = solve()
        print(f"[bench] warmup {i}: {infos[0]['iterations']} its, relres {infos[0]['relres_true']:.2e}, "
              f"{infos[0]['seconds'] * 1e3:.1f} ms", file=sys.stderr, flush=True)

    # untimed survey: kernel time per pass kind over one solve each
    survey = {}
    its = infos[0]["iterations"] if args.warmup else None
    if not args.no_survey:
        for name, kind in B.PROF_KINDS.items():
            B.csg_profile(op.op, kind, 1 << 16)
            infos = solve()
            ms, n, by = B.csg_profile_read(op.op)
            B.csg_profile(op.op, 0, 0)
            survey[name] = {"ms_per_solve": ms, "launches": n, "GBps": (by / (ms * 1e-3) / 1e9) if ms > 0 else 0.0}
            its = infos[0]["iterations"]
            print(f"[bench] survey {name}: {ms:.2f} ms over {n} launches, "
                  f"{survey[name]['GBps']:.0f} GB/s", file=sys.stderr, flush=True)
    passes = {k: v for k, v in survey.items() if k != "vcycle"}
    dominant = max(passes, key=lambda k: passes[k]["ms_per_solve"]) if passes else "outer_cgs1"

    # timed region: K solves as a user runs them (iterations replayed from
    # captured HIP graphs, no instrumentation)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        infos = solve()
        lat.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    graphs = B.csg_graphs_active(op.op)
    # the same K solves again with every launch of the dominant pass bracketed
    # by HIP events on its stream (timed launches run outside graphs: events
    # recorded inside a graph cannot be timed on this HIP)
    B.csg_profile(op.op, B.PROF_KINDS[dominant], 1 << 20)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        solve()
    torch.cuda.synchronize()
    elapsed_instr = time.perf_counter() - t1
    kms, kn, kbytes = B.csg_profile_read(op.op)
    B.csg_profile(op.op, 0, 0)
    its = infos[0]["iterations"]
    relres = max(i["relres_true"] for i in infos)

    # the same inputs with the V-cycle in complex64 (outer FGMRES complex128)
    mixed = None
    if not args.no_mixed and not w.cycle_prec:
        op = None
        torch.cuda.empty_cache()
        opm = Operator(dict(params, cycle_prec=1), w.phi, tuned=not args.no_tuned)

        def solve_m():
            rc, inf = B.helm_solve(opm.op, chi.data_ptr(), u.data_ptr(), nrhs, w.tol, w.restart, w.maxit, 0, stream)
            if rc != 0:
                raise RuntimeError(f"complex64-cycle solve did not converge: {B.STATUS.get(rc, rc)}")
            return inf

        for _ in range(max(1, args.warmup)):
            solve_m()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(args.steps):
            inf = solve_m()
        torch.cuda.synchronize()
        el_m = time.perf_counter() - t2
        mixed = {"value": args.steps * nrhs / el_m, "unit": "solves/s", "ms_per_step": el_m / args.steps * 1e3,
                 "gain_over_fp64": (args.steps * nrhs / el_m) / (args.steps * nrhs / elapsed),
                 "iterations_per_solve": inf[0]["iterations"],
                 "relres_true_max": max(i["relres_true"] for i in inf),
                 "cycle_dtype": "c64", "outer_dtype": "f64"}
        print(f"[bench] complex64 cycle: {mixed['ms_per_step']:.1f} ms per step, {inf[0]['iterations']} its, "
              f"gain {mixed['gain_over_fp64']:.3f}", file=sys.stderr, flush=True)
        del opm
    # (not in counter-calibration runs: their one plain copy must stay the largest)
    ceiling = copy_ceiling(torch) if args.calibrate_copy <= 0 else 0.0
    print(f"[bench] device copy ceiling {ceiling:.0f} GB/s", file=sys.stderr, flush=True)

    value = args.steps * nrhs / elapsed
    achieved = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else 0.0
    lat_ms = np.array(lat) * 1e3
    traffic = counted_traffic(dominant, args.workload)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.cycle_prec else "f64",
        "data": "synthetic",
        "config": {"workload": wname, "unknowns": int(w.unknowns), "nrhs": nrhs, "levels": n_levels,
                   "tol": w.tol, "restart": w.restart, "cycle": "V(1,1) GMRES(3)",
                   "outer_dtype": "f64", "parallelism": "single-gpu", "hip_graphs": graphs,
                   "tuned_knobs": knobs or "library defaults"},
        "iterations_per_solve": its,
        "relres_true": relres,
        "p50_latency_ms": float(np.percentile(lat_ms, 50)),
        "p99_latency_ms": float(np.percentile(lat_ms, 99)),
        "roofline": {
            "bound": "hbm",
            "kernel": dominant,
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic,
            "launches": kn,
            "avg_launch_us": kms * 1e3 / max(1, kn),
            "alg_bytes_per_launch": kbytes / max(1, kn),
            "region": f"{args.steps} solves right after the timed region, same inputs, each {dominant} launch "
                      f"timed with a HIP event pair ({elapsed_instr / args.steps * 1e3:.1f} ms per solve there)",
            "copy_ceiling": ceiling,
            "frac_of_copy_ceiling": achieved / ceiling if ceiling > 0 else None,
            # the counted HBM bytes over the same launch time: how close the
            # pass streams to the HBM limit, halo re-reads included
            "traffic_GBps": (traffic / (kms * 1e-3 / max(1, kn)) / 1e9) if traffic and kms > 0 else None,
            "traffic_frac": (traffic / (kms * 1e-3 / max(1, kn)) / 1e9 / HBM_PEAK_GBPS)
                            if traffic and kms > 0 else None,
        },
        "copy_ceiling_GBps": ceiling,
    }
    if mixed:
        out["mixed_precision"] = mixed
    if "vcycle" in survey:
        v = survey["vcycle"]
        out["vcycle_GBps"] = v["GBps"]
        out["vcycle_ms"] = v["ms_per_solve"] / max(1, v["launches"])
        out["vcycle_frac_of_hbm_peak"] = v["GBps"] / HBM_PEAK_GBPS
        # a working set inside the 256 MB Infinity Cache makes the rate an
        # effective one, not an HBM fraction
        ws = vcycle_working_set(op_levels, nrhs, 8 if w.cycle_prec else 16)
        out["vcycle_working_set_MB"] = ws / 1e6
        out["vcycle_rate_kind"] = "hbm" if ws > MALL_BYTES else "effective (Infinity-Cache resident working set)"
        out["pass_survey_ms_per_solve"] = {k: round(v["ms_per_solve"], 3) for k, v in survey.items()}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, its, args.cpu_sample_its)
    if args.second and args.second != args.workload:
        op = None
        torch.cuda.empty_cache()
        out["second_workload"] = second_workload(args.second, args.second_steps, not args.no_tuned)
    if args.serving_requests > 0:
        # a bounded serving stream beside the headline (its own workload: C5)
        op = None
        torch.cuda.empty_cache()
        out["serving"] = serving(args.serving_requests, args.streams, args.load, args.batch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
