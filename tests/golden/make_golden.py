"""Write the oracle's stored answers of the full-size 2-D workloads, which the
GPU tests compare against (the oracle is too slow to run inside them):

  c2_oracle.json  synth.workloads.c2(): 1024^2 + 32 layers, kh = 0.5, Gaussian
                  source, beta = 0.4, 8 levels, FGMRES(30) to 1e-6
  c3_oracle.json  synth.workloads.c3(cycle_prec=0): 2048^2 + 32 layers, three
                  wave-speed layers, beta = 0.3, 9 levels, FGMRES(30) to 1e-6
                  and to 1e-12 (the reference answer a solve stopping at 1e-6
                  is measured against, and the distance of the 1e-6 answer
                  from it: the error floor of any solve stopping there)
  c4_oracle.json  synth.workloads.c4(cycle_prec=0): 3-D 128^3 + 16 layers,
                  beta = 0.4, 6 levels, FGMRES(30) to 1e-6, complex128; the
                  first and the last of its 16 point sources (entries rhs0,
                  rhs15), 8192 sampled entries each, and the first again to
                  1e-12 (tight0) with the error floor of a 1e-6 solve (floor0)

Each file holds the iteration counts and true residuals, the solution norm, a
seeded sample of solution entries and the inner products of the solution with
a few seeded random vectors.  Calls only oracle/ and synth/; run from the repo
root:  python tests/golden/make_golden.py c2|c3|c4
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle, Params  # noqa: E402
from synth import workloads as W  # noqa: E402

NSAMPLE = 16384
NPROJ = 4


def sample_index(size, cfg_id, n=NSAMPLE):
    g = np.random.default_rng([W.SEED, cfg_id, 777])
    return np.sort(g.choice(size, size=min(n, size), replace=False))


def probes(shape, cfg_id):
    """Seeded random complex vectors whose inner products with u are stored."""
    return [W.rand_cvec(shape, item=900 + q, cfg_id=cfg_id) for q in range(NPROJ)]


def describe(u, idx, prb):
    flat = u.ravel()
    return {
        "u_norm": float(np.linalg.norm(flat)),
        "sample_re": flat[idx].real.tolist(),
        "sample_im": flat[idx].imag.tolist(),
        "proj": [[float(np.vdot(q.ravel(), flat).real), float(np.vdot(q.ravel(), flat).imag)] for q in prb],
    }


def solve(o, chi, tol, maxit):
    t = time.time()
    u, info = o.fgmres(chi, tol=tol, restart=30, maxit=maxit)
    dt = time.time() - t
    print(f"  tol {tol:g}: {info.iterations} iterations, relres {info.relres_true:.3e}, {dt:.0f} s", flush=True)
    assert info.converged
    return u, {"tol": tol, "iterations": info.iterations, "restarts": info.restarts,
               "relres_true": info.relres_true, "oracle_seconds": dt}


def main(name):
    if name == "c2":
        w, cfg, tight = W.c2(), 2, False
        what = "oracle FGMRES(30) solve of synth.workloads.c2(), tol 1e-6, complex128"
    elif name == "c3":
        w, cfg, tight = W.c3(cycle_prec=0), 3, True
        what = ("oracle FGMRES(30) solves of synth.workloads.c3(cycle_prec=0), tol 1e-6 and 1e-12, "
                "complex128")
    elif name == "c4":
        w, cfg = W.c4(cycle_prec=0), 4
        o = Oracle(Params(**w.params()), w.phi)
        idx = sample_index(w.unknowns, cfg, 8192)
        prb = probes(w.grid_shape, cfg)
        out = dict(what="oracle FGMRES(30) solves of synth.workloads.c4(cycle_prec=0), right-hand sides 0 and 15, "
                        "tol 1e-6, complex128", nsample=len(idx), sample_index=idx.tolist(),
                   probe_items=[900 + q for q in range(NPROJ)], probe_cfg_id=cfg)
        for r in (0, 15):
            u, info = solve(o, w.chi[r], 1e-6, 3000)
            out[f"rhs{r}"] = dict(info, **describe(u, idx, prb))
            if r == 0:
                # the reference a complex64-cycle solve stopping at 1e-6 is
                # measured against, and the error floor of any such solve
                ut, it = solve(o, w.chi[0], 1e-12, 20000)
                out["tight0"] = dict(it, **describe(ut, idx, prb))
                out["floor0"] = float(np.linalg.norm(u - ut) / np.linalg.norm(ut))
                print(f"  floor |u(1e-6) - u(1e-12)| / |u(1e-12)| = {out['floor0']:.3e}", flush=True)
        with open(os.path.join(ROOT, "tests", "golden", "c4_oracle.json"), "w") as f:
            json.dump(out, f)
        return
    else:
        raise SystemExit("usage: make_golden.py c2|c3|c4")
    o = Oracle(Params(**w.params()), w.phi)
    idx = sample_index(w.unknowns, cfg)
    prb = probes(w.grid_shape, cfg)
    u6, i6 = solve(o, w.chi[0], 1e-6, 6000)
    out = dict(what=what, nsample=len(idx), sample_index=idx.tolist(),
               probe_items=[900 + q for q in range(NPROJ)], probe_cfg_id=cfg)
    out.update(i6)
    out.update(describe(u6, idx, prb))
    if tight:
        ut, it = solve(o, w.chi[0], 1e-12, 20000)
        out["tight"] = dict(it, **describe(ut, idx, prb))
        out["floor"] = float(np.linalg.norm(u6 - ut) / np.linalg.norm(ut))
        print(f"  floor |u(1e-6) - u(1e-12)| / |u(1e-12)| = {out['floor']:.3e}", flush=True)
    with open(os.path.join(ROOT, "tests", "golden", f"{name}_oracle.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c2")
