"""Write tests/golden/c2_oracle.json: the FP64 CPU oracle's solve of the 2-D
1024^2 + 32-layer workload (kh = 0.5, Gaussian source, beta = 0.4, 8 levels,
FGMRES(30) to 1e-6).  Calls only oracle/ and synth/; run from the repo root:
    python tests/golden/make_golden.py
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


def main():
    w = W.c2()
    o = Oracle(Params(**w.params()), w.phi)
    t = time.time()
    u, info = o.fgmres(w.chi[0], tol=1e-6, restart=30, maxit=3000)
    dt = time.time() - t
    g = np.random.default_rng([W.SEED, 2, 777])
    idx = np.sort(g.choice(u.size, size=256, replace=False))
    flat = u.ravel()
    out = {
        "what": "oracle FGMRES(30) solve of synth.workloads.c2(), tol 1e-6, complex128",
        "iterations": info.iterations,
        "restarts": info.restarts,
        "relres_true": info.relres_true,
        "u_norm": float(np.linalg.norm(flat)),
        "sample_index": idx.tolist(),
        "sample_re": flat[idx].real.tolist(),
        "sample_im": flat[idx].imag.tolist(),
        "oracle_seconds": dt,
    }
    with open(os.path.join(ROOT, "tests", "golden", "c2_oracle.json"), "w") as f:
        json.dump(out, f)
    print(out["iterations"], out["relres_true"], dt)


if __name__ == "__main__":
    main()
