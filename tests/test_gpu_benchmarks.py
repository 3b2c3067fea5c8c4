"""The paper's own benchmark problems on the GPU at its settings (section 5:
theta_beta = 10.3132 degrees, tolerance 1e-7, kh <= 0.625): Benchmark 1
(constant k, point source, layers on every side) and Benchmark 3 (the
Gaussian model: Dirichlet on the south and west edges, layers on the north
and east), complex128 throughout, against the FP64 oracle on the same inputs
(iterations +-1, solution within 1e-10, or as close as the oracle is to
itself under rounding-size perturbations where the problem is that
sensitive).  The counts are printed beside the paper's tables (ballpark
only: layer width and restart are unstated)."""
import json
import os

import pytest

from oracle.oracle import Oracle, Params
from synth import workloads as W
from tests.gpu_common import dev, host, note, pair, rel, torch_cuda

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _check(w, restart, printed):
    """Iterations +-1 and solutions within 1e-10, unless the oracle itself is
    that sensitive: where relative perturbations of 1e-15 in the right-hand
    side move the oracle's own solution and iteration count (the bound states
    of Benchmark 3 at nu > 2.73 put isolated eigenvalues of H close to zero,
    section 5), the GPU must agree with the oracle as closely as the oracle
    agrees with itself over six such perturbations (10x margin on the
    solution, their iteration spread + 1).  The GPU solution's true residual
    is recomputed with the oracle's H either way."""
    import numpy as np
    import torch
    torch_cuda()
    op, orc = pair(w, max_rhs=1, cycle_prec=0, restart=restart)
    u, rc, infos = op.solve(dev(w.chi[:1], torch.complex128), tol=w.tol, restart=restart, maxit=3000)
    uo, io = orc.fgmres(w.chi[0], tol=w.tol, restart=restart, maxit=3000)
    ug = host(u)[0]
    e = rel(ug, uo)
    chi = w.chi[0].reshape(ug.shape)
    res = np.linalg.norm(chi - orc.apply(ug, which=0)) / np.linalg.norm(chi)
    note(f"  {w.name}: its gpu {infos[0]['iterations']} oracle {io.iterations} paper {printed}; "
         f"sol err {e:.2e}; gpu true relres {res:.2e}")
    assert rc == 0 and io.converged
    assert res <= w.tol * (1 + 1e-6)
    e_tol, it_tol = 1e-10, 1
    if e > e_tol or abs(infos[0]["iterations"] - io.iterations) > it_tol:
        # the oracle's own spread over six rounding-size perturbations
        spread, e_self = 0, 0.0
        for seed in range(6):
            noise = np.random.default_rng(12345 + seed).standard_normal(chi.shape)
            up, ip = orc.fgmres(chi * (1 + 1e-15 * noise), tol=w.tol, restart=restart, maxit=3000)
            spread = max(spread, abs(ip.iterations - io.iterations))
            e_self = max(e_self, rel(up, uo))
        note(f"    oracle self-sensitivity: sol {e_self:.2e}, iterations +-{spread}")
        e_tol = max(e_tol, 10 * e_self)
        it_tol += spread
    assert abs(infos[0]["iterations"] - io.iterations) <= it_tol
    assert e <= e_tol


@pytest.mark.parametrize("k", [20, 40, 60, 80])
def test_benchmark1_constant_k(k):
    with open(os.path.join(GOLDEN, "paper_table2_benchmark1.json")) as f:
        printed = json.load(f)["V(1,1)"][str(k)]["iterations"]
    _check(W.benchmark1(k), 30, printed)


@pytest.mark.parametrize("nu", [1, 7])
@pytest.mark.parametrize("k", [0.5, 1.5, 2.5])
def test_benchmark3_gaussian_model(k, nu):
    with open(os.path.join(GOLDEN, "paper_tables45_benchmark3.json")) as f:
        printed = json.load(f)[f"nu={nu}"]["V(1,1)"][str(k)]
    _check(W.benchmark3(k, nu), 64, printed)
