"""The paper's own benchmark problems on the GPU at its settings (section 5:
theta_beta = 10.3132 degrees, tolerance 1e-7, kh <= 0.625): Benchmark 1
(constant k, point source, layers on every side) and Benchmark 3 (the
Gaussian model: Dirichlet on the south and west edges, layers on the north
and east), complex128 throughout, against the FP64 oracle on the same inputs
(iterations +-1, solution within 1e-10).  The counts are printed beside the
paper's tables (ballpark only: layer width and restart are unstated)."""
import json
import os

import pytest

from oracle.oracle import Oracle, Params
from synth import workloads as W
from tests.gpu_common import dev, host, note, pair, rel, torch_cuda

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _check(w, restart, printed):
    import torch
    torch_cuda()
    op, orc = pair(w, max_rhs=1, cycle_prec=0, restart=restart)
    u, rc, infos = op.solve(dev(w.chi[:1], torch.complex128), tol=w.tol, restart=restart, maxit=3000)
    uo, io = orc.fgmres(w.chi[0], tol=w.tol, restart=restart, maxit=3000)
    e = rel(host(u)[0], uo)
    note(f"  {w.name}: its gpu {infos[0]['iterations']} oracle {io.iterations} paper {printed}; sol err {e:.2e}")
    assert rc == 0 and io.converged
    assert abs(infos[0]["iterations"] - io.iterations) <= 1
    assert e <= 1e-10


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
