"""Ballpark of the oracle against the paper's iteration tables at the paper's
settings (section 5: theta_beta = 10.3132 degrees, tolerance 1e-7, kh <=
0.625).  The ECS layer width, the restart length and the transfer operators
are not stated in the paper, so the counts are parity unpinned: they are
checked to lie within a factor two of the printed ones (layers of n/4 cells,
FGMRES restarted every 64 iterations, the longest restart the library
supports)."""
import json
import os

import numpy as np
import pytest

from oracle.oracle import Oracle, Params
from synth import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _its(w, restart=64):
    o = Oracle(Params(**w.params()), w.phi)
    _, info = o.fgmres(w.chi[0], tol=w.tol, restart=restart, maxit=3000)
    assert info.converged
    return info.iterations


@pytest.mark.parametrize("nu", [1, 7])
@pytest.mark.parametrize("k", [0.5, 1.5])
def test_benchmark3_gaussian_model_ballpark(k, nu):
    with open(os.path.join(GOLDEN, "paper_tables45_benchmark3.json")) as f:
        g = json.load(f)
    printed = g[f"nu={nu}"]["V(1,1)"][str(k)]
    w = W.benchmark3(k, nu)
    assert w.grid_shape == (g["grid"][str(k)] + g["grid"][str(k)] // 4 - 1,) * 2
    its = _its(w)
    print(f"benchmark 3 k={k} nu={nu}: oracle {its}, paper {printed}")
    assert printed / 2 <= its <= 2 * printed


@pytest.mark.parametrize("k", [40, 60])
def test_benchmark1_paper_settings_ballpark(k):
    with open(os.path.join(GOLDEN, "paper_table2_benchmark1.json")) as f:
        g = json.load(f)
    printed = g["V(1,1)"][str(k)]["iterations"]
    its = _its(W.benchmark1(k), restart=30)
    print(f"benchmark 1 k={k}: oracle {its}, paper {printed}")
    assert printed / 2 <= its <= 2 * printed


def test_benchmark3_setup_follows_the_model():
    """The Gaussian model's inputs: Dirichlet (no layer) on the low sides, n/4
    layer cells on the high sides, phi and chi sampled at the nodes x = j h."""
    w = W.benchmark3(0.5, 7)
    n, h = 64, 50.0 / 64
    assert w.layer_lo == (0, 0) and w.layer_hi == (16, 16)
    x = h * np.arange(1, n + 16)
    assert np.isclose(w.phi[0, 0], 7 * (np.exp(-x[0] ** 2) * 2) + 0.25)
    assert np.isclose(w.chi[0, 3, 5].real, 1.0 / (np.exp(x[5] ** 2) + np.exp(x[3] ** 2)))
    # beyond the interior box phi keeps its value at x = 50
    assert np.isclose(w.phi[-1, -1], 7 * 2 * np.exp(-50.0 ** 2) + 0.25)
