"""The third-order polynomial smoother (section 4) on the GPU against the FP64
CPU oracle: the per-level angle and Richardson weights built by the library's
setup, one sweep on every level, the polynomial-smoothed V-cycle (V(1,1),
V(2,1), V(1,0), V(0,2)) and the FGMRES solve it preconditions, 2-D and 3-D,
the tiled 2-D sweep and the three-pass one, both cycle precisions."""
import numpy as np
import pytest

from oracle.oracle import Oracle, Params
from synth import workloads as W
from tests.gpu_common import dev, host, note, rel, rvec, torch_cuda

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 6e-6


def _case(dim, **kw):
    if dim == 2:
        return W.small(dim=2, n=150, mlo=11, mhi=8, beta=0.35, kh=0.5, item=21, **kw)
    return W.small(dim=3, n=27, mlo=3, mhi=4, beta=0.4, kh=0.4, item=22, **kw)


def _pair(w, prec, max_rhs=2):
    from paper_1012_5379_amd import Operator
    params = dict(w.params(), cycle_prec=prec, max_rhs=max_rhs, restart=30, smoother=1)
    note(f"[case] {w.name} dims={w.grid_shape} poly prec={prec} nu=({w.nu1},{w.nu2})")
    op = Operator(params, w.phi)
    orc = Oracle(Params(**w.params(), smoother=1), w.phi)
    assert op.levels == orc.levels
    return op, orc


@pytest.mark.parametrize("dim", [2, 3])
def test_polynomial_per_level_matches_oracle(dim):
    from paper_1012_5379_amd import binding as B
    torch_cuda()
    op, orc = _pair(_case(dim), 0)
    for l in range(op.levels):
        vp, om, conds = B.csg_poly_info(op.op, l)
        d = orc.poly(l)
        e = max(abs(a - b) / abs(b) for a, b in zip(om, d["omega"]))
        note(f"  level {l}: varphi {np.degrees(vp):.6f} deg (oracle {np.degrees(d['varphi']):.6f}), "
             f"conds {conds}/{d['conds']}, weights rel err {e:.1e}")
        assert conds == d["conds"]
        assert abs(np.exp(1j * vp) - np.exp(1j * d["varphi"])) <= 1e-12
        assert e <= 1e-12


@pytest.mark.parametrize("tiles", ["1", "0"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dim", [2, 3])
def test_polynomial_sweep_every_level(dim, prec, tiles, monkeypatch):
    monkeypatch.setenv("CSG_POLY_TILES", tiles)
    torch_cuda()
    op, orc = _pair(_case(dim), prec)
    for l in range(op.levels):
        b = np.stack([rvec(orc.shape(l), 700 + l), rvec(orc.shape(l), 710 + l)])
        x0 = np.stack([rvec(orc.shape(l), 720 + l), rvec(orc.shape(l), 730 + l)]) * 1e-3
        x = host(op.smooth(dev(b, op.cdtype), dev(x0, op.cdtype), level=l))
        for r in range(2):
            e = rel(x[r], orc.poly_sweep(b[r], x0[r], l=l))
            note(f"  tiles {tiles} prec {prec} level {l} rhs {r}: {e:.2e}")
            assert e <= (TOL64 if prec == 0 else TOL32)


SHAPES = {"V(1,1)": (1, 1), "V(2,1)": (2, 1), "V(1,0)": (1, 0), "V(0,2)": (0, 2)}


@pytest.mark.parametrize("tiles", ["1", "0"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("shape", list(SHAPES))
def test_polynomial_vcycle(shape, dim, prec, tiles, monkeypatch):
    monkeypatch.setenv("CSG_POLY_TILES", tiles)
    torch_cuda()
    nu1, nu2 = SHAPES[shape]
    op, orc = _pair(_case(dim, nu1=nu1, nu2=nu2), prec)
    b = np.stack([rvec(orc.shape(0), 740), rvec(orc.shape(0), 741)])
    x = host(op.vcycle(dev(b, op.cdtype)))
    for r in range(2):
        e = rel(x[r], orc.vcycle(b[r]))
        note(f"  {shape} {dim}-D tiles {tiles} prec {prec} rhs {r}: {e:.2e}")
        assert e <= (TOL64 if prec == 0 else TOL32)


@pytest.mark.parametrize("dim", [2, 3])
def test_polynomial_fgmres_matches_oracle(dim):
    """FGMRES preconditioned by the polynomial-smoothed V(1,1)-cycle: outer
    iterations +-1 and solution within 1e-10 of the oracle's."""
    import torch
    w = _case(dim)
    op, orc = _pair(w, 0, max_rhs=1)
    u, rc, infos = op.solve(dev(w.chi[:1], torch.complex128), tol=1e-8, restart=30, maxit=1000)
    uo, io = orc.fgmres(w.chi[0], tol=1e-8, restart=30, maxit=1000)
    e = rel(host(u)[0], uo)
    note(f"  poly {dim}-D: its gpu {infos[0]['iterations']} oracle {io.iterations} sol err {e:.2e}")
    assert rc == 0 and io.converged
    assert abs(infos[0]["iterations"] - io.iterations) <= 1
    assert e <= 1e-10
