"""Cycle shapes of section 3.2 on the GPU against the FP64 CPU oracle:
V(1,0), V(2,1), V(0,1), GMRES(s) smoothing with s = 1, 2, 4 (s = 4 takes the
untiled passes), and the two-grid cycle (levels = 2), in 2-D and 3-D.  Each
shape: one V-cycle per precision (complex128 1e-12; complex64 the stated
single-precision bound) and the complex128 FGMRES solve (iterations +-1,
solution within 1e-10 of the oracle's)."""
import numpy as np
import pytest

from synth import workloads as W
from tests.gpu_common import dev, host, note, pair, rel, rvec, torch_cuda

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 6e-6   # about ten times the largest complex64 error observed

SHAPES = {
    "V(1,0)s3": dict(s=3, nu1=1, nu2=0),
    "V(2,1)s3": dict(s=3, nu1=2, nu2=1),
    "V(0,1)s3": dict(s=3, nu1=0, nu2=1),
    "V(1,1)s1": dict(s=1, nu1=1, nu2=1),
    "V(1,1)s2": dict(s=2, nu1=1, nu2=1),
    "V(1,1)s4": dict(s=4, nu1=1, nu2=1),
    "V(2,2)s4": dict(s=4, nu1=2, nu2=2),
    "2grid": dict(s=3, nu1=1, nu2=1, levels=2),
}


def _work(dim, shape):
    kw = SHAPES[shape]
    if kw.get("levels") == 2:
        # two grids: the coarse grid must stay within the dense-solve limit
        if dim == 2:
            return W.small(dim=2, n=40, mlo=5, mhi=6, beta=0.4, kh=0.5, item=11, **kw)
        return W.small(dim=3, n=12, mlo=2, mhi=3, beta=0.4, kh=0.4, item=12, **kw)
    if dim == 2:
        return W.small(dim=2, n=150, mlo=11, mhi=8, beta=0.35, kh=0.5, item=13, **kw)
    return W.small(dim=3, n=27, mlo=3, mhi=4, beta=0.4, kh=0.4, item=14, **kw)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("shape", list(SHAPES))
def test_vcycle_shape(shape, dim, prec):
    torch_cuda()
    w = _work(dim, shape)
    op, orc = pair(w, max_rhs=2, cycle_prec=prec)
    b = np.stack([rvec(orc.shape(0), 500), rvec(orc.shape(0), 501)])
    x = host(op.vcycle(dev(b, op.cdtype)))
    for r in range(2):
        e = rel(x[r], orc.vcycle(b[r]))
        note(f"  {shape} {dim}-D prec {prec} levels {op.levels} rhs {r}: {e:.2e}")
        assert e <= (TOL64 if prec == 0 else TOL32)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("shape", list(SHAPES))
def test_fgmres_shape(shape, dim):
    import torch
    w = _work(dim, shape)
    op, orc = pair(w, max_rhs=1, cycle_prec=0)
    u, rc, infos = op.solve(dev(w.chi[:1], torch.complex128), tol=1e-8, restart=30, maxit=800)
    uo, io = orc.fgmres(w.chi[0], tol=1e-8, restart=30, maxit=800)
    e = rel(host(u)[0], uo)
    note(f"  {shape} {dim}-D: its gpu {infos[0]['iterations']} oracle {io.iterations} sol err {e:.2e}")
    assert rc == 0 and io.converged
    assert abs(infos[0]["iterations"] - io.iterations) <= 1
    assert e <= 1e-10
