"""GPU parity of the complex-shifted preconditioner M = L(beta) - s phi
(beta = 0, s = 1 + i eps: the complex shifted Laplacian of sections 1-2;
beta > 0 with s != 1 as well) against the FP64 oracle on the same inputs:
M on every level, every level's GMRES(s) sweep and the V-cycle at 1e-12
(complex128), the FGMRES solve with iterations +-1 and solution within
1e-10, the complex64 cycle's solution against the oracle's tightly converged
answer; on the default passes (LDS tiles, slabs) and with every level on the
unfused multi-block passes.  Also the equivalence the paper relies on: on a
grid without ECS layers the CSG preconditioner is e^{-2i beta} times the one
with beta = 0 and s = e^{2i beta}, so FGMRES takes the same iterations."""
import cmath

import numpy as np
import pytest

from oracle.oracle import Oracle, Params
from tests.gpu_common import dev, host, note, rel, rvec, tight_oracle, torch_cuda
from synth import workloads as W

pytestmark = pytest.mark.gpu

UNFUSED = {"CSG_TILES": "0", "CSG_FUSE_MAX": "0", "CSG_TAIL_MAX": "0", "CSG_HDOT_TILES": "0", "CSG_SLABS": "0"}
CASES = {
    "2d_csl": (lambda: W.small(dim=2, n=101, mlo=7, mhi=4, beta=0.0, kh=0.45, item=1), 1 + 0.5j),
    "3d_csl": (lambda: W.small(dim=3, n=27, mlo=3, mhi=4, beta=0.0, kh=0.4, item=3), 1 + 0.5j),
    "2d_csg_shift": (lambda: W.small(dim=2, n=101, mlo=7, mhi=4, beta=0.35, kh=0.45, item=1), 0.9 + 0.3j),
}


def _pair(w, shift, prec, max_rhs=2):
    from paper_1012_5379_amd import Operator
    note(f"[case] {w.name} shift {shift} prec {prec}")
    op = Operator(dict(w.params(), cycle_prec=prec, max_rhs=max_rhs, restart=30, shift=shift), w.phi)
    orc = Oracle(Params(**w.params(), shift=shift), w.phi)
    assert op.levels == orc.levels
    return op, orc


@pytest.mark.parametrize("path", ["default", "unfused"])
@pytest.mark.parametrize("name", list(CASES))
def test_operators_sweeps_vcycle(name, path, monkeypatch):
    torch_cuda()
    if path == "unfused":
        for k, v in UNFUSED.items():
            monkeypatch.setenv(k, v)
    w, shift = CASES[name][0](), CASES[name][1]
    op, orc = _pair(w, shift, 0)
    for l in range(op.levels):
        x = np.stack([rvec(orc.shape(l), 600 + l), rvec(orc.shape(l), 610 + l)])
        y = host(op.apply(dev(x, op.cdtype), which=1, level=l))
        for r in range(2):
            e = rel(y[r], orc.apply(x[r], which=1, l=l))
            assert e <= 1e-12, (l, r, e)
        b = np.stack([rvec(orc.shape(l), 620 + l), rvec(orc.shape(l), 630 + l)])
        x0 = 1e-4 * np.stack([rvec(orc.shape(l), 640 + l), rvec(orc.shape(l), 650 + l)])
        xs = host(op.smooth(dev(b, op.cdtype), dev(x0, op.cdtype), level=l))
        for r in range(2):
            xo, _ = orc.gmres_sweep(b[r], x0[r], l=l)
            e = rel(xs[r], xo)
            note(f"  {path} level {l} rhs {r}: sweep {e:.2e}")
            assert e <= 1e-12
    b = np.stack([rvec(orc.shape(0), 660), rvec(orc.shape(0), 661)])
    v = host(op.vcycle(dev(b, op.cdtype)))
    for r in range(2):
        e = rel(v[r], orc.vcycle(b[r]))
        note(f"  {path} vcycle rhs {r}: {e:.2e}")
        assert e <= 1e-12


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_fgmres(name, prec):
    import torch
    torch_cuda()
    w, shift = CASES[name][0](), CASES[name][1]
    op, orc = _pair(w, shift, prec)
    chi = np.stack([w.chi[0], rvec(w.chi.shape[1:], 670)])
    tol = 1e-8
    u, rc, infos = op.solve(dev(chi, torch.complex128), tol=tol, restart=30, maxit=800)
    u = host(u)
    assert rc == 0
    for r in range(2):
        uo, io = orc.fgmres(chi[r], tol=tol, restart=30, maxit=800)
        if prec == 0:
            e = rel(u[r], uo)
            note(f"  rhs {r}: its gpu {infos[r]['iterations']} oracle {io.iterations} sol err {e:.2e}")
            assert abs(infos[r]["iterations"] - io.iterations) <= 1
            assert e <= 1e-10
        else:
            ref = tight_oracle(orc, chi[r], restart=30)
            floor = rel(uo, ref)
            e = rel(u[r], ref)
            note(f"  rhs {r}: its gpu {infos[r]['iterations']} oracle {io.iterations} sol err {e:.2e} "
                 f"(floor {floor:.2e})")
            assert e <= max(1e-5, 10 * floor)


@pytest.mark.parametrize("dim", [2, 3])
def test_csg_equals_scaled_csl_layer_free(dim):
    """Layer-free box, variable phi: CSG(beta) and CSL(beta = 0, s = e^{2i beta})
    take the same FGMRES iterations and reach the same solution."""
    import torch
    from paper_1012_5379_amd import Operator
    torch_cuda()
    beta = 0.3
    n = (60, 47, 0) if dim == 2 else (18, 15, 20)
    shape = tuple(reversed([m - 1 for m in n[:dim]]))
    phi = 100.0 * (1 + 0.3 * W.rng(78, dim).random(shape))
    z = (0, 0, 0)
    base = dict(dim=dim, n=n, h=1.0 / max(n), layer_lo=z, layer_hi=z, gamma=0.5, levels=0, s=3, nu1=1, nu2=1)
    chi = W.rand_cvec((1,) + shape, item=80 + dim)
    out = {}
    for tag, kw in (("csg", dict(beta=beta)), ("csl", dict(beta=0.0, shift=cmath.exp(2j * beta)))):
        op = Operator(dict(base, cycle_prec=0, max_rhs=1, restart=30, **kw), phi)
        u, rc, infos = op.solve(dev(chi, torch.complex128), tol=1e-9, restart=30, maxit=500)
        assert rc == 0
        out[tag] = (host(u)[0], infos[0]["iterations"])
    note(f"  dim {dim}: iterations csg {out['csg'][1]} csl {out['csl'][1]}")
    assert out["csg"][1] == out["csl"][1]
    assert rel(out["csg"][0], out["csl"][0]) <= 1e-9
