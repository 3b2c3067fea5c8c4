"""GPU parity of the Galerkin coarse operators (M_{l+1} = R M_l P stored as
9- or 27-point stencils; the remark in section 5) against the FP64 oracle,
which forms them independently (colour-class probing there, entry-by-entry
triple products in the library's setup): M on every level and every level's
GMRES(s) sweep and the V-cycle at 1e-12 (complex128), the FGMRES solve with
iterations +-1 and solution within 1e-10, the complex64 cycle against the
oracle's tightly converged answer; also with the complex-shifted
preconditioner."""
import numpy as np
import pytest

from oracle.oracle import Oracle, Params
from tests.gpu_common import dev, host, note, rel, rvec, tight_oracle, torch_cuda
from synth import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "2d": (lambda: W.small(dim=2, n=101, mlo=7, mhi=4, beta=0.35, kh=0.45, item=1), 0j),
    "3d": (lambda: W.small(dim=3, n=27, mlo=3, mhi=4, beta=0.4, kh=0.4, item=3), 0j),
    "2d_shifted": (lambda: W.small(dim=2, n=101, mlo=7, mhi=4, beta=0.0, kh=0.45, item=1), 1 + 0.5j),
}


def _pair(w, shift, prec, max_rhs=2):
    from paper_1012_5379_amd import Operator
    note(f"[case] {w.name} Galerkin shift {shift} prec {prec}")
    op = Operator(dict(w.params(), cycle_prec=prec, max_rhs=max_rhs, restart=30, shift=shift, coarse_op=1), w.phi)
    orc = Oracle(Params(**w.params(), shift=shift, coarse_op=1), w.phi)
    assert op.levels == orc.levels
    return op, orc


@pytest.mark.parametrize("name", list(CASES))
def test_operators_sweeps_vcycle(name):
    torch_cuda()
    w, shift = CASES[name][0](), CASES[name][1]
    op, orc = _pair(w, shift, 0)
    for l in range(op.levels):
        x = np.stack([rvec(orc.shape(l), 700 + l), rvec(orc.shape(l), 710 + l)])
        y = host(op.apply(dev(x, op.cdtype), which=1, level=l))
        for r in range(2):
            e = rel(y[r], orc.apply(x[r], which=1, l=l))
            note(f"  level {l} rhs {r}: M {e:.2e}")
            assert e <= 1e-12
        b = np.stack([rvec(orc.shape(l), 720 + l), rvec(orc.shape(l), 730 + l)])
        x0 = 1e-4 * np.stack([rvec(orc.shape(l), 740 + l), rvec(orc.shape(l), 750 + l)])
        xs = host(op.smooth(dev(b, op.cdtype), dev(x0, op.cdtype), level=l))
        for r in range(2):
            xo, _ = orc.gmres_sweep(b[r], x0[r], l=l)
            e = rel(xs[r], xo)
            note(f"  level {l} rhs {r}: sweep {e:.2e}")
            assert e <= 1e-12
    b = np.stack([rvec(orc.shape(0), 760), rvec(orc.shape(0), 761)])
    v = host(op.vcycle(dev(b, op.cdtype)))
    for r in range(2):
        e = rel(v[r], orc.vcycle(b[r]))
        note(f"  vcycle rhs {r}: {e:.2e}")
        assert e <= 1e-12


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_fgmres(name, prec):
    import torch
    torch_cuda()
    w, shift = CASES[name][0](), CASES[name][1]
    op, orc = _pair(w, shift, prec)
    chi = np.stack([w.chi[0], rvec(w.chi.shape[1:], 770)])
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


def test_polynomial_smoother_rejected():
    from paper_1012_5379_amd import binding as B
    w = CASES["2d"][0]()
    with pytest.raises(B.CsgError):
        B.csg_workspace_bytes(B.make_params(**dict(w.params(), coarse_op=1, smoother=1)))
