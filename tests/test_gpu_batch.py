"""Batched operators (several problems of one size class in one operator, all
advancing in the same launches) against each problem solved alone and
against the FP64 oracle: the FGMRES solves (2-D and 3-D, the 3-D ones on the
slab passes), the V-cycle in both precisions, and the class checks."""
import numpy as np
import pytest

from oracle.oracle import Oracle, Params
from synth import workloads as W
from tests.gpu_common import dev, host, note, rel, rvec, torch_cuda

pytestmark = pytest.mark.gpu


def _problems(dim):
    if dim == 2:
        return [W.small(dim=2, n=96, mlo=6, mhi=9, beta=b, kh=0.45, item=30 + q, nrhs=2)
                for q, b in enumerate((0.3, 0.35, 0.4))]
    return [W.small(dim=3, n=24, mlo=3, mhi=2, beta=b, kh=0.4, item=40 + q, nrhs=2) for q, b in enumerate((0.35, 0.4))]


def _params(w, prec, R):
    return dict(w.params(), cycle_prec=prec, max_rhs=R, restart=20)


@pytest.mark.parametrize("dim", [2, 3])
def test_batched_solves_equal_alone_and_oracle(dim, monkeypatch):
    import torch
    from paper_1012_5379_amd import BatchOperator, Operator
    torch_cuda()
    if dim == 3:
        monkeypatch.setenv("CSG_SLAB_MIN", "0")
    ws = _problems(dim)
    R = 2
    bop = BatchOperator([_params(w, 0, R) for w in ws], [w.phi for w in ws])
    chi = np.concatenate([w.chi for w in ws])
    u, rc, infos = bop.solve(dev(chi, torch.complex128), tol=1e-8, restart=20, maxit=600)
    u = host(u)
    assert rc == 0
    for q, w in enumerate(ws):
        op = Operator(_params(w, 0, R), w.phi)
        ua, rca, infa = op.solve(dev(w.chi, torch.complex128), tol=1e-8, restart=20, maxit=600)
        ua = host(ua)
        orc = Oracle(Params(**w.params()), w.phi)
        for r in range(R):
            k = q * R + r
            uo, io = orc.fgmres(w.chi[r], tol=1e-8, restart=20, maxit=600)
            e = rel(u[k], uo)
            note(f"  problem {q} rhs {r}: its batch {infos[k]['iterations']} alone {infa[r]['iterations']} "
                 f"oracle {io.iterations}; sol err {e:.2e}; batch == alone: {np.array_equal(u[k], ua[r])}")
            assert infos[k]["iterations"] == infa[r]["iterations"]
            assert np.array_equal(u[k], ua[r])
            assert abs(infos[k]["iterations"] - io.iterations) <= 1
            assert e <= 1e-10


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dim", [2, 3])
def test_batched_vcycle_equals_alone(dim, prec):
    from paper_1012_5379_amd import BatchOperator, Operator
    torch_cuda()
    ws = _problems(dim)
    R = 2
    bop = BatchOperator([_params(w, prec, R) for w in ws], [w.phi for w in ws])
    b = np.stack([rvec(ws[0].grid_shape, 800 + k) for k in range(len(ws) * R)])
    x = host(bop.vcycle(dev(b, bop.cdtype)))
    for q, w in enumerate(ws):
        op = Operator(_params(w, prec, R), w.phi)
        xa = host(op.vcycle(dev(b[q * R:(q + 1) * R], op.cdtype)))
        assert np.array_equal(x[q * R:(q + 1) * R], xa)
        if prec == 0:
            orc = Oracle(Params(**w.params()), w.phi)
            e = rel(x[q * R], orc.vcycle(b[q * R]))
            note(f"  problem {q}: vcycle vs oracle {e:.2e}")
            assert e <= 1e-12


def test_batch_rejects_mixed_classes():
    from paper_1012_5379_amd import BatchOperator
    from paper_1012_5379_amd import binding as B
    torch_cuda()
    import torch
    a = W.small(dim=2, n=96, m=6, item=50)
    b = W.small(dim=2, n=80, m=6, item=51)
    pa, pb = B.make_params(**_params(a, 0, 1)), B.make_params(**_params(b, 0, 1))
    nb = B.csg_batch_workspace_bytes(pa, 2)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    fa, fb = np.ascontiguousarray(a.phi), np.ascontiguousarray(b.phi)
    with pytest.raises(B.CsgError) as ei:
        B.csg_batch_create([pa, pb], [fa.ctypes.data, fb.ctypes.data], ws.data_ptr(), nb,
                           torch.cuda.current_stream().cuda_stream)
    assert ei.value.code == B.CSG_EINVAL
    with pytest.raises(B.CsgError):
        B.csg_batch_workspace_bytes(B.make_params(**dict(_params(a, 0, 1), smoother=1)), 2)
