"""csg_smooth_static (the sweep for callers that cannot allocate: its vectors,
partials and states in the library's static device array) against csg_smooth
(the same sweep on the operator's workspace) through the C ABI: two calls in a
row, the second on a smaller input, each equal to csg_smooth bit for bit and to
the oracle's sweep at 1e-12 (complex128) / the complex64 bound; inputs beyond
the array's size are rejected with CSG_ENOMEM."""
import numpy as np
import pytest

from synth import workloads as W
from tests.gpu_common import dev, host, note, pair, rel, rvec, torch_cuda

pytestmark = pytest.mark.gpu


def _static(op, level, b, x):
    import torch
    from paper_1012_5379_amd import binding as B
    b = op._vec(b, level, op.cdtype)
    x = op._vec(x, level, op.cdtype)
    B.csg_smooth_static(op.op, level, b.data_ptr(), x.data_ptr(), b.shape[0],
                        torch.cuda.current_stream().cuda_stream)
    return x


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dim", [2, 3])
def test_static_sweep_equals_workspace_sweep(dim, prec):
    torch_cuda()
    w = (W.small(dim=2, n=300, m=21, beta=0.4, kh=0.5, item=2) if dim == 2
         else W.small(dim=3, n=27, mlo=3, mhi=4, beta=0.4, kh=0.4, item=3))
    op, orc = pair(w, max_rhs=3, cycle_prec=prec)
    # a large call (finest level, 3 RHS), then a smaller one (level 1, 1 RHS)
    for level, nrhs, item in ((0, 3, 600), (1, 1, 610)):
        b = np.stack([rvec(orc.shape(level), item + r) for r in range(nrhs)])
        x0 = np.stack([rvec(orc.shape(level), item + 5 + r) for r in range(nrhs)]) * 1e-3
        xs = host(_static(op, level, dev(b, op.cdtype), dev(x0, op.cdtype)))
        xw = host(op.smooth(dev(b, op.cdtype), dev(x0, op.cdtype), level=level))
        assert np.array_equal(xs, xw)
        for r in range(nrhs):
            xo, _ = orc.gmres_sweep(b[r], x0[r], l=level)
            e = rel(xs[r], xo)
            note(f"  {dim}-D prec {prec} level {level} rhs {r}/{nrhs}: {e:.2e} vs oracle")
            assert e <= (1e-12 if prec == 0 else 6e-6)


def test_static_sweep_rejects_oversized_input():
    from paper_1012_5379_amd import binding as B
    torch_cuda()
    w = W.small(dim=2, n=300, m=21, beta=0.4, kh=0.5, item=2)
    op, orc = pair(w, max_rhs=16, cycle_prec=0)
    b = dev(np.zeros((16,) + orc.shape(0), complex), op.cdtype)
    x = dev(np.zeros((16,) + orc.shape(0), complex), op.cdtype)
    with pytest.raises(B.CsgError) as ei:
        _static(op, 0, b, x)
    assert ei.value.code == B.CSG_ENOMEM
    # the library stays usable: a fitting call right after matches csg_smooth
    b1 = rvec(orc.shape(0), 620)[None]
    xs = host(_static(op, 0, dev(b1, op.cdtype), dev(np.zeros_like(b1), op.cdtype)))
    xw = host(op.smooth(dev(b1, op.cdtype), dev(np.zeros_like(b1), op.cdtype), level=0))
    assert np.array_equal(xs, xw)
