"""GPU parity under the autotuner's knobs at their extremes.

The knobs the autotuner picks (slab workgroups per right-hand side, the level
size from which 3-D levels take the slab passes, LDS tiles per chunked-pass
block, the fused-pass size limit, the coarse-tail size) may only change how
the passes are laid out.  Each extreme setting below is checked like the
default one: every level's GMRES(s) sweep and the V-cycle against the FP64
oracle at 1e-12 (complex128), and the FGMRES solve with iterations +-1 and
solution within 1e-10."""
import numpy as np
import pytest

from tests.gpu_common import cases, dev, host, note, pair, rel, rvec, torch_cuda

pytestmark = pytest.mark.gpu

KNOBS = {
    "3d_ragged": [
        dict(slab_blocks=1, slab_min=1, tail_max=-1),        # one run of planes per column, every level slabbed
        dict(slab_blocks=4096, slab_min=1, tail_max=-1),     # runs as short as the geometry allows
        dict(slab_min=-1, tail_max=8000),                    # no slabs, a large coarse tail
    ],
    "2d_wide": [
        dict(tile_mult=4, tail_max=-1),                      # four times the tiles
        dict(tile_mult=64, fuse_max=-1, tail_max=-1),        # tiles overflow the partial buffers: untiled passes
        dict(fuse_max=4000000, tail_max=5000),               # fused passes on every level, a large tail
    ],
}
CASES = cases()


@pytest.mark.parametrize("name,knobs", [(n, k) for n, ks in KNOBS.items() for k in ks],
                         ids=lambda v: v if isinstance(v, str) else "-".join(f"{a}{b}" for a, b in v.items()))
def test_tuned_extremes_match_oracle(name, knobs):
    import torch
    from paper_1012_5379_amd import Operator
    from oracle.oracle import Oracle, Params
    torch_cuda()
    w = CASES[name]()
    params = dict(w.params(), cycle_prec=0, max_rhs=2, restart=30, **knobs)
    note(f"[case] {name} knobs {knobs}")
    op = Operator(params, w.phi)
    orc = Oracle(Params(**w.params()), w.phi)
    assert op.levels == orc.levels
    for l in range(op.levels):
        b = np.stack([rvec(orc.shape(l), 510 + l), rvec(orc.shape(l), 520 + l)])
        x0 = np.stack([rvec(orc.shape(l), 530 + l), rvec(orc.shape(l), 540 + l)]) * 1e-4
        x = host(op.smooth(dev(b, op.cdtype), dev(x0, op.cdtype), level=l))
        for r in range(2):
            xo, _ = orc.gmres_sweep(b[r], x0[r], l=l)
            e = rel(x[r], xo)
            note(f"  sweep level {l} rhs {r}: {e:.2e}")
            assert e <= 1e-12
    b = np.stack([rvec(orc.shape(0), 550), rvec(orc.shape(0), 551)])
    x = host(op.vcycle(dev(b, op.cdtype)))
    for r in range(2):
        e = rel(x[r], orc.vcycle(b[r]))
        note(f"  vcycle rhs {r}: {e:.2e}")
        assert e <= 1e-12
    chi = np.stack([w.chi[0], rvec(w.chi.shape[1:], 560)])
    u, rc, infos = op.solve(dev(chi, torch.complex128), tol=1e-8, restart=30, maxit=600)
    u = host(u)
    assert rc == 0
    for r in range(2):
        uo, io = orc.fgmres(chi[r], tol=1e-8, restart=30, maxit=600)
        e = rel(u[r], uo)
        note(f"  solve rhs {r}: its gpu {infos[r]['iterations']} oracle {io.iterations} sol err {e:.2e}")
        assert abs(infos[r]["iterations"] - io.iterations) <= 1
        assert e <= 1e-10
