"""GPU parity of the pass sequences that large grids take.

A level too large for the LDS-staged tiles and above the fused-pass size limit
runs one stencil pass and one Gram-Schmidt pass per Arnoldi step, the plain
closing/restriction and interpolation/residual passes, and (on the finest
level) the chunked w = H z; levels above the coarse-tail limit run the
multi-block passes.  The environment switches below force those sequences on
small grids, where every level can be compared with the FP64 CPU oracle:
each GMRES(s) sweep, each V-cycle and the FGMRES solve (complex128: 1e-12 per
operation, iterations +-1 and solution 1e-10 end to end; complex64 cycle:
the stated single-precision bounds, and the solution against the oracle's
tightly converged answer)."""
import numpy as np
import pytest

from tests.gpu_common import cases, dev, host, note, pair, rel, rvec, tight_oracle, torch_cuda

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = {"smooth": 6e-6, "vcycle": 6e-6}   # about ten times the largest error observed

# switch sets: every level unfused and untiled (the finest levels of the
# 2048^2, 128^3 and 192^3 grids), and the same with the fused untiled passes
# (the mid-size 3-D levels)
PATHS = {
    "unfused": {"CSG_TILES": "0", "CSG_FUSE_MAX": "0", "CSG_TAIL_MAX": "0", "CSG_HDOT_TILES": "0",
                "CSG_SLABS": "0"},
    "fused_untiled": {"CSG_TILES": "0", "CSG_FUSE_MAX": "1000000000", "CSG_TAIL_MAX": "0",
                      "CSG_HDOT_TILES": "0", "CSG_SLABS": "0"},
    # every 3-D level on z-marching slabs (the large 3-D levels' path)
    "slab": {"CSG_SLAB_MIN": "0", "CSG_TAIL_MAX": "0"},
    # slabs for the Arnoldi passes, the transfers as separate chunked passes
    "slab_chunked_transfers": {"CSG_SLAB_MIN": "0", "CSG_TAIL_MAX": "0", "CSG_SLAB_PR": "0", "CSG_SLAB_DOWN": "0"},
}
CASES = {k: v for k, v in cases().items() if k in ("2d_wide", "3d_ragged")}


def _env(monkeypatch, path):
    for k, v in PATHS[path].items():
        monkeypatch.setenv(k, v)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("name", list(CASES))
def test_sweep_and_vcycle(name, path, prec, monkeypatch):
    torch_cuda()
    _env(monkeypatch, path)
    w = CASES[name]()
    op, orc = pair(w, max_rhs=2, cycle_prec=prec)
    for l in range(op.levels):
        b = np.stack([rvec(orc.shape(l), 410 + l), rvec(orc.shape(l), 420 + l)])
        x0 = np.stack([rvec(orc.shape(l), 430 + l), rvec(orc.shape(l), 440 + l)]) * 1e-4
        x = host(op.smooth(dev(b, op.cdtype), dev(x0, op.cdtype), level=l))
        for r in range(2):
            xo, k = orc.gmres_sweep(b[r], x0[r], l=l)
            e = rel(x[r], xo)
            note(f"  {path} prec {prec} sweep level {l} rhs {r}: {e:.2e}")
            assert e <= (TOL64 if prec == 0 else TOL32["smooth"])
    b = np.stack([rvec(orc.shape(0), 450), rvec(orc.shape(0), 451)])
    x = host(op.vcycle(dev(b, op.cdtype)))
    for r in range(2):
        e = rel(x[r], orc.vcycle(b[r]))
        note(f"  {path} prec {prec} vcycle rhs {r}: {e:.2e}")
        assert e <= (TOL64 if prec == 0 else TOL32["vcycle"])


@pytest.mark.parametrize("path", ["unfused", "slab", "slab_chunked_transfers"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_fgmres_large_grid_paths(name, prec, path, monkeypatch):
    """The whole solve on the unfused, untiled passes, and on 3-D slabs: two RHS, complex128
    cycle iterations +-1 and solution within 1e-10 of the oracle; complex64
    cycle true residual at the tolerance and solution error against the
    oracle's tightly converged answer within ten times the error any solve
    stopping at that tolerance has."""
    import torch
    _env(monkeypatch, path)
    w = CASES[name]()
    chi = np.stack([w.chi[0], rvec(w.chi.shape[1:], 460)])
    op, orc = pair(w, max_rhs=2, cycle_prec=prec)
    tol = 1e-8
    u, rc, infos = op.solve(dev(chi, torch.complex128), tol=tol, restart=20, maxit=600)
    u = host(u)
    assert rc == 0
    for r in range(2):
        uo, io = orc.fgmres(chi[r], tol=tol, restart=20, maxit=600)
        if prec == 0:
            e = rel(u[r], uo)
            note(f"  rhs {r}: its gpu {infos[r]['iterations']} oracle {io.iterations} sol err {e:.2e}")
            assert abs(infos[r]["iterations"] - io.iterations) <= 1
            assert e <= 1e-10
        else:
            ref = tight_oracle(orc, chi[r], restart=20)
            floor = rel(uo, ref)
            e = rel(u[r], ref)
            rr = np.linalg.norm(chi[r] - orc.apply(u[r], which=0, l=0)) / np.linalg.norm(chi[r])
            note(f"  rhs {r}: its gpu {infos[r]['iterations']} oracle {io.iterations} relres {rr:.2e} "
                 f"sol err {e:.2e} (floor {floor:.2e})")
            assert rr <= tol
            assert e <= max(1e-5, 10 * floor)


@pytest.mark.parametrize("prec", [0, 1])
def test_slab_transfer_passes_bitwise(prec, monkeypatch):
    """On slab levels the fused transfer passes (interpolation with the
    residual that opens the post-sweep; the pre-sweep's closing update with
    the restriction) give the V-cycle bit for bit the values of the chunked
    passes they replace (the same formulas in the same order), two RHS."""
    torch_cuda()
    w = CASES["3d_ragged"]()
    monkeypatch.setenv("CSG_SLAB_MIN", "0")
    monkeypatch.setenv("CSG_TAIL_MAX", "0")
    fused, orc = pair(w, max_rhs=2, cycle_prec=prec)
    monkeypatch.setenv("CSG_SLAB_PR", "0")
    monkeypatch.setenv("CSG_SLAB_DOWN", "0")
    chunked, _ = pair(w, max_rhs=2, cycle_prec=prec)
    b = np.stack([rvec(orc.shape(0), 470), rvec(orc.shape(0), 471)])
    xf = host(fused.vcycle(dev(b, fused.cdtype)))
    xc = host(chunked.vcycle(dev(b, chunked.cdtype)))
    note(f"  prec {prec}: max |fused - chunked| {np.abs(xf - xc).max():.2e}")
    assert np.array_equal(xf, xc)
