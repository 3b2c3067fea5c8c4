"""Shared helpers of the GPU parity tests (the HIP path vs the CPU oracle)."""
import sys

import numpy as np

from oracle.oracle import Oracle, Params
from synth import workloads as W


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch


def pair(w: W.Workload, max_rhs=2, cycle_prec=None, restart=30):
    """Build the GPU operator and the oracle on the same seeded workload."""
    from paper_1012_5379_amd import Operator
    cp = w.cycle_prec if cycle_prec is None else cycle_prec
    params = dict(w.params(), cycle_prec=cp, max_rhs=max_rhs, restart=restart)
    note(f"[case] {w.name} dims={w.grid_shape} cycle_prec={cp} max_rhs={max_rhs}")
    op = Operator(params, w.phi)
    orc = Oracle(Params(**w.params()), w.phi)
    assert op.levels == orc.levels
    return op, orc


def dev(a, dtype):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch = torch_cuda()
    torch.cuda.synchronize()
    return t.detach().to("cpu").to(torch.complex128).numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def rvec(shape, item):
    return W.rand_cvec(shape, item=item)


# Grids with odd interval counts, unequal layers and several blocks with a
# ragged tail, in 2-D and 3-D (shared by the per-operation parity suites).
def cases():
    return {
        "c1": lambda: W.c1(),
        "2d_ragged": lambda: W.small(dim=2, n=101, mlo=7, mhi=4, beta=0.35, kh=0.45, item=1),
        "2d_wide": lambda: W.small(dim=2, n=300, m=21, beta=0.4, kh=0.5, item=2),
        "3d_ragged": lambda: W.small(dim=3, n=27, mlo=3, mhi=4, beta=0.4, kh=0.4, item=3),
    }


def tight_oracle(orc, chi, restart=30, maxit=4000):
    """The oracle's answer at tol 1e-12: the reference a solve stopping at a
    looser tolerance is measured against."""
    u, info = orc.fgmres(chi, tol=1e-12, restart=restart, maxit=maxit)
    assert info.converged
    return u
