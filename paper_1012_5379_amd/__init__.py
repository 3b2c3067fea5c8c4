"""MI355X-native GMRES-smoothed CSG multigrid / FGMRES solver for the ECS
Helmholtz problem (Reps, Vanroose, bin Zubair).

``Operator`` wraps one hierarchy built by libcsg inside a torch-allocated
workspace; vectors are torch complex CUDA tensors shaped (nrhs, [z,] y, x).
torch provides device memory and the current stream only; every step of the
solver runs in the library's HIP kernels (see include/csg.h).
"""
from __future__ import annotations

import numpy as np

from . import binding as B

__all__ = ["Operator", "BatchOperator", "B"]


def _torch():
    import torch
    return torch


class Operator:
    """One CSG multigrid hierarchy + FGMRES state resident on the GPU."""

    def __init__(self, params: dict, phi: np.ndarray, device: str = "cuda", tuned: bool = False):
        """tuned: take the execution knobs the caller left at 0 from the
        autotuner's table (paper_1012_5379_amd/tuned.json) for this problem's
        dimension, precision, smoother and size class."""
        torch = _torch()
        self.params = dict(params)
        if tuned:
            from . import tune
            self.params = tune.apply(self.params)
        self.p = B.make_params(**self.params)
        self.nbytes = B.csg_workspace_bytes(self.p)
        self.device = torch.device(device)
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        self.levels, self.dims = B.csg_plan_levels(self.p)
        if phi.size != int(np.prod(self.dims[0])):
            raise ValueError("phi must have one value per finest-level unknown")
        self._phi = phi
        self.op = B.csg_operator_create(self.p, phi.ctypes.data, self.ws.data_ptr(), self.nbytes,
                                        self._stream())
        self.cdtype = torch.complex64 if self.p.cycle_prec else torch.complex128

    def __del__(self):
        op = getattr(self, "op", None)
        if op:
            try:
                B.csg_operator_destroy(op)
            except Exception:
                pass
            self.op = None

    # ------------------------------------------------------------------ helpers
    def _stream(self) -> int:
        torch = _torch()
        return torch.cuda.current_stream(self.device).cuda_stream

    def shape(self, level: int = 0) -> tuple:
        d = self.dims[level][: self.p.dim]
        return tuple(reversed(d))

    def _vec(self, t, level, dtype):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError("vectors must be CUDA tensors")
        if t.dtype != dtype:
            raise TypeError(f"expected {dtype}, got {t.dtype}")
        sh = self.shape(level)
        if t.dim() == len(sh):
            t = t.unsqueeze(0)
        if tuple(t.shape[1:]) != sh or not t.is_contiguous():
            raise ValueError(f"expected a contiguous (nrhs, {sh}) tensor, got {tuple(t.shape)}")
        return t

    def empty(self, nrhs=1, level=0, dtype=None):
        torch = _torch()
        return torch.empty((nrhs,) + self.shape(level), dtype=dtype or self.cdtype, device=self.device)

    # --------------------------------------------------------------- operations
    def apply(self, x, which: int = 1, level: int = 0):
        """y = A x with A = H (which=0, level 0, complex128) or M_level (which=1)."""
        torch = _torch()
        dt = torch.complex128 if which == 0 else self.cdtype
        x = self._vec(x, level, dt)
        y = torch.empty_like(x)
        B.csg_stencil_apply(self.op, which, level, x.data_ptr(), y.data_ptr(), x.shape[0], self._stream())
        return y

    def vcycle(self, b):
        b = self._vec(b, 0, self.cdtype)
        x = _torch().empty_like(b)
        B.csg_vcycle(self.op, b.data_ptr(), x.data_ptr(), b.shape[0], self._stream())
        return x

    def smooth(self, b, x, level: int = 0):
        b = self._vec(b, level, self.cdtype)
        x = self._vec(x, level, self.cdtype)
        B.csg_smooth(self.op, level, b.data_ptr(), x.data_ptr(), b.shape[0], self._stream())
        return x

    def residual_restrict(self, b, x, level: int = 0):
        b = self._vec(b, level, self.cdtype)
        xp = 0 if x is None else self._vec(x, level, self.cdtype).data_ptr()
        bc = self.empty(b.shape[0], level + 1)
        B.csg_residual_restrict(self.op, level, b.data_ptr(), xp, bc.data_ptr(), b.shape[0], self._stream())
        return bc

    def prolong_correct(self, ec, x, level: int = 0):
        ec = self._vec(ec, level + 1, self.cdtype)
        x = self._vec(x, level, self.cdtype)
        B.csg_prolong_correct(self.op, level, ec.data_ptr(), x.data_ptr(), ec.shape[0], self._stream())
        return x

    def coarse_solve(self, b):
        L = self.levels - 1
        b = self._vec(b, L, self.cdtype)
        x = _torch().empty_like(b)
        B.csg_coarse_solve(self.op, b.data_ptr(), x.data_ptr(), b.shape[0], self._stream())
        return x

    def solve(self, chi, tol=1e-6, restart=None, maxit=1000, u0=None):
        """FGMRES(restart) preconditioned by one V-cycle per step.  Returns
        (u, status, [info per RHS])."""
        torch = _torch()
        chi = self._vec(chi, 0, torch.complex128)
        restart = self.p.restart if restart is None else restart
        if u0 is None:
            u = torch.empty_like(chi)
            use = 0
        else:
            u = self._vec(u0, 0, torch.complex128).clone()
            use = 1
        rc, infos = B.helm_solve(self.op, chi.data_ptr(), u.data_ptr(), chi.shape[0], float(tol), int(restart),
                                 int(maxit), use, self._stream())
        return u, rc, infos


class BatchOperator(Operator):
    """Problems of one size class in one operator (csg_batch_create): problem q
    owns right-hand sides q*max_rhs .. (q+1)*max_rhs - 1 of every vector, and
    every operation runs all problems in the same launches."""

    def __init__(self, params_list: list, phis: list, device: str = "cuda"):
        torch = _torch()
        self.nprob = len(params_list)
        self.params = dict(params_list[0])
        ps = [B.make_params(**dict(p)) for p in params_list]
        self.p = ps[0]
        self.rpp = self.p.max_rhs
        self.nbytes = B.csg_batch_workspace_bytes(self.p, self.nprob)
        self.device = torch.device(device)
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.levels, self.dims = B.csg_plan_levels(self.p)
        self._phis = [np.ascontiguousarray(f, dtype=np.float64) for f in phis]
        for f in self._phis:
            if f.size != int(np.prod(self.dims[0])):
                raise ValueError("phi must have one value per finest-level unknown")
        self._ps = ps
        self.op = B.csg_batch_create(ps, [f.ctypes.data for f in self._phis], self.ws.data_ptr(), self.nbytes,
                                     self._stream())
        self.cdtype = torch.complex64 if self.p.cycle_prec else torch.complex128
