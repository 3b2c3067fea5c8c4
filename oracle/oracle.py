"""ctypes shim over the FP64 CPU oracle (``libcsg_oracle.so``).

TEST INFRASTRUCTURE ONLY: the oracle is the plain CPU implementation the GPU
library is checked against.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark import this module; the product path never does,
and this module imports nothing from the GPU package.

Arrays are numpy ``complex128`` (interleaved re, im) and ``float64``; unknowns of
a grid are stored x fastest.  ``Oracle`` mirrors the oracle's C entry points,
each of which cites the passage of the paper it follows (see csg_oracle.c).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsg_oracle.so")
SRC = os.path.join(HERE, "csg_oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, IEEE semantics kept)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Params(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("h", C.c_double),
                ("layer_lo", C.c_int * 3), ("layer_hi", C.c_int * 3),
                ("gamma", C.c_double), ("beta", C.c_double), ("levels", C.c_int),
                ("s", C.c_int), ("nu1", C.c_int), ("nu2", C.c_int), ("smoother", C.c_int),
                ("poly_k2", C.c_double), ("shift_re", C.c_double), ("shift_im", C.c_double),
                ("coarse_op", C.c_int)]


class _Cplx(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class _Poly(C.Structure):
    _fields_ = [("k2", C.c_double), ("H", C.c_double), ("t", _Cplx * 3), ("e", _Cplx * 3),
                ("f", _Cplx * 3), ("varphi", C.c_double), ("c", _Cplx * 4), ("omega", _Cplx * 3),
                ("conds", C.c_int)]


class _Info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("vcycles", C.c_int),
                ("converged", C.c_int), ("relres_true", C.c_double),
                ("relres_est", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        vp, ip, dp = C.c_void_p, C.c_int, C.c_double
        L.ora_build.restype = vp
        L.ora_build.argtypes = [C.POINTER(_Params), vp, C.POINTER(C.c_int)]
        L.ora_free.argtypes = [vp]
        L.ora_levels.argtypes = [vp]
        L.ora_level_dims.argtypes = [vp, ip, C.POINTER(C.c_int)]
        for nm in ("ora_axis_nodes", "ora_axis_sw"):
            getattr(L, nm).argtypes = [vp, ip, ip, ip, vp]
        L.ora_level_phi.argtypes = [vp, ip, vp]
        L.ora_apply.argtypes = [vp, ip, ip, vp, vp]
        L.ora_restrict.argtypes = [vp, ip, vp, vp]
        L.ora_prolong_add.argtypes = [vp, ip, vp, vp]
        L.ora_coarse_solve.argtypes = [vp, vp, vp]
        L.ora_gmres_sweep.argtypes = [vp, ip, ip, vp, vp, ip]
        L.ora_vcycle_level.argtypes = [vp, ip, vp, vp]
        L.ora_vcycle.argtypes = [vp, vp, vp]
        L.ora_fgmres.argtypes = [vp, vp, vp, dp, ip, ip, ip, C.POINTER(_Info), vp, ip]
        L.ora_poly_level.argtypes = [vp, ip, C.POINTER(_Poly)]
        L.ora_poly_conditions.argtypes = [dp, dp, ip, dp, dp, dp, C.POINTER(C.c_double),
                                          C.POINTER(C.c_double)]
        L.ora_poly_sweep.argtypes = [vp, ip, vp, vp, ip]
        L.ora_galerkin_stencil.argtypes = [vp, ip, vp]
        L.ora_threads.restype = C.c_int
        L.ora_threads.argtypes = []
        L.ora_dot.restype = _Cplx
        L.ora_dot.argtypes = [C.c_long, vp, vp]
        _lib = L
    return _lib


@dataclass
class Params:
    """Problem and cycle parameters (problem statement; eq. csggrid; section 3)."""
    dim: int = 2
    n: tuple = (64, 64, 0)
    h: float = 1.0 / 64
    layer_lo: tuple = (8, 8, 0)
    layer_hi: tuple = (8, 8, 0)
    gamma: float = np.pi / 6
    beta: float = 0.4
    levels: int = 0
    s: int = 3
    nu1: int = 1
    nu2: int = 1
    smoother: int = 0        # 0 = GMRES(s), 1 = third-order polynomial (section 4)
    poly_k2: float = 0.0     # k^2 of the polynomial's vertex t0; 0 = mean of phi
    shift: complex = 0j      # factor s of phi in M = L(beta) - s phi; 0 means 1 (beta = 0, s = 1 + i eps: CSL)
    coarse_op: int = 0       # 0 = rediscretisation (section 3), 1 = Galerkin R M P

    def c(self) -> _Params:
        p = _Params()
        p.dim = self.dim
        for a in range(3):
            p.n[a] = int(self.n[a]) if a < len(self.n) else 0
            p.layer_lo[a] = int(self.layer_lo[a]) if a < len(self.layer_lo) else 0
            p.layer_hi[a] = int(self.layer_hi[a]) if a < len(self.layer_hi) else 0
        p.h, p.gamma, p.beta = float(self.h), float(self.gamma), float(self.beta)
        p.levels, p.s, p.nu1, p.nu2 = int(self.levels), int(self.s), int(self.nu1), int(self.nu2)
        p.smoother, p.poly_k2 = int(self.smoother), float(self.poly_k2)
        p.shift_re, p.shift_im = float(complex(self.shift).real), float(complex(self.shift).imag)
        p.coarse_op = int(self.coarse_op)
        return p

    def unknown_shape(self) -> tuple:
        """numpy shape of one grid vector, slowest axis first ((z,) y, x)."""
        nu = [self.n[a] + self.layer_lo[a] + self.layer_hi[a] - 1 for a in range(self.dim)]
        return tuple(reversed(nu))


@dataclass
class Info:
    iterations: int
    restarts: int
    vcycles: int
    converged: bool
    relres_true: float
    relres_est: float
    history: np.ndarray = field(default_factory=lambda: np.zeros(0))


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


class Oracle:
    """One built hierarchy of the oracle (finest level 0)."""

    def __init__(self, params: Params, phi: np.ndarray):
        self.params = params
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        st = C.c_int(0)
        self._h = lib().ora_build(C.byref(params.c()), phi.ctypes.data, C.byref(st))
        if not self._h:
            raise ValueError(f"oracle rejected parameters (status {st.value})")
        self.levels = lib().ora_levels(self._h)
        self.dims = []
        for l in range(self.levels):
            d = (C.c_int * 3)()
            lib().ora_level_dims(self._h, l, d)
            self.dims.append(tuple(d))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().ora_free(h)
            self._h = None

    # -- shapes ---------------------------------------------------------
    def shape(self, l: int) -> tuple:
        d = self.dims[l]
        return tuple(reversed(d[: self.params.dim]))

    def size(self, l: int) -> int:
        return int(np.prod(self.dims[l]))

    def _out(self, l):
        return np.zeros(self.shape(l), dtype=np.complex128)

    # -- tables ---------------------------------------------------------
    def axis_nodes(self, which: int, l: int, a: int) -> np.ndarray:
        nint = self.dims[l][a] + 1
        out = np.zeros(nint + 1, dtype=np.complex128)
        if lib().ora_axis_nodes(self._h, which, l, a, out.ctypes.data):
            raise ValueError("bad axis/level")
        return out

    def axis_sw(self, which: int, l: int, a: int) -> np.ndarray:
        nu = self.dims[l][a]
        out = np.zeros(3 * nu, dtype=np.complex128)
        if lib().ora_axis_sw(self._h, which, l, a, out.ctypes.data):
            raise ValueError("bad axis/level")
        return out.reshape(3, nu)

    def level_phi(self, l: int) -> np.ndarray:
        out = np.zeros(self.shape(l), dtype=np.float64)
        lib().ora_level_phi(self._h, l, out.ctypes.data)
        return out

    # -- operations -----------------------------------------------------
    def apply(self, x: np.ndarray, which: int = 1, l: int = 0) -> np.ndarray:
        x, px = _c(x.reshape(self.shape(l)), np.complex128)
        y = self._out(l)
        if lib().ora_apply(self._h, which, l, px, y.ctypes.data):
            raise ValueError("bad operator/level")
        return y

    def restrict(self, r: np.ndarray, l: int) -> np.ndarray:
        r, pr = _c(r.reshape(self.shape(l)), np.complex128)
        bc = self._out(l + 1)
        if lib().ora_restrict(self._h, l, pr, bc.ctypes.data):
            raise ValueError("bad level")
        return bc

    def prolong_add(self, ec: np.ndarray, x: np.ndarray, l: int) -> np.ndarray:
        ec, pe = _c(ec.reshape(self.shape(l + 1)), np.complex128)
        x = np.array(x, dtype=np.complex128, order="C").reshape(self.shape(l))
        if lib().ora_prolong_add(self._h, l, pe, x.ctypes.data):
            raise ValueError("bad level")
        return x

    def coarse_solve(self, b: np.ndarray) -> np.ndarray:
        l = self.levels - 1
        b, pb = _c(b.reshape(self.shape(l)), np.complex128)
        x = self._out(l)
        lib().ora_coarse_solve(self._h, pb, x.ctypes.data)
        return x

    def gmres_sweep(self, b, x=None, l: int = 0, s: int | None = None):
        """One GMRES(s) sweep; returns (x_new, steps)."""
        s = self.params.s if s is None else s
        b, pb = _c(b.reshape(self.shape(l)), np.complex128)
        zero = x is None
        x = self._out(l) if zero else np.array(x, dtype=np.complex128, order="C").reshape(self.shape(l))
        k = lib().ora_gmres_sweep(self._h, l, s, pb, x.ctypes.data, int(zero))
        return x, k

    def galerkin_stencil(self, l: int) -> np.ndarray:
        """Level l's Galerkin operator (coarse_op = 1) as (3^d, *shape) coefficients,
        offset index sum_a (o_a + 1) 3^a over the used axes (x first)."""
        np_ = 3 ** self.params.dim
        out = np.zeros((np_,) + self.shape(l), dtype=np.complex128)
        if lib().ora_galerkin_stencil(self._h, l, out.ctypes.data):
            raise ValueError("no Galerkin operator on this level")
        return out

    def poly(self, l: int) -> dict:
        """The level's third-order polynomial smoother (section 4)."""
        pl = _Poly()
        if lib().ora_poly_level(self._h, l, C.byref(pl)):
            raise ValueError("bad level")
        cx = lambda a: np.array([complex(v.re, v.im) for v in a])
        return dict(k2=pl.k2, H=pl.H, t=cx(pl.t), e=cx(pl.e), f=cx(pl.f), varphi=pl.varphi,
                    c=cx(pl.c), omega=cx(pl.omega), conds=pl.conds)

    def poly_sweep(self, b, x=None, l: int = 0):
        """One polynomial smoothing sweep: x + q(M) (b - M x), error times p(M)."""
        b, pb = _c(b.reshape(self.shape(l)), np.complex128)
        zero = x is None
        x = self._out(l) if zero else np.array(x, dtype=np.complex128, order="C").reshape(self.shape(l))
        lib().ora_poly_sweep(self._h, l, pb, x.ctypes.data, int(zero))
        return x

    def vcycle(self, b, l: int = 0) -> np.ndarray:
        b, pb = _c(b.reshape(self.shape(l)), np.complex128)
        x = self._out(l)
        lib().ora_vcycle_level(self._h, l, pb, x.ctypes.data)
        return x

    def fgmres(self, chi, tol=1e-6, restart=30, maxit=1000, u0=None, hist_len=100000):
        chi, pc = _c(chi.reshape(self.shape(0)), np.complex128)
        use_x0 = u0 is not None
        u = (np.array(u0, dtype=np.complex128, order="C").reshape(self.shape(0))
             if use_x0 else self._out(0))
        info = _Info()
        hist = np.zeros(max(1, min(hist_len, maxit)), dtype=np.float64)
        rc = lib().ora_fgmres(self._h, pc, u.ctypes.data, float(tol), int(restart), int(maxit),
                              int(use_x0), C.byref(info), hist.ctypes.data, hist.size)
        if rc < 0:
            raise FloatingPointError(f"oracle fgmres failed ({rc})")
        inf = Info(info.iterations, info.restarts, info.vcycles, bool(info.converged),
                   info.relres_true, info.relres_est, hist[: info.iterations].copy())
        return u, inf


def poly_conditions(k2, H, dim, beta, gamma, varphi):
    """(F, S): |p(t0 + rho e^{-2i beta})|^2 = 1 + 2 rho F + rho^2 S + O(rho^3)."""
    F, S = C.c_double(0), C.c_double(0)
    if lib().ora_poly_conditions(float(k2), float(H), int(dim), float(beta), float(gamma), float(varphi),
                                 C.byref(F), C.byref(S)):
        raise ValueError("bad arguments")
    return F.value, S.value


def dot(x: np.ndarray, y: np.ndarray) -> complex:
    x, px = _c(x.ravel(), np.complex128)
    y, py = _c(y.ravel(), np.complex128)
    r = lib().ora_dot(x.size, px, py)
    return complex(r.re, r.im)


def threads() -> int:
    return int(lib().ora_threads())
