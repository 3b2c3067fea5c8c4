"""ctypes binding of libcsg (include/csg.h): argument marshalling only.

Every function here has the name of the C entry point it calls and does nothing
but convert Python arguments to the C types; all arithmetic of the solver runs
in the library's HIP kernels.  The library must have been built in-tree
(``python -m paper_1012_5379_amd.build``); importing this module without it
raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "csg.h")

CSG_OK, CSG_EINVAL, CSG_ENOMEM, CSG_EDEVICE, CSG_ENOCONV, CSG_ENUMERIC = 0, -1, -2, -3, -4, -5
CSG_MAX_LEVELS, CSG_MAX_S, CSG_MAX_RESTART, CSG_MAX_RHS = 16, 8, 64, 64
STATUS = {0: "CSG_OK", -1: "CSG_EINVAL", -2: "CSG_ENOMEM", -3: "CSG_EDEVICE", -4: "CSG_ENOCONV",
          -5: "CSG_ENUMERIC"}


class csg_params(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("h", C.c_double),
                ("layer_lo", C.c_int * 3), ("layer_hi", C.c_int * 3), ("gamma", C.c_double),
                ("beta", C.c_double), ("levels", C.c_int), ("s", C.c_int), ("nu1", C.c_int),
                ("nu2", C.c_int), ("cycle_prec", C.c_int), ("max_rhs", C.c_int), ("restart", C.c_int),
                ("tail_max", C.c_int), ("fuse_max", C.c_int), ("graphs", C.c_int),
                ("smoother", C.c_int), ("poly_k2", C.c_double),
                ("slab_blocks", C.c_int), ("tile_mult", C.c_int), ("slab_min", C.c_int),
                ("shift_re", C.c_double), ("shift_im", C.c_double), ("coarse_op", C.c_int)]


class csg_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("vcycles", C.c_int),
                ("converged", C.c_int), ("relres_true", C.c_double), ("relres_est", C.c_double),
                ("seconds", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class CsgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None
vp, ip, dp = C.c_void_p, C.c_int, C.c_double
Dims = (C.c_int * 3) * CSG_MAX_LEVELS

_SIGS = {
    "csg_last_error": (C.c_char_p, []),
    "csg_workspace_bytes": (ip, [C.POINTER(csg_params), C.POINTER(C.c_size_t)]),
    "csg_plan_levels": (ip, [C.POINTER(csg_params), C.POINTER(C.c_int), vp]),
    "csg_operator_create": (ip, [C.POINTER(csg_params), vp, vp, C.c_size_t, vp, C.POINTER(vp)]),
    "csg_operator_destroy": (ip, [vp]),
    "csg_operator_info": (ip, [vp, C.POINTER(C.c_int), vp]),
    "csg_stencil_apply": (ip, [vp, ip, ip, vp, vp, ip, vp]),
    "csg_vcycle": (ip, [vp, vp, vp, ip, vp]),
    "csg_smooth": (ip, [vp, ip, vp, vp, ip, vp]),
    "csg_smooth_static": (ip, [vp, ip, vp, vp, ip, vp]),
    "csg_poly_info": (ip, [vp, ip, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "csg_residual_restrict": (ip, [vp, ip, vp, vp, vp, ip, vp]),
    "csg_prolong_correct": (ip, [vp, ip, vp, vp, ip, vp]),
    "csg_coarse_solve": (ip, [vp, vp, vp, ip, vp]),
    "helm_solve": (ip, [vp, vp, vp, ip, dp, ip, ip, ip, C.POINTER(csg_solve_info), vp]),
    "csg_solve_begin": (ip, [vp, vp, vp, ip, dp, ip, ip, ip, vp, C.POINTER(vp)]),
    "csg_solve_step": (ip, [vp]),
    "csg_solve_poll": (ip, [vp, C.POINTER(C.c_int)]),
    "csg_solve_end": (ip, [vp, C.POINTER(csg_solve_info)]),
    "csg_batch_workspace_bytes": (ip, [C.POINTER(csg_params), ip, C.POINTER(C.c_size_t)]),
    "csg_batch_create": (ip, [vp, ip, vp, vp, C.c_size_t, vp, C.POINTER(vp)]),
    "helm_step_batch": (ip, [vp, C.POINTER(C.c_int)]),
    "csg_profile": (ip, [vp, ip, ip]),
    "csg_profile_read": (ip, [vp, C.POINTER(C.c_double), C.POINTER(C.c_long), C.POINTER(C.c_double)]),
    "csg_graphs_active": (ip, [vp]),
}

PROF_KINDS = {"vcycle": 1, "stencil_dots": 2, "orth": 3, "upd_restrict": 4, "prolong_resid": 5,
              "update": 6, "outer_h": 7, "outer_cgs1": 8, "outer_cgs2": 9, "outer_norm": 10,
              "outer_proj2": 11, "fused": 12}


def lib() -> C.CDLL:
    """Load the in-tree libcsg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1012_5379_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_symbols() -> list:
    """Names of the functions include/csg.h declares."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(csg_\w+|helm_\w+)\s*\(", src)))


def check(code: int) -> int:
    if code < 0:
        raise CsgError(code, lib().csg_last_error().decode())
    return code


def make_params(dim=2, n=(64, 64, 0), h=1 / 64, layer_lo=(8, 8, 0), layer_hi=(8, 8, 0),
                gamma=0.5235987755982988, beta=0.4, levels=0, s=3, nu1=1, nu2=1, cycle_prec=0,
                max_rhs=1, restart=30, tail_max=0, fuse_max=0, graphs=0, smoother=0,
                poly_k2=0.0, slab_blocks=0, tile_mult=0, slab_min=0, shift=0j, coarse_op=0) -> csg_params:
    p = csg_params()
    p.dim = int(dim)
    for a in range(3):
        p.n[a] = int(n[a]) if a < len(n) else 0
        p.layer_lo[a] = int(layer_lo[a]) if a < len(layer_lo) else 0
        p.layer_hi[a] = int(layer_hi[a]) if a < len(layer_hi) else 0
    p.h, p.gamma, p.beta = float(h), float(gamma), float(beta)
    p.levels, p.s, p.nu1, p.nu2 = int(levels), int(s), int(nu1), int(nu2)
    p.cycle_prec, p.max_rhs, p.restart = int(cycle_prec), int(max_rhs), int(restart)
    p.tail_max, p.fuse_max, p.graphs = int(tail_max), int(fuse_max), int(graphs)
    p.smoother, p.poly_k2 = int(smoother), float(poly_k2)
    p.slab_blocks, p.tile_mult, p.slab_min = int(slab_blocks), int(tile_mult), int(slab_min)
    p.shift_re, p.shift_im = float(complex(shift).real), float(complex(shift).imag)
    p.coarse_op = int(coarse_op)
    return p


# --- one wrapper per exported symbol ------------------------------------------------

def csg_last_error() -> str:
    return lib().csg_last_error().decode()


def csg_workspace_bytes(p: csg_params) -> int:
    out = C.c_size_t(0)
    check(lib().csg_workspace_bytes(C.byref(p), C.byref(out)))
    return out.value


def csg_plan_levels(p: csg_params):
    L = C.c_int(0)
    dims = Dims()
    check(lib().csg_plan_levels(C.byref(p), C.byref(L), dims))
    return L.value, [tuple(dims[l]) for l in range(L.value)]


def csg_operator_create(p: csg_params, phi_host_ptr: int, ws_ptr: int, ws_bytes: int, stream: int) -> int:
    op = vp()
    check(lib().csg_operator_create(C.byref(p), phi_host_ptr, ws_ptr, ws_bytes, stream, C.byref(op)))
    return op.value


def csg_operator_destroy(op: int) -> None:
    check(lib().csg_operator_destroy(op))


def csg_operator_info(op: int):
    L = C.c_int(0)
    dims = Dims()
    check(lib().csg_operator_info(op, C.byref(L), dims))
    return L.value, [tuple(dims[l]) for l in range(L.value)]


def csg_stencil_apply(op, which, level, x, y, nrhs, stream):
    return check(lib().csg_stencil_apply(op, which, level, x, y, nrhs, stream))


def csg_vcycle(op, b, x, nrhs, stream):
    return check(lib().csg_vcycle(op, b, x, nrhs, stream))


def csg_smooth(op, level, b, x, nrhs, stream):
    return check(lib().csg_smooth(op, level, b, x, nrhs, stream))


def csg_smooth_static(op, level, b, x, nrhs, stream):
    return check(lib().csg_smooth_static(op, level, b, x, nrhs, stream))


def csg_poly_info(op, level):
    """(varphi, [w1, w2, w3] as complex, conds) of the level's polynomial smoother."""
    vphi, om, conds = C.c_double(0), (C.c_double * 6)(), C.c_int(0)
    check(lib().csg_poly_info(op, level, C.byref(vphi), om, C.byref(conds)))
    return vphi.value, [complex(om[2 * i], om[2 * i + 1]) for i in range(3)], conds.value


def csg_residual_restrict(op, level, b, x, bc, nrhs, stream):
    return check(lib().csg_residual_restrict(op, level, b, x, bc, nrhs, stream))


def csg_prolong_correct(op, level, ec, x, nrhs, stream):
    return check(lib().csg_prolong_correct(op, level, ec, x, nrhs, stream))


def csg_coarse_solve(op, b, x, nrhs, stream):
    return check(lib().csg_coarse_solve(op, b, x, nrhs, stream))


def helm_solve(op, chi, u, nrhs, tol, restart, maxit, use_initial_guess, stream):
    """Returns (status, [info dict per RHS]); CSG_ENOCONV is returned, not raised."""
    infos = (csg_solve_info * max(1, nrhs))()
    rc = lib().helm_solve(op, chi, u, nrhs, tol, restart, maxit, use_initial_guess, infos, stream)
    if rc < 0 and rc != CSG_ENOCONV:
        check(rc)
    return rc, [infos[r].as_dict() for r in range(nrhs)]


def csg_solve_begin(op, chi, u, nrhs, tol, restart, maxit, use_initial_guess, stream) -> int:
    sv = vp()
    check(lib().csg_solve_begin(op, chi, u, nrhs, tol, restart, maxit, use_initial_guess, stream,
                                C.byref(sv)))
    return sv.value


def csg_solve_step(sv) -> int:
    return check(lib().csg_solve_step(sv))


def csg_solve_poll(sv):
    done = C.c_int(0)
    r = check(lib().csg_solve_poll(sv, C.byref(done)))
    return r, bool(done.value)


def csg_solve_end(sv, nrhs):
    infos = (csg_solve_info * max(1, nrhs))()
    rc = lib().csg_solve_end(sv, infos)
    if rc < 0 and rc != CSG_ENOCONV:
        check(rc)
    return rc, [infos[r].as_dict() for r in range(nrhs)]


def csg_batch_workspace_bytes(p: csg_params, nprob: int) -> int:
    n = C.c_size_t(0)
    check(lib().csg_batch_workspace_bytes(C.byref(p), int(nprob), C.byref(n)))
    return n.value


def csg_batch_create(params: list, phi_ptrs: list, ws_ptr: int, ws_bytes: int, stream: int) -> int:
    """params: csg_params per problem; phi_ptrs: host addresses of their phi."""
    k = len(params)
    parr = (C.POINTER(csg_params) * k)(*[C.pointer(p) for p in params])
    farr = (C.c_void_p * k)(*phi_ptrs)
    op = vp()
    check(lib().csg_batch_create(parr, k, farr, ws_ptr, ws_bytes, stream, C.byref(op)))
    return op.value


def helm_step_batch(sv) -> bool:
    done = C.c_int(0)
    check(lib().helm_step_batch(sv, C.byref(done)))
    return bool(done.value)


def csg_profile(op, kind: int, cap: int) -> None:
    check(lib().csg_profile(op, kind, cap))


def csg_profile_read(op):
    """Returns (kernel ms summed, launches, algorithmic bytes summed)."""
    ms, n, by = C.c_double(0), C.c_long(0), C.c_double(0)
    check(lib().csg_profile_read(op, C.byref(ms), C.byref(n), C.byref(by)))
    return ms.value, n.value, by.value


def csg_graphs_active(op) -> bool:
    return check(lib().csg_graphs_active(op)) == 1
