"""Host-only checks of libcsg: it loads, exports every symbol include/csg.h
declares, and its level planning and parameter validation behave as documented
(no device work is done by these calls)."""
import ctypes as C

import numpy as np
import pytest

from paper_1012_5379_amd import binding as B


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = B.header_symbols()
    assert len(names) >= 17
    for n in names:
        assert hasattr(L, n), n


CONFIG_LEVELS = [
    # (interior n, layer m, dim, expected level count, finest unknowns, coarsest unknowns per axis)
    (64, 8, 2, 5, 79, 4),        # 64^2 + 8-cell layers
    (1024, 32, 2, 8, 1087, 8),   # 1024^2 + 32-cell layers
    (2048, 32, 2, 9, 2111, 8),   # 2048^2 + 32-cell layers
    (128, 16, 3, 6, 159, 4),     # 128^3 + 16-cell layers
]


@pytest.mark.parametrize("n,m,dim,L,nf,nc", CONFIG_LEVELS)
def test_plan_levels_of_the_benchmark_grids(n, m, dim, L, nf, nc):
    p = B.make_params(dim=dim, n=(n,) * dim, h=1.0 / n, layer_lo=(m,) * dim, layer_hi=(m,) * dim)
    levels, dims = B.csg_plan_levels(p)
    assert levels == L
    assert dims[0][:dim] == (nf,) * dim
    assert dims[-1][:dim] == (nc,) * dim
    for l in range(1, levels):
        for a in range(dim):
            assert dims[l][a] == (dims[l - 1][a] + 2) // 2 - 1   # ceil-halved intervals


@pytest.mark.parametrize("dim,n,mlo,mhi,levels", [(2, 20, 3, 2, 0), (3, 10, 2, 1, 3), (2, 13, 0, 4, 2)])
def test_plan_matches_oracle_hierarchy(dim, n, mlo, mhi, levels):
    from oracle.oracle import Oracle, Params
    pad = lambda v: tuple([v] * dim + [0] * (3 - dim))
    op = Params(dim=dim, n=pad(n), h=1.0 / n, layer_lo=pad(mlo), layer_hi=pad(mhi), levels=levels)
    o = Oracle(op, np.zeros(op.unknown_shape()))
    p = B.make_params(dim=dim, n=pad(n), h=1.0 / n, layer_lo=pad(mlo), layer_hi=pad(mhi), levels=levels)
    L, dims = B.csg_plan_levels(p)
    assert L == o.levels
    assert [d[:dim] for d in dims] == [d[:dim] for d in o.dims]


def test_workspace_bytes_grows_with_rhs_and_restart():
    p1 = B.make_params(max_rhs=1)
    p4 = B.make_params(max_rhs=4)
    pr = B.make_params(max_rhs=1, restart=10)
    assert B.csg_workspace_bytes(p4) > B.csg_workspace_bytes(p1) > B.csg_workspace_bytes(pr) > 0
    pm = B.make_params(cycle_prec=1)
    assert B.csg_workspace_bytes(pm) < B.csg_workspace_bytes(p1)


@pytest.mark.parametrize("bad", [
    dict(dim=1), dict(dim=4), dict(beta=0.6, gamma=0.5), dict(beta=-0.1), dict(gamma=0.8),
    dict(s=0), dict(s=9), dict(nu1=-1), dict(max_rhs=0), dict(max_rhs=65), dict(restart=0),
    dict(restart=65), dict(h=0.0), dict(h=float("nan")), dict(cycle_prec=2),
    dict(n=(0, 64, 0)), dict(layer_lo=(-1, 8, 0)),
    dict(levels=9),                               # 80 intervals cannot be halved 8 times
    dict(n=(200, 200, 0), levels=2),              # coarsest would exceed 4096 unknowns
])
def test_invalid_parameters_rejected(bad):
    p = B.make_params(**bad)
    with pytest.raises(B.CsgError) as e:
        B.csg_workspace_bytes(p)
    assert e.value.code == B.CSG_EINVAL
    assert B.csg_last_error()


def test_beta_zero_is_allowed():
    """beta = 0 makes M equal to H; it is a valid (test) configuration."""
    assert B.csg_workspace_bytes(B.make_params(beta=0.0)) > 0


def test_create_rejects_small_workspace_without_device_work():
    p = B.make_params()
    need = B.csg_workspace_bytes(p)
    phi = np.zeros(79 * 79)
    op = C.c_void_p()
    # non-null, aligned fake address: the size check happens before any device access
    rc = B.lib().csg_operator_create(C.byref(p), phi.ctypes.data, 4096 * 256, need - 1, None, C.byref(op))
    assert rc == B.CSG_ENOMEM and not op.value
