"""Pins of the oracle's grid and operator against facts the paper and the
mathematics fix (section 2: eq. csggrid, the Shortley-Weller scheme, the
Kronecker-sum operators and Lemma 2.1 / Proposition 3.1)."""
import numpy as np
import pytest

from oracle.oracle import Oracle, Params


def P(dim=2, n=16, m=4, beta=0.4, gamma=np.pi / 6, levels=0, h=None, mlo=None, mhi=None, **kw):
    mlo = m if mlo is None else mlo
    mhi = m if mhi is None else mhi
    nn = tuple([n] * dim + [0] * (3 - dim))
    lo = tuple([mlo] * dim + [0] * (3 - dim))
    hi = tuple([mhi] * dim + [0] * (3 - dim))
    return Params(dim=dim, n=nn, h=1.0 / n if h is None else h, layer_lo=lo, layer_hi=hi,
                  gamma=gamma, beta=beta, levels=levels, **kw)


def const_phi(p, val):
    return np.full(p.unknown_shape(), float(val))


def test_axis_nodes_follow_csggrid():
    """eq. csggrid: n intervals of h e^{i theta_beta} between ECS layers of
    h e^{i theta_gamma} (on both sides, per the two-sided-layer remark)."""
    p = P(dim=1, n=10, m=3, beta=0.3)
    o = Oracle(p, const_phi(p, 0))
    h = p.h
    for which, th in ((0, 0.0), (1, p.beta)):
        z = o.axis_nodes(which, 0, 0)
        d = np.diff(z)
        assert np.allclose(d[:3], h * np.exp(1j * p.gamma), rtol=0, atol=1e-15)
        assert np.allclose(d[3:13], h * np.exp(1j * th), rtol=0, atol=1e-15)
        assert np.allclose(d[13:], h * np.exp(1j * p.gamma), rtol=0, atol=1e-15)
        # |h_beta| = h: the edge parametrisation of section 4.3 needs the rotation form
        assert np.allclose(np.abs(d), h, rtol=1e-14)


def test_zero_row_sum_every_axis_every_level():
    """Shortley-Weller weights annihilate constants: west + centre + east = 0."""
    p = P(dim=2, n=24, m=5, beta=0.35, levels=4)
    o = Oracle(p, const_phi(p, 0))
    for l in range(o.levels):
        for a in range(2):
            sw = o.axis_sw(1, l, a)
            scale = np.max(np.abs(sw))
            assert np.max(np.abs(sw.sum(axis=0))) <= 1e-14 * scale


def _plane(shape, xi):
    idx = np.indices(shape)  # (z?, y, x) order
    phase = sum(xi[k] * idx[k] for k in range(len(shape)))
    return np.exp(1j * phase)


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("which", [0, 1])
def test_plane_wave_symbol(dim, which):
    """On a region of uniform spacing s_a with constant phi the 3-point scheme
    has the symbol sum_a 4 sin^2(xi_a/2)/s_a^2 - phi (discrete plane waves)."""
    n = {1: 40, 2: 24, 3: 10}[dim]
    m = {1: 6, 2: 4, 3: 3}[dim]
    p = P(dim=dim, n=n, m=m, beta=0.37)
    phi0 = 123.5
    o = Oracle(p, const_phi(p, phi0))
    shape = p.unknown_shape()
    rng = np.random.default_rng(7)
    xi = rng.uniform(-np.pi, np.pi, size=dim)
    x = _plane(shape, xi)
    y = o.apply(x, which=which, l=0)
    th = 0.0 if which == 0 else p.beta
    s_int = p.h * np.exp(1j * th)
    s_lay = p.h * np.exp(1j * p.gamma)
    # unknown index i is node i+1; interior intervals are nodes m..m+n.
    # Nodes whose 3-point stencil lies entirely in the interior: m+1 .. m+n-1.
    inner = slice(m, m + n - 1)             # unknown indices of those nodes
    # nodes whose stencil lies inside the low layer and off the Dirichlet end:
    # 2 .. m-1 -> unknown 1 .. m-2
    lay = slice(1, m - 1)
    sel_int = tuple([inner] * dim)
    sel_lay = tuple([lay] * dim)
    sym_int = sum(4 * np.sin(xi[k] / 2) ** 2 / s_int ** 2 for k in range(dim)) - phi0
    sym_lay = sum(4 * np.sin(xi[k] / 2) ** 2 / s_lay ** 2 for k in range(dim)) - phi0
    # symbol uses xi per numpy axis; the spacing is the same on every axis
    err_i = np.max(np.abs(y[sel_int] - sym_int * x[sel_int])) / np.max(np.abs(sym_int * x[sel_int]))
    err_l = np.max(np.abs(y[sel_lay] - sym_lay * x[sel_lay])) / np.max(np.abs(sym_lay * x[sel_lay]))
    assert err_i < 1e-13
    assert err_l < 1e-13


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("level", [0, 1, 2])
def test_quadratic_exactness_across_interfaces(dim, level):
    """Shortley-Weller is exact for quadratics in the complex coordinate, also
    at the ECS interfaces and on the nested coarse grids: A(sum_a z_a^2) =
    -2d - phi * sum_a z_a^2 at nodes not next to the Dirichlet ends."""
    n = {1: 22, 2: 14, 3: 8}[dim]
    p = P(dim=dim, n=n, m=5, mlo=5, mhi=3, beta=0.31, levels=3)
    rng = np.random.default_rng(3)
    phi = rng.uniform(10, 50, size=p.unknown_shape())
    o = Oracle(p, phi)
    shape = o.shape(level)
    phil = o.level_phi(level)
    zs = [o.axis_nodes(1, level, a)[1:-1] for a in range(dim)]   # unknown nodes per axis
    grids = np.meshgrid(*reversed(zs), indexing="ij")
    q = sum(g ** 2 for g in grids)
    y = o.apply(q, which=1, l=level)
    expect = -2.0 * dim - phil * q
    sel = tuple(slice(1, s - 1) for s in shape)
    err = np.max(np.abs(y[sel] - expect[sel])) / np.max(np.abs(expect[sel]))
    assert err < 1e-12
    if level == 0:
        zs = [o.axis_nodes(0, 0, a)[1:-1] for a in range(dim)]
        grids = np.meshgrid(*reversed(zs), indexing="ij")
        q = sum(g ** 2 for g in grids)
        y = o.apply(q, which=0, l=0)
        expect = -2.0 * dim - phil * q
        err = np.max(np.abs(y[sel] - expect[sel])) / np.max(np.abs(expect[sel]))
        assert err < 1e-12


@pytest.mark.parametrize("beta", [0.0, 0.25])
def test_dirichlet_sine_modes(beta):
    """Uniform spacing s, no layers: the 1-D Dirichlet eigenpairs are
    sin(k pi j / N) with eigenvalue 4 sin^2(k pi/(2N))/s^2 (textbook)."""
    N = 20
    p = P(dim=1, n=N, m=0, beta=beta, gamma=np.pi / 6)
    phi0 = 17.0
    o = Oracle(p, const_phi(p, phi0))
    s = p.h * np.exp(1j * beta)
    j = np.arange(1, N)
    for k in (1, 2, 7, N - 1):
        v = np.sin(k * np.pi * j / N).astype(np.complex128)
        lam = 4 * np.sin(k * np.pi / (2 * N)) ** 2 / s ** 2 - phi0
        y = o.apply(v, which=1, l=0)
        assert np.max(np.abs(y - lam * v)) <= 1e-12 * np.abs(lam)
    # 2-D Kronecker sum: eigenvalue is the sum of the 1-D ones
    p2 = P(dim=2, n=N, m=0, beta=beta)
    o2 = Oracle(p2, const_phi(p2, phi0))
    for k1, k2 in ((1, 3), (5, 19)):
        v = np.outer(np.sin(k2 * np.pi * j / N), np.sin(k1 * np.pi * j / N)).astype(np.complex128)
        lam = (4 * np.sin(k1 * np.pi / (2 * N)) ** 2 + 4 * np.sin(k2 * np.pi / (2 * N)) ** 2) / s ** 2 - phi0
        y = o2.apply(v, which=1, l=0)
        assert np.max(np.abs(y - lam * v)) <= 1e-12 * np.abs(lam)


def _dense(o, which, l):
    n = o.size(l)
    A = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for c in range(n):
        e[:] = 0
        e[c] = 1
        A[:, c] = o.apply(e, which=which, l=l).ravel()
    return A


def _in_triangle(z, t0, t1, t2, tol):
    # barycentric coordinates
    T = np.array([[t1.real - t0.real, t2.real - t0.real], [t1.imag - t0.imag, t2.imag - t0.imag]])
    rhs = np.vstack([z.real - t0.real, z.imag - t0.imag])
    lam = np.linalg.solve(T, rhs)
    l1, l2 = lam
    l0 = 1 - l1 - l2
    return np.all(l0 >= -tol) and np.all(l1 >= -tol) and np.all(l2 >= -tol)


@pytest.mark.parametrize("dim,n,m", [(1, 32, 8), (2, 16, 8)])
def test_spectrum_in_triangle_every_level(dim, n, m):
    """Lemma 2.1 / Proposition 3.1: on every level the spectrum of M lies in the
    triangle t0 = -k^2, t1 = -k^2 + 4d/(2^l h_beta)^2, t2 = -k^2 + 4d/(2^l h_gamma)^2,
    in the lower half-plane (layer widths chosen so no coarse interval straddles
    an interface)."""
    k = 9.0
    p = P(dim=dim, n=n, m=m, beta=0.4, levels=3)
    o = Oracle(p, const_phi(p, k * k))
    for l in range(o.levels):
        hl = p.h * 2 ** l
        t0 = -k * k + 0j
        t1 = -k * k + 4 * dim / (hl * np.exp(1j * p.beta)) ** 2
        t2 = -k * k + 4 * dim / (hl * np.exp(1j * p.gamma)) ** 2
        ev = np.linalg.eigvals(_dense(o, 1, l))
        assert np.all(ev.imag <= 1e-9 * np.abs(t2))
        assert _in_triangle(ev, t0, t1, t2, 1e-9)
    # H (theta = 0) is the special case beta = 0 (remark after Lemma 2.1)
    evH = np.linalg.eigvals(_dense(o, 0, 0))
    t1 = -k * k + 4 * dim / p.h ** 2 + 0j
    t2 = -k * k + 4 * dim / (p.h * np.exp(1j * p.gamma)) ** 2
    assert _in_triangle(evH, -k * k + 0j, t1, t2, 1e-9)


def test_two_sided_layers_give_double_eigenvalues():
    """Remark after Lemma 2.1: equal layers on both sides of a symmetric interior
    give (nearly) double eigenvalues on the layer branch.  The two layers couple
    weakly through the interior, so the twins agree to a small relative gap, not
    to rounding; a one-sided or differently rotated layer has no twins at all."""
    p = P(dim=1, n=16, m=6, beta=0.0)
    o = Oracle(p, const_phi(p, 0.0))
    ev = np.linalg.eigvals(_dense(o, 1, 0))
    lay = ev[np.abs(ev.imag) > 0.5 * np.max(np.abs(ev.imag))]   # layer-branch tips
    # every strongly complex (layer) eigenvalue has a near twin
    for z in lay:
        d = np.sort(np.abs(lay - z))
        assert d[1] < 1e-4 * np.abs(z)


def test_phi_injection_and_level_dims():
    """Coarse operators by rediscretisation (section 3.1) on ceil-halved grids;
    phi injected from fine node 2J to coarse node J."""
    p = P(dim=2, n=20, m=3, mlo=3, mhi=2, beta=0.3)   # 25 intervals: odd
    rng = np.random.default_rng(11)
    phi = rng.uniform(0, 10, size=p.unknown_shape())
    o = Oracle(p, phi)
    assert [d[0] for d in o.dims] == [24, 12, 6]   # 25 -> 13 -> 7 intervals
    f = o.level_phi(0)
    c = o.level_phi(1)
    assert np.array_equal(c, f[1::2, 1::2][: c.shape[0], : c.shape[1]])
    # nested complex coordinates: coarse node J = fine node 2J, last = last
    for l in range(1, o.levels):
        zf = o.axis_nodes(1, l - 1, 0)
        zc = o.axis_nodes(1, l, 0)
        assert np.array_equal(zc[:-1], zf[: 2 * (len(zc) - 1): 2])
        assert zc[-1] == zf[-1]
