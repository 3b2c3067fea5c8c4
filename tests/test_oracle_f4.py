"""Pins of the oracle's two preconditioner variants.

Complex shifted Laplacian (section 1, section 2: M = L - (1 + i eps) k^2):
the oracle's M = L(beta) - s phi with a complex factor s.
  * Dirichlet sine modes of a layer-free box are eigenvectors with
    eigenvalue sum_a (4 / h^2) sin^2(m_a pi / (2 n_a)) - s k^2 (constant phi).
  * On a layer-free grid every interval of the CSG grid is e^{i beta} times
    the real one, so L(beta) = e^{-2i beta} L(0) on every level and
    M_CSG(beta) = e^{-2i beta} M(s = e^{2i beta}, beta = 0): the two
    preconditioners differ by a constant factor, their V-cycles by its
    inverse, and flexible GMRES takes the same iterates (the equivalence of
    the two approaches the paper relies on in section 6).

Galerkin coarse operators (M_{l+1} = R M_l P, the remark in section 5):
  * On a layer-free box with constant phi the operator is a Kronecker sum,
    the transfers tensor products (linear interpolation P_1, full weighting
    R_1 = P_1^T / 2 per axis), so level l's Galerkin operator equals
    sum_a (x)_{b != a} (R_1 P_1)_b (x) (R_1 A_1 P_1)_a - s k^2 (x)_b (R_1 P_1)_b
    built here from dense 1-D textbook matrices, not from the oracle.
  * With ECS layers and a variable phi the stored stencil must reproduce
    R (M_{l-1} (P x)) for random x, from the oracle's separately pinned
    transfers and fine operator, and the coarsest solve inverts it.
  * Galerkin and rediscretised hierarchies give FGMRES counts of the same
    size (the paper reports similar results; ballpark only)."""
import cmath
import math

import numpy as np
import pytest

from oracle.oracle import Oracle, Params
from synth import workloads as W


def _box(dim, n, beta=0.0, **kw):
    n3 = tuple(list(n) + [0] * (3 - len(n)))
    z = (0, 0, 0)
    return Params(dim=dim, n=n3, h=1.0 / max(n), layer_lo=z, layer_hi=z, gamma=0.5, beta=beta, **kw)


@pytest.mark.parametrize("dim,n", [(2, (16, 12)), (3, (8, 6, 10))])
def test_csl_sine_modes(dim, n):
    k2 = 30.0
    s = 1 + 0.5j
    p = _box(dim, n, shift=s)
    shape = tuple(reversed([m - 1 for m in n]))
    o = Oracle(p, np.full(shape, k2))
    h = p.h
    rng = np.random.default_rng(4)
    for _ in range(4):
        m = [int(rng.integers(1, nn)) for nn in n]
        axes = [np.sin(m[a] * np.pi * np.arange(1, n[a]) / n[a]) for a in range(dim)]
        mode = axes[0]
        for a in range(1, dim):
            mode = np.multiply.outer(axes[a], mode)
        lam = sum(4 / h ** 2 * math.sin(m[a] * math.pi / (2 * n[a])) ** 2 for a in range(dim)) - s * k2
        y = o.apply(mode.astype(complex), which=1, l=0)
        assert np.linalg.norm(y - lam * mode) <= 1e-12 * abs(lam) * np.linalg.norm(mode)


def _pair_csg_csl(dim, n, beta, levels=3):
    shape = tuple(reversed([m - 1 for m in n]))
    phi = 20.0 * (1 + 0.3 * W.rng(77, dim).random(shape))
    csg = Oracle(_box(dim, n, beta=beta, levels=levels), phi)
    csl = Oracle(_box(dim, n, beta=0.0, levels=levels, shift=cmath.exp(2j * beta)), phi)
    return csg, csl, shape


@pytest.mark.parametrize("dim,n", [(2, (24, 17)), (3, (10, 9, 12))])
def test_csg_is_scaled_csl(dim, n):
    beta = 0.3
    a = cmath.exp(-2j * beta)
    csg, csl, shape = _pair_csg_csl(dim, n, beta)
    for l in range(csg.levels):
        x = W.rand_cvec(csg.shape(l), item=l)
        y1, y2 = csg.apply(x, which=1, l=l), a * csl.apply(x, which=1, l=l)
        assert np.linalg.norm(y1 - y2) <= 1e-13 * np.linalg.norm(y1)
    b = W.rand_cvec(shape, item=9)
    v1, v2 = csg.vcycle(b), csl.vcycle(b) / a
    assert np.linalg.norm(v1 - v2) <= 1e-11 * np.linalg.norm(v1)
    chi = W.rand_cvec(shape, item=10)
    u1, i1 = csg.fgmres(chi, tol=1e-9, restart=20)
    u2, i2 = csl.fgmres(chi, tol=1e-9, restart=20)
    assert i1.converged and i2.converged and i1.iterations == i2.iterations
    assert np.linalg.norm(u1 - u2) <= 1e-9 * np.linalg.norm(u1)


def _p1(nf):
    """Dense 1-D linear interpolation from the ceil-halved grid: fine unknowns
    1..nf-1 (node index), coarse unknowns 1..nc-1 with coarse node c at fine 2c."""
    nc = (nf + 1) // 2
    P = np.zeros((nf - 1, nc - 1))
    for c in range(1, nc):
        f = 2 * c
        if f <= nf - 1:
            P[f - 1, c - 1] = 1.0
        for g in (f - 1, f + 1):
            if 1 <= g <= nf - 1:
                P[g - 1, c - 1] = 0.5
    return P


def _a1(nf, h, beta):
    """Dense 1-D negative Laplacian on a uniform complex grid h e^{i beta}."""
    m = nf - 1
    A = (np.diag(np.full(m, 2.0)) - np.diag(np.ones(m - 1), 1) - np.diag(np.ones(m - 1), -1)) / h ** 2
    return A * cmath.exp(-2j * beta)


def _kron_all(mats):
    out = mats[-1]
    for m in reversed(mats[:-1]):
        out = np.kron(out, m)   # numpy order: slowest axis first, so the last axis is outermost
    return out


def _stencil_dense(st, shape, dim):
    """Assemble a [offset][unknown] stencil (x fastest) into a dense matrix."""
    N = int(np.prod(shape))
    nu = list(reversed(shape)) + [1] * (3 - dim)
    A = np.zeros((N, N), dtype=complex)
    flat = st.reshape(3 ** dim, N)
    for p in range(N):
        i, j, k = p % nu[0], (p // nu[0]) % nu[1], p // (nu[0] * nu[1])
        for oi in range(3 ** dim):
            o = [(oi // 3 ** a) % 3 - 1 if a < dim else 0 for a in range(3)]
            q = [i + o[0], j + o[1], k + o[2]]
            if all(0 <= q[a] < nu[a] for a in range(3)):
                A[p, q[0] + nu[0] * (q[1] + nu[1] * q[2])] = flat[oi, p]
    return A


@pytest.mark.parametrize("dim,n", [(2, (16, 12)), (2, (13, 10)), (3, (8, 8, 6))])
def test_galerkin_closed_form_layer_free(dim, n):
    beta, k2, s = 0.25, 15.0, 1 + 0.2j
    p = _box(dim, n, beta=beta, levels=3, shift=s, coarse_op=1)
    shape = tuple(reversed([m - 1 for m in n]))
    o = Oracle(p, np.full(shape, k2))
    # 1-D pieces per axis and level (x first)
    A = [[_a1(n[a], p.h, beta)] for a in range(dim)]
    Mm = [[np.eye(n[a] - 1)] for a in range(dim)]
    nf = list(n)
    for l in range(1, 3):
        for a in range(dim):
            P = _p1(nf[a])
            R = 0.5 * P.T
            A[a].append(R @ A[a][-1] @ P)
            Mm[a].append(R @ Mm[a][-1] @ P)
        nf = [(m + 1) // 2 for m in nf]
        ref = -s * k2 * _kron_all([Mm[a][l] for a in range(dim)])
        for a in range(dim):
            ref = ref + _kron_all([A[b][l] if b == a else Mm[b][l] for b in range(dim)])
        got = _stencil_dense(o.galerkin_stencil(l), o.shape(l), dim)
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref), l


@pytest.mark.parametrize("dim", [2, 3])
def test_galerkin_reproduces_product_with_layers(dim):
    w = W.small(dim=dim, n=20 if dim == 2 else 9, mlo=4, mhi=3, beta=0.35, kh=0.4, item=5)
    p = Params(**w.params(), coarse_op=1)
    o = Oracle(p, w.phi)
    for l in range(1, o.levels):
        x = W.rand_cvec(o.shape(l), item=20 + l)
        ref = o.restrict(o.apply(o.prolong_add(x, np.zeros(o.shape(l - 1), complex), l - 1), which=1, l=l - 1), l - 1)
        y = o.apply(x, which=1, l=l)
        assert np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref), l
    L = o.levels - 1
    x = W.rand_cvec(o.shape(L), item=31)
    assert np.linalg.norm(o.coarse_solve(o.apply(x, which=1, l=L)) - x) <= 1e-11 * np.linalg.norm(x)


def test_galerkin_and_rediscretisation_similar():
    w = W.benchmark1(40)
    it = {}
    for op in (0, 1):
        o = Oracle(Params(**w.params(), coarse_op=op), w.phi)
        _, info = o.fgmres(w.chi[0], tol=w.tol, restart=30, maxit=600)
        assert info.converged
        it[op] = info.iterations
    print(f"Benchmark 1 k=40: rediscretised {it[0]}, Galerkin {it[1]} iterations")
    assert 0.5 <= it[1] / it[0] <= 2.0


def test_invalid_combinations_rejected():
    w = W.small(dim=2, n=20, m=4)
    for bad in (dict(smoother=1, coarse_op=1), dict(smoother=1, shift=1 + 0.5j), dict(coarse_op=2)):
        with pytest.raises(Exception):
            Oracle(Params(**w.params(), **bad), w.phi)
