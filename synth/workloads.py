"""Seeded synthetic workloads standing in for the paper's benchmark problems.

Every array is drawn from ``numpy.random.default_rng([10125379, cfg_id, item])``
so the CPU oracle and the GPU library always see identical inputs.  Nothing here
is solver arithmetic: these are the wavenumber fields phi (real FP64 on every
unknown, ECS layers included), the sources chi (complex128, leading RHS axis)
and the cycle/solver settings of each workload.

Grid convention: per axis there are ``layer_lo + n + layer_hi`` intervals of the
mesh width h; node j sits at the real coordinate (j - layer_lo) h, and the
unknowns are the nodes 1 .. N-1 (the far ends of the layers are Dirichlet).
Inside the ECS layers phi is the value at the nearest interior-box node
(constant extension).  Arrays are shaped slowest axis first: (y, x) or (z, y, x).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

SEED = 10125379

__all__ = ["Workload", "rng", "axis_nodes_real", "c1", "c2", "c3", "c4", "c5_request",
           "c5_stream", "small", "rand_cvec", "smooth_field", "SEED", "by_name", "benchmark1", "benchmark3"]


def rng(cfg_id: int, item: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED, cfg_id, item])


@dataclass
class Workload:
    """Problem + cycle + solver settings for one seeded solve."""
    name: str
    dim: int
    n: tuple
    h: float
    layer_lo: tuple
    layer_hi: tuple
    gamma: float
    beta: float
    levels: int
    phi: np.ndarray
    chi: np.ndarray                 # (nrhs, *grid)
    s: int = 3
    nu1: int = 1
    nu2: int = 1
    cycle_prec: int = 0             # 0 = complex128 cycle, 1 = complex64 cycle
    tol: float = 1e-6
    restart: int = 30
    maxit: int = 3000
    meta: dict = field(default_factory=dict)

    @property
    def nrhs(self) -> int:
        return int(self.chi.shape[0])

    @property
    def grid_shape(self) -> tuple:
        return tuple(self.phi.shape)

    @property
    def unknowns(self) -> int:
        return int(np.prod(self.phi.shape))

    def params(self) -> dict:
        """Plain parameter dict (keys of both the oracle and the GPU library)."""
        pad = lambda t: tuple(list(t) + [0] * (3 - len(t)))
        return dict(dim=self.dim, n=pad(self.n), h=self.h, layer_lo=pad(self.layer_lo),
                    layer_hi=pad(self.layer_hi), gamma=self.gamma, beta=self.beta,
                    levels=self.levels, s=self.s, nu1=self.nu1, nu2=self.nu2)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def axis_nodes_real(n: int, mlo: int, mhi: int, h: float) -> np.ndarray:
    """Real coordinates of the unknown nodes 1..N-1 of one axis, clamped to the
    interior box [0, n h] (constant extension of phi into the layers)."""
    j = np.arange(1, n + mlo + mhi)
    x = (j - mlo) * h
    return np.clip(x, 0.0, n * h)


def _mesh(dim, n, mlo, mhi, h):
    axes = [axis_nodes_real(n[a], mlo[a], mhi[a], h) for a in range(dim)]
    # slowest axis first
    return np.meshgrid(*reversed(axes), indexing="ij")  # returns (z?, y, x) order


def _interior_index(n: int, mlo: int, mhi: int) -> np.ndarray:
    """Index of the interior-box node (0..n) nearest to each unknown node."""
    j = np.arange(1, n + mlo + mhi)
    return np.clip(j - mlo, 0, n)


def smooth_field(g: np.random.Generator, dim: int, n: tuple, corr_cells: float = 8.0) -> np.ndarray:
    """Gaussian-filtered i.i.d. N(0,1) noise on the interior-box nodes (n+1 per
    axis), sigma = corr_cells cells, reflecting edges, truncated at 4 sigma,
    normalised to max |g| = 1.  Shape slowest axis first."""
    from scipy.ndimage import gaussian_filter

    shape = tuple(n[a] + 1 for a in reversed(range(dim)))
    noise = g.standard_normal(shape)
    f = gaussian_filter(noise, sigma=corr_cells, mode="reflect", truncate=4.0)
    return f / np.max(np.abs(f))


def _extend(field_box: np.ndarray, dim, n, mlo, mhi) -> np.ndarray:
    """Sample an interior-box nodal field at every unknown (constant extension)."""
    idx = [_interior_index(n[a], mlo[a], mhi[a]) for a in range(dim)]
    return field_box[np.ix_(*reversed(idx))]


def _point_source(shape, index) -> np.ndarray:
    chi = np.zeros(shape, dtype=np.complex128)
    chi[tuple(index)] = 1.0
    return chi


def c1() -> Workload:
    """2-D, 64^2 interior + 8-cell ECS layers, phi = 20^2, unit point source at
    the centre node, beta = 0.4, 5 levels, complex128 (deterministic case)."""
    n, m, h = 64, 8, 1.0 / 64
    shape = (n + 2 * m - 1,) * 2
    phi = np.full(shape, 400.0)
    # centre of the box: node m + n/2 on each axis -> unknown index m + n/2 - 1
    c = m + n // 2 - 1
    chi = _point_source(shape, (c, c))[None]
    return Workload("c1_2d_64_k20_fp64", 2, (n, n), h, (m, m), (m, m), np.pi / 6, 0.4, 5,
                    phi, chi, meta=dict(cfg_id=1))


def c2(item: int = 0) -> Workload:
    """2-D, 1024^2 interior + 32-cell layers, phi = k0^2 (1 - 0.5 exp(-|x-c|^2/0.02)),
    k0 = 0.5/h, Gaussian source of width 2h, beta = 0.4, 8 levels, complex128."""
    g = rng(2, item)
    n, m, h = 1024, 32, 1.0 / 1024
    k0 = 0.5 / h
    cx, cy = g.uniform(0.25, 0.75, size=2)
    sx, sy = g.uniform(0.2, 0.8, size=2)
    Y, X = _mesh(2, (n, n), (m, m), (m, m), h)
    phi = k0 ** 2 * (1.0 - 0.5 * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / 0.02))
    # source uses the unclamped node coordinates
    ax = (np.arange(1, n + 2 * m) - m) * h
    Ys, Xs = np.meshgrid(ax, ax, indexing="ij")
    sig = 2 * h
    chi = np.exp(-((Xs - sx) ** 2 + (Ys - sy) ** 2) / (2 * sig ** 2)).astype(np.complex128)[None]
    return Workload("c2_2d_1024_kh0.5_fp64", 2, (n, n), h, (m, m), (m, m), np.pi / 6, 0.4, 8,
                    phi, chi, meta=dict(cfg_id=2, centre=(cx, cy), source=(sx, sy), k0=k0))


def c3(item: int = 0, cycle_prec: int = 1) -> Workload:
    """2-D, 2048^2 interior + 32-cell layers, three horizontal wave-speed layers
    (interfaces at seeded depths, speeds U[1,2], max kh = 0.5), unit point source
    near (1/2, 1/32), beta = 0.3, 9 levels; complex64 cycle by default."""
    g = rng(3, item)
    n, m, h = 2048, 32, 1.0 / 2048
    d1, d2 = np.sort(g.uniform(0.1, 0.9, size=2))
    r = g.uniform(1.0, 2.0, size=3)
    k = (0.5 / h) * r.min() / r
    Y, X = _mesh(2, (n, n), (m, m), (m, m), h)
    layer = np.where(Y >= d2, 2, np.where(Y >= d1, 1, 0))
    phi = (k ** 2)[layer]
    shape = phi.shape
    ix = m + n // 2 - 1
    iy = m + n // 32 - 1
    chi = _point_source(shape, (iy, ix))[None]
    return Workload("c3_2d_2048_layers_mixed", 2, (n, n), h, (m, m), (m, m), np.pi / 6, 0.3, 9,
                    phi, chi, cycle_prec=cycle_prec,
                    meta=dict(cfg_id=3, depths=(d1, d2), speeds=tuple(r)))


def c4(item: int = 0, nrhs: int = 16, cycle_prec: int = 1) -> Workload:
    """3-D, 128^3 interior + 16-cell layers, phi = k^2 (1 + 0.3 g) with g a
    smooth random field (correlation 8h, max kh = 0.5), 16 unit point sources,
    beta = 0.4, 6 levels; complex64 cycle by default."""
    g = rng(4, item)
    n, m, h = 128, 16, 1.0 / 128
    f = smooth_field(g, 3, (n, n, n))
    k2 = (0.5 / h) ** 2 / np.max(1 + 0.3 * f)
    phi = _extend(k2 * (1 + 0.3 * f), 3, (n,) * 3, (m,) * 3, (m,) * 3)
    shape = phi.shape
    nodes = set()
    chi = np.zeros((nrhs,) + shape, dtype=np.complex128)
    r = 0
    while r < nrhs:
        p = tuple(int(v) for v in g.integers(m, m + n - 1, size=3))  # interior unknowns
        if p in nodes:
            continue
        nodes.add(p)
        chi[r][p] = 1.0
        r += 1
    return Workload("c4_3d_128_16rhs_mixed", 3, (n,) * 3, h, (m,) * 3, (m,) * 3, np.pi / 6, 0.4, 6,
                    phi, chi, cycle_prec=cycle_prec, meta=dict(cfg_id=4))


C5_2D = (256, 512, 1024, 2048)
C5_3D = (64, 96, 128, 192)


def c5_request(item: int, dim: int | None = None, n: int | None = None) -> Workload:
    """One request of the serving stream: 70% 2-D (N in {256..2048}), 30% 3-D
    (N in {64..192}); kh ~ U[0.3,0.6], beta ~ U[0.3,0.5], layers N/16, phi with
    +-30% smooth variation, 1-8 unit point sources; complex64 cycle."""
    g = rng(5, item)
    u = g.uniform()
    if dim is None:
        dim = 2 if u < 0.7 else 3
    if n is None:
        n = int(g.choice(C5_2D if dim == 2 else C5_3D))
    kh = g.uniform(0.3, 0.6)
    beta = g.uniform(0.3, 0.5)
    nrhs = int(g.integers(1, 9))
    m = n // 16
    h = 1.0 / n
    f = smooth_field(g, dim, (n,) * dim)
    k2 = (kh / h) ** 2 / np.max(1 + 0.3 * f)
    phi = _extend(k2 * (1 + 0.3 * f), dim, (n,) * dim, (m,) * dim, (m,) * dim)
    shape = phi.shape
    chi = np.zeros((nrhs,) + shape, dtype=np.complex128)
    for r in range(nrhs):
        p = tuple(int(v) for v in g.integers(m, m + n - 1, size=dim))
        chi[r][p] = 1.0
    return Workload(f"c5_{dim}d_{n}_{item}", dim, (n,) * dim, h, (m,) * dim, (m,) * dim,
                    np.pi / 6, beta, 0, phi, chi, cycle_prec=1,
                    meta=dict(cfg_id=5, item=item, kh=kh))


def c5_stream(count: int, rate: float, start_item: int = 0):
    """Poisson arrival times (seconds) and request ids of the serving stream."""
    g = rng(5, 10 ** 6 + start_item)
    gaps = g.exponential(1.0 / rate, size=count)
    return np.cumsum(gaps), list(range(start_item, start_item + count))


def small(dim: int = 2, n: int = 16, m: int = 4, beta: float = 0.4, kh: float = 0.3,
          item: int = 0, nrhs: int = 1, levels: int = 0, random_phi: bool = True,
          mlo: int | None = None, mhi: int | None = None, gamma: float = np.pi / 6,
          s: int = 3, nu1: int = 1, nu2: int = 1, cycle_prec: int = 0,
          n_axes: tuple | None = None) -> Workload:
    """Small seeded problem for per-operation and end-to-end checks: smooth
    +-30% phi (or constant), random complex sources."""
    g = rng(100 + dim, item)
    mlo = m if mlo is None else mlo
    mhi = m if mhi is None else mhi
    nax = tuple(n_axes) if n_axes is not None else (n,) * dim
    h = 1.0 / n
    k2 = (kh / h) ** 2
    if random_phi:
        f = smooth_field(g, dim, nax, corr_cells=max(1.0, min(nax) / 8))
        phi = _extend(k2 / 1.3 * (1 + 0.3 * f), dim, nax, (mlo,) * dim, (mhi,) * dim)
    else:
        shape = tuple(nax[a] + mlo + mhi - 1 for a in reversed(range(dim)))
        phi = np.full(shape, k2)
    shape = phi.shape
    chi = (g.standard_normal((nrhs,) + shape) + 1j * g.standard_normal((nrhs,) + shape))
    return Workload(f"small_{dim}d_{'x'.join(map(str, nax))}_{item}", dim, nax, h, (mlo,) * dim,
                    (mhi,) * dim, gamma, beta, levels, phi, chi.astype(np.complex128), s=s,
                    nu1=nu1, nu2=nu2, cycle_prec=cycle_prec, meta=dict(cfg_id=100 + dim, item=item))


# The paper's numerical experiments (section 5): theta_beta = 10.3132 degrees,
# theta_gamma = pi/6, V(1,1) with GMRES(3), FGMRES to relative residual 1e-7,
# kh <= 0.625.  The ECS layer width is not stated; m = n/4 cells per layer (the
# width of the hierarchy figure of section 4) is the reading taken here.
PAPER_BETA = 10.3132 * np.pi / 180.0
BENCH1_GRID = {20: 32, 40: 64, 60: 128, 80: 128, 100: 256}
BENCH3_GRID = {0.5: 64, 1.5: 128, 2.5: 256, 3.5: 512, 4.5: 512}


def benchmark1(k: float, n: int | None = None) -> Workload:
    """Benchmark 1 (constant k model): unit square, phi = k^2, unit point
    source at (1/2, 1/2), ECS layers of n/4 cells on every side; the interior
    grid of the paper's table for this k."""
    n = BENCH1_GRID[int(k)] if n is None else n
    m = n // 4
    h = 1.0 / n
    shape = (n + 2 * m - 1,) * 2
    phi = np.full(shape, float(k) ** 2)
    c = m + n // 2 - 1
    chi = _point_source(shape, (c, c))[None]
    return Workload(f"bench1_k{k:g}_{n}", 2, (n, n), h, (m, m), (m, m), np.pi / 6, PAPER_BETA, 0, phi, chi,
                    tol=1e-7, restart=30, maxit=3000, meta=dict(cfg_id=11, k=k))


def benchmark3(k: float, nu: float, n: int | None = None) -> Workload:
    """Benchmark 3 (Gaussian model): the square (0, 50)^2 with
    phi = nu (e^{-x^2} + e^{-y^2}) + k^2 and chi = 1 / (e^{x^2} + e^{y^2}),
    homogeneous Dirichlet on the south and west edges (no layer there), ECS
    layers of n/4 cells on the north and east edges; the interior grid of the
    paper's tables for this k."""
    n = BENCH3_GRID[float(k)] if n is None else n
    m = n // 4
    L = 50.0
    h = L / n
    # unknown nodes 1 .. n + m - 1 per axis; x = j h, phi constant beyond x = L
    x = np.arange(1, n + m) * h
    xc = np.minimum(x, L)
    Y, X = np.meshgrid(xc, xc, indexing="ij")
    phi = nu * (np.exp(-X ** 2) + np.exp(-Y ** 2)) + float(k) ** 2
    Ys, Xs = np.meshgrid(x, x, indexing="ij")
    with np.errstate(over="ignore"):
        chi = (1.0 / (np.exp(Xs ** 2) + np.exp(Ys ** 2))).astype(np.complex128)[None]
    return Workload(f"bench3_k{k:g}_nu{nu:g}_{n}", 2, (n, n), h, (0, 0), (m, m), np.pi / 6, PAPER_BETA, 0, phi, chi,
                    tol=1e-7, restart=30, maxit=3000, meta=dict(cfg_id=13, k=k, nu=nu))


def rand_cvec(shape, item: int = 0, cfg_id: int = 99) -> np.ndarray:
    g = rng(cfg_id, item)
    return (g.standard_normal(shape) + 1j * g.standard_normal(shape)).astype(np.complex128)


def by_name(name: str) -> Workload:
    return {"c1": c1, "c2": c2, "c3": c3, "c4": c4}[name]()
