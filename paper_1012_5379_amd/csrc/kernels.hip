// kernels.hip -- gfx950 kernels of libcsg.
//
// Every level pass walks a contiguous chunk of grid points per block (x
// fastest), so loads and stores of interleaved complex values are coalesced.
// Chunks are remapped so the blocks an XCD receives cover one contiguous
// eighth of the grid, keeping the y/z stencil neighbours inside that XCD's L2.
// Passes that feed a global inner product write one partial sum per block; the
// blocks of the next pass re-reduce those partials in a fixed order, so results
// are deterministic, no atomics are used and no pass waits on another block.
// Inner products and norms accumulate in FP64 even when vectors are complex64.
#include <cfloat>
#include <cmath>

#include "kernels.h"

namespace csg {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ unsigned chunk_id(int nb)
{
    const unsigned b = blockIdx.x;
    if ((nb & 7) == 0) return (b & 7u) * (unsigned)(nb >> 3) + (b >> 3);
    return b;
}

template <int DIM>
__device__ __forceinline__ void decomp(unsigned p, unsigned nx, unsigned ny, unsigned &i, unsigned &j, unsigned &k)
{
    if (DIM == 2) {
        j = p / nx;
        i = p - j * nx;
        k = 0;
    } else {
        const unsigned t = p / nx;
        i = p - t * nx;
        k = t / ny;
        j = t - k * ny;
    }
}

// (A x)_p for the Kronecker-sum operator: per axis west/centre/east weights,
// diagonal minus phi.  Boundary weights are zero in the tables, so the clamped
// neighbour index only keeps the load in range.
template <typename T, int DIM, typename TI>
__device__ __forceinline__ Cx<T> apply_pt(const LvlK<T> &L, const Cx<TI> *__restrict__ x, unsigned i, unsigned j,
                                          unsigned k, unsigned p)
{
    const Cx<T> *tx = L.tab[0];
    Cx<T> d = tx[L.nx + i];
    if (DIM >= 2) d = d + L.tab[1][L.ny + j];
    if (DIM == 3) d = d + L.tab[2][L.nz + k];
    d.re -= L.phi[p];
    Cx<T> acc = d * cvt<T>(x[p]);
    acc = cfma(tx[i], cvt<T>(x[i ? p - 1 : p]), acc);
    acc = cfma(tx[2 * L.nx + i], cvt<T>(x[i + 1 < L.nx ? p + 1 : p]), acc);
    if (DIM >= 2) {
        const Cx<T> *ty = L.tab[1];
        acc = cfma(ty[j], cvt<T>(x[j ? p - L.nx : p]), acc);
        acc = cfma(ty[2 * L.ny + j], cvt<T>(x[j + 1 < L.ny ? p + L.nx : p]), acc);
    }
    if (DIM == 3) {
        const Cx<T> *tz = L.tab[2];
        const unsigned sz = L.nx * L.ny;
        acc = cfma(tz[k], cvt<T>(x[k ? p - sz : p]), acc);
        acc = cfma(tz[2 * L.nz + k], cvt<T>(x[k + 1 < L.nz ? p + sz : p]), acc);
    }
    return acc;
}

// Wavefront (64 lanes) butterfly, then the 4 wavefronts in order.  Every lane
// ends with bit-identical sums (pairwise additions are commutative).
template <int NV>
__device__ __forceinline__ void block_sum(zc (&v)[NV], int nv, zc *sh, zc *res)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        if (q < nv) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                v[q].re += __shfl_xor(v[q].re, off, 64);
                v[q].im += __shfl_xor(v[q].im, off, 64);
            }
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q)
            if (q < nv) sh[wv * NV + q] = v[q];
    }
    __syncthreads();
    if (threadIdx.x < nv) {
        const int q = threadIdx.x;
        zc a = sh[q];
        a = a + sh[NV + q];
        a = a + sh[2 * NV + q];
        a = a + sh[3 * NV + q];
        res[q] = a;
    }
    __syncthreads();
}

// Sum the per-block partials of one RHS (layout [value][NBMAX]).
template <int NV>
__device__ __forceinline__ void reduce_parts(const zc *part, int nb, int nv, zc *sh, zc *res)
{
    zc v[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        v[q] = mkc(0.0, 0.0);
        if (q < nv)
            for (int b = threadIdx.x; b < nb; b += BLK) v[q] = v[q] + part[q * NBMAX + b];
    }
    block_sum<NV>(v, nv, sh, res);
}

// Complex Givens rotation [c s; -conj(s) c] (c real) taking (a, b) to (r, 0).
__device__ __forceinline__ void rot(zc a, zc b, double &c, zc &s)
{
    const double aa = sqrt(cabs2(a)), bb = sqrt(cabs2(b));
    if (bb == 0.0) { c = 1.0; s = mkc(0.0, 0.0); return; }
    if (aa == 0.0) { c = 0.0; s = mkc(b.re / bb, -b.im / bb); return; }
    const double nu = hypot(aa, bb);
    c = aa / nu;
    const zc ph = mkc(a.re / aa, a.im / aa);
    s = (1.0 / nu) * (ph * mkc(b.re, -b.im));
}

// Least squares of one GMRES(s) sweep: y = argmin || beta0 e1 - Hbar y || over
// the first k Arnoldi columns, and the residual coefficients
// cres = beta0 e1 - Hbar y (so that r = sum_i cres_i v_i).  R is caller
// scratch of (CSG_MAX_S+1) * CSG_MAX_S values.  Returns k.
__device__ int gmres_ls(const GState *gs, int s, double hn_last, zc *R, zc *y, zc *cres)
{
    const double beta0 = gs->beta0;
    int k = gs->k;
    if (k > s) k = s;
    if (!(beta0 > 0.0)) k = 0;
    auto hget = [&](int i, int c) -> zc {
        if (i > c + 1) return mkc(0.0, 0.0);
        return (i == s && c == s - 1) ? mkc(hn_last, 0.0) : gs->H[i * CSG_MAX_S + c];
    };
    for (int i = 0; i <= k; ++i)
        for (int c = 0; c < k; ++c) R[i * CSG_MAX_S + c] = hget(i, c);
    zc g[CSG_MAX_S + 1];
    for (int i = 0; i <= CSG_MAX_S; ++i) g[i] = mkc(0.0, 0.0);
    g[0] = mkc(beta0, 0.0);
    double cs[CSG_MAX_S];
    zc sn[CSG_MAX_S];
    for (int c = 0; c < k; ++c) {
        for (int i = 0; i < c; ++i) {
            const zc t1 = R[i * CSG_MAX_S + c], t2 = R[(i + 1) * CSG_MAX_S + c];
            R[i * CSG_MAX_S + c] = cs[i] * t1 + sn[i] * t2;
            R[(i + 1) * CSG_MAX_S + c] = cs[i] * t2 - mkc(sn[i].re, -sn[i].im) * t1;
        }
        rot(R[c * CSG_MAX_S + c], R[(c + 1) * CSG_MAX_S + c], cs[c], sn[c]);
        const zc t1 = R[c * CSG_MAX_S + c], t2 = R[(c + 1) * CSG_MAX_S + c];
        R[c * CSG_MAX_S + c] = cs[c] * t1 + sn[c] * t2;
        R[(c + 1) * CSG_MAX_S + c] = mkc(0.0, 0.0);
        const zc gc = g[c];
        g[c + 1] = mkc(0.0, 0.0) - mkc(sn[c].re, -sn[c].im) * gc;
        g[c] = cs[c] * gc;
    }
    for (int i = k - 1; i >= 0; --i) {
        zc acc = g[i];
        for (int c = i + 1; c < k; ++c) acc = acc - R[i * CSG_MAX_S + c] * y[c];
        const zc d = R[i * CSG_MAX_S + i];
        y[i] = (1.0 / cabs2(d)) * (acc * mkc(d.re, -d.im));
    }
    for (int i = 0; i <= k; ++i) {
        zc acc = (i == 0) ? mkc(beta0, 0.0) : mkc(0.0, 0.0);
        for (int c = 0; c < k; ++c) acc = acc - hget(i, c) * y[c];
        cres[i] = acc;
    }
    return k;
}

// ---------------------------------------------------------------------------
// operator application
// ---------------------------------------------------------------------------

template <typename T, int DIM>
__global__ __launch_bounds__(BLK) void k_apply(LvlK<T> L, const Cx<T> *__restrict__ x, Cx<T> *__restrict__ y,
                                               size_t ld, unsigned chunk, int nb, const int *active)
{
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    x += rhs * ld;
    y += rhs * ld;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(L.N, p0 + chunk);
    for (unsigned p = p0 + threadIdx.x; p < p1; p += BLK) {
        unsigned i, j, k;
        decomp<DIM>(p, L.nx, L.ny, i, j, k);
        y[p] = apply_pt<T, DIM>(L, x, i, j, k, p);
    }
}

// ---------------------------------------------------------------------------
// GMRES(s) sweep passes
// ---------------------------------------------------------------------------

// Arnoldi step j, first half: w = A u_j (raw basis vector) and the inner
// products <u_i, w>, i <= j (plus <u_0, u_0> when j = 0).  Block 0 first
// finishes the previous step's norm: h_{j,j-1} and the scale of u_j.
template <typename T, int DIM>
__global__ __launch_bounds__(BLK) void k_st(LvlK<T> L, Basis<T> B, int j, size_t ld, const zc *__restrict__ pin,
                                            int nbin, zc *__restrict__ pout, GState *gsb, double tiny,
                                            unsigned chunk, int nb, const int *active)
{
    __shared__ zc sh[4 * NVAL];
    __shared__ zc res[NVAL];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    GState *gs = gsb + rhs;
    if (j >= 1 && blockIdx.x == 0) {
        reduce_parts<1>(pin + (size_t)rhs * NVAL * NBMAX, nbin, 1, sh, res);
        if (threadIdx.x == 0) {
            const double hn = sqrt(res[0].re);
            const bool brk = !(hn > tiny * gs->beta0);
            gs->H[j * CSG_MAX_S + (j - 1)] = mkc(hn, 0.0);
            gs->sig[j] = brk ? 0.0 : 1.0 / hn;
            if (brk && gs->k > j) gs->k = j;
        }
    }
    const size_t off = rhs * ld;
    const Cx<T> *uj = B.u[j] + off;
    Cx<T> *w = B.u[j + 1] + off;
    const int nv = j + 1 + (j == 0);
    zc acc[NVAL];
#pragma unroll
    for (int q = 0; q < NVAL; ++q) acc[q] = mkc(0.0, 0.0);
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(L.N, p0 + chunk);
    for (unsigned p = p0 + threadIdx.x; p < p1; p += BLK) {
        unsigned i, jj, k;
        decomp<DIM>(p, L.nx, L.ny, i, jj, k);
        const Cx<T> wv = apply_pt<T, DIM>(L, uj, i, jj, k, p);
        w[p] = wv;
        const zc wd = cvt<double>(wv);
#pragma unroll
        for (int q = 0; q < NVAL - 1; ++q)
            if (q <= j) acc[q] = cjfma(cvt<double>(B.u[q][off + p]), wd, acc[q]);
        if (j == 0) acc[1].re += cabs2(cvt<double>(uj[p]));
    }
    block_sum<NVAL>(acc, nv, sh, res);
    if (threadIdx.x < nv) pout[((size_t)rhs * NVAL + threadIdx.x) * NBMAX + c] = res[threadIdx.x];
}

// Arnoldi step j, second half: h_ij = sig_i sig_j <u_i, w>, then
// u_{j+1} = sig_j w - sum_i h_ij sig_i u_i (classical Gram-Schmidt) and the
// partial ||u_{j+1}||^2.
template <typename T>
__global__ __launch_bounds__(BLK) void k_orth(Basis<T> B, int j, unsigned N, size_t ld, const zc *__restrict__ pin,
                                              int nbin, zc *__restrict__ pout, GState *gsb, unsigned chunk, int nb,
                                              int s, const int *active)
{
    __shared__ zc sh[4 * NVAL];
    __shared__ zc res[NVAL];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    GState *gs = gsb + rhs;
    const int nv = j + 1 + (j == 0);
    reduce_parts<NVAL>(pin + (size_t)rhs * NVAL * NBMAX, nbin, nv, sh, res);
    double sig[NVAL];
    double beta0;
    if (j == 0) {
        beta0 = sqrt(res[1].re);
        sig[0] = beta0 > 0.0 ? 1.0 / beta0 : 0.0;
    } else {
        beta0 = gs->beta0;
#pragma unroll
        for (int q = 0; q < NVAL; ++q)
            if (q <= j) sig[q] = gs->sig[q];
    }
    double sj = 0.0;
#pragma unroll
    for (int q = 0; q < NVAL; ++q)
        if (q == j) sj = sig[q];
    zc h[NVAL];
    Cx<T> cu[NVAL];
#pragma unroll
    for (int q = 0; q < NVAL; ++q) {
        if (q <= j) {
            h[q] = (sig[q] * sj) * res[q];
            cu[q] = cvt<T>(sig[q] * h[q]);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (j == 0) {
            gs->beta0 = beta0;
            gs->sig[0] = sig[0];
            gs->k = s;
        }
#pragma unroll
        for (int q = 0; q < NVAL; ++q)
            if (q <= j) gs->H[q * CSG_MAX_S + j] = h[q];
    }
    const size_t off = rhs * ld;
    Cx<T> *w = B.u[j + 1] + off;
    const T aw = (T)sj;
    zc acc[1] = {mkc(0.0, 0.0)};
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(N, p0 + chunk);
    for (unsigned p = p0 + threadIdx.x; p < p1; p += BLK) {
        Cx<T> v = aw * w[p];
#pragma unroll
        for (int q = 0; q < NVAL - 1; ++q)
            if (q <= j) v = v - cu[q] * B.u[q][off + p];
        w[p] = v;
        acc[0].re += cabs2(cvt<double>(v));
    }
    block_sum<1>(acc, 1, sh, res);
    if (threadIdx.x == 0) pout[((size_t)rhs * NVAL) * NBMAX + c] = res[0];
}

// Shared prologue of the sweep's closing passes: finish h_{s,s-1}, solve the
// small least-squares problem and publish coefficients in shared memory:
// ax[i] = y_i sig_i (update), ar[i] = cres_i sig_i (Arnoldi residual).
__device__ int close_sweep(const zc *pin, int nbin, GState *gs, int s, double tiny, zc *sh, zc *res, zc *ax, zc *ar)
{
    reduce_parts<1>(pin, nbin, 1, sh, res);
    __shared__ int ks;
    __shared__ zc Rs[(CSG_MAX_S + 1) * CSG_MAX_S], ys[CSG_MAX_S], crs[CSG_MAX_S + 1];
    if (threadIdx.x == 0) {
        const double hn = sqrt(res[0].re);
        const bool brk = !(hn > tiny * gs->beta0);
        const double sig_s = brk ? 0.0 : 1.0 / hn;
        zc *y = ys, *cr = crs;
        const int k = gmres_ls(gs, s, hn, Rs, y, cr);
        for (int i = 0; i < k; ++i) ax[i] = gs->sig[i] * y[i];
        for (int i = 0; i <= k; ++i) ar[i] = ((i == s) ? sig_s : gs->sig[i]) * cr[i];
        ks = k;
        if (blockIdx.x == 0) {
            gs->H[s * CSG_MAX_S + (s - 1)] = mkc(hn, 0.0);
            gs->sig[s] = sig_s;
            for (int i = 0; i < k; ++i) gs->y[i] = y[i];
        }
    }
    __syncthreads();
    return ks;
}

// x (+)= sum_i y_i sig_i u_i
template <typename T>
__global__ __launch_bounds__(BLK) void k_upd(Cx<T> *x, int accumulate, Basis<T> B, int s, unsigned N, size_t ld,
                                             const zc *__restrict__ pin, int nbin, GState *gsb, double tiny,
                                             unsigned chunk, int nb, const int *active)
{
    __shared__ zc sh[4];
    __shared__ zc res[1];
    __shared__ zc ax[CSG_MAX_S], ar[CSG_MAX_S + 1];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const int k = close_sweep(pin + (size_t)rhs * NVAL * NBMAX, nbin, gsb + rhs, s, tiny, sh, res, ax, ar);
    Cx<T> cx[CSG_MAX_S];
#pragma unroll
    for (int q = 0; q < CSG_MAX_S; ++q)
        if (q < k) cx[q] = cvt<T>(ax[q]);
    const size_t off = rhs * ld;
    Cx<T> *xx = x + off;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(N, p0 + chunk);
    for (unsigned p = p0 + threadIdx.x; p < p1; p += BLK) {
        Cx<T> v = accumulate ? xx[p] : mkc<T>(0, 0);
#pragma unroll
        for (int q = 0; q < CSG_MAX_S; ++q)
            if (q < k) v = cfma(cx[q], B.u[q][off + p], v);
        xx[p] = v;
    }
}

// --- per-axis index helpers for the transfers -------------------------------
// Fine unknown i (node f = i+1) interpolates from coarse node f/2 (f even,
// weight 1) or nodes (f-1)/2 and (f+1)/2 (f odd, weight 1/2); coarse node c is
// an unknown (index c-1) when 1 <= c <= nuc.
struct PAx {
    int n;
    unsigned idx[2];
    float w[2];
};
__device__ __forceinline__ PAx paxis(unsigned i, unsigned nuc)
{
    PAx a;
    a.n = 0;
    const unsigned f = i + 1;
    if ((f & 1u) == 0) {
        const unsigned c = f >> 1;
        if (c >= 1 && c <= nuc) { a.idx[0] = c - 1; a.w[0] = 1.f; a.n = 1; }
    } else {
        const unsigned c0 = (f - 1) >> 1, c1 = (f + 1) >> 1;
        if (c0 >= 1) { a.idx[a.n] = c0 - 1; a.w[a.n] = 0.5f; a.n++; }
        if (c1 <= nuc) { a.idx[a.n] = c1 - 1; a.w[a.n] = 0.5f; a.n++; }
    }
    return a;
}

template <typename T, int DIM>
__device__ __forceinline__ Cx<T> prolong_pt(const Cx<T> *__restrict__ ec, unsigned i, unsigned j, unsigned k,
                                            unsigned ncx, unsigned ncy, unsigned ncz)
{
    const PAx ax = paxis(i, ncx);
    Cx<T> acc = mkc<T>(0, 0);
    if (DIM == 2) {
        const PAx ay = paxis(j, ncy);
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a)
                if (b < ay.n && a < ax.n)
                    acc = acc + (T)(ax.w[a] * ay.w[b]) * ec[ay.idx[b] * ncx + ax.idx[a]];
    } else {
        const PAx ay = paxis(j, ncy), az = paxis(k, ncz);
#pragma unroll
        for (int cz = 0; cz < 2; ++cz)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 2; ++a)
                    if (cz < az.n && b < ay.n && a < ax.n)
                        acc = acc + (T)(ax.w[a] * ay.w[b] * az.w[cz]) *
                                        ec[(az.idx[cz] * ncy + ay.idx[b]) * ncx + ax.idx[a]];
    }
    return acc;
}

// Fine nodes 2c-1, 2c, 2c+1 of coarse node c = I+1 along one axis, as fine
// unknown indices 2I, 2I+1, 2I+2 with weights 1/2, 1, 1/2; a node outside the
// unknown range contributes nothing.  `own` marks the nodes whose x this
// coarse point writes (2c-1, 2c, and 2c+1 for the last coarse unknown).
struct RAx {
    unsigned lo;
    int n;
    int own;   // bit q set: node lo+q is owned
};
__device__ __forceinline__ RAx raxis(unsigned I, unsigned nuc, unsigned nuf)
{
    RAx r;
    r.lo = 2 * I;
    r.n = (2 * I + 2 < nuf) ? 3 : (2 * I + 1 < nuf ? 2 : 1);
    r.own = 3;
    if (I + 1 == nuc && r.n == 3) r.own = 7;
    r.own &= (1 << r.n) - 1;
    return r;
}
__device__ __forceinline__ float rw(int q) { return q == 1 ? 1.f : 0.5f; }

// Closing pass of the last pre-smoothing sweep fused with the restriction:
// x (+)= sum y_i sig_i u_i on the fine grid, and
// bc = 2^-d P^T r with the Arnoldi residual r = sum_i cres_i sig_i u_i.
template <typename T, int DIM>
__global__ __launch_bounds__(BLK) void k_upd_res(Cx<T> *x, int accumulate, Basis<T> B, int s, LvlK<T> F, LvlK<T> C,
                                                 Cx<T> *bc, size_t ldf, size_t ldc, const zc *__restrict__ pin,
                                                 int nbin, GState *gsb, double tiny, unsigned chunk, int nb,
                                                 const int *active)
{
    __shared__ zc sh[4];
    __shared__ zc res[1];
    __shared__ zc ax[CSG_MAX_S], ar[CSG_MAX_S + 1];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const int k = close_sweep(pin + (size_t)rhs * NVAL * NBMAX, nbin, gsb + rhs, s, tiny, sh, res, ax, ar);
    Cx<T> cx[CSG_MAX_S], cr[CSG_MAX_S + 1];
#pragma unroll
    for (int q = 0; q <= CSG_MAX_S; ++q) {
        if (q < k) cx[q] = cvt<T>(ax[q]);
        if (q <= k) cr[q] = cvt<T>(ar[q]);
    }
    const size_t offf = rhs * ldf;
    Cx<T> *xx = x + offf;
    Cx<T> *bb = bc + rhs * ldc;
    const T scale = (DIM == 2) ? (T)0.25 : (T)0.125;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(C.N, p0 + chunk);
    for (unsigned pc = p0 + threadIdx.x; pc < p1; pc += BLK) {
        unsigned I, J, K;
        decomp<DIM>(pc, C.nx, C.ny, I, J, K);
        const RAx rx = raxis(I, C.nx, F.nx);
        const RAx ry = raxis(J, C.ny, F.ny);
        const RAx rz = (DIM == 3) ? raxis(K, C.nz, F.nz) : RAx{0, 1, 1};
        Cx<T> acc = mkc<T>(0, 0);
        for (int qz = 0; qz < rz.n; ++qz)
            for (int qy = 0; qy < ry.n; ++qy)
                for (int qx = 0; qx < rx.n; ++qx) {
                    const unsigned fp = ((rz.lo + qz) * F.ny + (ry.lo + qy)) * F.nx + (rx.lo + qx);
                    Cx<T> uv[CSG_MAX_S + 1];
#pragma unroll
                    for (int q = 0; q <= CSG_MAX_S; ++q)
                        if (q <= k) uv[q] = B.u[q][offf + fp];
                    Cx<T> r = mkc<T>(0, 0);
#pragma unroll
                    for (int q = 0; q <= CSG_MAX_S; ++q)
                        if (q <= k) r = cfma(cr[q], uv[q], r);
                    T wgt = (T)(rw(qx) * rw(qy));
                    if (DIM == 3) wgt *= (T)rw(qz);
                    acc = acc + wgt * r;
                    const bool own = ((rx.own >> qx) & 1) && ((ry.own >> qy) & 1) && ((rz.own >> qz) & 1);
                    if (own) {
                        Cx<T> v = accumulate ? xx[fp] : mkc<T>(0, 0);
#pragma unroll
                        for (int q = 0; q < CSG_MAX_S; ++q)
                            if (q < k) v = cfma(cx[q], uv[q], v);
                        xx[fp] = v;
                    }
                }
        bb[pc] = scale * acc;
    }
}

// r = b - A x
template <typename T, int DIM>
__global__ __launch_bounds__(BLK) void k_resid(LvlK<T> L, const Cx<T> *__restrict__ x, const Cx<T> *__restrict__ b,
                                               Cx<T> *__restrict__ r, size_t ld, unsigned chunk, int nb,
                                               const int *active)
{
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const size_t off = rhs * ld;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(L.N, p0 + chunk);
    for (unsigned p = p0 + threadIdx.x; p < p1; p += BLK) {
        unsigned i, j, k;
        decomp<DIM>(p, L.nx, L.ny, i, j, k);
        r[off + p] = b[off + p] - apply_pt<T, DIM>(L, x + off, i, j, k, p);
    }
}

// bc = 2^-d P^T (b - A x)   (x may be null: bc = 2^-d P^T b)
template <typename T, int DIM>
__global__ __launch_bounds__(BLK) void k_restrict(LvlK<T> F, LvlK<T> C, const Cx<T> *__restrict__ x,
                                                  const Cx<T> *__restrict__ b, Cx<T> *__restrict__ bc, size_t ldf,
                                                  size_t ldc, unsigned chunk, int nb, const int *active)
{
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const size_t offf = rhs * ldf;
    const Cx<T> *xx = x ? x + offf : nullptr;
    const T scale = (DIM == 2) ? (T)0.25 : (T)0.125;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(C.N, p0 + chunk);
    for (unsigned pc = p0 + threadIdx.x; pc < p1; pc += BLK) {
        unsigned I, J, K;
        decomp<DIM>(pc, C.nx, C.ny, I, J, K);
        const RAx rx = raxis(I, C.nx, F.nx);
        const RAx ry = raxis(J, C.ny, F.ny);
        const RAx rz = (DIM == 3) ? raxis(K, C.nz, F.nz) : RAx{0, 1, 1};
        Cx<T> acc = mkc<T>(0, 0);
        for (int qz = 0; qz < rz.n; ++qz)
            for (int qy = 0; qy < ry.n; ++qy)
                for (int qx = 0; qx < rx.n; ++qx) {
                    const unsigned fi = rx.lo + qx, fj = ry.lo + qy, fk = rz.lo + qz;
                    const unsigned fp = (fk * F.ny + fj) * F.nx + fi;
                    Cx<T> r = b[offf + fp];
                    if (xx) r = r - apply_pt<T, DIM>(F, xx, fi, fj, fk, fp);
                    T wgt = (T)(rw(qx) * rw(qy));
                    if (DIM == 3) wgt *= (T)rw(qz);
                    acc = acc + wgt * r;
                }
        bc[rhs * ldc + pc] = scale * acc;
    }
}

// xout = xin + P ec   (xin may be null; xin == xout allowed)
template <typename T, int DIM>
__global__ __launch_bounds__(BLK) void k_prolong(LvlK<T> F, LvlK<T> C, const Cx<T> *ec, const Cx<T> *xin,
                                                 Cx<T> *xout, size_t ldf, size_t ldc, unsigned chunk, int nb,
                                                 const int *active)
{
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const size_t off = rhs * ldf;
    const Cx<T> *e = ec + rhs * ldc;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(F.N, p0 + chunk);
    for (unsigned p = p0 + threadIdx.x; p < p1; p += BLK) {
        unsigned i, j, k;
        decomp<DIM>(p, F.nx, F.ny, i, j, k);
        Cx<T> v = prolong_pt<T, DIM>(e, i, j, k, C.nx, C.ny, C.nz);
        if (xin) v = v + xin[off + p];
        xout[off + p] = v;
    }
}

// Interpolated correction fused with the residual that opens the next sweep:
// xout = xin + P ec and r = b - A xout (xout at the neighbours recomputed).
template <typename T, int DIM>
__device__ __forceinline__ Cx<T> corrected(const Cx<T> *xin, const Cx<T> *e, unsigned i, unsigned j, unsigned k,
                                           unsigned p, const LvlK<T> &C)
{
    Cx<T> v = prolong_pt<T, DIM>(e, i, j, k, C.nx, C.ny, C.nz);
    if (xin) v = v + xin[p];
    return v;
}

template <typename T, int DIM>
__global__ __launch_bounds__(BLK) void k_prc(LvlK<T> F, LvlK<T> C, const Cx<T> *ec, const Cx<T> *xin, Cx<T> *xout,
                                             const Cx<T> *__restrict__ b, Cx<T> *__restrict__ r, size_t ldf,
                                             size_t ldc, unsigned chunk, int nb, const int *active)
{
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const size_t off = rhs * ldf;
    const Cx<T> *e = ec + rhs * ldc;
    const Cx<T> *xi = xin ? xin + off : nullptr;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(F.N, p0 + chunk);
    for (unsigned p = p0 + threadIdx.x; p < p1; p += BLK) {
        unsigned i, j, k;
        decomp<DIM>(p, F.nx, F.ny, i, j, k);
        const Cx<T> *tx = F.tab[0];
        Cx<T> d = tx[F.nx + i];
        if (DIM >= 2) d = d + F.tab[1][F.ny + j];
        if (DIM == 3) d = d + F.tab[2][F.nz + k];
        d.re -= F.phi[p];
        const Cx<T> xc = corrected<T, DIM>(xi, e, i, j, k, p, C);
        Cx<T> acc = d * xc;
        if (i) acc = cfma(tx[i], corrected<T, DIM>(xi, e, i - 1, j, k, p - 1, C), acc);
        if (i + 1 < F.nx) acc = cfma(tx[2 * F.nx + i], corrected<T, DIM>(xi, e, i + 1, j, k, p + 1, C), acc);
        if (DIM >= 2) {
            const Cx<T> *ty = F.tab[1];
            if (j) acc = cfma(ty[j], corrected<T, DIM>(xi, e, i, j - 1, k, p - F.nx, C), acc);
            if (j + 1 < F.ny) acc = cfma(ty[2 * F.ny + j], corrected<T, DIM>(xi, e, i, j + 1, k, p + F.nx, C), acc);
        }
        if (DIM == 3) {
            const Cx<T> *tz = F.tab[2];
            const unsigned sz = F.nx * F.ny;
            if (k) acc = cfma(tz[k], corrected<T, DIM>(xi, e, i, j, k - 1, p - sz, C), acc);
            if (k + 1 < F.nz) acc = cfma(tz[2 * F.nz + k], corrected<T, DIM>(xi, e, i, j, k + 1, p + sz, C), acc);
        }
        xout[off + p] = xc;
        r[off + p] = b[off + p] - acc;
    }
}

// x = M_L^{-1} b with the transposed dense inverse (column c contiguous).
template <typename T>
__global__ __launch_bounds__(BLK) void k_coarse(const Cx<T> *__restrict__ minvT, int n, const Cx<T> *__restrict__ b,
                                                Cx<T> *__restrict__ x, size_t ld, const int *active)
{
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const Cx<T> *bb = b + rhs * ld;
    for (int i = blockIdx.x * BLK + threadIdx.x; i < n; i += gridDim.x * BLK) {
        Cx<T> acc = mkc<T>(0, 0);
        for (int c = 0; c < n; ++c) acc = cfma(minvT[(size_t)c * n + i], bb[c], acc);
        x[rhs * ld + i] = acc;
    }
}

// ---------------------------------------------------------------------------
// outer flexible GMRES passes (FP64)
// ---------------------------------------------------------------------------

template <int JB>
__device__ __forceinline__ void store_parts(zc (&acc)[JB], int nv, zc *pout, int rhs, unsigned c, zc *sh, zc *res)
{
    block_sum<JB>(acc, nv, sh, res);
    for (int q = threadIdx.x; q < nv; q += BLK) pout[((size_t)rhs * OVAL + q) * NBMAX + c] = res[q];
}

// w = H z and the first-round inner products <v_i, w>, i <= j.
template <typename TZ, int DIM, int JB>
__global__ __launch_bounds__(BLK) void k_hst(LvlK<double> H, const Cx<TZ> *__restrict__ z, zc *__restrict__ w,
                                             const zc *__restrict__ V, size_t vstride, int j, size_t ld,
                                             zc *__restrict__ pout, unsigned chunk, int nb, const int *active)
{
    __shared__ zc sh[4 * JB];
    __shared__ zc res[JB];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const size_t off = rhs * ld;
    zc acc[JB];
#pragma unroll
    for (int q = 0; q < JB; ++q) acc[q] = mkc(0.0, 0.0);
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(H.N, p0 + chunk);
    for (unsigned p = p0 + threadIdx.x; p < p1; p += BLK) {
        unsigned i, jj, k;
        decomp<DIM>(p, H.nx, H.ny, i, jj, k);
        const zc wv = apply_pt<double, DIM>(H, z + off, i, jj, k, p);
        w[off + p] = wv;
#pragma unroll
        for (int q = 0; q < JB; ++q)
            if (q <= j) acc[q] = cjfma(V[q * vstride + off + p], wv, acc[q]);
    }
    store_parts<JB>(acc, j + 1, pout, rhs, c, sh, res);
}

// w -= sum_i h_i v_i, then the second-round inner products <v_i, w>.
template <int JB>
__global__ __launch_bounds__(BLK) void k_cgs1(zc *__restrict__ w, const zc *__restrict__ V, size_t vstride, int j,
                                              unsigned N, size_t ld, const FState *fsb, zc *__restrict__ pout,
                                              unsigned chunk, int nb, const int *active)
{
    __shared__ zc sh[4 * JB];
    __shared__ zc res[JB];
    __shared__ zc hh[JB];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    if (threadIdx.x <= j) hh[threadIdx.x] = fsb[rhs].hcol[threadIdx.x];
    __syncthreads();
    const size_t off = rhs * ld;
    zc acc[JB];
#pragma unroll
    for (int q = 0; q < JB; ++q) acc[q] = mkc(0.0, 0.0);
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(N, p0 + chunk);
    for (unsigned p = p0 + threadIdx.x; p < p1; p += BLK) {
        zc vv[JB];
        zc x = w[off + p];
#pragma unroll
        for (int q = 0; q < JB; ++q)
            if (q <= j) {
                vv[q] = V[q * vstride + off + p];
                x = x - hh[q] * vv[q];
            }
        w[off + p] = x;
#pragma unroll
        for (int q = 0; q < JB; ++q)
            if (q <= j) acc[q] = cjfma(vv[q], x, acc[q]);
    }
    store_parts<JB>(acc, j + 1, pout, rhs, c, sh, res);
}

// w -= sum_i c_i v_i (second round) and the partial ||w||^2.
__global__ __launch_bounds__(BLK) void k_cgs2(zc *__restrict__ w, const zc *__restrict__ V, size_t vstride, int j,
                                              unsigned N, size_t ld, const FState *fsb, zc *__restrict__ pout,
                                              unsigned chunk, int nb, const int *active)
{
    __shared__ zc sh[4];
    __shared__ zc res[1];
    __shared__ zc cc[OVAL];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    if (threadIdx.x <= j) cc[threadIdx.x] = fsb[rhs].corr[threadIdx.x];
    __syncthreads();
    const size_t off = rhs * ld;
    zc acc[1] = {mkc(0.0, 0.0)};
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(N, p0 + chunk);
    for (unsigned p = p0 + threadIdx.x; p < p1; p += BLK) {
        zc x = w[off + p];
        for (int q = 0; q <= j; ++q) x = x - cc[q] * V[q * vstride + off + p];
        w[off + p] = x;
        acc[0].re += cabs2(x);
    }
    block_sum<1>(acc, 1, sh, res);
    if (threadIdx.x == 0) pout[((size_t)rhs * OVAL) * NBMAX + c] = res[0];
}

// v = w / h (scale from the FGMRES state), optional cycle-precision copy.
template <typename TB>
__global__ __launch_bounds__(BLK) void k_vnorm(const zc *w, zc *v, Cx<TB> *__restrict__ bc,
                                               unsigned N, size_t ld, const FState *fsb, unsigned chunk, int nb,
                                               const int *active)
{
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const double sc = fsb[rhs].inv_hn;
    const size_t off = rhs * ld;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(N, p0 + chunk);
    for (unsigned p = p0 + threadIdx.x; p < p1; p += BLK) {
        const zc x = sc * w[off + p];
        v[off + p] = x;
        if (bc) bc[off + p] = cvt<TB>(x);
    }
}

// r = chi - H u, partial ||r||^2 (value 0) and ||chi||^2 (value 1).
template <int DIM>
__global__ __launch_bounds__(BLK) void k_tres(LvlK<double> H, const zc *__restrict__ chi, const zc *__restrict__ u,
                                              zc *__restrict__ r, size_t ld, int with_chi, zc *__restrict__ pout,
                                              unsigned chunk, int nb, const int *active)
{
    __shared__ zc sh[8];
    __shared__ zc res[2];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const size_t off = rhs * ld;
    zc acc[2] = {mkc(0.0, 0.0), mkc(0.0, 0.0)};
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(H.N, p0 + chunk);
    for (unsigned p = p0 + threadIdx.x; p < p1; p += BLK) {
        unsigned i, j, k;
        decomp<DIM>(p, H.nx, H.ny, i, j, k);
        const zc ch = chi[off + p];
        const zc x = ch - apply_pt<double, DIM>(H, u + off, i, j, k, p);
        r[off + p] = x;
        acc[0].re += cabs2(x);
        acc[1].re += cabs2(ch);
    }
    const int nv = with_chi ? 2 : 1;
    block_sum<2>(acc, nv, sh, res);
    if (threadIdx.x < nv) pout[((size_t)rhs * OVAL + threadIdx.x) * NBMAX + c] = res[threadIdx.x];
}

// u += sum_{i < kcols} y_i z_i
template <typename TZ>
__global__ __launch_bounds__(BLK) void k_uupd(zc *__restrict__ u, const Cx<TZ> *__restrict__ Z, size_t zstride,
                                              unsigned N, size_t ld, const FState *fsb, unsigned chunk, int nb,
                                              const int *active)
{
    __shared__ zc yy[CSG_MAX_RESTART];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const int kc = fsb[rhs].kcols;
    if (threadIdx.x < kc) yy[threadIdx.x] = fsb[rhs].y[threadIdx.x];
    __syncthreads();
    const size_t off = rhs * ld;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(N, p0 + chunk);
    for (unsigned p = p0 + threadIdx.x; p < p1; p += BLK) {
        zc x = u[off + p];
        for (int q = 0; q < kc; ++q) x = cfma(yy[q], cvt<double>(Z[q * zstride + off + p]), x);
        u[off + p] = x;
    }
}

// One block per RHS: finish an outer reduction and advance the small FGMRES
// state (Hessenberg column, Givens rotations, residual estimate, LS solve).
__global__ __launch_bounds__(BLK) void k_fin(int mode, const zc *__restrict__ pin, int nbin, int j, FState *fsb,
                                             Report *rep, const int *active)
{
    __shared__ zc sh[4];
    __shared__ zc res[1];
    const int rhs = blockIdx.x;
    if (!active[rhs]) return;
    FState *fs = fsb + rhs;
    const zc *pp = pin + (size_t)rhs * OVAL * NBMAX;
    if (mode == FIN_H || mode == FIN_C) {
        for (int q = 0; q <= j; ++q) {
            reduce_parts<1>(pp + q * NBMAX, nbin, 1, sh, res);
            if (threadIdx.x == 0) {
                if (mode == FIN_H) {
                    fs->hcol[q] = res[0];
                } else {
                    fs->corr[q] = res[0];
                    fs->hcol[q] = fs->hcol[q] + res[0];
                }
            }
        }
        return;
    }
    if (mode == FIN_LS) {
        if (threadIdx.x == 0) {
            const int k = fs->kcols;
            for (int i = k - 1; i >= 0; --i) {
                zc acc = fs->g[i];
                for (int c = i + 1; c < k; ++c) acc = acc - fs->R[i * CSG_MAX_RESTART + c] * fs->y[c];
                const zc d = fs->R[i * CSG_MAX_RESTART + i];
                fs->y[i] = (1.0 / cabs2(d)) * (acc * mkc(d.re, -d.im));
            }
        }
        return;
    }
    double nchi2 = 0.0;
    if (mode == FIN_BEGIN) {
        reduce_parts<1>(pp + NBMAX, nbin, 1, sh, res);
        nchi2 = res[0].re;
    }
    reduce_parts<1>(pp, nbin, 1, sh, res);
    if (threadIdx.x != 0) return;
    if (mode == FIN_N) {
        const double hn = sqrt(res[0].re);
        const int m = CSG_MAX_RESTART;
        for (int q = 0; q <= j; ++q) fs->R[q * m + j] = fs->hcol[q];
        fs->R[(j + 1) * m + j] = mkc(hn, 0.0);
        for (int q = 0; q < j; ++q) {
            const zc t1 = fs->R[q * m + j], t2 = fs->R[(q + 1) * m + j];
            fs->R[q * m + j] = fs->cs[q] * t1 + fs->sn[q] * t2;
            fs->R[(q + 1) * m + j] = fs->cs[q] * t2 - mkc(fs->sn[q].re, -fs->sn[q].im) * t1;
        }
        double cs;
        zc sn;
        rot(fs->R[j * m + j], fs->R[(j + 1) * m + j], cs, sn);
        fs->cs[j] = cs;
        fs->sn[j] = sn;
        const zc t1 = fs->R[j * m + j], t2 = fs->R[(j + 1) * m + j];
        fs->R[j * m + j] = cs * t1 + sn * t2;
        fs->R[(j + 1) * m + j] = mkc(0.0, 0.0);
        const zc gj = fs->g[j];
        fs->g[j + 1] = mkc(0.0, 0.0) - mkc(sn.re, -sn.im) * gj;
        fs->g[j] = cs * gj;
        fs->hn = hn;
        fs->inv_hn = hn > 0.0 ? 1.0 / hn : 0.0;
        fs->kcols = j + 1;
        const double est = sqrt(cabs2(fs->g[j + 1])) / fs->nchi;
        rep[rhs].est = est;
        rep[rhs].hn = hn;
        rep[rhs].finite = isfinite(est) && isfinite(hn);
        return;
    }
    // FIN_BEGIN / FIN_BETA: start of a restart cycle
    const double beta = sqrt(res[0].re);
    if (mode == FIN_BEGIN) fs->nchi = sqrt(nchi2);
    fs->beta = beta;
    for (int q = 0; q <= CSG_MAX_RESTART; ++q) fs->g[q] = mkc(0.0, 0.0);
    fs->g[0] = mkc(beta, 0.0);
    fs->inv_hn = beta > 0.0 ? 1.0 / beta : 0.0;
    fs->kcols = 0;
    const double est = fs->nchi > 0.0 ? beta / fs->nchi : 0.0;
    rep[rhs].est = est;
    rep[rhs].hn = fs->nchi;
    rep[rhs].finite = isfinite(est) && isfinite(fs->nchi);
}

__global__ void k_copy_mask(const int *src, int *dst, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline dim3 grid(const Launch &g) { return dim3(g.nb, g.nrhs); }

template <typename T, int DIM>
void launch_apply(const LvlK<T> &L, const void *x, void *y, size_t ld, const Launch &g, const int *active)
{
    hipLaunchKernelGGL((k_apply<T, DIM>), grid(g), dim3(BLK), 0, g.st, L, (const Cx<T> *)x, (Cx<T> *)y, ld, g.chunk,
                       g.nb, active);
}

template <typename T, int DIM>
void launch_st(const LvlK<T> &L, const Basis<T> &B, int j, size_t ld, const zc *pin, int nbin, zc *pout, GState *gs,
               double tiny, const Launch &g, const int *active)
{
    hipLaunchKernelGGL((k_st<T, DIM>), grid(g), dim3(BLK), 0, g.st, L, B, j, ld, pin, nbin, pout, gs, tiny, g.chunk,
                       g.nb, active);
}

template <typename T>
void launch_orth(const Basis<T> &B, int j, int s, unsigned N, size_t ld, const zc *pin, int nbin, zc *pout,
                 GState *gs, const Launch &g, const int *active)
{
    hipLaunchKernelGGL((k_orth<T>), grid(g), dim3(BLK), 0, g.st, B, j, N, ld, pin, nbin, pout, gs, g.chunk, g.nb, s,
                       active);
}

template <typename T>
void launch_upd(Cx<T> *x, int accumulate, const Basis<T> &B, int s, unsigned N, size_t ld, const zc *pin, int nbin,
                GState *gs, double tiny, const Launch &g, const int *active)
{
    hipLaunchKernelGGL((k_upd<T>), grid(g), dim3(BLK), 0, g.st, x, accumulate, B, s, N, ld, pin, nbin, gs, tiny,
                       g.chunk, g.nb, active);
}

template <typename T, int DIM>
void launch_upd_res(Cx<T> *x, int accumulate, const Basis<T> &B, int s, const LvlK<T> &F, const LvlK<T> &C,
                    Cx<T> *bc, size_t ldf, size_t ldc, const zc *pin, int nbin, GState *gs, double tiny,
                    const Launch &gc, const int *active)
{
    hipLaunchKernelGGL((k_upd_res<T, DIM>), grid(gc), dim3(BLK), 0, gc.st, x, accumulate, B, s, F, C, bc, ldf, ldc,
                       pin, nbin, gs, tiny, gc.chunk, gc.nb, active);
}

template <typename T, int DIM>
void launch_resid(const LvlK<T> &L, const Cx<T> *x, const Cx<T> *b, Cx<T> *r, size_t ld, const Launch &g,
                  const int *active)
{
    hipLaunchKernelGGL((k_resid<T, DIM>), grid(g), dim3(BLK), 0, g.st, L, x, b, r, ld, g.chunk, g.nb, active);
}

template <typename T, int DIM>
void launch_restrict(const LvlK<T> &F, const LvlK<T> &C, const Cx<T> *x, const Cx<T> *b, Cx<T> *bc, size_t ldf,
                     size_t ldc, const Launch &gc, const int *active)
{
    hipLaunchKernelGGL((k_restrict<T, DIM>), grid(gc), dim3(BLK), 0, gc.st, F, C, x, b, bc, ldf, ldc, gc.chunk,
                       gc.nb, active);
}

template <typename T, int DIM>
void launch_prolong(const LvlK<T> &F, const LvlK<T> &C, const Cx<T> *ec, const Cx<T> *xin, Cx<T> *xout, size_t ldf,
                    size_t ldc, const Launch &g, const int *active)
{
    hipLaunchKernelGGL((k_prolong<T, DIM>), grid(g), dim3(BLK), 0, g.st, F, C, ec, xin, xout, ldf, ldc, g.chunk,
                       g.nb, active);
}

template <typename T, int DIM>
void launch_prc(const LvlK<T> &F, const LvlK<T> &C, const Cx<T> *ec, const Cx<T> *xin, Cx<T> *xout, const Cx<T> *b,
                Cx<T> *r, size_t ldf, size_t ldc, const Launch &g, const int *active)
{
    hipLaunchKernelGGL((k_prc<T, DIM>), grid(g), dim3(BLK), 0, g.st, F, C, ec, xin, xout, b, r, ldf, ldc, g.chunk,
                       g.nb, active);
}

template <typename T>
void launch_coarse(const Cx<T> *minvT, int n, const Cx<T> *b, Cx<T> *x, size_t ld, int nrhs, hipStream_t st,
                   const int *active)
{
    const int nbx = (n + BLK - 1) / BLK;
    hipLaunchKernelGGL((k_coarse<T>), dim3(nbx, nrhs), dim3(BLK), 0, st, minvT, n, b, x, ld, active);
}

template <typename TZ, int DIM>
void launch_hst(const LvlK<double> &H, const Cx<TZ> *z, zc *w, const zc *V, size_t vstride, int j, size_t ld,
                zc *pout, const Launch &g, const int *active)
{
    if (j < 8)
        hipLaunchKernelGGL((k_hst<TZ, DIM, 8>), grid(g), dim3(BLK), 0, g.st, H, z, w, V, vstride, j, ld, pout, g.chunk,
                           g.nb, active);
    else if (j < 16)
        hipLaunchKernelGGL((k_hst<TZ, DIM, 16>), grid(g), dim3(BLK), 0, g.st, H, z, w, V, vstride, j, ld, pout,
                           g.chunk, g.nb, active);
    else if (j < 32)
        hipLaunchKernelGGL((k_hst<TZ, DIM, 32>), grid(g), dim3(BLK), 0, g.st, H, z, w, V, vstride, j, ld, pout,
                           g.chunk, g.nb, active);
    else
        hipLaunchKernelGGL((k_hst<TZ, DIM, 64>), grid(g), dim3(BLK), 0, g.st, H, z, w, V, vstride, j, ld, pout,
                           g.chunk, g.nb, active);
}

void launch_cgs1(zc *w, const zc *V, size_t vstride, int j, unsigned N, size_t ld, const FState *fs, zc *pout,
                 const Launch &g, const int *active)
{
    if (j < 8)
        hipLaunchKernelGGL((k_cgs1<8>), grid(g), dim3(BLK), 0, g.st, w, V, vstride, j, N, ld, fs, pout, g.chunk, g.nb,
                           active);
    else if (j < 16)
        hipLaunchKernelGGL((k_cgs1<16>), grid(g), dim3(BLK), 0, g.st, w, V, vstride, j, N, ld, fs, pout, g.chunk,
                           g.nb, active);
    else if (j < 32)
        hipLaunchKernelGGL((k_cgs1<32>), grid(g), dim3(BLK), 0, g.st, w, V, vstride, j, N, ld, fs, pout, g.chunk,
                           g.nb, active);
    else
        hipLaunchKernelGGL((k_cgs1<64>), grid(g), dim3(BLK), 0, g.st, w, V, vstride, j, N, ld, fs, pout, g.chunk,
                           g.nb, active);
}

void launch_cgs2(zc *w, const zc *V, size_t vstride, int j, unsigned N, size_t ld, const FState *fs, zc *pout,
                 const Launch &g, const int *active)
{
    hipLaunchKernelGGL(k_cgs2, grid(g), dim3(BLK), 0, g.st, w, V, vstride, j, N, ld, fs, pout, g.chunk, g.nb, active);
}

template <typename TB>
void launch_vnorm(const zc *w, zc *v, Cx<TB> *bcast, unsigned N, size_t ld, const FState *fs, const Launch &g,
                  const int *active)
{
    hipLaunchKernelGGL((k_vnorm<TB>), grid(g), dim3(BLK), 0, g.st, w, v, bcast, N, ld, fs, g.chunk, g.nb, active);
}

template <int DIM>
void launch_tres(const LvlK<double> &H, const zc *chi, const zc *u, zc *r, size_t ld, int with_chi, zc *pout,
                 const Launch &g, const int *active)
{
    hipLaunchKernelGGL((k_tres<DIM>), grid(g), dim3(BLK), 0, g.st, H, chi, u, r, ld, with_chi, pout, g.chunk, g.nb,
                       active);
}

template <typename TZ>
void launch_uupd(zc *u, const Cx<TZ> *Z, size_t zstride, unsigned N, size_t ld, const FState *fs, const Launch &g,
                 const int *active)
{
    hipLaunchKernelGGL((k_uupd<TZ>), grid(g), dim3(BLK), 0, g.st, u, Z, zstride, N, ld, fs, g.chunk, g.nb, active);
}

void launch_fin(int mode, const zc *pin, int nbin, int j, FState *fs, Report *rep, int nrhs, hipStream_t st,
                const int *active)
{
    hipLaunchKernelGGL(k_fin, dim3(nrhs), dim3(BLK), 0, st, mode, pin, nbin, j, fs, rep, active);
}

void launch_copy_mask(const int *src, int *dst, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy_mask, dim3((n + 255) / 256), dim3(256), 0, st, src, dst, n);
}

// ---------------------------------------------------------------------------
// explicit instantiations
// ---------------------------------------------------------------------------

#define INST_TD(T, D)                                                                                               \
    template void launch_apply<T, D>(const LvlK<T> &, const void *, void *, size_t, const Launch &, const int *);  \
    template void launch_st<T, D>(const LvlK<T> &, const Basis<T> &, int, size_t, const zc *, int, zc *, GState *, \
                                  double, const Launch &, const int *);                                            \
    template void launch_upd_res<T, D>(Cx<T> *, int, const Basis<T> &, int, const LvlK<T> &, const LvlK<T> &,      \
                                       Cx<T> *, size_t, size_t, const zc *, int, GState *, double, const Launch &, \
                                       const int *);                                                               \
    template void launch_resid<T, D>(const LvlK<T> &, const Cx<T> *, const Cx<T> *, Cx<T> *, size_t,               \
                                     const Launch &, const int *);                                                 \
    template void launch_restrict<T, D>(const LvlK<T> &, const LvlK<T> &, const Cx<T> *, const Cx<T> *, Cx<T> *,   \
                                        size_t, size_t, const Launch &, const int *);                              \
    template void launch_prolong<T, D>(const LvlK<T> &, const LvlK<T> &, const Cx<T> *, const Cx<T> *, Cx<T> *,    \
                                       size_t, size_t, const Launch &, const int *);                               \
    template void launch_prc<T, D>(const LvlK<T> &, const LvlK<T> &, const Cx<T> *, const Cx<T> *, Cx<T> *,        \
                                   const Cx<T> *, Cx<T> *, size_t, size_t, const Launch &, const int *);           \
    template void launch_hst<T, D>(const LvlK<double> &, const Cx<T> *, zc *, const zc *, size_t, int, size_t,     \
                                   zc *, const Launch &, const int *);

INST_TD(double, 2)
INST_TD(double, 3)
INST_TD(float, 2)
INST_TD(float, 3)

#define INST_T(T)                                                                                                  \
    template void launch_orth<T>(const Basis<T> &, int, int, unsigned, size_t, const zc *, int, zc *, GState *,    \
                                 const Launch &, const int *);                                                     \
    template void launch_upd<T>(Cx<T> *, int, const Basis<T> &, int, unsigned, size_t, const zc *, int, GState *, \
                                double, const Launch &, const int *);                                              \
    template void launch_coarse<T>(const Cx<T> *, int, const Cx<T> *, Cx<T> *, size_t, int, hipStream_t,          \
                                   const int *);                                                                   \
    template void launch_vnorm<T>(const zc *, zc *, Cx<T> *, unsigned, size_t, const FState *, const Launch &,     \
                                  const int *);                                                                    \
    template void launch_uupd<T>(zc *, const Cx<T> *, size_t, unsigned, size_t, const FState *, const Launch &,    \
                                 const int *);

INST_T(double)
INST_T(float)

template void launch_tres<2>(const LvlK<double> &, const zc *, const zc *, zc *, size_t, int, zc *, const Launch &,
                             const int *);
template void launch_tres<3>(const LvlK<double> &, const zc *, const zc *, zc *, size_t, int, zc *, const Launch &,
                             const int *);

}  // namespace csg
