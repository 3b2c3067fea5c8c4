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
#include <algorithm>
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

// A scalar zero the compiler cannot see through: added to the index of a
// block-uniform coefficient in shared memory inside a point loop, it keeps
// the coefficient a broadcast read at its point of use instead of a value
// held in vector registers for the whole pass (the first projection's
// coefficients, two per basis vector, would otherwise take 4 registers each
// per lane and lower the kernel's occupancy or spill).
__device__ __forceinline__ int opaque_zero()
{
    int z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    return z;
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

// diagonal d -= s phi_p with the operator's factor s (exactly d.re -= phi_p
// for s = 1)
template <typename T>
__device__ __forceinline__ void sub_phi(Cx<T> &d, const LvlK<T> &K, T ph)
{
    d.re -= (T)K.sre * ph;
    d.im -= (T)K.sim * ph;
}

// (A x)_p for a Galerkin level's stored stencil (neighbours outside the grid
// have coefficient 0; their loads are clamped to p).
template <typename T, int DIM, typename TI>
__device__ __forceinline__ Cx<T> apply_gal(const LvlK<T> &L, const Cx<TI> *__restrict__ x, unsigned i, unsigned j,
                                           unsigned k, unsigned p)
{
    Cx<T> acc = mkc(T(0), T(0));
    const unsigned sz = L.nx * L.ny;
#pragma unroll
    for (int oz = (DIM == 3 ? -1 : 0); oz <= (DIM == 3 ? 1 : 0); ++oz)
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) {
                const int oi = (ox + 1) + 3 * (oy + 1) + (DIM == 3 ? 9 * (oz + 1) : 0);
                const bool in = (ox >= 0 || i > 0) && (ox <= 0 || i + 1 < L.nx) && (oy >= 0 || j > 0) &&
                                (oy <= 0 || j + 1 < L.ny) && (oz >= 0 || k > 0) && (oz <= 0 || k + 1 < L.nz);
                const unsigned q = in ? (unsigned)((int)p + ox + oy * (int)L.nx + oz * (int)sz) : p;
                acc = cfma(L.gst[(size_t)oi * L.N + p], cvt<T>(x[q]), acc);
            }
    return acc;
}

// (A x)_p for the Kronecker-sum operator: per axis west/centre/east weights,
// diagonal minus phi.  Boundary weights are zero in the tables, so the clamped
// neighbour index only keeps the load in range.  Galerkin levels take the
// stored stencil instead.
template <typename T, int DIM, typename TI>
__device__ __forceinline__ Cx<T> apply_pt(const LvlK<T> &L, const Cx<TI> *__restrict__ x, unsigned i, unsigned j,
                                          unsigned k, unsigned p)
{
    if (L.gst) return apply_gal<T, DIM>(L, x, i, j, k, p);
    const Cx<T> *tx = L.tab[0];
    Cx<T> d = tx[L.nx + i];
    if (DIM >= 2) d = d + L.tab[1][L.ny + j];
    if (DIM == 3) d = d + L.tab[2][L.nz + k];
    sub_phi(d, L, L.phi[p]);
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

// One DPP step on a double (both 32-bit halves moved alike; lanes without a
// source or masked off contribute 0).
template <int CTRL, int ROWS, int BANKS, bool BC>
__device__ __forceinline__ double dpp64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, BANKS, BC);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, BANKS, BC);
    return __hiloint2double(hi, lo);
}

// Exchanges of a double between lane pairs of a wavefront.  permlane32/16
// swaps (gfx950) trade the upper half of a with the lower half of b across
// lanes L and L^32 (rows 1, 3 of a with rows 0, 2 of b across L and L^16), so
// a + b afterwards holds, in lanes with that lane bit clear, the pair sum of a
// and in the others the pair sum of b.
__device__ __forceinline__ void swap32(double &a, double &b)
{
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
    a = __hiloint2double(hi[0], lo[0]);
    b = __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ void swap16(double &a, double &b)
{
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
    a = __hiloint2double(hi[0], lo[0]);
    b = __hiloint2double(hi[1], lo[1]);
}

// Partner lanes of the in-row steps: L^15 (row mirror), L^7 (half-row
// mirror), L^2 and L^1 (quad permutations); each differs from L in bit 3, 2,
// 1, 0 respectively and agrees with it on every higher bit.
template <int B>
__device__ __forceinline__ double partner(double v)
{
    constexpr int CTRL = B == 3 ? 0x140 : B == 2 ? 0x141 : B == 1 ? 0x4E : 0xB1;
    return dpp64<CTRL, 0xF, 0xF, false>(v);
}

// One halving step of the reduce-scatter at lane bit B: value k pairs with
// value k + n/2; the lane keeps k when its bit B is clear, k + n/2 otherwise,
// and adds the partner lane's copy of the value it keeps.
template <int B, int N, int ND>
__device__ __forceinline__ void halve(double (&d)[ND])
{
    constexpr int H = N / 2;
    if constexpr (B >= 4) {
#pragma unroll
        for (int k = 0; k < H; ++k) {
            if constexpr (B == 5) swap32(d[k], d[k + H]);
            else swap16(d[k], d[k + H]);
            d[k] = d[k] + d[k + H];
        }
    } else {
        const bool up = (threadIdx.x >> B) & 1;
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const double keep = up ? d[k + H] : d[k], send = up ? d[k] : d[k + H];
            d[k] = keep + partner<B>(send);
        }
    }
}

// Wavefront totals of d[0..ND-1] (ND a power of two, 2..64): a reduce-scatter
// over lane bits 5, 4, ... (log2 ND steps, each exchanging half the values a
// lane holds) and sums over the lower lane bits.  Every lane returns the total
// of value lane >> (6 - log2 ND).  The additions follow a fixed order; the
// cost is at most about 4 VALU operations per value (a scan of one value at a
// time across the wavefront takes 21).
template <int ND>
__device__ __forceinline__ double wave_totals(double (&d)[ND])
{
    static_assert(ND >= 2 && ND <= 64 && (ND & (ND - 1)) == 0, "power of two");
    halve<5, ND>(d);
    if constexpr (ND >= 4) halve<4, ND / 2>(d);
    if constexpr (ND >= 8) halve<3, ND / 4>(d);
    if constexpr (ND >= 16) halve<2, ND / 8>(d);
    if constexpr (ND >= 32) halve<1, ND / 16>(d);
    if constexpr (ND >= 64) halve<0, ND / 32>(d);
    double s = d[0];
    if constexpr (ND < 4) {
        double t = s;
        swap16(s, t);
        s = s + t;
    }
    if constexpr (ND < 8) s = s + partner<3>(s);
    if constexpr (ND < 16) s = s + partner<2>(s);
    if constexpr (ND < 32) s = s + partner<1>(s);
    if constexpr (ND < 64) s = s + partner<0>(s);
    return s;
}

constexpr int pow2_at_least(int n)
{
    int p = 2;
    while (p < n) p *= 2;
    return p;
}

// Wavefront totals of v[0..NV-1] into this wave's row of sh (row layout
// [NV] complex, as re/im doubles): one lane per total writes it.
template <int NV>
__device__ __forceinline__ void wave_totals_to(const zc (&v)[NV], int nv, zc *sh, int wv)
{
    constexpr int ND = pow2_at_least(2 * NV);
    constexpr int SH = ND == 2 ? 5 : ND == 4 ? 4 : ND == 8 ? 3 : ND == 16 ? 2 : ND == 32 ? 1 : 0;
    double d[ND];
#pragma unroll
    for (int q = 0; q < ND / 2; ++q) {
        const bool on = q < NV && q < nv;
        const zc x = v[q < NV ? q : 0];
        d[2 * q] = on ? x.re : 0.0;
        d[2 * q + 1] = on ? x.im : 0.0;
    }
    const double t = wave_totals<ND>(d);
    const int lane = threadIdx.x & 63, idx = lane >> SH;
    if ((lane & ((1 << SH) - 1)) == 0 && idx < 2 * nv) reinterpret_cast<double *>(sh)[wv * 2 * NV + idx] = t;
}

// Wavefront totals, then the BLK/64 wavefronts in order; every thread reads
// the same totals from res.
template <int NV>
__device__ __forceinline__ void block_sum(zc (&v)[NV], int nv, zc *sh, zc *res)
{
    constexpr int NW = BLK / 64;
    wave_totals_to<NV>(v, nv, sh, threadIdx.x >> 6);
    __syncthreads();
    if (threadIdx.x < nv) {
        const int q = threadIdx.x;
        zc a = sh[q];
#pragma unroll
        for (int w = 1; w < NW; ++w) a = a + sh[w * NV + q];
        res[q] = a;
    }
    __syncthreads();
}

// This thread's share of the per-block partials of one RHS (layout
// [value][NBMAX]): partials b and b + BLK of every row, all loaded at once
// (rows >= nv and blocks >= nb are read inside the buffer and dropped), so the
// reduction waits for memory once; the second is added only when present.
template <int NV>
__device__ __forceinline__ void load_parts(const zc *part, int nb, int nv, zc (&v)[NV])
{
    static_assert(NBMAX <= 2 * BLK && NV <= NVAL, "partials layout");
    const int b = (int)threadIdx.x;
    const bool ok = b < nb, ok2 = b + BLK < nb;
    zc v2[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        v[q] = part[q * NBMAX + b];
        v2[q] = part[q * NBMAX + min(b + BLK, NBMAX - 1)];
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        if (ok2) v[q] = v[q] + v2[q];
        if (!(ok && q < nv)) v[q] = mkc(0.0, 0.0);
    }
}

// block_sum at the end of a pass: thread q < nv stores the total it formed
// itself (res[q]), so the closing barrier is left out.
template <int NV>
__device__ __forceinline__ void block_sum_last(zc (&v)[NV], int nv, zc *sh, zc *res)
{
    constexpr int NW = BLK / 64;
    wave_totals_to<NV>(v, nv, sh, threadIdx.x >> 6);
    __syncthreads();
    if (threadIdx.x < nv) {
        const int q = threadIdx.x;
        zc a = sh[q];
#pragma unroll
        for (int w = 1; w < NW; ++w) a = a + sh[w * NV + q];
        res[q] = a;
    }
}

// Sum the per-block partials of one RHS into res[0..nv-1].
template <int NV>
__device__ __forceinline__ void reduce_parts(const zc *part, int nb, int nv, zc *sh, zc *res)
{
    zc v[NV];
    load_parts<NV>(part, nb, nv, v);
    block_sum<NV>(v, nv, sh, res);
}

// Complex Givens rotation [c s; -conj(s) c] (c real) taking (a, b) to (r, 0).
__device__ __forceinline__ void rot(zc a, zc b, double &c, zc &s)
{
    const double a2 = cabs2(a), b2 = cabs2(b), n2 = a2 + b2;
    if (n2 > 1e-280 && n2 < 1e280 && a2 > 0.0) {
        // c = |a| / nu, s = (a / |a|) conj(b) / nu with nu = sqrt(|a|^2 + |b|^2):
        // one division on the dependent chain (squares far from under/overflow)
        const double inv = 1.0 / (sqrt(a2) * sqrt(n2));
        c = a2 * inv;
        s = inv * (a * mkc(b.re, -b.im));
        return;
    }
    const double aa = sqrt(a2), bb = sqrt(b2);
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
// scratch of (CSG_MAX_S+1) * CSG_MAX_S values.  Returns k.  SB - 1 bounds s:
// the loops are unrolled to it so the rotations, g and y stay in registers.
template <int SB>
__device__ int gmres_ls(const GState *gs, int s, double hn_last, zc *R, zc *y, zc *cres)
{
    constexpr int K = SB - 1;
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
    zc g[K + 1], yl[K];
    double cs[K];
    zc sn[K];
#pragma unroll
    for (int i = 0; i <= K; ++i) g[i] = mkc(0.0, 0.0);
    g[0] = mkc(beta0, 0.0);
#pragma unroll
    for (int c = 0; c < K; ++c) {
        if (c >= k) break;
#pragma unroll
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
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
        if (i < k) {
            zc acc = g[i];
#pragma unroll
            for (int c = i + 1; c < K; ++c)
                if (c < k) acc = acc - R[i * CSG_MAX_S + c] * yl[c];
            const zc d = R[i * CSG_MAX_S + i];
            yl[i] = (1.0 / cabs2(d)) * (acc * mkc(d.re, -d.im));
        }
    }
#pragma unroll
    for (int i = 0; i < K; ++i)
        if (i < k) y[i] = yl[i];
#pragma unroll
    for (int i = 0; i <= K; ++i) {
        if (i > k) break;
        zc acc = (i == 0) ? mkc(beta0, 0.0) : mkc(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < K; ++c)
            if (c < k) acc = acc - hget(i, c) * yl[c];
        cres[i] = acc;
    }
    return k;
}

// ---------------------------------------------------------------------------
// pass bodies: one loop over a range of points, shared by the multi-block
// passes (range = one block's chunk) and the single-workgroup coarse tail
// (range = the whole level)
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ Cx<T> *pick(const Basis<T> &B, int j)
{
    Cx<T> *r = B.u[0];
#pragma unroll
    for (int q = 1; q <= CSG_MAX_S; ++q)
        if (q == j) r = B.u[q];
    return r;
}

// B.u[j] = v with a run-time j, written as a select per slot: an indexed
// store would place the whole pointer array in scratch memory, and pointers
// read back from there lose their address space (shared-memory vectors are
// then reached by flat accesses behind scratch loads).
template <typename T>
__device__ __forceinline__ void place(Basis<T> &B, int j, Cx<T> *v)
{
#pragma unroll
    for (int q = 0; q <= CSG_MAX_S; ++q)
        if (q == j) B.u[q] = v;
}

template <typename T, int DIM>
__device__ __forceinline__ void body_apply(const LvlK<T> &L, const Cx<T> *x, Cx<T> *y, unsigned p0, unsigned p1,
                                           unsigned st)
{
    for (unsigned p = p0; p < p1; p += st) {
        unsigned i, j, k;
        decomp<DIM>(p, L.nx, L.ny, i, j, k);
        y[p] = apply_pt<T, DIM>(L, x, i, j, k, p);
    }
}

// Points a thread handles per iteration: their loads are issued together
// (indices clamped to the last point of the range, stores masked), so each
// iteration pays one memory latency for U points.
template <typename T>
struct Ubatch {
    static constexpr int U = sizeof(T) == 8 ? 2 : 4;
};

// h_{s,s-1} of a sweep, two ways.  FP64 cycles take it from the sums of the
// last Arnoldi pass (below) and never form u_s.  complex64 cycles form u_s in
// an explicit last Gram-Schmidt pass and take its norm: with single-pass
// classical Gram-Schmidt on float vectors the basis is orthonormal only to
// float accuracy, too little for the identity when A v_{s-1} nearly lies in the
// basis span (under-resolved coarse levels).
template <typename T>
constexpr bool norm_from_sums() { return sizeof(T) == 8; }

// Arnoldi bookkeeping on the raw (unnormalised) basis u_0..u_s of one sweep,
// v_i = sig_i u_i: pass 0 forms w_0 = A u_0; pass j+1 (j < s-1) forms
// u_{j+1} = sig_j w_j - sum_{i<=j} sig_i h_ij u_i (classical Gram-Schmidt) and,
// in the same sweep over the grid, w_{j+1} = A u_{j+1} with u_{j+1} recomputed at
// the stencil neighbours; the last pass forms u_s only.  Every pass emits the
// partial sums <u_i, w> (i up to its newest vector) and ||newest u||^2.

// pass 0: w = A u_0, acc[0] += <u_0, w>, acc[1] += ||u_0||^2 (and, with NA = 3,
// acc[2] += ||w||^2 for a sweep of one step)
template <typename T, int DIM, int NA = 2>
__device__ __forceinline__ void body_st0(const LvlK<T> &L, const Cx<T> *u0, Cx<T> *w, unsigned p0, unsigned p1,
                                         unsigned st, zc (&acc)[NA])
{
    constexpr int U = Ubatch<T>::U;
    if (p0 >= p1) return;
    const unsigned last = p1 - 1;
    for (unsigned p = p0; p < p1; p += U * st) {
        Cx<T> wv[U], uc[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const unsigned pk = min(p + k * st, last);
            unsigned i, jj, kk;
            decomp<DIM>(pk, L.nx, L.ny, i, jj, kk);
            wv[k] = apply_pt<T, DIM>(L, u0, i, jj, kk, pk);
            uc[k] = u0[pk];
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (p + k * st >= p1) break;
            w[p + k * st] = wv[k];
            const zc wd = cvt<double>(wv[k]), ud = cvt<double>(uc[k]);
            acc[0] = cjfma(ud, wd, acc[0]);
            acc[1].re += cabs2(ud);
            if (NA > 2) acc[NA - 1].re += cabs2(wd);
        }
    }
}

// unfused pass 2j: w_j = A u_j, acc[i] += <u_i, w_j> (i <= j), acc[j+1] += ||u_j||^2,
// and with wn (the last step of a sweep) acc[j+2] += ||w_j||^2
template <typename T, int DIM, int SB>
__device__ __forceinline__ void body_stj(const LvlK<T> &L, const Basis<T> &B, Cx<T> *w, int j, size_t off,
                                         unsigned p0, unsigned p1, unsigned st, zc (&acc)[SB + 1], bool wn)
{
    constexpr int U = Ubatch<T>::U;
    const Cx<T> *uj = pick(B, j) + off;
    Cx<T> *wo = w + off;
    if (p0 >= p1) return;
    const unsigned last = p1 - 1;
    for (unsigned p = p0; p < p1; p += U * st) {
        Cx<T> wv[U], uq[U][SB - 1];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const unsigned pk = min(p + k * st, last);
            unsigned i, jj, kk;
            decomp<DIM>(pk, L.nx, L.ny, i, jj, kk);
            wv[k] = apply_pt<T, DIM>(L, uj, i, jj, kk, pk);
#pragma unroll
            for (int q = 0; q < SB - 1; ++q)
                if (q <= j) uq[k][q] = B.u[q][off + pk];
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (p + k * st >= p1) break;
            wo[p + k * st] = wv[k];
            const zc wd = cvt<double>(wv[k]);
#pragma unroll
            for (int q = 0; q < SB - 1; ++q) {
                if (q <= j) acc[q] = cjfma(cvt<double>(uq[k][q]), wd, acc[q]);
                if (q == j) acc[q + 1].re += cabs2(cvt<double>(uq[k][q]));
                if (q == j && wn) acc[q + 2].re += cabs2(wd);
            }
        }
    }
}

// u_{j+1}(q) = sj w_j(q) - sum_{i<=j} cu_i u_i(q)
template <typename T, int SB>
__device__ __forceinline__ Cx<T> next_u(const Basis<T> &B, const Cx<T> *win, int j, T sj, const Cx<T> (&cu)[SB],
                                        size_t off, unsigned q)
{
    Cx<T> v = sj * win[q];
#pragma unroll
    for (int i = 0; i < SB - 1; ++i)
        if (i <= j) v = v - cu[i] * B.u[i][off + q];
    return v;
}

// pass j+1: u_{j+1} (written to B.u[j+1]), w_{j+1} = A u_{j+1} (written to wout),
// acc[i] += <u_i, w_{j+1}> for i <= j+1, acc[j+2] += ||u_{j+1}||^2
// (with wn, the last step of a sweep: acc[j+3] += ||w_{j+1}||^2; NA >= SB + 1)
template <typename T, int DIM, int SB, int NA>
__device__ __forceinline__ void body_os(const LvlK<T> &L, const Basis<T> &B, const Cx<T> *win, Cx<T> *wout, int j,
                                        T sj, const Cx<T> (&cu)[SB], size_t off, unsigned p0, unsigned p1,
                                        unsigned st, zc (&acc)[NA], bool wn)
{
    Cx<T> *un = pick(B, j + 1) + off;
    const Cx<T> *wi = win + off;
    Cx<T> *wo = wout + off;
    for (unsigned p = p0; p < p1; p += st) {
        unsigned i, jj, k;
        decomp<DIM>(p, L.nx, L.ny, i, jj, k);
        Cx<T> uq[SB - 1];
        Cx<T> uc = sj * wi[p];
#pragma unroll
        for (int q = 0; q < SB - 1; ++q)
            if (q <= j) {
                uq[q] = B.u[q][off + p];
                uc = uc - cu[q] * uq[q];
            }
        const Cx<T> *tx = L.tab[0];
        Cx<T> d = tx[L.nx + i];
        if (DIM >= 2) d = d + L.tab[1][L.ny + jj];
        if (DIM == 3) d = d + L.tab[2][L.nz + k];
        sub_phi(d, L, L.phi[p]);
        Cx<T> a = d * uc;
        if (i) a = cfma(tx[i], next_u<T, SB>(B, wi, j, sj, cu, off, p - 1), a);
        if (i + 1 < L.nx) a = cfma(tx[2 * L.nx + i], next_u<T, SB>(B, wi, j, sj, cu, off, p + 1), a);
        if (DIM >= 2) {
            const Cx<T> *ty = L.tab[1];
            if (jj) a = cfma(ty[jj], next_u<T, SB>(B, wi, j, sj, cu, off, p - L.nx), a);
            if (jj + 1 < L.ny) a = cfma(ty[2 * L.ny + jj], next_u<T, SB>(B, wi, j, sj, cu, off, p + L.nx), a);
        }
        if (DIM == 3) {
            const Cx<T> *tz = L.tab[2];
            const unsigned sz = L.nx * L.ny;
            if (k) a = cfma(tz[k], next_u<T, SB>(B, wi, j, sj, cu, off, p - sz), a);
            if (k + 1 < L.nz) a = cfma(tz[2 * L.nz + k], next_u<T, SB>(B, wi, j, sj, cu, off, p + sz), a);
        }
        un[p] = uc;
        wo[p] = a;
        const zc wd = cvt<double>(a), ud = cvt<double>(uc);
#pragma unroll
        for (int q = 0; q < SB - 1; ++q)
            if (q <= j) acc[q] = cjfma(cvt<double>(uq[q]), wd, acc[q]);
#pragma unroll
        for (int q = 1; q < SB; ++q) {
            if (q == j + 1) acc[q] = cjfma(ud, wd, acc[q]);
            if (q == j + 2) acc[q].re += cabs2(ud);
        }
        if (wn) {
#pragma unroll
            for (int q = 3; q < NA; ++q)
                if (q == j + 3) acc[q].re += cabs2(wd);
        }
    }
}

// last pass: u_s = sj w - sum_i cu_i u_i into B.u[j+1], nrm += ||u_s||^2
template <typename T, int SB>
__device__ __forceinline__ void body_orthl(const Basis<T> &B, const Cx<T> *win, int j, T sj, const Cx<T> (&cu)[SB],
                                           size_t off, unsigned p0, unsigned p1, unsigned st, double &nrm)
{
    constexpr int U = Ubatch<T>::U;
    Cx<T> *un = pick(B, j + 1) + off;
    if (p0 >= p1) return;
    const unsigned last = p1 - 1;
    for (unsigned p = p0; p < p1; p += U * st) {
        Cx<T> v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = next_u<T, SB>(B, win, j, sj, cu, off, min(p + k * st, last));
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (p + k * st >= p1) break;
            un[p + k * st] = v[k];
            nrm += cabs2(cvt<double>(v[k]));
        }
    }
}

// x (+)= sum_{i<k} cx_i u_i
template <typename T, int SB>
__device__ __forceinline__ void body_upd(Cx<T> *x, int accumulate, const Basis<T> &B, int k,
                                         const Cx<T> (&cx)[SB], size_t off, unsigned p0, unsigned p1,
                                         unsigned st)
{
    constexpr int U = Ubatch<T>::U;
    if (p0 >= p1) return;
    const unsigned last = p1 - 1;
    for (unsigned p = p0; p < p1; p += U * st) {
        Cx<T> v[U];
#pragma unroll
        for (int kk = 0; kk < U; ++kk) {
            const unsigned pk = min(p + kk * st, last);
            v[kk] = accumulate ? x[pk] : mkc<T>(0, 0);
#pragma unroll
            for (int q = 0; q < SB - 1; ++q)
                if (q < k) v[kk] = cfma(cx[q], B.u[q][off + pk], v[kk]);
        }
#pragma unroll
        for (int kk = 0; kk < U; ++kk) {
            if (p + kk * st >= p1) break;
            x[p + kk * st] = v[kk];
        }
    }
}

// x (+)= sum_{i<k} cx_i u_i and r = sum_{i<=k} cr_i u_i (the Arnoldi residual
// of the sweep), pointwise on the fine grid
template <typename T, int SB>
__device__ __forceinline__ void body_upd_r(Cx<T> *x, int accumulate, Cx<T> *r, const Basis<T> &B, int k,
                                           const Cx<T> (&cx)[SB], const Cx<T> (&cr)[SB], size_t off, unsigned p0,
                                           unsigned p1, unsigned st)
{
    constexpr int U = Ubatch<T>::U;
    if (p0 >= p1) return;
    const unsigned last = p1 - 1;
    for (unsigned p = p0; p < p1; p += U * st) {
        Cx<T> v[U], rr[U];
#pragma unroll
        for (int kk = 0; kk < U; ++kk) {
            const unsigned pk = min(p + kk * st, last);
            v[kk] = accumulate ? x[pk] : mkc<T>(0, 0);
            rr[kk] = mkc<T>(0, 0);
#pragma unroll
            for (int q = 0; q < SB; ++q)
                if (q <= k) {
                    const Cx<T> u = B.u[q][off + pk];
                    rr[kk] = cfma(cr[q], u, rr[kk]);
                    if (q < k) v[kk] = cfma(cx[q], u, v[kk]);
                }
        }
#pragma unroll
        for (int kk = 0; kk < U; ++kk) {
            if (p + kk * st >= p1) break;
            x[p + kk * st] = v[kk];
            r[p + kk * st] = rr[kk];
        }
    }
}

// --- per-axis index helpers for the transfers -------------------------------
// Fine unknown i (node f = i+1) interpolates from coarse node f/2 (f even,
// weight 1) or nodes (f-1)/2 and (f+1)/2 (f odd, weight 1/2); coarse node c is
// an unknown (index c-1) when 1 <= c <= nuc.
struct PAx {
    unsigned idx[2];
    float w[2];
};
// Both candidate coarse nodes always present (indices clamped into range,
// weight 0 for a node that is absent or a Dirichlet end), so the loads of a
// point issue without branches.
__device__ __forceinline__ PAx paxis(unsigned i, unsigned nuc)
{
    PAx a;
    const unsigned f = i + 1, c0 = f >> 1;
    const bool odd = (f & 1u) != 0;
    a.w[0] = (c0 >= 1 && c0 <= nuc) ? (odd ? 0.5f : 1.f) : 0.f;
    a.w[1] = (odd && c0 + 1 <= nuc) ? 0.5f : 0.f;
    a.idx[0] = min(max(c0, 1u), nuc) - 1;
    a.idx[1] = min(c0 + 1, nuc) - 1;
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
            for (int a = 0; a < 2; ++a) acc = acc + (T)(ax.w[a] * ay.w[b]) * ec[ay.idx[b] * ncx + ax.idx[a]];
    } else {
        const PAx ay = paxis(j, ncy), az = paxis(k, ncz);
#pragma unroll
        for (int cz = 0; cz < 2; ++cz)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 2; ++a)
                    acc = acc + (T)(ax.w[a] * ay.w[b] * az.w[cz]) * ec[(az.idx[cz] * ncy + ay.idx[b]) * ncx + ax.idx[a]];
    }
    return acc;
}

// prolong_pt in 2-D split into its loads and its sum, so that the loads of
// several points can be issued before any of them is used.
template <typename T>
struct PLoads2 {
    Cx<T> e[4];
    float w[4];
};
// Coarse node (I, J) is read at ec[(J - oy) * ld + I - ox]: the whole coarse
// level (ox = oy = 0, ld = ncx) or a staged window of it.
template <typename T>
__device__ __forceinline__ void prolong_load2(const Cx<T> *__restrict__ ec, unsigned i, unsigned j, unsigned ncx,
                                              unsigned ncy, PLoads2<T> &pl, unsigned ox = 0, unsigned oy = 0,
                                              unsigned ld = 0)
{
    const PAx ax = paxis(i, ncx), ay = paxis(j, ncy);
    if (ld == 0) ld = ncx;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            pl.e[2 * b + a] = ec[(ay.idx[b] - oy) * ld + ax.idx[a] - ox];
            pl.w[2 * b + a] = ax.w[a] * ay.w[b];
        }
}
template <typename T>
__device__ __forceinline__ Cx<T> prolong_sum2(const PLoads2<T> &pl)
{
    Cx<T> acc = mkc<T>(0, 0);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc = acc + (T)pl.w[k] * pl.e[k];
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

// Closing pass of the last pre-smoothing sweep fused with the restriction, per
// coarse point: x (+)= sum cx_i u_i on the fine points it owns, and
// bc = 2^-d P^T r with the Arnoldi residual r = sum_i cr_i u_i.
template <typename T, int DIM, int SB>
__device__ __forceinline__ void body_upd_res(Cx<T> *xx, int accumulate, const Basis<T> &B, int k,
                                             const Cx<T> (&cx)[SB], const Cx<T> (&cr)[SB],
                                             const LvlK<T> &F, const LvlK<T> &C, Cx<T> *bb, size_t offf,
                                             unsigned p0, unsigned p1, unsigned st)
{
    const T scale = (DIM == 2) ? (T)0.25 : (T)0.125;
    for (unsigned pc = p0; pc < p1; pc += st) {
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
                    Cx<T> uv[SB];
#pragma unroll
                    for (int q = 0; q < SB; ++q)
                        if (q <= k) uv[q] = B.u[q][offf + fp];
                    Cx<T> r = mkc<T>(0, 0);
#pragma unroll
                    for (int q = 0; q < SB; ++q)
                        if (q <= k) r = cfma(cr[q], uv[q], r);
                    T wgt = (T)(rw(qx) * rw(qy));
                    if (DIM == 3) wgt *= (T)rw(qz);
                    acc = acc + wgt * r;
                    const bool own = ((rx.own >> qx) & 1) && ((ry.own >> qy) & 1) && ((rz.own >> qz) & 1);
                    if (own) {
                        Cx<T> v = accumulate ? xx[fp] : mkc<T>(0, 0);
#pragma unroll
                        for (int q = 0; q < SB - 1; ++q)
                            if (q < k) v = cfma(cx[q], uv[q], v);
                        xx[fp] = v;
                    }
                }
        bb[pc] = scale * acc;
    }
}

// r = b - A x
template <typename T, int DIM>
__device__ __forceinline__ void body_resid(const LvlK<T> &L, const Cx<T> *x, const Cx<T> *b, Cx<T> *r, unsigned p0,
                                           unsigned p1, unsigned st)
{
    constexpr int U = Ubatch<T>::U;
    if (p0 >= p1) return;
    const unsigned last = p1 - 1;
    for (unsigned p = p0; p < p1; p += U * st) {
        Cx<T> v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const unsigned pk = min(p + k * st, last);
            unsigned i, j, kk;
            decomp<DIM>(pk, L.nx, L.ny, i, j, kk);
            v[k] = b[pk] - apply_pt<T, DIM>(L, x, i, j, kk, pk);
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (p + k * st >= p1) break;
            r[p + k * st] = v[k];
        }
    }
}

// bc = 2^-d P^T (b - A x)   (x may be null: bc = 2^-d P^T b)
template <typename T, int DIM>
__device__ __forceinline__ void body_restrict(const LvlK<T> &F, const LvlK<T> &C, const Cx<T> *xx, const Cx<T> *b,
                                              Cx<T> *bc, unsigned p0, unsigned p1, unsigned st)
{
    const T scale = (DIM == 2) ? (T)0.25 : (T)0.125;
    for (unsigned pc = p0; pc < p1; pc += st) {
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
                    Cx<T> r = b[fp];
                    if (xx) r = r - apply_pt<T, DIM>(F, xx, fi, fj, fk, fp);
                    T wgt = (T)(rw(qx) * rw(qy));
                    if (DIM == 3) wgt *= (T)rw(qz);
                    acc = acc + wgt * r;
                }
        bc[pc] = scale * acc;
    }
}

// xout = xin + P ec   (xin may be null; xin == xout allowed)
template <typename T, int DIM>
__device__ __forceinline__ void body_prolong(const LvlK<T> &F, const LvlK<T> &C, const Cx<T> *e, const Cx<T> *xin,
                                             Cx<T> *xout, unsigned p0, unsigned p1, unsigned st)
{
    constexpr int U = Ubatch<T>::U;
    if (p0 >= p1) return;
    const unsigned last = p1 - 1;
    for (unsigned p = p0; p < p1; p += U * st) {
        Cx<T> v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const unsigned pk = min(p + k * st, last);
            unsigned i, j, kk;
            decomp<DIM>(pk, F.nx, F.ny, i, j, kk);
            v[k] = prolong_pt<T, DIM>(e, i, j, kk, C.nx, C.ny, C.nz);
            if (xin) v[k] = v[k] + xin[pk];
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (p + k * st >= p1) break;
            xout[p + k * st] = v[k];
        }
    }
}

template <typename T, int DIM>
__device__ __forceinline__ Cx<T> corrected(const Cx<T> *xin, const Cx<T> *e, unsigned i, unsigned j, unsigned k,
                                           unsigned p, const LvlK<T> &C)
{
    Cx<T> v = prolong_pt<T, DIM>(e, i, j, k, C.nx, C.ny, C.nz);
    if (xin) v = v + xin[p];
    return v;
}

// Interpolated correction fused with the residual that opens the next sweep:
// xout = xin + P ec and r = b - A xout (xout at the neighbours recomputed).
template <typename T, int DIM>
__device__ __forceinline__ void prc_pt(const LvlK<T> &F, const LvlK<T> &C, const Cx<T> *e, const Cx<T> *xi,
                                       const Cx<T> *b, unsigned p, Cx<T> &xc, Cx<T> &rr)
{
    unsigned i, j, k;
    decomp<DIM>(p, F.nx, F.ny, i, j, k);
    const Cx<T> *tx = F.tab[0];
    Cx<T> d = tx[F.nx + i];
    if (DIM >= 2) d = d + F.tab[1][F.ny + j];
    if (DIM == 3) d = d + F.tab[2][F.nz + k];
    sub_phi(d, F, F.phi[p]);
    xc = corrected<T, DIM>(xi, e, i, j, k, p, C);
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
    rr = b[p] - acc;
}

template <typename T, int DIM>
__device__ __forceinline__ void body_prc(const LvlK<T> &F, const LvlK<T> &C, const Cx<T> *e, const Cx<T> *xi,
                                         Cx<T> *xout, const Cx<T> *b, Cx<T> *r, unsigned p0, unsigned p1,
                                         unsigned st)
{
    constexpr int U = Ubatch<T>::U;
    if (p0 >= p1) return;
    const unsigned last = p1 - 1;
    for (unsigned p = p0; p < p1; p += U * st) {
        Cx<T> xc[U], rr[U];
#pragma unroll
        for (int k = 0; k < U; ++k) prc_pt<T, DIM>(F, C, e, xi, b, min(p + k * st, last), xc[k], rr[k]);
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (p + k * st >= p1) break;
            xout[p + k * st] = xc[k];
            r[p + k * st] = rr[k];
        }
    }
}

// x = M^{-1} b with the transposed dense inverse (column c contiguous), by NT
// threads: rows in blocks of R = min(n, NT), NT/R column groups per row,
// group sums combined in a fixed order through shared memory `part`.
template <typename T, int NT>
__device__ __forceinline__ void body_coarse(const Cx<T> *minvT, int n, const Cx<T> *b, Cx<T> *x, Cx<T> *part)
{
    const int R = n < NT ? n : NT;
    const int G = NT / R;
    const int t = threadIdx.x;
    for (int r0 = 0; r0 < n; r0 += R) {
        const int row = r0 + t % R, g = t / R;
        Cx<T> acc = mkc<T>(0, 0);
        if (g < G && row < n)
            for (int c = g; c < n; c += G) acc = cfma(minvT[(size_t)c * n + row], b[c], acc);
        if (g < G) part[g * R + t % R] = acc;
        __syncthreads();
        if (t < R && r0 + t < n) {
            Cx<T> s = part[t];
            for (int q = 1; q < G; ++q) s = s + part[q * R + t];
            x[r0 + t] = s;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// scalar logic of a GMRES(s) sweep (Arnoldi coefficients, breakdown, small
// least squares), identical for the multi-block passes and the tail
// ---------------------------------------------------------------------------

// Consumer of the partials of pass j (res[i] = <u_i, w_j> for i <= j,
// res[j+1] = ||u_j||^2): the scale sig_j of u_j (j = 0: beta0 = ||u_0||;
// j > 0: h_{j,j-1} = ||u_j||, with the breakdown test against tiny * beta0),
// h_ij = sig_i sig_j <u_i, w_j>, and the Gram-Schmidt coefficients
// cu_i = sig_i h_ij of u_{j+1}.  Returns sig_j.  `store` publishes the state
// (sig_i for i < j come from the state written by earlier passes).
// State of the earlier passes of a sweep that coef_step reads (beta0, sig_i),
// loaded at kernel entry so the loads overlap the partial-sum reduction.
template <int SB>
struct GPrev {
    double beta0;
    double sig[SB];
};
template <int SB>
__device__ __forceinline__ GPrev<SB> load_prev(const GState *gs, int j)
{
    GPrev<SB> g;
    g.beta0 = gs->beta0;
#pragma unroll
    for (int q = 0; q < SB; ++q) g.sig[q] = q < j ? gs->sig[q] : 0.0;
    return g;
}

template <typename T, int SB>
__device__ __forceinline__ double coef_step(const zc *res, int j, int s, double tiny, const GPrev<SB> &pv, GState *gs,
                                            bool store, Cx<T> (&cu)[SB])
{
    double sig[SB];
    double nrm2 = 0.0;
#pragma unroll
    for (int q = 0; q < SB; ++q)
        if (q == j + 1) nrm2 = res[q].re;
    const double hn = sqrt(nrm2);
    double beta0, sj;
    bool brk = false;
    if (j == 0) {
        beta0 = hn;
        sj = beta0 > 0.0 ? 1.0 / beta0 : 0.0;
    } else {
        beta0 = pv.beta0;
        brk = !(hn > tiny * beta0);
        sj = brk ? 0.0 : 1.0 / hn;
    }
#pragma unroll
    for (int q = 0; q < SB; ++q) {
        if (q < j) sig[q] = pv.sig[q];
        if (q == j) sig[q] = sj;
    }
    zc h[SB];
#pragma unroll
    for (int q = 0; q < SB; ++q) {
        if (q <= j) {
            h[q] = (sig[q] * sj) * res[q];
            cu[q] = cvt<T>(sig[q] * h[q]);
        }
    }
    if (store) {
        if (j == 0) {
            gs->beta0 = beta0;
            gs->k = s;
        } else {
            gs->H[j * CSG_MAX_S + (j - 1)] = mkc(hn, 0.0);
            if (brk && gs->k > j) gs->k = j;
        }
        gs->sig[j] = sj;
#pragma unroll
        for (int q = 0; q < SB; ++q)
            if (q <= j) gs->H[q * CSG_MAX_S + j] = h[q];
    }
    return sj;
}

// ---------------------------------------------------------------------------
// multi-block passes
// ---------------------------------------------------------------------------

template <typename T, int DIM>
__global__ __launch_bounds__(BLK) void k_apply(LvlK<T> L, const Cx<T> *__restrict__ x, Cx<T> *__restrict__ y,
                                               size_t ld, unsigned chunk, int nb, const int *active)
{
    const int rhs = blockIdx.y;
    L = L.at(rhs);
    if (!active[rhs]) return;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(L.N, p0 + chunk);
    body_apply<T, DIM>(L, x + rhs * ld, y + rhs * ld, p0 + threadIdx.x, p1, BLK);
}

// pass 0 of a sweep: w_0 = A u_0 with <u_0, w_0> and ||u_0||^2 (NA = 3: and
// ||w_0||^2, when the sweep has one step)
template <typename T, int DIM, int NA>
__global__ __launch_bounds__(BLK) void k_st0(LvlK<T> L, const Cx<T> *u0, Cx<T> *w, size_t ld, zc *__restrict__ pout,
                                             unsigned chunk, int nb, const int *active)
{
    __shared__ zc sh[(BLK / 64) * NA];
    __shared__ zc res[NA];
    const int rhs = blockIdx.y;
    L = L.at(rhs);
    if (!active[rhs]) return;
    zc acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = mkc(0.0, 0.0);
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(L.N, p0 + chunk);
    body_st0<T, DIM, NA>(L, u0 + rhs * ld, w + rhs * ld, p0 + threadIdx.x, p1, BLK, acc);
    block_sum_last<NA>(acc, NA, sh, res);
    if (threadIdx.x < NA) pout[((size_t)rhs * NVAL + threadIdx.x) * NBMAX + c] = res[threadIdx.x];
}

// unfused pass 2j: w_j = A u_j with <u_i, w_j> (i <= j) and ||u_j||^2
template <typename T, int DIM, int SB>
__global__ __launch_bounds__(BLK) void k_stj(LvlK<T> L, Basis<T> B, Cx<T> *w, int j, int wn, size_t ld,
                                             zc *__restrict__ pout, unsigned chunk, int nb, const int *active)
{
    __shared__ zc sh[(BLK / 64) * (SB + 1)];
    __shared__ zc res[SB + 1];
    const int rhs = blockIdx.y;
    L = L.at(rhs);
    if (!active[rhs]) return;
    zc acc[SB + 1];
#pragma unroll
    for (int q = 0; q <= SB; ++q) acc[q] = mkc(0.0, 0.0);
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(L.N, p0 + chunk);
    body_stj<T, DIM, SB>(L, B, w, j, rhs * ld, p0 + threadIdx.x, p1, BLK, acc, wn != 0);
    const int nv = j + 2 + (wn ? 1 : 0);
    block_sum_last<SB + 1>(acc, nv, sh, res);
    if (threadIdx.x < nv) pout[((size_t)rhs * NVAL + threadIdx.x) * NBMAX + c] = res[threadIdx.x];
}

// pass j+1 (j < s-1): u_{j+1} and w_{j+1} = A u_{j+1} in one sweep of the grid
template <typename T, int DIM, int SB>
__global__ __launch_bounds__(BLK) void k_os(LvlK<T> L, Basis<T> B, const Cx<T> *win, Cx<T> *wout, int j, int s,
                                            size_t ld, const zc *__restrict__ pin, int nbin, zc *__restrict__ pout,
                                            GState *gsb, double tiny, unsigned chunk, int nb, const int *active)
{
    __shared__ zc sh[(BLK / 64) * (SB + 1)];
    __shared__ zc res[SB + 1];
    const int rhs = blockIdx.y;
    L = L.at(rhs);
    if (!active[rhs]) return;
    GState *gs = gsb + rhs;
    const GPrev<SB> pv = load_prev<SB>(gs, j);
    reduce_parts<SB + 1>(pin + (size_t)rhs * NVAL * NBMAX, nbin, j + 2, sh, res);
    Cx<T> cu[SB];
    const double sj = coef_step<T, SB>(res, j, s, tiny, pv, gs, blockIdx.x == 0 && threadIdx.x == 0, cu);
    zc acc[SB + 1];
#pragma unroll
    for (int q = 0; q <= SB; ++q) acc[q] = mkc(0.0, 0.0);
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(L.N, p0 + chunk);
    const bool wn = norm_from_sums<T>() && j + 2 == s;   // last step of the sweep
    body_os<T, DIM, SB, SB + 1>(L, B, win, wout, j, (T)sj, cu, rhs * ld, p0 + threadIdx.x, p1, BLK, acc, wn);
    const int nv = j + 3 + (wn ? 1 : 0);
    block_sum_last<SB + 1>(acc, nv, sh, res);
    if (threadIdx.x < nv) pout[((size_t)rhs * NVAL + threadIdx.x) * NBMAX + c] = res[threadIdx.x];
}

// Fused pass j+1 on one 2-D tile (see launch_os_tile), J = j.  Phase 1: every
// point of the tile and its one-point halo forms u_{j+1} = sj w_j - sum_i cu_i
// u_i (zero outside the level) into shared memory, the tile's own points also
// to global memory, keeping their u_i and phi in registers.  Phase 2: the
// tile's points apply the stencil to the shared copy, write w_{j+1} and sum
// <u_i, w_{j+1}> (i <= j+1), ||u_{j+1}||^2 and, on the last step,
// ||w_{j+1}||^2.  A thread owns the same points in both phases.  The loads of
// the partials go first, then those of the tile's stencil tables (into shared
// memory) and of the first TILE_PRE points, all before the partial-sum
// reduction; phase 1 goes in batches of TILE_PB points per thread whose loads
// are issued together (the address of an absent point clamped to the tile's
// corner), so a batch waits for memory once.
template <typename T, int SB, int J>
__global__ __launch_bounds__(BLK) void k_os_tile(LvlK<T> L, Basis<T> B, const Cx<T> *win, Cx<T> *wout, int s,
                                                 size_t ld, const zc *__restrict__ pin, int nbin,
                                                 zc *__restrict__ pout, GState *gsb, double tiny, TileGeo tg,
                                                 int ntile, const int *active)
{
    static_assert(J + 3 <= SB, "basis and sum slots");
    constexpr int j = J;
    __shared__ zc sh[(BLK / 64) * (SB + 1)];
    __shared__ zc res[SB + 1];
    __shared__ Cx<T> lu[TILE_MAXN];
    __shared__ Cx<T> ltab[6 * TAB_MAXD];   // x lower, diag, upper; y lower, diag, upper
    const int rhs = blockIdx.y;
    L = L.at(rhs);
    // the mask is tested after the prologue's loads are issued (every read
    // below is harmless for a RHS that no longer iterates)
    const int act = active[rhs];
    GState *gs = gsb + rhs;
    const GPrev<SB> pv = load_prev<SB>(gs, j);
    const unsigned t = chunk_id(ntile);
    const unsigned tyi = t / tg.ntx, txi = t - tyi * tg.ntx;
    const int nx = (int)L.nx, ny = (int)L.ny;
    const int x0 = (int)(txi * tg.tx), y0 = (int)(tyi * tg.ty);
    const int TX = min(x0 + (int)tg.tx, nx) - x0, TY = min(y0 + (int)tg.ty, ny) - y0;
    const int HX = TX + 2, HY = TY + 2;
    const int HN = HX * HY;
    const size_t off = rhs * ld;
    const size_t pc = (size_t)y0 * nx + x0;   // a point of the level every clamped address goes to
    const Cx<T> *wi = win + off;
    Cx<T> *un = pick(B, j + 1) + off;
    Cx<T> *wo = wout + off;
    // stencil tables of the tile's columns x0 .. x0+TX-1 and rows y0 .. y0+TY-1,
    // one entry per thread, loaded ahead of the partials (so the reduction's
    // wait covers it) and stored to shared memory after the reduction
    int tslot = -1;
    const Cx<T> *tsrc;
    {
        const int q = threadIdx.x;
        const bool xs = q < 3 * TX;
        const int qq = xs ? q : min(q - 3 * TX, 3 * TY - 1);
        const int c = qq / 3, a = qq - 3 * c;
        tsrc = (xs ? L.tab[0] + a * nx + x0 : L.tab[1] + a * ny + y0) + c;
        if (q < 3 * TX + 3 * TY) tslot = (xs ? a : 3 + a) * TAB_MAXD + c;
    }
    // field by field: a whole-struct copy into shared memory later would keep
    // the value in a per-thread shared-memory slot, written as soon as it lands
    const T tre = tsrc->re, tim = tsrc->im;
    zc pv_parts[SB + 1];
    load_parts<SB + 1>(pin + (size_t)rhs * NVAL * NBMAX, nbin, j + 2, pv_parts);
    // halo-tile point e: its index in the level (clamped when absent), whether present
    auto locate = [&](int e, size_t &p) {
        const int ey = e / HX, ex = e - ey * HX;
        const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
        const bool ok = e < HN && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        p = ok ? (size_t)gy * nx + gx : pc;
        return ok;
    };
    auto inner = [&](int e) {
        const int ey = e / HX, ex = e - ey * HX;
        return e < HN && ex >= 1 && ex <= HX - 2 && ey >= 1 && ey <= HY - 2;
    };
    // the first TILE_PRE points of each thread are loaded before the
    // partial-sum reduction, so their memory latency overlaps it
    Cx<T> uq[TILE_MAXE][J + 1], wq[TILE_PRE];
    T phq[TILE_MAXE];
    size_t pq[TILE_MAXE];
    bool okq[TILE_MAXE];
#pragma unroll
    for (int it = 0; it < TILE_PRE; ++it) {
        okq[it] = locate(threadIdx.x + it * BLK, pq[it]);
        wq[it] = wi[pq[it]];
#pragma unroll
        for (int q = 0; q <= J; ++q) uq[it][q] = B.u[q][off + pq[it]];
        phq[it] = L.phi[pq[it]];
    }
    if (!act) return;
    block_sum<SB + 1>(pv_parts, j + 2, sh, res);
    if (tslot >= 0) ltab[tslot] = mkc<T>(tre, tim);
    Cx<T> cu[SB];
    const double sjd = coef_step<T, SB>(res, j, s, tiny, pv, gs, blockIdx.x == 0 && threadIdx.x == 0, cu);
    const T sj = (T)sjd;
#pragma unroll
    for (int b0 = 0; b0 < TILE_MAXE; b0 += TILE_PB) {
        if (b0 * BLK >= HN) break;   // the same for every thread of the block
        Cx<T> wv[TILE_PB];
#pragma unroll
        for (int i = 0; i < TILE_PB; ++i) {
            const int it = b0 + i;
            if (it >= TILE_MAXE) break;
            if (it < TILE_PRE) {
                wv[i] = wq[it < TILE_PRE ? it : 0];
            } else {
                okq[it] = locate(threadIdx.x + it * BLK, pq[it]);
                wv[i] = wi[pq[it]];
#pragma unroll
                for (int q = 0; q <= J; ++q) uq[it][q] = B.u[q][off + pq[it]];
                phq[it] = L.phi[pq[it]];
            }
        }
#pragma unroll
        for (int i = 0; i < TILE_PB; ++i) {
            const int it = b0 + i;
            if (it >= TILE_MAXE) break;
            const int e = threadIdx.x + it * BLK;
            Cx<T> v = sj * wv[i];
#pragma unroll
            for (int q = 0; q <= J; ++q) v = v - cu[q] * uq[it][q];
            if (!okq[it]) v = mkc<T>(0, 0);
            if (okq[it] && inner(e)) un[pq[it]] = v;
            if (e < HN) lu[e] = v;
        }
    }
    __syncthreads();
    zc acc[SB + 1];
#pragma unroll
    for (int q = 0; q <= SB; ++q) acc[q] = mkc(0.0, 0.0);
    const bool wlast = norm_from_sums<T>() && j + 2 == s;   // last step of the sweep
#pragma unroll
    for (int it = 0; it < TILE_MAXE; ++it) {
        const int e = threadIdx.x + it * BLK;
        if (it * BLK >= HN) break;   // the same for every thread of the block
        if (!inner(e)) continue;
        const int ey = e / HX, ex = e - ey * HX;
        const int c = ex - 1, r = ey - 1;
        const Cx<T> uc = lu[e];
        Cx<T> d = ltab[1 * TAB_MAXD + c] + ltab[4 * TAB_MAXD + r];
        sub_phi(d, L, phq[it]);
        Cx<T> a = d * uc;
        a = cfma(ltab[0 * TAB_MAXD + c], lu[e - 1], a);
        a = cfma(ltab[2 * TAB_MAXD + c], lu[e + 1], a);
        a = cfma(ltab[3 * TAB_MAXD + r], lu[e - HX], a);
        a = cfma(ltab[5 * TAB_MAXD + r], lu[e + HX], a);
        wo[pq[it]] = a;
        const zc wd = cvt<double>(a), ud = cvt<double>(uc);
#pragma unroll
        for (int q = 0; q <= J; ++q) acc[q] = cjfma(cvt<double>(uq[it][q]), wd, acc[q]);
        acc[j + 1] = cjfma(ud, wd, acc[j + 1]);
        acc[j + 2].re += cabs2(ud);
        if (wlast) acc[j + 3].re += cabs2(wd);
    }
    const int nv = j + 3 + (wlast ? 1 : 0);
    block_sum_last<SB + 1>(acc, nv, sh, res);
    if (threadIdx.x < nv) pout[((size_t)rhs * NVAL + threadIdx.x) * NBMAX + t] = res[threadIdx.x];
}

// ---------------------------------------------------------------------------
// 3-D Arnoldi passes on z-marching slabs.  A block owns a column of
// SX x SY points of the x-y plane over a run of planes; it forms the pass's
// vector u (u_0 itself for pass 0, else u_{j+1} = sj w_j - sum cu_i u_i) on the
// column's points and their one-point x-y halo, one plane at a time, into a
// ring of three shared-memory planes, and applies the 7-point stencil to the
// middle plane from there.  Every point of u is read (or formed) once per
// block plus the halo (x-y ring, one plane above and below the run), instead
// of once per stencil neighbour as in the chunked passes, whose z neighbours
// lie a whole plane away.  Outputs match k_st0 (J = -1) and k_os (J = j):
// w = A u, u_{j+1} stored for the run's own planes, and the partial sums
// <u_i, w> (i < m), <u_m, w>, ||u_m||^2 (and ||w||^2 on the sweep's last
// step), m = J + 1, one partial per block.
// ---------------------------------------------------------------------------
constexpr int SX = 32, SY = 16;             // slab column: SX * SY = BLK points per plane
constexpr int SHX = SX + 2, SHY = SY + 2;   // with the x-y halo
constexpr int SRING = 2 * SHX + 2 * SY;     // halo points of one plane
static_assert(SX * SY == BLK && SRING <= BLK, "one column point and at most one halo point per thread");

// The unit value at halo-plane position of ring index r (x-y halo of a TX x TY
// column): (ex, ey) in [0, TX + 1] x [0, TY + 1].
__device__ __forceinline__ void ring_pos(int r, int TX, int TY, int &ex, int &ey)
{
    const int W = TX + 2;
    if (r < W) { ex = r; ey = 0; }
    else if (r < 2 * W) { ex = r - W; ey = TY + 1; }
    else if (r < 2 * W + TY) { ex = 0; ey = 1 + r - 2 * W; }
    else { ex = TX + 1; ey = 1 + r - 2 * W - TY; }
}

template <typename T, int SB, int J>
__global__ __launch_bounds__(BLK) void k_slab(LvlK<T> L, Basis<T> B, const Cx<T> *win, Cx<T> *wout, int s, size_t ld,
                                              const zc *__restrict__ pin, int nbin, zc *__restrict__ pout,
                                              GState *gsb, double tiny, unsigned ntx, unsigned nty, unsigned nzc,
                                              unsigned zrun, int wnorm, int nslab, const int *active)
{
    constexpr int M = J + 1;                   // index of the pass's vector
    constexpr int NU = J + 1;                  // older basis vectors read for the dots (J >= 0)
    static_assert(M + 3 <= SB + 1, "sum slots");
    __shared__ zc sh[(BLK / 64) * (SB + 1)];
    __shared__ zc res[SB + 1];
    __shared__ Cx<T> ring[3][SHX * SHY];
    __shared__ Cx<T> ltab[3 * SX + 3 * SY];
    const int rhs = blockIdx.y;
    L = L.at(rhs);
    if (!active[rhs]) return;
    const size_t off = rhs * ld;
    // GMRES coefficients of this step from the previous pass's partials
    Cx<T> cu[SB];
    T sj = (T)1;
    if (J >= 0) {
        GState *gs = gsb + rhs;
        const GPrev<SB> pv = load_prev<SB>(gs, J);
        reduce_parts<SB + 1>(pin + (size_t)rhs * NVAL * NBMAX, nbin, J + 2, sh, res);
        sj = (T)coef_step<T, SB>(res, J, s, tiny, pv, gs, blockIdx.x == 0 && threadIdx.x == 0, cu);
    }
    const unsigned slot = chunk_id(nslab);
    const unsigned col = slot / nzc, zci = slot - col * nzc;
    if (col >= ntx * nty) {
        // padding block: zero partials
        if ((int)threadIdx.x < M + 3) pout[((size_t)rhs * NVAL + threadIdx.x) * NBMAX + slot] = mkc(0.0, 0.0);
        return;
    }
    const unsigned cyi = col / ntx, cxi = col - cyi * ntx;
    const int nx = (int)L.nx, ny = (int)L.ny, nz = (int)L.nz;
    const int x0 = (int)cxi * SX, y0 = (int)cyi * SY;
    const int TX = min(SX, nx - x0), TY = min(SY, ny - y0);
    const int z0 = (int)(zci * zrun), z1 = min(nz, z0 + (int)zrun);
    // this thread's column point and (maybe) one halo point of every plane
    const int tx = threadIdx.x % SX, ty = threadIdx.x / SX;
    const bool own = tx < TX && ty < TY;
    const int eo = (ty + 1) * SHX + tx + 1;
    const unsigned po = (unsigned)(y0 + min(ty, TY - 1)) * nx + (x0 + min(tx, TX - 1));
    int er = -1;
    unsigned pr = 0;
    bool rin = false;
    if ((int)threadIdx.x < 2 * (TX + 2) + 2 * TY) {
        int ex, ey;
        ring_pos(threadIdx.x, TX, TY, ex, ey);
        er = ey * SHX + ex;
        const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
        rin = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        pr = rin ? (unsigned)gy * nx + gx : po;
    }
    // the column's x and y stencil rows
    for (int q = threadIdx.x; q < 3 * (TX + TY); q += BLK) {
        if (q < 3 * TX) {
            const int a = q / TX, c = q - a * TX;
            ltab[a * SX + c] = L.tab[0][a * nx + x0 + c];
        } else {
            const int qq = q - 3 * TX, a = qq / TY, c = qq - a * TY;
            ltab[3 * SX + a * SY + c] = L.tab[1][a * ny + y0 + c];
        }
    }
    const unsigned plane = (unsigned)nx * ny;
    // the values a plane's u is formed from at one point (w_j and u_0..u_j,
    // or u_0 itself), loaded one plane ahead of their use
    struct Raw {
        Cx<T> w;
        Cx<T> u[NU > 0 ? NU : 1];
    };
    // (only the threads holding a halo point load it: wavefronts 2..7 hold
    // none and issue no halo loads)
    auto load = [&](int k, Raw &ro, Raw &rr, T &ph) {
        const unsigned kp = (unsigned)max(0, min(k, nz - 1)) * plane;
        if (J < 0) {
            ro.w = B.u[0][off + kp + po];
            if (er >= 0) rr.w = B.u[0][off + kp + pr];
        } else {
            ro.w = win[off + kp + po];
#pragma unroll
            for (int q = 0; q < NU; ++q) ro.u[q] = B.u[q][off + kp + po];
            if (er >= 0) {
                rr.w = win[off + kp + pr];
#pragma unroll
                for (int q = 0; q < NU; ++q) rr.u[q] = B.u[q][off + kp + pr];
            }
        }
        ph = L.phi[kp + po];
    };
    auto combine = [&](const Raw &r) -> Cx<T> {
        if (J < 0) return r.w;
        Cx<T> v = sj * r.w;
#pragma unroll
        for (int q = 0; q < NU; ++q) v = v - cu[q] * r.u[q];
        return v;
    };
    Cx<T> *un = J >= 0 ? B.u[M] + off : nullptr;
    // plane k into ring slot k % 3 (zero outside the level); u_{j+1} of the
    // run's own planes also to memory; returns the column point's u
    auto stage = [&](int k, const Raw &ro, const Raw &rr) -> Cx<T> {
        Cx<T> *R = ring[(k + 3) % 3];
        const bool kin = k >= 0 && k < nz;
        const Cx<T> uo = combine(ro);
        if (er >= 0) R[er] = (kin && rin) ? combine(rr) : mkc<T>(0, 0);
        R[eo] = (kin && own) ? uo : mkc<T>(0, 0);
        if (J >= 0 && kin && own && k >= z0 && k < z1) un[(size_t)k * plane + po] = uo;
        return uo;
    };
    zc acc[SB + 1];
#pragma unroll
    for (int q = 0; q <= SB; ++q) acc[q] = mkc(0.0, 0.0);
    const bool wn = wnorm != 0;
    Raw ro, rr, ro2, rr2;
    T phc, phn, dph;
    load(z0 - 1, ro, rr, dph);
    stage(z0 - 1, ro, rr);
    load(z0, ro, rr, phc);
    Cx<T> uc = stage(z0, ro, rr);
    Cx<T> ucq[NU > 0 ? NU : 1];
#pragma unroll
    for (int q = 0; q < NU; ++q) ucq[q] = ro.u[q];
    load(z0 + 1, ro, rr, phn);
    for (int k = z0; k < z1; ++k) {
        const Cx<T> unx = stage(k + 1, ro, rr);
        // the plane after next is in flight while this plane's stencil runs
        T ph2 = phn;
        if (k + 2 <= z1) load(k + 2, ro2, rr2, ph2);
        __syncthreads();
        if (own) {
            const Cx<T> *Rm = ring[(k + 2) % 3], *R0 = ring[k % 3], *Rp = ring[(k + 1) % 3];
            const Cx<T> *tz = L.tab[2];
            Cx<T> d = ltab[SX + tx] + ltab[3 * SX + SY + ty] + tz[nz + k];
            sub_phi(d, L, phc);
            Cx<T> a = d * R0[eo];
            a = cfma(ltab[tx], R0[eo - 1], a);
            a = cfma(ltab[2 * SX + tx], R0[eo + 1], a);
            a = cfma(ltab[3 * SX + ty], R0[eo - SHX], a);
            a = cfma(ltab[3 * SX + 2 * SY + ty], R0[eo + SHX], a);
            a = cfma(tz[k], Rm[eo], a);
            a = cfma(tz[2 * nz + k], Rp[eo], a);
            wout[off + (size_t)k * plane + po] = a;
            const zc wd = cvt<double>(a), ud = cvt<double>(uc);
#pragma unroll
            for (int q = 0; q < NU; ++q) acc[q] = cjfma(cvt<double>(ucq[q]), wd, acc[q]);
            acc[M] = cjfma(ud, wd, acc[M]);
            acc[M + 1].re += cabs2(ud);
            if (wn) acc[M + 2].re += cabs2(wd);
        }
        __syncthreads();
        uc = unx;
        phc = phn;
#pragma unroll
        for (int q = 0; q < NU; ++q) ucq[q] = ro.u[q];
        ro = ro2;
        rr = rr2;
        phn = ph2;
    }
    const int nv = M + 2 + (wn ? 1 : 0);
    block_sum_last<SB + 1>(acc, nv, sh, res);
    if ((int)threadIdx.x < nv) pout[((size_t)rhs * NVAL + threadIdx.x) * NBMAX + slot] = res[threadIdx.x];
}

// w = H z on the z-marching slabs of the finest 3-D level, with the
// first-round inner products <v_i, w> (i <= j) and ||w||^2 (the outer
// analogue of k_slab, same column/run geometry): z of each plane is staged
// into the ring (column points and their x-y halo, complex128), the 7-point
// stencil of H is applied to the middle plane and w stored; the first group of
// up to 8 basis vectors, loaded at the column point before the plane's
// barrier, meets w in registers (later groups: k_hdot_groups).  One partial
// per block; the padding blocks write zeros.
template <typename TZ>
__global__ __launch_bounds__(BLK) void k_slab_hdot(LvlK<double> H, const Cx<TZ> *__restrict__ z,
                                                   zc *__restrict__ w, const zc *__restrict__ V, size_t vstride,
                                                   int j, size_t ld, zc *__restrict__ pout, unsigned ntx,
                                                   unsigned nty, unsigned nzc, unsigned zrun, int nslab,
                                                   const int *active)
{
    __shared__ zc sh[(BLK / 64) * 9];
    __shared__ zc res[9];
    __shared__ zc ring[3][SHX * SHY];
    __shared__ zc ltab[3 * SX + 3 * SY];
    const int rhs = blockIdx.y;
    H = H.at(rhs);
    if (!active[rhs]) return;
    const size_t off = rhs * ld;
    zc *po = pout + (size_t)rhs * OVAL * NBMAX;
    const unsigned slot = chunk_id(nslab);
    const unsigned col = slot / nzc, zci = slot - col * nzc;
    if (col >= ntx * nty) {
        if ((int)threadIdx.x <= min(j, 7) || (int)threadIdx.x == j + 1)
            po[(size_t)threadIdx.x * NBMAX + slot] = mkc(0.0, 0.0);
        return;
    }
    const unsigned cyi = col / ntx, cxi = col - cyi * ntx;
    const int nx = (int)H.nx, ny = (int)H.ny, nz = (int)H.nz;
    const int x0 = (int)cxi * SX, y0 = (int)cyi * SY;
    const int TX = min(SX, nx - x0), TY = min(SY, ny - y0);
    const int z0 = (int)(zci * zrun), z1 = min(nz, z0 + (int)zrun);
    const int tx = threadIdx.x % SX, ty = threadIdx.x / SX;
    const bool own = tx < TX && ty < TY;
    const int eo = (ty + 1) * SHX + tx + 1;
    const unsigned pp = (unsigned)(y0 + min(ty, TY - 1)) * nx + (x0 + min(tx, TX - 1));
    int er = -1;
    unsigned pr = 0;
    bool rin = false;
    if ((int)threadIdx.x < 2 * (TX + 2) + 2 * TY) {
        int ex, ey;
        ring_pos(threadIdx.x, TX, TY, ex, ey);
        er = ey * SHX + ex;
        const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
        rin = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        pr = rin ? (unsigned)gy * nx + gx : pp;
    }
    for (int q = threadIdx.x; q < 3 * (TX + TY); q += BLK) {
        if (q < 3 * TX) {
            const int a = q / TX, c = q - a * TX;
            ltab[a * SX + c] = H.tab[0][a * nx + x0 + c];
        } else {
            const int qq = q - 3 * TX, a = qq / TY, c = qq - a * TY;
            ltab[3 * SX + a * SY + c] = H.tab[1][a * ny + y0 + c];
        }
    }
    const unsigned plane = (unsigned)nx * ny;
    const int g0 = min(j, 7);   // the first group: v_0 .. v_g0
    // z of plane k at the column point and (threads holding one) the halo
    // point (clamped plane: the values outside the level are replaced by zeros
    // when staged)
    auto load_z = [&](int k, Cx<TZ> &zo, Cx<TZ> &zr) {
        const unsigned kp = (unsigned)max(0, min(k, nz - 1)) * plane;
        zo = z[off + kp + pp];
        if (er >= 0) zr = z[off + kp + pr];
    };
    // the first group's basis values and phi at the column point of plane k
    auto load_v = [&](int k, zc (&v)[8], double &ph) {
        const unsigned kp = (unsigned)max(0, min(k, nz - 1)) * plane;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q <= g0) v[q] = V[q * vstride + off + kp + pp];
        ph = H.phi[kp + pp];
    };
    auto stage = [&](int k, const Cx<TZ> &zo, const Cx<TZ> &zr) {
        zc *R = ring[(k + 3) % 3];
        const bool kin = k >= 0 && k < nz;
        if (er >= 0) R[er] = (kin && rin) ? cvt<double>(zr) : mkc(0.0, 0.0);
        R[eo] = (kin && own) ? cvt<double>(zo) : mkc(0.0, 0.0);
    };
    zc acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = mkc(0.0, 0.0);
    Cx<TZ> zo, zr;
    load_z(z0 - 1, zo, zr);
    stage(z0 - 1, zo, zr);
    load_z(z0, zo, zr);
    stage(z0, zo, zr);
    load_z(z0 + 1, zo, zr);
    for (int k = z0; k < z1; ++k) {
        stage(k + 1, zo, zr);
        // z of the plane after next, and this plane's basis values, are in
        // flight across the barrier (values loaded a plane ahead would hold
        // twice the registers and halve the resident workgroups)
        if (k + 2 <= z1) load_z(k + 2, zo, zr);
        zc vc[8];
        double phc;
        load_v(k, vc, phc);
        __syncthreads();
        if (own) {
            const zc *Rm = ring[(k + 2) % 3], *R0 = ring[k % 3], *Rp = ring[(k + 1) % 3];
            const zc *tz = H.tab[2];
            zc d = ltab[SX + tx] + ltab[3 * SX + SY + ty] + tz[nz + k];
            sub_phi(d, H, phc);
            zc a = d * R0[eo];
            a = cfma(ltab[tx], R0[eo - 1], a);
            a = cfma(ltab[2 * SX + tx], R0[eo + 1], a);
            a = cfma(ltab[3 * SX + ty], R0[eo - SHX], a);
            a = cfma(ltab[3 * SX + 2 * SY + ty], R0[eo + SHX], a);
            a = cfma(tz[k], Rm[eo], a);
            a = cfma(tz[2 * nz + k], Rp[eo], a);
            w[off + (size_t)k * plane + pp] = a;
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q <= g0) acc[q] = cjfma(vc[q], a, acc[q]);
            acc[8].re += cabs2(a);
        }
        __syncthreads();
    }
    block_sum_last<9>(acc, 9, sh, res);
    if ((int)threadIdx.x <= g0) po[(size_t)threadIdx.x * NBMAX + slot] = res[threadIdx.x];
    if (threadIdx.x == 8) po[(size_t)(j + 1) * NBMAX + slot] = res[8];
}

// Pass 0 on one 2-D tile (see launch_st0_tile): u_0 on the tile and its
// one-point halo into shared memory (zero outside the level), then w_0 = A u_0
// on the tile's points with <u_0, w_0>, ||u_0||^2 and (NA = 3) ||w_0||^2.  All
// of a thread's loads are issued together (phi kept for phase 2), the tile's
// stencil tables are staged in shared memory, as in k_os_tile.
template <typename T, int NA>
__global__ __launch_bounds__(BLK) void k_st0_tile(LvlK<T> L, const Cx<T> *__restrict__ u0, Cx<T> *__restrict__ w,
                                                  size_t ld, zc *__restrict__ pout, TileGeo tg, int ntile,
                                                  const int *active)
{
    __shared__ zc sh[(BLK / 64) * NA];
    __shared__ zc res[NA];
    __shared__ Cx<T> lu[TILE_MAXN];
    __shared__ Cx<T> ltab[6 * TAB_MAXD];
    const int rhs = blockIdx.y;
    L = L.at(rhs);
    const int act = active[rhs];   // tested before the first store (reads below are harmless)
    const unsigned t = chunk_id(ntile);
    const unsigned tyi = t / tg.ntx, txi = t - tyi * tg.ntx;
    const int nx = (int)L.nx, ny = (int)L.ny;
    const int x0 = (int)(txi * tg.tx), y0 = (int)(tyi * tg.ty);
    const int TX = min(x0 + (int)tg.tx, nx) - x0, TY = min(y0 + (int)tg.ty, ny) - y0;
    const int HX = TX + 2, HY = TY + 2, HN = HX * HY;
    const size_t off = rhs * ld;
    const size_t pc = (size_t)y0 * nx + x0;
    const Cx<T> *ui = u0 + off;
    int tslot = -1;
    const Cx<T> *tsrc;
    {
        const int q = threadIdx.x;
        const bool xs = q < 3 * TX;
        const int qq = xs ? q : min(q - 3 * TX, 3 * TY - 1);
        const int c = qq / 3, a = qq - 3 * c;
        tsrc = (xs ? L.tab[0] + a * nx + x0 : L.tab[1] + a * ny + y0) + c;
        if (q < 3 * TX + 3 * TY) tslot = (xs ? a : 3 + a) * TAB_MAXD + c;
    }
    const T tre = tsrc->re, tim = tsrc->im;
    T phq[TILE_MAXE];
    size_t pq[TILE_MAXE];
    // one batch: this pass holds a single vector per point, so all of a
    // thread's points fit in registers and the tile waits for memory once
    constexpr int PB = TILE_MAXE;
#pragma unroll
    for (int b0 = 0; b0 < TILE_MAXE; b0 += PB) {
        if (b0 * BLK >= HN) break;   // the same for every thread of the block
        Cx<T> v[PB];
        bool ok[PB];
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int it = b0 + i;
            if (it >= TILE_MAXE) break;
            const int e = threadIdx.x + it * BLK;
            const int ey = e / HX, ex = e - ey * HX;
            const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
            ok[i] = e < HN && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
            pq[it] = ok[i] ? (size_t)gy * nx + gx : pc;
            v[i] = ui[pq[it]];
            phq[it] = L.phi[pq[it]];
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int it = b0 + i;
            if (it >= TILE_MAXE) break;
            const int e = threadIdx.x + it * BLK;
            if (e < HN) lu[e] = ok[i] ? v[i] : mkc<T>(0, 0);
        }
    }
    if (tslot >= 0) ltab[tslot] = mkc<T>(tre, tim);
    if (!act) return;
    __syncthreads();
    zc acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = mkc(0.0, 0.0);
#pragma unroll
    for (int it = 0; it < TILE_MAXE; ++it) {
        if (it * BLK >= HN) break;   // the same for every thread of the block
        const int e = threadIdx.x + it * BLK;
        const int ey = e / HX, ex = e - ey * HX;
        if (e >= HN || ex < 1 || ex > HX - 2 || ey < 1 || ey > HY - 2) continue;
        const int c = ex - 1, r = ey - 1;
        const Cx<T> uc = lu[e];
        Cx<T> d = ltab[1 * TAB_MAXD + c] + ltab[4 * TAB_MAXD + r];
        sub_phi(d, L, phq[it]);
        Cx<T> a = d * uc;
        a = cfma(ltab[0 * TAB_MAXD + c], lu[e - 1], a);
        a = cfma(ltab[2 * TAB_MAXD + c], lu[e + 1], a);
        a = cfma(ltab[3 * TAB_MAXD + r], lu[e - HX], a);
        a = cfma(ltab[5 * TAB_MAXD + r], lu[e + HX], a);
        w[off + pq[it]] = a;
        const zc wd = cvt<double>(a), ud = cvt<double>(uc);
        acc[0] = cjfma(ud, wd, acc[0]);
        acc[1].re += cabs2(ud);
        if (NA > 2) acc[NA - 1].re += cabs2(wd);
    }
    block_sum_last<NA>(acc, NA, sh, res);
    if (threadIdx.x < NA) pout[((size_t)rhs * NVAL + threadIdx.x) * NBMAX + t] = res[threadIdx.x];
}


// last pass: u_s and ||u_s||^2
template <typename T, int SB>
__global__ __launch_bounds__(BLK) void k_orthl(Basis<T> B, const Cx<T> *win, int j, int s, unsigned N, size_t ld,
                                               const zc *__restrict__ pin, int nbin, zc *__restrict__ pout,
                                               GState *gsb, double tiny, unsigned chunk, int nb, const int *active)
{
    __shared__ zc sh[(BLK / 64) * NVAL];
    __shared__ zc res[NVAL];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    GState *gs = gsb + rhs;
    const GPrev<SB> pv = load_prev<SB>(gs, j);
    reduce_parts<SB>(pin + (size_t)rhs * NVAL * NBMAX, nbin, j + 2, sh, res);
    Cx<T> cu[SB];
    const double sj = coef_step<T, SB>(res, j, s, tiny, pv, gs, blockIdx.x == 0 && threadIdx.x == 0, cu);
    zc acc[1] = {mkc(0.0, 0.0)};
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(N, p0 + chunk);
    body_orthl<T, SB>(B, win + rhs * ld, j, (T)sj, cu, rhs * ld, p0 + threadIdx.x, p1, BLK, acc[0].re);
    block_sum_last<1>(acc, 1, sh, res);
    if (threadIdx.x == 0) pout[((size_t)rhs * NVAL) * NBMAX + c] = res[0];
}

// Shared prologue of the sweep's closing passes.  The last Arnoldi pass left
// <u_i, w_{s-1}> (i < s), ||u_{s-1}||^2 and ||w_{s-1}||^2 with w_{s-1} = A u_{s-1}:
// finish column s-1 of the Hessenberg matrix (coef_step), take h_{s,s-1} from
// ||A v_{s-1}||^2 = sum_i |h_{i,s-1}|^2 + h_{s,s-1}^2 (v_i orthonormal), so u_s
// itself is never formed, solve the small least-squares problem and publish
// ax[i] = y_i sig_i (update) and the Arnoldi residual on {u_0..u_{s-1}, w_{s-1}}:
// r = sum_{i<s} ar_i u_i + ar_s w_{s-1} (u_s = sig_{s-1} w_{s-1} - sum_i cu_i u_i
// folded in).  Every block finishes the column in its own shared copy of the
// state; block 0 publishes it.
// Register-resident form of the closing least squares for s <= SB - 1 <= 3,
// run by one thread: gathers columns 0..s-2 of the sweep's state, finishes
// column s-1 and h_{s,s-1} as described above, and writes ax, ar (shared) and
// k.  With `publish` the finished state goes back to gs.  The arithmetic is the
// same, operation for operation, as coef_step followed by gmres_ls.
template <int SB>
struct CloseIn {
    zc H[SB][SB - 1];
    double sig[SB];
    double beta0;
    int k;
};

// The sweep's state as far as earlier passes finished it (loaded before the
// partial-sum reduction): columns 0..s-2 (sums form) or 0..s-1 (explicit form,
// all but h_{s,s-1}).
template <int SB>
__device__ __forceinline__ void close_gather(const GState *gs, int s, bool sums, CloseIn<SB> &in)
{
    constexpr int K = SB - 1;
    const int j = s - 1;
    const int ncol = sums ? s - 1 : s;
#pragma unroll
    for (int c = 0; c < K; ++c) {
#pragma unroll
        for (int r = 0; r < SB; ++r) in.H[r][c] = mkc(0.0, 0.0);
        in.sig[c] = 0.0;
        if (c < ncol) {
            in.sig[c] = gs->sig[c];
#pragma unroll
            for (int r = 0; r < SB; ++r)
                if (r <= c + 1 && !(sums && c + 1 == j && r == j) && !(!sums && r == s))
                    in.H[r][c] = gs->H[r * CSG_MAX_S + c];
        }
    }
    in.sig[K] = 0.0;
    in.k = gs->k;
    in.beta0 = gs->beta0;
}

// y = argmin || beta0 e1 - Hbar y || over the first k columns (gmres_ls on a
// register copy of Hbar)
template <int SB>
__device__ __forceinline__ void ls_regs(const zc (&H)[SB][SB - 1], double beta0, int k, zc (&yl)[SB - 1])
{
    constexpr int K = SB - 1;
    zc R[SB][K], g[SB];
    double cs[K];
    zc sn[K];
#pragma unroll
    for (int r = 0; r < SB; ++r) {
        g[r] = mkc(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < K; ++c) R[r][c] = H[r][c];
    }
    g[0] = mkc(beta0, 0.0);
#pragma unroll
    for (int c = 0; c < K; ++c) {
        if (c >= k) break;
#pragma unroll
        for (int i = 0; i < c; ++i) {
            const zc t1 = R[i][c], t2 = R[i + 1][c];
            R[i][c] = cs[i] * t1 + sn[i] * t2;
            R[i + 1][c] = cs[i] * t2 - mkc(sn[i].re, -sn[i].im) * t1;
        }
        rot(R[c][c], R[c + 1][c], cs[c], sn[c]);
        const zc t1 = R[c][c], t2 = R[c + 1][c];
        R[c][c] = cs[c] * t1 + sn[c] * t2;
        R[c + 1][c] = mkc(0.0, 0.0);
        const zc gc = g[c];
        g[c + 1] = mkc(0.0, 0.0) - mkc(sn[c].re, -sn[c].im) * gc;
        g[c] = cs[c] * gc;
    }
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
        yl[i] = mkc(0.0, 0.0);
        if (i < k) {
            zc acc = g[i];
#pragma unroll
            for (int c = i + 1; c < K; ++c)
                if (c < k) acc = acc - R[i][c] * yl[c];
            const zc d = R[i][i];
            yl[i] = (1.0 / cabs2(d)) * (acc * mkc(d.re, -d.im));
        }
    }
}

template <typename T, int SB>
__device__ __forceinline__ void close_regs(const CloseIn<SB> &in, GState *gs, const zc *res, int s, double tiny, bool publish, zc *ax,
                           zc *ar, int *ks)
{
    constexpr int K = SB - 1;
    const int j = s - 1;
    zc H[SB][K];
    double sig[SB];
#pragma unroll
    for (int r = 0; r < SB; ++r) {
        sig[r] = in.sig[r];
#pragma unroll
        for (int c = 0; c < K; ++c) H[r][c] = in.H[r][c];
    }
    int k = in.k;
    double beta0 = in.beta0;
    if constexpr (!norm_from_sums<T>()) {
        // explicit form: column s-1 is complete, res[0] = ||u_s||^2
        const double hn = sqrt(res[0].re);
        const double sig_s = !(hn > tiny * beta0) ? 0.0 : 1.0 / hn;
#pragma unroll
        for (int c = 0; c < K; ++c)
#pragma unroll
            for (int r = 1; r < SB; ++r)
                if (c == j && r == s) H[r][c] = mkc(hn, 0.0);
#pragma unroll
        for (int i = 0; i < SB; ++i)
            if (i == s) sig[i] = sig_s;
        if (k > s) k = s;
        if (!(beta0 > 0.0)) k = 0;
        zc yl[K];
        ls_regs<SB>(H, beta0, k, yl);
#pragma unroll
        for (int i = 0; i < SB; ++i) {
            zc acc = (i == 0) ? mkc(beta0, 0.0) : mkc(0.0, 0.0);
#pragma unroll
            for (int c = 0; c < K; ++c)
                if (c < k && i <= c + 1) acc = acc - H[i][c] * yl[c];
            if (i <= k) ar[i] = sig[i] * acc;
        }
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (i < k) ax[i] = sig[i] * yl[i];
        *ks = k;
        if (publish) {
            gs->H[s * CSG_MAX_S + (s - 1)] = mkc(hn, 0.0);
            gs->sig[s] = sig_s;
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (i < k) gs->y[i] = yl[i];
        }
        return;
    }
    // column j (coef_step)
    const double hnj = sqrt(res[j + 1].re);
    double sj;
    if (j == 0) {
        beta0 = hnj;
        sj = beta0 > 0.0 ? 1.0 / beta0 : 0.0;
        k = s;
    } else {
        const bool brk = !(hnj > tiny * beta0);
        sj = brk ? 0.0 : 1.0 / hnj;
        if (brk && k > j) k = j;
    }
    zc cu[SB];
    double w2 = sj * sj * res[j + 2].re, c2 = 0.0;
#pragma unroll
    for (int q = 0; q < SB; ++q) {
        if (q == j) sig[q] = sj;
#pragma unroll
        for (int c = 0; c < K; ++c)
            if (c == j && q <= j) {
                const zc h = (sig[q] * sj) * res[q];
                H[q][c] = h;
                cu[q] = cvt<double>(cvt<T>(sig[q] * h));
                c2 += cabs2(h);
            }
#pragma unroll
        for (int c = 1; c < K; ++c)
            if (c == j && q == j) H[q][c - 1] = mkc(hnj, 0.0);
    }
    // h_{s,s-1}: a difference at rounding level of ||A v_{s-1}||^2 means A v_{s-1}
    // lies in the basis span
    const double h2 = w2 - c2;
    const double hn = h2 > 1e-13 * w2 ? sqrt(h2) : 0.0;
    const double sig_s = !(hn > tiny * beta0) ? 0.0 : 1.0 / hn;
#pragma unroll
    for (int c = 0; c < K; ++c)
#pragma unroll
        for (int r = 1; r < SB; ++r)
            if (c == j && r == s) H[r][c] = mkc(hn, 0.0);
    if (k > s) k = s;
    if (!(beta0 > 0.0)) k = 0;
    zc yl[K];
    ls_regs<SB>(H, beta0, k, yl);
    zc arl[SB];
#pragma unroll
    for (int i = 0; i < SB; ++i) {
        zc acc = (i == 0) ? mkc(beta0, 0.0) : mkc(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < K; ++c)
            if (c < k && i <= c + 1) acc = acc - H[i][c] * yl[c];
        arl[i] = ((i == s) ? sig_s : sig[i]) * acc;
    }
    if (k == s) {
        zc as = mkc(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < SB; ++i)
            if (i == s) as = arl[i];
#pragma unroll
        for (int i = 0; i < SB - 1; ++i)
            if (i < s) arl[i] = arl[i] - as * cu[i];
#pragma unroll
        for (int i = 0; i < SB; ++i)
            if (i == s) arl[i] = sj * as;
    }
#pragma unroll
    for (int i = 0; i < K; ++i)
        if (i < k) ax[i] = sig[i] * yl[i];
#pragma unroll
    for (int i = 0; i < SB; ++i)
        if (i <= k) ar[i] = arl[i];
    *ks = k;
    if (publish) {
        gs->beta0 = beta0;
        gs->k = k;
#pragma unroll
        for (int c = 0; c < K; ++c)
            if (c == j) {
#pragma unroll
                for (int r = 0; r < SB; ++r)
                    if (r <= s) gs->H[r * CSG_MAX_S + c] = H[r][c];
                if (j > 0) gs->H[j * CSG_MAX_S + (j - 1)] = mkc(hnj, 0.0);
            }
#pragma unroll
        for (int i = 0; i < SB; ++i) {
            if (i == j) gs->sig[i] = sj;
            if (i == s) gs->sig[i] = sig_s;
        }
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (i < k) gs->y[i] = yl[i];
    }
}

// The closing prologue (s <= 3) in two halves, so that a pass can issue its
// own loads in between: close_begin issues the loads of the sweep state
// (thread 0) and of this thread's partials; close_end sums the partials and
// solves the least squares (ax, ar and the returned k as close_sweep).
// The sweep state is copied with one vector load per thread (8 bytes each) and
// staged in shared memory, so that no scalar load of it (each waited for in
// turn) stands before the pass's other loads.
constexpr int GS_WORDS = (int)(sizeof(GState) / sizeof(double));
static_assert(sizeof(GState) % sizeof(double) == 0 && GS_WORDS <= BLK, "state copy");
template <int SB>
struct CloseLoads {
    double gv;
    zc v[SB + 1];
};
template <typename T, int SB>
__device__ __forceinline__ void close_begin(const zc *pin, int nbin, const GState *gs, int s, CloseLoads<SB> &cl)
{
    static_assert(SB <= 4, "register form");
    constexpr bool sums = norm_from_sums<T>();
    cl.gv = reinterpret_cast<const double *>(gs)[min((int)threadIdx.x, GS_WORDS - 1)];
    load_parts<SB + 1>(pin, nbin, sums ? s + 2 : 1, cl.v);
}
template <typename T, int SB>
__device__ __forceinline__ int close_end(CloseLoads<SB> &cl, GState *gs, int s, double tiny, zc *sh, zc *res,
                                         zc *ax, zc *ar)
{
    __shared__ int ks;
    __shared__ __align__(16) double lgs[GS_WORDS];
    constexpr bool sums = norm_from_sums<T>();
    if (threadIdx.x < GS_WORDS) lgs[threadIdx.x] = cl.gv;
    block_sum<SB + 1>(cl.v, sums ? s + 2 : 1, sh, res);
    if (threadIdx.x == 0) {
        CloseIn<SB> in;
        close_gather<SB>(reinterpret_cast<const GState *>(lgs), s, sums, in);
        close_regs<T, SB>(in, gs, res, s, tiny, blockIdx.x == 0, ax, ar, &ks);
    }
    __syncthreads();
    return ks;
}

template <typename T, int SB>
__device__ __forceinline__ int close_sweep(const zc *pin, int nbin, GState *gs, int s, double tiny, zc *sh, zc *res, zc *ax, zc *ar)
{
    __shared__ int ks;
    constexpr bool sums = norm_from_sums<T>();
    if constexpr (SB <= 4) {
        CloseIn<SB> in;
        if (threadIdx.x == 0) close_gather<SB>(gs, s, sums, in);
        reduce_parts<SB + 1>(pin, nbin, sums ? s + 2 : 1, sh, res);
        if (threadIdx.x == 0) close_regs<T, SB>(in, gs, res, s, tiny, blockIdx.x == 0, ax, ar, &ks);
        __syncthreads();
        return ks;
    }
    if constexpr (!sums) {
        __shared__ zc Rs[(CSG_MAX_S + 1) * CSG_MAX_S], ys[CSG_MAX_S], crs[CSG_MAX_S + 1];
        reduce_parts<1>(pin, nbin, 1, sh, res);
        if (threadIdx.x == 0) {
            const double hn = sqrt(res[0].re);
            const bool brk = !(hn > tiny * gs->beta0);
            const double sig_s = brk ? 0.0 : 1.0 / hn;
            const int k = gmres_ls<SB>(gs, s, hn, Rs, ys, crs);
            for (int i = 0; i < k; ++i) ax[i] = gs->sig[i] * ys[i];
            for (int i = 0; i <= k; ++i) ar[i] = ((i == s) ? sig_s : gs->sig[i]) * crs[i];
            ks = k;
            if (blockIdx.x == 0) {
                gs->H[s * CSG_MAX_S + (s - 1)] = mkc(hn, 0.0);
                gs->sig[s] = sig_s;
                for (int i = 0; i < k; ++i) gs->y[i] = ys[i];
            }
        }
        __syncthreads();
        return ks;
    }
    __shared__ GState lg;
    __shared__ zc Rs[(CSG_MAX_S + 1) * CSG_MAX_S], ys[CSG_MAX_S], crs[CSG_MAX_S + 1];
    {
        const double *src = (const double *)gs;
        double *dst = (double *)&lg;
        for (int i = threadIdx.x; i < (int)(sizeof(GState) / sizeof(double)); i += blockDim.x) dst[i] = src[i];
    }
    reduce_parts<SB + 1>(pin, nbin, s + 2, sh, res);
    if (threadIdx.x == 0) {
        Cx<T> cu[SB];
        const double sj = coef_step<T, SB>(res, s - 1, s, tiny, load_prev<SB>(&lg, s - 1), &lg, true, cu);
        double h2 = sj * sj * res[s + 1].re;
        for (int i = 0; i < s; ++i) h2 -= cabs2(lg.H[i * CSG_MAX_S + (s - 1)]);
        // a difference at rounding level of ||A v_{s-1}||^2: A v_{s-1} lies in the basis span
        const double hn = h2 > 1e-13 * (sj * sj * res[s + 1].re) ? sqrt(h2) : 0.0;
        const bool brk = !(hn > tiny * lg.beta0);
        const double sig_s = brk ? 0.0 : 1.0 / hn;
        const int k = gmres_ls<SB>(&lg, s, hn, Rs, ys, crs);
        for (int i = 0; i < k; ++i) ax[i] = lg.sig[i] * ys[i];
        for (int i = 0; i <= k; ++i) ar[i] = ((i == s) ? sig_s : lg.sig[i]) * crs[i];
        if (k == s) {
            const zc as = ar[s];
            for (int i = 0; i < s; ++i) ar[i] = ar[i] - as * cvt<double>(cu[i]);
            ar[s] = sj * as;
        }
        ks = k;
        if (blockIdx.x == 0) {
            lg.H[s * CSG_MAX_S + (s - 1)] = mkc(hn, 0.0);
            lg.sig[s] = sig_s;
            for (int i = 0; i < k; ++i) lg.y[i] = ys[i];
            *gs = lg;
        }
    }
    __syncthreads();
    return ks;
}

template <typename T, int SB>
__device__ __forceinline__ void coefs_to_T(int k, const zc *ax, const zc *ar, Cx<T> (&cx)[SB], Cx<T> (&cr)[SB])
{
#pragma unroll
    for (int q = 0; q < SB; ++q) {
        if (q < k) cx[q] = cvt<T>(ax[q]);
        if (q <= k) cr[q] = cvt<T>(ar[q]);
    }
}

// x (+)= sum_i y_i sig_i u_i.  For s <= 3 the loads of the closing prologue
// go first, then those of the thread's first TILE_PB points (every basis
// vector the update can use, u_0..u_{s-1}, and x), then the mask test, so
// that the least squares overlaps the first batch's memory latency; later
// batches issue all their loads together.
template <typename T, int SB>
__global__ __launch_bounds__(BLK) void k_upd(Cx<T> *x, int accumulate, Basis<T> B, int s, unsigned N, size_t ld,
                                             const zc *__restrict__ pin, int nbin, GState *gsb, double tiny,
                                             unsigned chunk, int nb, const int *active)
{
    __shared__ zc sh[(BLK / 64) * (SB + 1)];
    __shared__ zc res[SB + 1];
    __shared__ zc ax[CSG_MAX_S], ar[CSG_MAX_S + 1];
    const int rhs = blockIdx.y;
    if constexpr (SB <= 4) {
        constexpr int PB = TILE_PB;
        const int act = active[rhs];
        CloseLoads<SB> cls;
        close_begin<T, SB>(pin + (size_t)rhs * NVAL * NBMAX, nbin, gsb + rhs, s, cls);
        const unsigned c = chunk_id(nb);
        const unsigned p0 = c * chunk, p1 = min(N, p0 + chunk);
        const size_t off = rhs * ld;
        Cx<T> *xr = x + off;
        Cx<T> u[PB][SB - 1], xv[PB];
        // every load unconditional (slots past s-1 read slot s-1 again; x read
        // and dropped when not accumulating), so that the wait before the least
        // squares leaves the first batch in flight
        const Cx<T> *bu[SB - 1];
#pragma unroll
        for (int q = 0; q < SB - 1; ++q) bu[q] = B.u[min(q, s - 1)] + off;
        auto load = [&](unsigned p) {
#pragma unroll
            for (int i = 0; i < PB; ++i) {
                const unsigned pk = min(p + i * BLK, N - 1);
#pragma unroll
                for (int q = 0; q < SB - 1; ++q) u[i][q] = bu[q][pk];
                xv[i] = xr[pk];
            }
        };
        const unsigned pt = p0 + threadIdx.x;
        load(pt);
        if (!act) return;
        const int k = close_end<T, SB>(cls, gsb + rhs, s, tiny, sh, res, ax, ar);
        Cx<T> cx[SB], cr[SB];
        coefs_to_T<T, SB>(k, ax, ar, cx, cr);
        for (unsigned p = pt; p < p1; p += PB * BLK) {
            if (p != pt) load(p);
#pragma unroll
            for (int i = 0; i < PB; ++i) {
                Cx<T> v = accumulate ? xv[i] : mkc<T>(0, 0);
#pragma unroll
                for (int q = 0; q < SB - 1; ++q)
                    if (q < k) v = cfma(cx[q], u[i][q], v);
                if (p + i * BLK < p1) xr[p + i * BLK] = v;
            }
        }
    } else {
        if (!active[rhs]) return;
        const int k = close_sweep<T, SB>(pin + (size_t)rhs * NVAL * NBMAX, nbin, gsb + rhs, s, tiny, sh, res, ax, ar);
        Cx<T> cx[SB], cr[SB];
        coefs_to_T<T, SB>(k, ax, ar, cx, cr);
        const unsigned c = chunk_id(nb);
        const unsigned p0 = c * chunk, p1 = min(N, p0 + chunk);
        body_upd<T, SB>(x + rhs * ld, accumulate, B, k, cx, rhs * ld, p0 + threadIdx.x, p1, BLK);
    }
}

template <typename T, int DIM, int SB>
__global__ __launch_bounds__(BLK) void k_upd_res(Cx<T> *x, int accumulate, Basis<T> B, int s, LvlK<T> F, LvlK<T> C,
                                                 Cx<T> *bc, size_t ldf, size_t ldc, const zc *__restrict__ pin,
                                                 int nbin, GState *gsb, double tiny, unsigned chunk, int nb,
                                                 const int *active)
{
    __shared__ zc sh[(BLK / 64) * (SB + 1)];
    __shared__ zc res[SB + 1];
    __shared__ zc ax[CSG_MAX_S], ar[CSG_MAX_S + 1];
    const int rhs = blockIdx.y;
    F = F.at(rhs);
    C = C.at(rhs);
    if (!active[rhs]) return;
    const int k = close_sweep<T, SB>(pin + (size_t)rhs * NVAL * NBMAX, nbin, gsb + rhs, s, tiny, sh, res, ax, ar);
    Cx<T> cx[SB], cr[SB];
    coefs_to_T<T, SB>(k, ax, ar, cx, cr);
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(C.N, p0 + chunk);
    body_upd_res<T, DIM, SB>(x + rhs * ldf, accumulate, B, k, cx, cr, F, C, bc + rhs * ldc, rhs * ldf, p0 + threadIdx.x,
                         p1, BLK);
}

// Up-path pass on one 2-D tile (see launch_up_tile).  Phase 1: x = xin + P ec
// on the tile and a two-point halo into shared memory (zero outside the level;
// the tile's own points also to xout).  Phase 2: r = b - A x on the tile and a
// one-point halo, held in registers (the tile's points also to r), then moved
// into the shared buffer once every thread is done reading x.  Phase 3: w_0 =
// A r on the tile with <r, w_0>, ||r||^2 and (NA = 3) ||w_0||^2.  A thread owns
// the same points in phases 2 and 3 (phi loaded once).  The stencil tables of
// the tile's columns and rows are staged in shared memory, and b and phi of
// the first TILE_PB points of phase 2 are loaded with phase 1's first batch;
// every phase goes in batches of TILE_PB points per thread whose loads are
// issued together (absent points clamped to the tile's corner).
template <typename T, int NA, bool FU>
__global__ __launch_bounds__(BLK) void k_up_tile(LvlK<T> F, LvlK<T> C, const Cx<T> *__restrict__ ec,
                                                 const Cx<T> *__restrict__ xin, Cx<T> *__restrict__ xout,
                                                 const Cx<T> *__restrict__ b, Cx<T> *__restrict__ r,
                                                 Cx<T> *__restrict__ w, size_t ldf, size_t ldc,
                                                 zc *__restrict__ pout, TileGeo tg, int ntile, UpClose<T> uc,
                                                 const int *active)
{
    constexpr int SB = 4;
    __shared__ zc sh[(BLK / 64) * (NA > SB + 1 ? NA : SB + 1)];
    __shared__ zc res[SB + 1];
    __shared__ Cx<T> lx[UP_MAXN];
    __shared__ Cx<T> ltab[6 * TAB_MAXD];   // x lower, diag, upper; y lower, diag, upper
    __shared__ Cx<T> lc[FU ? UPC_MAXN : 1];   // the coarse correction on the tile's coarse window
    __shared__ zc axc[CSG_MAX_S], arc[CSG_MAX_S + 1];
    const int rhs = blockIdx.y;
    F = F.at(rhs);
    C = C.at(rhs);
    const int act = active[rhs];   // tested before the first store (reads below are harmless)
    const unsigned t = chunk_id(ntile);
    const unsigned tyi = t / tg.ntx, txi = t - tyi * tg.ntx;
    const int nx = (int)F.nx, ny = (int)F.ny;
    const int x0 = (int)(txi * tg.tx), y0 = (int)(tyi * tg.ty);
    const int TX = min(x0 + (int)tg.tx, nx) - x0, TY = min(y0 + (int)tg.ty, ny) - y0;
    const int AX = TX + 4, AN = AX * (TY + 4);   // x: tile and two-point halo
    const int RX = TX + 2, RN = RX * (TY + 2);   // r: tile and one-point halo
    const size_t off = rhs * ldf;
    const size_t pc = (size_t)y0 * nx + x0;      // a point of the level every clamped address goes to
    const Cx<T> *e = ec + rhs * ldc;
    const Cx<T> *xi = xin ? xin + off : nullptr;
    // stencil tables of the columns x0-1 .. x0+TX and rows y0-1 .. y0+TY (zero
    // outside the level), one entry per thread, stored before phase 1's barrier
    T tre, tim;
    bool tzero;
    int tslot = -1;
    {
        const int q = threadIdx.x;
        const bool xs = q < 3 * RX;
        const int qq = xs ? q : min(q - 3 * RX, 3 * (TY + 2) - 1);
        const int c = qq / 3, a = qq - 3 * c;
        const int g = (xs ? x0 : y0) - 1 + c, n = xs ? nx : ny;
        const Cx<T> *tab = xs ? F.tab[0] : F.tab[1];
        const Cx<T> *tp = tab + a * n + min(max(g, 0), n - 1);
        tre = tp->re;
        tim = tp->im;
        tzero = g < 0 || g >= n;
        if (q < 3 * RX + 3 * (TY + 2)) tslot = (xs ? a : 3 + a) * TAB_MAXD + c;
    }
    // phase-2 point q (tile and one-point halo): its index (clamped when absent), whether present
    auto locate2 = [&](int q, size_t &p) {
        const int qy = q / RX, qx = q - qy * RX;
        const int gx = x0 - 1 + qx, gy = y0 - 1 + qy;
        const bool ok = q < RN && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        p = ok ? (size_t)gy * nx + gx : pc;
        return ok;
    };
    // FU: the coarse sweep's closing update x_c + sum_{i<k} cx_i u_i, formed on
    // the coarse nodes the tile's interpolation reads (its coarse window) and
    // staged in shared memory; its prologue loads go first
    CloseLoads<SB> cls;
    unsigned cx0 = 0, cy0 = 0, CX = 1;
    int CN = 0;
    Cx<T> xbq[UPC_E], ucq[UPC_E][SB - 1];
    if constexpr (FU) {
        close_begin<T, SB>(uc.pin + (size_t)rhs * NVAL * NBMAX, uc.nbin, uc.gs + rhs, uc.s, cls);
        cx0 = paxis((unsigned)max(x0 - 2, 0), C.nx).idx[0];
        cy0 = paxis((unsigned)max(y0 - 2, 0), C.ny).idx[0];
        CX = paxis((unsigned)min(x0 + TX + 1, nx - 1), C.nx).idx[1] - cx0 + 1;
        const unsigned CY = paxis((unsigned)min(y0 + TY + 1, ny - 1), C.ny).idx[1] - cy0 + 1;
        CN = (int)(CX * CY);
        const size_t offc = rhs * ldc;
#pragma unroll
        for (int i = 0; i < UPC_E; ++i) {
            const int q = min((int)threadIdx.x + i * BLK, CN - 1);
            const unsigned qy = (unsigned)q / CX, qx = (unsigned)q - qy * CX;
            const size_t P = offc + (size_t)(cy0 + qy) * C.nx + cx0 + qx;
            xbq[i] = uc.xb[P];
#pragma unroll
            for (int q2 = 0; q2 < SB - 1; ++q2) ucq[i][q2] = uc.B.u[min(q2, uc.s - 1)][P];   // slots past s-1 unused
        }
    }
    Cx<T> bq[TILE_MAXE];
    T phq[TILE_MAXE];
    size_t pq[TILE_MAXE];
    bool okq[TILE_MAXE];
#pragma unroll
    for (int it = 0; it < TILE_PB; ++it) {
        okq[it] = locate2(threadIdx.x + it * BLK, pq[it]);
        bq[it] = b[off + pq[it]];
        phq[it] = F.phi[pq[it]];
    }
    // phase 1's first batch: coordinates and x_in loads ahead of the prologue
    size_t pp0[TILE_PB];
    bool ok0[TILE_PB], own0[TILE_PB];
    Cx<T> xl0[TILE_PB];
#pragma unroll
    for (int i = 0; i < TILE_PB; ++i) {
        const int q = threadIdx.x + i * BLK;
        const int qy = q / AX, qx = q - qy * AX;
        const int gx = x0 - 2 + qx, gy = y0 - 2 + qy;
        ok0[i] = q < AN && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        own0[i] = ok0[i] && qx >= 2 && qx < TX + 2 && qy >= 2 && qy < TY + 2;
        pp0[i] = ok0[i] ? (size_t)gy * nx + gx : pc;
        if (xi) xl0[i] = xi[pp0[i]];
    }
    if constexpr (FU) {
        if (!act) return;
        const int k = close_end<T, SB>(cls, uc.gs + rhs, uc.s, uc.tiny, sh, res, axc, arc);
        Cx<T> cxc[SB], crc[SB];
        coefs_to_T<T, SB>(k, axc, arc, cxc, crc);
#pragma unroll
        for (int i = 0; i < UPC_E; ++i) {
            const int q = threadIdx.x + i * BLK;
            Cx<T> v = xbq[i];
#pragma unroll
            for (int q2 = 0; q2 < SB - 1; ++q2)
                if (q2 < k) v = cfma(cxc[q2], ucq[i][q2], v);
            if (q < CN) lc[q] = v;
        }
        __syncthreads();
    }
#pragma unroll
    for (int b0 = 0; b0 < UP_MAXE; b0 += TILE_PB) {
        if (b0 * BLK >= AN) break;   // the same for every thread of the block
        PLoads2<T> pl[TILE_PB];
        Cx<T> xl[TILE_PB];
        size_t pp[TILE_PB];
        bool ok[TILE_PB], own[TILE_PB];
#pragma unroll
        for (int i = 0; i < TILE_PB; ++i) {
            if (b0 + i >= UP_MAXE) break;
            const int q = threadIdx.x + (b0 + i) * BLK;
            const int qy = q / AX, qx = q - qy * AX;
            int gx = x0 - 2 + qx, gy = y0 - 2 + qy;
            if (b0 == 0) {
                ok[i] = ok0[i];
                own[i] = own0[i];
            } else {
                ok[i] = q < AN && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
                own[i] = ok[i] && qx >= 2 && qx < TX + 2 && qy >= 2 && qy < TY + 2;
            }
            if (!ok[i]) gx = x0, gy = y0;
            pp[i] = (size_t)gy * nx + gx;
            if constexpr (FU)
                prolong_load2<T>(lc, gx, gy, C.nx, C.ny, pl[i], cx0, cy0, CX);
            else
                prolong_load2<T>(e, gx, gy, C.nx, C.ny, pl[i]);
        }
        if (xi) {
#pragma unroll
            for (int i = 0; i < TILE_PB; ++i)
                if (b0 + i < UP_MAXE) xl[i] = b0 == 0 ? xl0[i] : xi[pp[i]];
        }
        if (b0 == 0 && !act) return;
#pragma unroll
        for (int i = 0; i < TILE_PB; ++i) {
            if (b0 + i >= UP_MAXE) break;
            const int q = threadIdx.x + (b0 + i) * BLK;
            Cx<T> v = prolong_sum2<T>(pl[i]);
            if (xi) v = v + xl[i];
            if (own[i]) xout[off + pp[i]] = v;
            if (q < AN) lx[q] = ok[i] ? v : mkc<T>(0, 0);
        }
    }
    asm volatile("" ::: "memory");   // the table store stays after phase 1's loads
    if (tslot >= 0) ltab[tslot] = tzero ? mkc<T>(0, 0) : mkc<T>(tre, tim);
    __syncthreads();
    Cx<T> rq[TILE_MAXE];
#pragma unroll
    for (int b0 = 0; b0 < TILE_MAXE; b0 += TILE_PB) {
        if (b0 * BLK >= RN) break;
        if (b0 > 0) {
#pragma unroll
            for (int i = 0; i < TILE_PB; ++i) {
                const int it = b0 + i;
                if (it >= TILE_MAXE) break;
                okq[it] = locate2(threadIdx.x + it * BLK, pq[it]);
                bq[it] = b[off + pq[it]];
                phq[it] = F.phi[pq[it]];
            }
        }
#pragma unroll
        for (int i = 0; i < TILE_PB; ++i) {
            const int it = b0 + i;
            if (it >= TILE_MAXE) break;
            const int q = threadIdx.x + it * BLK;
            const int qy = q / RX, qx = q - qy * RX;
            const bool ok = okq[it];
            const int a = ok ? (qy + 1) * AX + qx + 1 : 2 * AX + 2;
            const int c = ok ? qx : 1, rr = ok ? qy : 1;
            Cx<T> d = ltab[1 * TAB_MAXD + c] + ltab[4 * TAB_MAXD + rr];
            sub_phi(d, F, phq[it]);
            Cx<T> ax = d * lx[a];
            ax = cfma(ltab[0 * TAB_MAXD + c], lx[a - 1], ax);
            ax = cfma(ltab[2 * TAB_MAXD + c], lx[a + 1], ax);
            ax = cfma(ltab[3 * TAB_MAXD + rr], lx[a - AX], ax);
            ax = cfma(ltab[5 * TAB_MAXD + rr], lx[a + AX], ax);
            const Cx<T> v = bq[it] - ax;
            if (ok && qx >= 1 && qx <= TX && qy >= 1 && qy <= TY) r[off + pq[it]] = v;
            rq[it] = ok ? v : mkc<T>(0, 0);
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < TILE_MAXE; ++it) {
        const int q = threadIdx.x + it * BLK;
        if (q >= RN) break;
        lx[q] = rq[it];
    }
    __syncthreads();
    zc acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = mkc(0.0, 0.0);
#pragma unroll
    for (int it = 0; it < TILE_MAXE; ++it) {
        if (it * BLK >= RN) break;   // the same for every thread of the block
        const int q = threadIdx.x + it * BLK;
        const int qy = q / RX, qx = q - qy * RX;
        if (q >= RN || qx < 1 || qx > TX || qy < 1 || qy > TY) continue;
        const Cx<T> uc = rq[it];
        Cx<T> d = ltab[1 * TAB_MAXD + qx] + ltab[4 * TAB_MAXD + qy];
        sub_phi(d, F, phq[it]);
        Cx<T> a = d * uc;
        a = cfma(ltab[0 * TAB_MAXD + qx], lx[q - 1], a);
        a = cfma(ltab[2 * TAB_MAXD + qx], lx[q + 1], a);
        a = cfma(ltab[3 * TAB_MAXD + qy], lx[q - RX], a);
        a = cfma(ltab[5 * TAB_MAXD + qy], lx[q + RX], a);
        w[off + pq[it]] = a;
        const zc wd = cvt<double>(a), ud = cvt<double>(uc);
        acc[0] = cjfma(ud, wd, acc[0]);
        acc[1].re += cabs2(ud);
        if (NA > 2) acc[NA - 1].re += cabs2(wd);
    }
    block_sum_last<NA>(acc, NA, sh, res);
    if (threadIdx.x < NA) pout[((size_t)rhs * NVAL + threadIdx.x) * NBMAX + t] = res[threadIdx.x];
}

// Down-path pass on one 2-D tile of the coarse level (see launch_down_tile).
// Prologue: the sweep's closing coefficients (as k_upd_r), with the loads of
// the first batch of phase 1, the coarse stencil tables of the tile (into
// shared memory) and phi of phase 3 already issued.  Phase 1: per fine point
// under the coarse tile and its one-point halo (fine nodes 2I .. 2I+2 of
// coarse unknown I), the Arnoldi residual r = sum cr_i u_i into shared memory
// (zero outside the fine level), and x (+)= sum cx_i u_i on the fine points the
// tile owns: 2X0 .. 2(X0+TX)-1 per axis, up to the last fine point for the
// tile at the far end.  Phase 1 goes in batches of TILE_PB points per thread
// whose loads are issued together (absent points clamped to the tile's first
// fine point).  Phase 2: bc = 2^-2 P^T r on the coarse tile and its halo into
// shared memory (zero outside the coarse level), the tile's points also to bc.
// Phase 3 (NA > 0): w_0 = A_c bc on the tile with <bc, w_0>, ||bc||^2 and
// (NA = 3) ||w_0||^2.
template <typename T, int SB, int NA>
__global__ __launch_bounds__(BLK) void k_down_tile(Cx<T> *__restrict__ x, int accumulate, Basis<T> B, int s,
                                                   LvlK<T> F, LvlK<T> C, Cx<T> *__restrict__ bc,
                                                   Cx<T> *__restrict__ wc, size_t ldf, size_t ldc,
                                                   const zc *__restrict__ pin, int nbin, GState *gsb, double tiny,
                                                   zc *__restrict__ pout, TileGeo tg, int ntile, const int *active)
{
    __shared__ zc sh[(BLK / 64) * (SB + 1)];
    __shared__ zc res[SB + 1];
    __shared__ zc ax[CSG_MAX_S], ar[CSG_MAX_S + 1];
    __shared__ Cx<T> lr[UP_MAXN];
    __shared__ Cx<T> lb[DN_MAXB];
    __shared__ Cx<T> ltab[6 * TAB_MAXD];   // coarse tables: x lower, diag, upper; y lower, diag, upper
    const int rhs = blockIdx.y;
    F = F.at(rhs);
    C = C.at(rhs);
    const int act = active[rhs];   // tested before the closing writes (reads below are harmless)
    const unsigned t = chunk_id(ntile);
    const unsigned tyi = t / tg.ntx, txi = t - tyi * tg.ntx;
    const int fnx = (int)F.nx, fny = (int)F.ny, cnx = (int)C.nx, cny = (int)C.ny;
    const int X0 = (int)(txi * tg.tx), Y0 = (int)(tyi * tg.ty);
    const int TX = min(X0 + (int)tg.tx, cnx) - X0, TY = min(Y0 + (int)tg.ty, cny) - Y0;
    const int FX = 2 * TX + 5, FN = FX * (2 * TY + 5);
    const int fx0 = 2 * X0 - 2, fy0 = 2 * Y0 - 2;
    const int ox1 = (X0 + TX == cnx) ? fnx : 2 * (X0 + TX), oy1 = (Y0 + TY == cny) ? fny : 2 * (Y0 + TY);
    const size_t offf = rhs * ldf, offc = rhs * ldc;
    const int BX = TX + 2, BN = BX * (TY + 2);
    CloseLoads<SB> cls;
    close_begin<T, SB>(pin + (size_t)rhs * NVAL * NBMAX, nbin, gsb + rhs, s, cls);
    // coarse tables of the tile's columns X0 .. X0+TX-1 and rows Y0 .. Y0+TY-1,
    // one entry per thread (stored to shared memory after the prologue)
    T tre = 0, tim = 0;
    int tslot = -1;
    if (NA > 0) {
        const int q = threadIdx.x;
        const bool xs = q < 3 * TX;
        const int qq = xs ? q : min(q - 3 * TX, 3 * TY - 1);
        const int c = qq / 3, a = qq - 3 * c;
        const Cx<T> *tab = xs ? C.tab[0] + a * cnx + X0 : C.tab[1] + a * cny + Y0;
        tre = tab[c].re;
        tim = tab[c].im;
        if (q < 3 * TX + 3 * TY) tslot = (xs ? a : 3 + a) * TAB_MAXD + c;
    }
    // phi of the coarse tile points of phase 3
    T phq[DN_MAXE];
    if (NA > 0) {
#pragma unroll
        for (int it = 0; it < DN_MAXE; ++it) {
            const int q = threadIdx.x + it * BLK;
            const int qy = q / BX, qx = q - qy * BX;
            const bool in = q < BN && qx >= 1 && qx <= TX && qy >= 1 && qy <= TY;
            phq[it] = C.phi[in ? (size_t)(Y0 - 1 + qy) * cnx + X0 - 1 + qx : (size_t)Y0 * cnx + X0];
        }
    }
    Cx<T> u[TILE_PB][SB], xv[TILE_PB];
    size_t pp[TILE_PB];
    bool ok[TILE_PB], own[TILE_PB];
    // basis slots 0..s; slots past s read slot s again (every load unconditional,
    // so the wait before the least squares leaves this batch in flight)
    const Cx<T> *bu[SB];
#pragma unroll
    for (int q2 = 0; q2 < SB; ++q2) bu[q2] = B.u[min(q2, s)];
    Cx<T> *const xw = x;
    // loads of the batch of phase 1 starting at b0 (x after the least squares
    // for the first batch: a sweep from zero never reads it)
    auto load_batch = [&](int b0, bool with_x) {
#pragma unroll
        for (int i = 0; i < TILE_PB; ++i) {
            if (b0 + i >= UP_MAXE) break;
            const int q = threadIdx.x + (b0 + i) * BLK;
            const int qy = q / FX, qx = q - qy * FX;
            int gx = fx0 + qx, gy = fy0 + qy;
            ok[i] = q < FN && gx >= 0 && gx < fnx && gy >= 0 && gy < fny;
            own[i] = ok[i] && gx >= 2 * X0 && gx < ox1 && gy >= 2 * Y0 && gy < oy1;
            if (!ok[i]) gx = 2 * X0, gy = 2 * Y0;
            pp[i] = offf + (size_t)gy * fnx + gx;
#pragma unroll
            for (int q2 = 0; q2 < SB; ++q2) u[i][q2] = bu[q2][pp[i]];
            xv[i] = mkc<T>(0, 0);
        }
        if (with_x && accumulate) {
#pragma unroll
            for (int i = 0; i < TILE_PB; ++i)
                if (b0 + i < UP_MAXE) xv[i] = xw[pp[i]];
        }
    };
    load_batch(0, false);
    if (!act) return;
    const int k = close_end<T, SB>(cls, gsb + rhs, s, tiny, sh, res, ax, ar);
    if (accumulate) {
#pragma unroll
        for (int i = 0; i < TILE_PB; ++i) xv[i] = xw[pp[i]];
    }
    Cx<T> cx[SB], cr[SB];
    coefs_to_T<T, SB>(k, ax, ar, cx, cr);
    if (tslot >= 0) ltab[tslot] = mkc<T>(tre, tim);
#pragma unroll
    for (int b0 = 0; b0 < UP_MAXE; b0 += TILE_PB) {
        if (b0 * BLK >= FN) break;   // the same for every thread of the block
        if (b0 > 0) load_batch(b0, true);
#pragma unroll
        for (int i = 0; i < TILE_PB; ++i) {
            if (b0 + i >= UP_MAXE) break;
            const int q = threadIdx.x + (b0 + i) * BLK;
            Cx<T> rr = mkc<T>(0, 0);
#pragma unroll
            for (int q2 = 0; q2 < SB; ++q2)
                if (q2 <= k) {
                    rr = cfma(cr[q2], u[i][q2], rr);
                    if (q2 < k) xv[i] = cfma(cx[q2], u[i][q2], xv[i]);
                }
            if (own[i]) xw[pp[i]] = xv[i];
            if (q < FN) lr[q] = ok[i] ? rr : mkc<T>(0, 0);
        }
    }
    __syncthreads();
    Cx<T> bq[DN_MAXE];
#pragma unroll
    for (int it = 0; it < DN_MAXE; ++it) {
        const int q = threadIdx.x + it * BLK;
        if (q >= BN) break;
        const int qy = q / BX, qx = q - qy * BX;
        const int I = X0 - 1 + qx, J = Y0 - 1 + qy;
        Cx<T> v = mkc<T>(0, 0);
        if (I >= 0 && I < cnx && J >= 0 && J < cny) {
            // fine nodes 2I + a, 2J + b sit at footprint offsets 2qx + a, 2qy + b
            const int f0 = 2 * qy * FX + 2 * qx;
            const int na = 2 * I + 2 < fnx ? 3 : (2 * I + 1 < fnx ? 2 : 1);
            const int nbb = 2 * J + 2 < fny ? 3 : (2 * J + 1 < fny ? 2 : 1);
            Cx<T> acc = mkc<T>(0, 0);
            for (int b2 = 0; b2 < nbb; ++b2)
                for (int a2 = 0; a2 < na; ++a2) acc = acc + (T)(rw(a2) * rw(b2)) * lr[f0 + b2 * FX + a2];
            v = (T)0.25 * acc;
            if (qx >= 1 && qx <= TX && qy >= 1 && qy <= TY) bc[offc + (size_t)J * cnx + I] = v;
        }
        bq[it] = v;
        lb[q] = v;
    }
    if constexpr (NA > 0) {
        __syncthreads();
        zc acc[NA];
#pragma unroll
        for (int q = 0; q < NA; ++q) acc[q] = mkc(0.0, 0.0);
#pragma unroll
        for (int it = 0; it < DN_MAXE; ++it) {
            const int q = threadIdx.x + it * BLK;
            if (q >= BN) break;
            const int qy = q / BX, qx = q - qy * BX;
            if (qx < 1 || qx > TX || qy < 1 || qy > TY) continue;
            const int c = qx - 1, r = qy - 1;
            const size_t p = (size_t)(Y0 + r) * cnx + X0 + c;
            const Cx<T> uc = bq[it];
            Cx<T> d = ltab[1 * TAB_MAXD + c] + ltab[4 * TAB_MAXD + r];
            sub_phi(d, C, phq[it]);
            Cx<T> a = d * uc;
            a = cfma(ltab[0 * TAB_MAXD + c], lb[q - 1], a);
            a = cfma(ltab[2 * TAB_MAXD + c], lb[q + 1], a);
            a = cfma(ltab[3 * TAB_MAXD + r], lb[q - BX], a);
            a = cfma(ltab[5 * TAB_MAXD + r], lb[q + BX], a);
            wc[offc + p] = a;
            const zc wd = cvt<double>(a), ud = cvt<double>(uc);
            acc[0] = cjfma(ud, wd, acc[0]);
            acc[1].re += cabs2(ud);
            if (NA > 2) acc[NA - 1].re += cabs2(wd);
        }
        block_sum_last<NA>(acc, NA, sh, res);
        if (threadIdx.x < NA) pout[((size_t)rhs * NVAL + threadIdx.x) * NBMAX + t] = res[threadIdx.x];
    }
}

template <typename T, int SB>
__global__ __launch_bounds__(BLK) void k_upd_r(Cx<T> *x, int accumulate, Cx<T> *r, Basis<T> B, int s, unsigned N,
                                               size_t ld, const zc *__restrict__ pin, int nbin, GState *gsb,
                                               double tiny, unsigned chunk, int nb, const int *active)
{
    __shared__ zc sh[(BLK / 64) * (SB + 1)];
    __shared__ zc res[SB + 1];
    __shared__ zc ax[CSG_MAX_S], ar[CSG_MAX_S + 1];
    const int rhs = blockIdx.y;
    if constexpr (SB <= 4) {
        // as k_upd: the first batch of points (u_0..u_s and x) is loaded
        // before the least squares, which runs while the loads are in flight
        constexpr int PB = TILE_PB;
        const int act = active[rhs];
        CloseLoads<SB> cls;
        close_begin<T, SB>(pin + (size_t)rhs * NVAL * NBMAX, nbin, gsb + rhs, s, cls);
        const unsigned c = chunk_id(nb);
        const unsigned p0 = c * chunk, p1 = min(N, p0 + chunk);
        const size_t off = rhs * ld;
        Cx<T> *xr = x + off, *rr = r + off;
        Cx<T> u[PB][SB], xv[PB];
        // every load unconditional (slots past s read slot s again; x read
        // and dropped when not accumulating)
        const Cx<T> *bu[SB];
#pragma unroll
        for (int q = 0; q < SB; ++q) bu[q] = B.u[min(q, s)] + off;
        auto load = [&](unsigned p) {
#pragma unroll
            for (int i = 0; i < PB; ++i) {
                const unsigned pk = min(p + i * BLK, N - 1);
#pragma unroll
                for (int q = 0; q < SB; ++q) u[i][q] = bu[q][pk];
                xv[i] = xr[pk];
            }
        };
        const unsigned pt = p0 + threadIdx.x;
        load(pt);
        if (!act) return;
        const int k = close_end<T, SB>(cls, gsb + rhs, s, tiny, sh, res, ax, ar);
        Cx<T> cx[SB], cr[SB];
        coefs_to_T<T, SB>(k, ax, ar, cx, cr);
        for (unsigned p = pt; p < p1; p += PB * BLK) {
            if (p != pt) load(p);
#pragma unroll
            for (int i = 0; i < PB; ++i) {
                Cx<T> v = accumulate ? xv[i] : mkc<T>(0, 0), rv = mkc<T>(0, 0);
#pragma unroll
                for (int q = 0; q < SB; ++q)
                    if (q <= k) {
                        rv = cfma(cr[q], u[i][q], rv);
                        if (q < k) v = cfma(cx[q], u[i][q], v);
                    }
                if (p + i * BLK < p1) {
                    xr[p + i * BLK] = v;
                    rr[p + i * BLK] = rv;
                }
            }
        }
    } else {
        if (!active[rhs]) return;
        const int k = close_sweep<T, SB>(pin + (size_t)rhs * NVAL * NBMAX, nbin, gsb + rhs, s, tiny, sh, res, ax, ar);
        Cx<T> cx[SB], cr[SB];
        coefs_to_T<T, SB>(k, ax, ar, cx, cr);
        const unsigned c = chunk_id(nb);
        const unsigned p0 = c * chunk, p1 = min(N, p0 + chunk);
        body_upd_r<T, SB>(x + rhs * ld, accumulate, r + rhs * ld, B, k, cx, cr, rhs * ld, p0 + threadIdx.x, p1, BLK);
    }
}

template <typename T, int DIM>
__global__ __launch_bounds__(BLK) void k_resid(LvlK<T> L, const Cx<T> *__restrict__ x, const Cx<T> *__restrict__ b,
                                               Cx<T> *__restrict__ r, size_t ld, unsigned chunk, int nb,
                                               const int *active)
{
    const int rhs = blockIdx.y;
    L = L.at(rhs);
    if (!active[rhs]) return;
    const size_t off = rhs * ld;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(L.N, p0 + chunk);
    body_resid<T, DIM>(L, x + off, b + off, r + off, p0 + threadIdx.x, p1, BLK);
}

template <typename T, int DIM>
__global__ __launch_bounds__(BLK) void k_restrict(LvlK<T> F, LvlK<T> C, const Cx<T> *__restrict__ x,
                                                  const Cx<T> *__restrict__ b, Cx<T> *__restrict__ bc, size_t ldf,
                                                  size_t ldc, unsigned chunk, int nb, const int *active)
{
    const int rhs = blockIdx.y;
    F = F.at(rhs);
    C = C.at(rhs);
    if (!active[rhs]) return;
    const size_t offf = rhs * ldf;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(C.N, p0 + chunk);
    body_restrict<T, DIM>(F, C, x ? x + offf : nullptr, b + offf, bc + rhs * ldc, p0 + threadIdx.x, p1, BLK);
}

template <typename T, int DIM>
__global__ __launch_bounds__(BLK) void k_prolong(LvlK<T> F, LvlK<T> C, const Cx<T> *ec, const Cx<T> *xin,
                                                 Cx<T> *xout, size_t ldf, size_t ldc, unsigned chunk, int nb,
                                                 const int *active)
{
    const int rhs = blockIdx.y;
    F = F.at(rhs);
    C = C.at(rhs);
    if (!active[rhs]) return;
    const size_t off = rhs * ldf;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(F.N, p0 + chunk);
    body_prolong<T, DIM>(F, C, ec + rhs * ldc, xin ? xin + off : nullptr, xout + off, p0 + threadIdx.x, p1, BLK);
}

template <typename T, int DIM>
__global__ __launch_bounds__(BLK) void k_prc(LvlK<T> F, LvlK<T> C, const Cx<T> *ec, const Cx<T> *xin, Cx<T> *xout,
                                             const Cx<T> *__restrict__ b, Cx<T> *__restrict__ r, size_t ldf,
                                             size_t ldc, unsigned chunk, int nb, const int *active)
{
    const int rhs = blockIdx.y;
    F = F.at(rhs);
    C = C.at(rhs);
    if (!active[rhs]) return;
    const size_t off = rhs * ldf;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk, p1 = min(F.N, p0 + chunk);
    body_prc<T, DIM>(F, C, ec + rhs * ldc, xin ? xin + off : nullptr, xout + off, b + off, r + off, p0 + threadIdx.x,
                     p1, BLK);
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_coarse(const Cx<T> *__restrict__ minvT, int n, const Cx<T> *__restrict__ b,
                                                Cx<T> *__restrict__ x, size_t ld, size_t mstride, unsigned rpp,
                                                const int *active)
{
    __shared__ Cx<T> part[BLK];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    if (rpp) minvT += (size_t)((unsigned)rhs / rpp) * mstride;
    body_coarse<T, BLK>(minvT, n, b + rhs * ld, x + rhs * ld, part);
}

// ---------------------------------------------------------------------------
// coarse tail: one workgroup per right-hand side runs every level from lt down
// to the coarsest and back (section 3.1 V-cycle), with __syncthreads between
// passes instead of kernel boundaries.  Same bodies and scalar logic as the
// multi-block passes; block-wide sums replace the partials.
// ---------------------------------------------------------------------------

constexpr int TB = 512;
constexpr int TW = TB / 64;

// sum of v[0..nv-1] over the workgroup, result in res (all threads see it)
template <int NV>
__device__ __forceinline__ void tail_sum(zc (&v)[NV], int nv, zc *sh, zc *res)
{
    wave_totals_to<NV>(v, nv, sh, threadIdx.x >> 6);
    __syncthreads();
    if (threadIdx.x < nv) {
        const int q = threadIdx.x;
        zc a = sh[q];
        for (int w = 1; w < TW; ++w) a = a + sh[w * NV + q];
        res[q] = a;
    }
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ LvlK<T> tlvl(const TLev<T> &d, int rhs)
{
    LvlK<T> L;
    for (int a = 0; a < 3; ++a) {
        L.tab[a] = d.tab[a];
        L.tstride[a] = d.tstride[a];
    }
    L.phi = d.phi;
    L.nx = d.nx;
    L.ny = d.ny;
    L.nz = d.nz;
    L.N = d.N;
    L.rpp = d.rpp;
    L.pstride = d.pstride;
    L.sre = d.sre;
    L.sim = d.sim;
    return L.at(rhs);
}

// Arnoldi passes of one sweep on the raw basis B (u_0 given), whole level;
// w0, w1 hold the stencil outputs (ping-pong), w_{s-1} ends in w[(s-1) % 2].
// As on the multi-block levels the last pass also sums ||w_{s-1}||^2 and
// h_{s,s-1} follows from ||A v_{s-1}||^2 = sum_i |h_{i,s-1}|^2 + h_{s,s-1}^2;
// fold[0..s-1] = cu_i and fold[s] = sig_{s-1} (u_s = fold[s] w_{s-1} -
// sum_i fold[i] u_i) are left for the closing pass.
template <typename T, int DIM, int SB>
__device__ void tail_steps(const LvlK<T> &L, const Basis<T> &B, Cx<T> *w0, Cx<T> *w1, size_t off, int s,
                           double tiny, GState *gs, zc *sh, zc *res, zc *fold)
{
    if (norm_from_sums<T>() && s == 1) {
        zc acc[3] = {mkc(0.0, 0.0), mkc(0.0, 0.0), mkc(0.0, 0.0)};
        body_st0<T, DIM, 3>(L, B.u[0] + off, w0 + off, threadIdx.x, L.N, TB, acc);
        tail_sum<3>(acc, 3, sh, res);
    } else {
        zc acc[2] = {mkc(0.0, 0.0), mkc(0.0, 0.0)};
        body_st0<T, DIM>(L, B.u[0] + off, w0 + off, threadIdx.x, L.N, TB, acc);
        tail_sum<2>(acc, 2, sh, res);
    }
    for (int j = 0; j < s; ++j) {
        Cx<T> cu[SB];
        const double sj = coef_step<T, SB>(res, j, s, tiny, load_prev<SB>(gs, j), gs, threadIdx.x == 0, cu);
        Cx<T> *win = (j & 1) ? w1 : w0;
        Cx<T> *wout = (j & 1) ? w0 : w1;
        if (j + 1 < s) {
            zc acc[SB + 1];
#pragma unroll
            for (int q = 0; q <= SB; ++q) acc[q] = mkc(0.0, 0.0);
            const bool wn = norm_from_sums<T>() && j + 2 == s;
            body_os<T, DIM, SB, SB + 1>(L, B, win, wout, j, (T)sj, cu, off, threadIdx.x, L.N, TB, acc, wn);
            tail_sum<SB + 1>(acc, j + 3 + (wn ? 1 : 0), sh, res);
        } else if constexpr (!norm_from_sums<T>()) {
            // explicit form: u_s and its norm
            zc nr[1] = {mkc(0.0, 0.0)};
            body_orthl<T, SB>(B, win + off, j, (T)sj, cu, off, threadIdx.x, L.N, TB, nr[0].re);
            tail_sum<1>(nr, 1, sh, res);
            if (threadIdx.x == 0) {
                const double hn = sqrt(res[0].re);
                const bool brk = !(hn > tiny * gs->beta0);
                gs->H[s * CSG_MAX_S + (s - 1)] = mkc(hn, 0.0);
                gs->sig[s] = brk ? 0.0 : 1.0 / hn;
            }
            __syncthreads();
        } else {
            if (threadIdx.x == 0) {
                // h_{s,s-1} (a difference at rounding level of ||A v_{s-1}||^2:
                // A v_{s-1} lies in the basis span), the scale of u_s, the breakdown test
                const double w2 = sj * sj * res[s + 1].re;
                double h2 = w2;
                for (int i = 0; i < s; ++i) h2 -= cabs2(gs->H[i * CSG_MAX_S + (s - 1)]);
                const double hn = h2 > 1e-13 * w2 ? sqrt(h2) : 0.0;
                const bool brk = !(hn > tiny * gs->beta0);
                gs->H[s * CSG_MAX_S + (s - 1)] = mkc(hn, 0.0);
                gs->sig[s] = brk ? 0.0 : 1.0 / hn;
#pragma unroll
                for (int i = 0; i < SB; ++i)
                    if (i < s) fold[i] = cvt<double>(cu[i]);
                fold[s] = mkc(sj, 0.0);
            }
            __syncthreads();
        }
    }
}

// Least squares of the sweep (thread 0) -> coefficients for every thread; the
// residual coefficients are those on {u_0..u_{s-1}, w_{s-1}} (u_s folded in).
template <typename T, int SB>
__device__ __forceinline__ int tail_close(const GState *gs, int s, zc *Rs, zc *ys, zc *crs, zc *ax, zc *ar, int *ks, const zc *fold,
                          Cx<T> (&cx)[SB], Cx<T> (&cr)[SB])
{
    if (SB <= 4 && threadIdx.x == 0) {
        // register copy of Hbar (s <= 3), the same arithmetic as gmres_ls
        constexpr int K = SB - 1;
        zc H[SB][K];
#pragma unroll
        for (int r = 0; r < SB; ++r)
#pragma unroll
            for (int c = 0; c < K; ++c) H[r][c] = (c < s && r <= c + 1) ? gs->H[r * CSG_MAX_S + c] : mkc(0.0, 0.0);
        const double beta0 = gs->beta0;
        int k = gs->k;
        if (k > s) k = s;
        if (!(beta0 > 0.0)) k = 0;
        zc yl[K];
        ls_regs<SB>(H, beta0, k, yl);
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (i < k) ax[i] = gs->sig[i] * yl[i];
#pragma unroll
        for (int i = 0; i < SB; ++i) {
            zc acc = (i == 0) ? mkc(beta0, 0.0) : mkc(0.0, 0.0);
#pragma unroll
            for (int c = 0; c < K; ++c)
                if (c < k && i <= c + 1) acc = acc - H[i][c] * yl[c];
            if (i <= k) ar[i] = gs->sig[i] * acc;
        }
        if (norm_from_sums<T>() && k == s) {
            const zc as = ar[s];
            for (int i = 0; i < s; ++i) ar[i] = ar[i] - as * fold[i];
            ar[s] = fold[s].re * as;
        }
        *ks = k;
    } else if (threadIdx.x == 0) {
        const double hn = gs->H[s * CSG_MAX_S + (s - 1)].re;
        const int k = gmres_ls<SB>(gs, s, hn, Rs, ys, crs);
        for (int i = 0; i < k; ++i) ax[i] = gs->sig[i] * ys[i];
        for (int i = 0; i <= k; ++i) ar[i] = gs->sig[i] * crs[i];
        if (norm_from_sums<T>() && k == s) {
            const zc as = ar[s];
            for (int i = 0; i < s; ++i) ar[i] = ar[i] - as * fold[i];
            ar[s] = fold[s].re * as;
        }
        *ks = k;
    }
    __syncthreads();
    const int k = *ks;
    coefs_to_T<T, SB>(k, ax, ar, cx, cr);
    return k;
}

// --- register stencils of the shared-memory tail -----------------------------
// The points a thread owns on a tail level are p = t + k TB, k < MP; their
// stencils are loaded once per visit of the level: the diagonal (centre table
// entries minus phi) and the neighbour weights in the order apply_pt adds
// them, with the neighbours' indices (clamped to the point itself at the
// level's edge, where the weight is zero).  Every stencil application of the
// visit then reads only shared memory.
template <typename T>
constexpr int tail_mp()
{
    return sizeof(T) == 8 ? 3 : 5;
}
template <typename T, int DIM, int MP>
struct TSten {
    Cx<T> d[MP], c[MP][2 * DIM];
    unsigned nb[MP][2 * DIM];
};

template <typename T, int DIM, int MP>
__device__ __forceinline__ void tsten_load(const LvlK<T> &L, TSten<T, DIM, MP> &S)
{
#pragma unroll
    for (int k = 0; k < MP; ++k) {
        const unsigned p = min(threadIdx.x + k * TB, L.N - 1);
        unsigned i, j, kk;
        decomp<DIM>(p, L.nx, L.ny, i, j, kk);
        const Cx<T> *tx = L.tab[0];
        Cx<T> d = tx[L.nx + i];
        if (DIM >= 2) d = d + L.tab[1][L.ny + j];
        if (DIM == 3) d = d + L.tab[2][L.nz + kk];
        sub_phi(d, L, L.phi[p]);
        S.d[k] = d;
        S.c[k][0] = tx[i];
        S.nb[k][0] = i ? p - 1 : p;
        S.c[k][1] = tx[2 * L.nx + i];
        S.nb[k][1] = i + 1 < L.nx ? p + 1 : p;
        if (DIM >= 2) {
            S.c[k][2] = L.tab[1][j];
            S.nb[k][2] = j ? p - L.nx : p;
            S.c[k][3] = L.tab[1][2 * L.ny + j];
            S.nb[k][3] = j + 1 < L.ny ? p + L.nx : p;
        }
        if (DIM == 3) {
            const unsigned sz = L.nx * L.ny;
            S.c[k][4] = L.tab[2][kk];
            S.nb[k][4] = kk ? p - sz : p;
            S.c[k][5] = L.tab[2][2 * L.nz + kk];
            S.nb[k][5] = kk + 1 < L.nz ? p + sz : p;
        }
    }
}

// (A x)(p) for the thread's k-th point p, x in shared memory
template <typename T, int DIM, int MP>
__device__ __forceinline__ Cx<T> tsten_apply(const TSten<T, DIM, MP> &S, int k, const Cx<T> *x, unsigned p)
{
    Cx<T> a = S.d[k] * x[p];
#pragma unroll
    for (int m = 0; m < 2 * DIM; ++m) a = cfma(S.c[k][m], x[S.nb[k][m]], a);
    return a;
}

// pass 0 (as body_st0)
template <typename T, int DIM, int MP, int NA>
__device__ __forceinline__ void tsten_st0(const TSten<T, DIM, MP> &S, const Cx<T> *u0, Cx<T> *w, unsigned N,
                                          zc (&acc)[NA])
{
#pragma unroll
    for (int k = 0; k < MP; ++k) {
        const unsigned p = threadIdx.x + k * TB;
        if (p >= N) break;
        const Cx<T> wv = tsten_apply(S, k, u0, p);
        w[p] = wv;
        const zc wd = cvt<double>(wv), ud = cvt<double>(u0[p]);
        acc[0] = cjfma(ud, wd, acc[0]);
        acc[1].re += cabs2(ud);
        if (NA > 2) acc[NA - 1].re += cabs2(wd);
    }
}

// r = b - A x
template <typename T, int DIM, int MP>
__device__ __forceinline__ void tsten_resid(const TSten<T, DIM, MP> &S, const Cx<T> *x, const Cx<T> *b, Cx<T> *r,
                                            unsigned N)
{
#pragma unroll
    for (int k = 0; k < MP; ++k) {
        const unsigned p = threadIdx.x + k * TB;
        if (p >= N) break;
        r[p] = b[p] - tsten_apply(S, k, x, p);
    }
}

// pass j+1 (as body_os): u_{j+1} at the thread's points into B.u[j+1], then,
// after a barrier, w_{j+1} = A u_{j+1} from there, with the same sums
template <typename T, int DIM, int SB, int MP, int NA>
__device__ __forceinline__ void tsten_os(const TSten<T, DIM, MP> &S, const Basis<T> &B, Cx<T> *un,
                                         const Cx<T> *win, Cx<T> *wout, int j, T sj, const Cx<T> (&cu)[SB],
                                         unsigned N, zc (&acc)[NA], bool wn)
{
    Cx<T> uq[MP][SB - 1], uc[MP];
#pragma unroll
    for (int k = 0; k < MP; ++k) {
        const unsigned p = min(threadIdx.x + k * TB, N - 1);
        uc[k] = sj * win[p];
#pragma unroll
        for (int q = 0; q < SB - 1; ++q)
            if (q <= j) {
                uq[k][q] = B.u[q][p];
                uc[k] = uc[k] - cu[q] * uq[k][q];
            }
        if (threadIdx.x + k * TB < N) un[p] = uc[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < MP; ++k) {
        const unsigned p = threadIdx.x + k * TB;
        if (p >= N) break;
        const Cx<T> a = tsten_apply(S, k, un, p);
        wout[p] = a;
        const zc wd = cvt<double>(a), ud = cvt<double>(uc[k]);
#pragma unroll
        for (int q = 0; q < SB - 1; ++q)
            if (q <= j) acc[q] = cjfma(cvt<double>(uq[k][q]), wd, acc[q]);
#pragma unroll
        for (int q = 1; q < SB; ++q) {
            if (q == j + 1) acc[q] = cjfma(ud, wd, acc[q]);
            if (q == j + 2) acc[q].re += cabs2(ud);
        }
        if (wn) {
#pragma unroll
            for (int q = 3; q < NA; ++q)
                if (q == j + 3) acc[q].re += cabs2(wd);
        }
    }
}

// Closing pass of the last pre-smoothing sweep on a shared-memory tail level,
// then the restriction (as body_upd_res, in two phases): each thread forms
// the Arnoldi residual r = sum_i cr_i u_i at its own fine points into rbuf
// (a stencil output the closing does not read) and updates x there; after a
// barrier, bc = 2^-d P^T r per coarse point from rbuf.  Every fine value is
// formed once instead of once per coarse footprint that covers it; the sums
// are the same, in the same order.
template <typename T, int DIM, int SB, int MP>
__device__ __forceinline__ void tail_upd_res(Cx<T> *xx, int accumulate, const Basis<T> &B, int k,
                                             const Cx<T> (&cx)[SB], const Cx<T> (&cr)[SB], const LvlK<T> &F,
                                             const LvlK<T> &C, Cx<T> *rbuf, Cx<T> *bb)
{
#pragma unroll
    for (int kk = 0; kk < MP; ++kk) {
        const unsigned p = threadIdx.x + kk * TB;
        if (p >= F.N) break;
        Cx<T> uv[SB];
#pragma unroll
        for (int q = 0; q < SB; ++q)
            if (q <= k) uv[q] = B.u[q][p];
        Cx<T> r = mkc<T>(0, 0);
#pragma unroll
        for (int q = 0; q < SB; ++q)
            if (q <= k) r = cfma(cr[q], uv[q], r);
        rbuf[p] = r;
        Cx<T> v = accumulate ? xx[p] : mkc<T>(0, 0);
#pragma unroll
        for (int q = 0; q < SB - 1; ++q)
            if (q < k) v = cfma(cx[q], uv[q], v);
        xx[p] = v;
    }
    __syncthreads();
    const T scale = (DIM == 2) ? (T)0.25 : (T)0.125;
    for (unsigned pc = threadIdx.x; pc < C.N; pc += TB) {
        unsigned I, J, K;
        decomp<DIM>(pc, C.nx, C.ny, I, J, K);
        const RAx rx = raxis(I, C.nx, F.nx);
        const RAx ry = raxis(J, C.ny, F.ny);
        const RAx rz = (DIM == 3) ? raxis(K, C.nz, F.nz) : RAx{0, 1, 1};
        Cx<T> acc = mkc<T>(0, 0);
#pragma unroll
        for (int qz = 0; qz < (DIM == 3 ? 3 : 1); ++qz)
#pragma unroll
            for (int qy = 0; qy < 3; ++qy)
#pragma unroll
                for (int qx = 0; qx < 3; ++qx) {
                    if (qz >= rz.n || qy >= ry.n || qx >= rx.n) continue;
                    const unsigned fp = ((rz.lo + qz) * F.ny + (ry.lo + qy)) * F.nx + (rx.lo + qx);
                    T wgt = (T)(rw(qx) * rw(qy));
                    if (DIM == 3) wgt *= (T)rw(qz);
                    acc = acc + wgt * rbuf[fp];
                }
        bb[pc] = scale * acc;
    }
}

// tail_steps on one shared-memory level with its register stencils
template <typename T, int DIM, int SB, int MP>
__device__ __forceinline__ void tsten_steps(const TSten<T, DIM, MP> &S, unsigned N, const Basis<T> &B, Cx<T> *u1,
                                            Cx<T> *w0, Cx<T> *w1, int s,
                            double tiny, GState *gs, zc *sh, zc *res, zc *fold)
{
    if (norm_from_sums<T>() && s == 1) {
        zc acc[3] = {mkc(0.0, 0.0), mkc(0.0, 0.0), mkc(0.0, 0.0)};
        tsten_st0<T, DIM, MP, 3>(S, B.u[0], w0, N, acc);
        tail_sum<3>(acc, 3, sh, res);
    } else {
        zc acc[2] = {mkc(0.0, 0.0), mkc(0.0, 0.0)};
        tsten_st0<T, DIM, MP, 2>(S, B.u[0], w0, N, acc);
        tail_sum<2>(acc, 2, sh, res);
    }
    for (int j = 0; j < s; ++j) {
        Cx<T> cu[SB];
        const double sj = coef_step<T, SB>(res, j, s, tiny, load_prev<SB>(gs, j), gs, threadIdx.x == 0, cu);
        Cx<T> *win = (j & 1) ? w1 : w0;
        Cx<T> *wout = (j & 1) ? w0 : w1;
        if (j + 1 < s) {
            zc acc[SB + 1];
#pragma unroll
            for (int q = 0; q <= SB; ++q) acc[q] = mkc(0.0, 0.0);
            const bool wn = norm_from_sums<T>() && j + 2 == s;
            // u_{j+1} at u1 + j N: an offset from a shared-memory base rather than
            // a pick among the basis pointers (which the compiler turns into an
            // indexed table in scratch memory, and flat accesses behind it)
            tsten_os<T, DIM, SB, MP, SB + 1>(S, B, u1 + (size_t)j * N, win, wout, j, (T)sj, cu, N, acc, wn);
            tail_sum<SB + 1>(acc, j + 3 + (wn ? 1 : 0), sh, res);
        } else if constexpr (!norm_from_sums<T>()) {
            // explicit form: u_s and its norm
            zc nr[1] = {mkc(0.0, 0.0)};
            body_orthl<T, SB>(B, win, j, (T)sj, cu, 0, threadIdx.x, N, TB, nr[0].re);
            tail_sum<1>(nr, 1, sh, res);
            if (threadIdx.x == 0) {
                const double hn = sqrt(res[0].re);
                const bool brk = !(hn > tiny * gs->beta0);
                gs->H[s * CSG_MAX_S + (s - 1)] = mkc(hn, 0.0);
                gs->sig[s] = brk ? 0.0 : 1.0 / hn;
            }
            __syncthreads();
        } else {
            if (threadIdx.x == 0) {
                // h_{s,s-1} (a difference at rounding level of ||A v_{s-1}||^2:
                // A v_{s-1} lies in the basis span), the scale of u_s, the breakdown test
                const double w2 = sj * sj * res[s + 1].re;
                double h2 = w2;
                for (int i = 0; i < s; ++i) h2 -= cabs2(gs->H[i * CSG_MAX_S + (s - 1)]);
                const double hn = h2 > 1e-13 * w2 ? sqrt(h2) : 0.0;
                const bool brk = !(hn > tiny * gs->beta0);
                gs->H[s * CSG_MAX_S + (s - 1)] = mkc(hn, 0.0);
                gs->sig[s] = brk ? 0.0 : 1.0 / hn;
#pragma unroll
                for (int i = 0; i < SB; ++i)
                    if (i < s) fold[i] = cvt<double>(cu[i]);
                fold[s] = mkc(sj, 0.0);
            }
            // no barrier: only thread 0 reads these, in the closing least
            // squares that follows, whose own barrier publishes its results
        }
    }
}

// Vectors of one level of the shared-memory tail: [b | x | u_0 .. | w_0 | w_1],
// N elements each (the coarsest level uses b and x only).
template <typename T>
struct LdsLev {
    Cx<T> *b, *x, *u[CSG_MAX_S + 1], *w[2];
};

// Elements of one tail level's block: b, x, the basis (u_0..u_{s-1}, and u_s
// when the sweep forms it) and the two stencil outputs.
template <typename T>
__host__ __device__ __forceinline__ int tail_vectors(int s)
{
    return 2 + s + (norm_from_sums<T>() ? 0 : 1) + 2;
}

// The coarse tail with every level's vectors in shared memory: the top
// level's b is copied in once, its x out once; tables, phi and the coarsest
// inverse stay in global memory (read-only).  Same passes as k_tail, except
// that the interpolated correction is applied in place and the residual that
// opens the post-sweep is a separate pass (no second x buffer).
template <typename T, int DIM, int SB>
__global__ __launch_bounds__(TB) void k_tail_lds(const TLev<T> *__restrict__ lev, int lt, int L, const Cx<T> *b_in,
                                                 Cx<T> *x_out, const Cx<T> *__restrict__ minvT, int nc, int s,
                                                 int nu1, int nu2, double tiny, size_t mstride, const int *active)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ GState gs;
    __shared__ zc sh[TW * NVAL];
    __shared__ zc res[NVAL];
    __shared__ zc Rs[(CSG_MAX_S + 1) * CSG_MAX_S], ys[CSG_MAX_S], crs[CSG_MAX_S + 1], ax[CSG_MAX_S],
        ar[CSG_MAX_S + 1];
    __shared__ int ks;
    __shared__ zc fold[CSG_MAX_S + 1];
    const int rhs = blockIdx.x;
    if (lev[0].rpp) minvT += (size_t)((unsigned)rhs / lev[0].rpp) * mstride;
    if (!active[rhs]) return;
    const int t = threadIdx.x;
    const int nv = tail_vectors<T>(s);
    const int nbas = nv - 4;   // basis vectors kept
    auto level = [&](int l) {
        size_t o = 0;
        for (int k = lt; k < l; ++k) o += (size_t)nv * lev[k].N;
        Cx<T> *p = reinterpret_cast<Cx<T> *>(smem) + o;
        const size_t N = lev[l].N;
        LdsLev<T> v;
        v.b = p;
        v.x = p + N;
        for (int q = 0; q <= CSG_MAX_S; ++q) v.u[q] = q < nbas ? p + (2 + q) * N : nullptr;
        v.w[0] = p + (2 + nbas) * N;
        v.w[1] = p + (3 + nbas) * N;
        return v;
    };
    {
        const LdsLev<T> top = level(lt);
        const Cx<T> *src = b_in + rhs * lev[lt].ld;
        for (unsigned p = t; p < lev[lt].N; p += TB) top.b[p] = src[p];
        __syncthreads();
    }
    constexpr int MP = tail_mp<T>();
    TSten<T, DIM, MP> S;
    // down: pre-smoothing and restriction
    for (int l = lt; l < L - 1; ++l) {
        const LvlK<T> F = tlvl(lev[l], rhs), C = tlvl(lev[l + 1], rhs);
        const LdsLev<T> f = level(l), c = level(l + 1);
        if (nu1 > 0) tsten_load<T, DIM, MP>(F, S);
        if (nu1 == 0) {
            body_restrict<T, DIM>(F, C, nullptr, f.b, c.b, t, C.N, TB);
            __syncthreads();
            continue;
        }
        Basis<T> B;
        for (int q = 0; q <= CSG_MAX_S; ++q) B.u[q] = f.u[q];
        if (norm_from_sums<T>()) place(B, s, ((s - 1) & 1) ? f.w[1] : f.w[0]);   // closing combines w_{s-1} in place of u_s
        for (int k = 0; k < nu1; ++k) {
            if (k == 0) {
                B.u[0] = f.b;
            } else {
                tsten_resid<T, DIM, MP>(S, f.x, f.b, f.u[0], F.N);
                __syncthreads();
                B.u[0] = f.u[0];
            }
            tsten_steps<T, DIM, SB, MP>(S, F.N, B, f.u[1], f.w[0], f.w[1], s, tiny, &gs, sh, res, fold);
            Cx<T> cx[SB], cr[SB];
            const int kk = tail_close<T, SB>(&gs, s, Rs, ys, crs, ax, ar, &ks, fold, cx, cr);
            if (k == nu1 - 1)
                tail_upd_res<T, DIM, SB, MP>(f.x, k > 0, B, kk, cx, cr, F, C, (s & 1) ? f.w[1] : f.w[0], c.b);
            else
                body_upd<T, SB>(f.x, k > 0, B, kk, cx, 0, t, F.N, TB);
            __syncthreads();
        }
    }
    // coarsest level: exact solve (partials in the top level's idle scratch
    // vectors, or past the coarsest block when those are too short)
    {
        const LdsLev<T> c = level(L - 1);
        const bool inside = lt < L - 1 && (size_t)(nv - 2) * lev[lt].N >= TB;
        Cx<T> *cpart = inside ? level(lt).u[0] : c.x + lev[L - 1].N;
        body_coarse<T, TB>(minvT, nc, c.b, c.x, cpart);
        __syncthreads();
    }
    // up: interpolated correction (in place) and post-smoothing
    for (int l = L - 2; l >= lt; --l) {
        const LvlK<T> F = tlvl(lev[l], rhs), C = tlvl(lev[l + 1], rhs);
        const LdsLev<T> f = level(l), c = level(l + 1);
        // the last pre-smoothed level's stencils are still in S
        if (nu2 > 0 && !(l == L - 2 && nu1 > 0)) tsten_load<T, DIM, MP>(F, S);
        body_prolong<T, DIM>(F, C, c.x, nu1 > 0 ? f.x : nullptr, f.x, t, F.N, TB);
        __syncthreads();
        if (nu2 == 0) continue;
        Basis<T> B;
        for (int q = 0; q <= CSG_MAX_S; ++q) B.u[q] = f.u[q];
        if (norm_from_sums<T>()) place(B, s, ((s - 1) & 1) ? f.w[1] : f.w[0]);
        for (int k = 0; k < nu2; ++k) {
            tsten_resid<T, DIM, MP>(S, f.x, f.b, f.u[0], F.N);
            __syncthreads();
            tsten_steps<T, DIM, SB, MP>(S, F.N, B, f.u[1], f.w[0], f.w[1], s, tiny, &gs, sh, res, fold);
            Cx<T> cx[SB], cr[SB];
            const int kk = tail_close<T, SB>(&gs, s, Rs, ys, crs, ax, ar, &ks, fold, cx, cr);
            body_upd<T, SB>(f.x, 1, B, kk, cx, 0, t, F.N, TB);
            __syncthreads();
        }
    }
    {
        const LdsLev<T> top = level(lt);
        Cx<T> *dst = x_out + rhs * lev[lt].ld;
        for (unsigned p = t; p < lev[lt].N; p += TB) dst[p] = top.x[p];
    }
}

template <typename T, int DIM, int SB>
__global__ __launch_bounds__(TB) void k_tail(const TLev<T> *__restrict__ lev, int lt, int L, const Cx<T> *b_in,
                                             Cx<T> *x_out, const Cx<T> *__restrict__ minvT, int nc, int s, int nu1,
                                             int nu2, double tiny, size_t mstride, const int *active)
{
    __shared__ GState gs;
    __shared__ zc sh[TW * NVAL];
    __shared__ zc res[NVAL];
    __shared__ zc Rs[(CSG_MAX_S + 1) * CSG_MAX_S], ys[CSG_MAX_S], crs[CSG_MAX_S + 1], ax[CSG_MAX_S],
        ar[CSG_MAX_S + 1];
    __shared__ int ks;
    __shared__ zc fold[CSG_MAX_S + 1];
    __shared__ Cx<T> cpart[TB];
    const int rhs = blockIdx.x;
    if (lev[0].rpp) minvT += (size_t)((unsigned)rhs / lev[0].rpp) * mstride;
    if (!active[rhs]) return;
    const int t = threadIdx.x;

    // down: pre-smoothing and restriction
    for (int l = lt; l < L - 1; ++l) {
        const TLev<T> &Fd = lev[l];
        const TLev<T> &Cd = lev[l + 1];
        const LvlK<T> F = tlvl(Fd, rhs), C = tlvl(Cd, rhs);
        const size_t offf = rhs * Fd.ld, offc = rhs * Cd.ld;
        const Cx<T> *b = (l == lt ? b_in : Fd.b) + offf;
        if (nu1 == 0) {
            body_restrict<T, DIM>(F, C, nullptr, b, Cd.b + offc, t, C.N, TB);
            __syncthreads();
            continue;
        }
        Basis<T> B;
        for (int q = 0; q <= CSG_MAX_S; ++q) B.u[q] = Fd.u[q];
        if (norm_from_sums<T>()) place(B, s, ((s - 1) & 1) ? Fd.w[1] : Fd.w[0]);   // closing combines w_{s-1} in place of u_s
        for (int k = 0; k < nu1; ++k) {
            if (k == 0) {
                B.u[0] = const_cast<Cx<T> *>(b) - offf;
            } else {
                body_resid<T, DIM>(F, Fd.xa + offf, b, Fd.r + offf, t, F.N, TB);
                __syncthreads();
                B.u[0] = Fd.r;
            }
            tail_steps<T, DIM, SB>(F, B, Fd.w[0], Fd.w[1], offf, s, tiny, &gs, sh, res, fold);
            Cx<T> cx[SB], cr[SB];
            const int kk = tail_close<T, SB>(&gs, s, Rs, ys, crs, ax, ar, &ks, fold, cx, cr);
            if (k == nu1 - 1)
                body_upd_res<T, DIM, SB>(Fd.xa + offf, k > 0, B, kk, cx, cr, F, C, Cd.b + offc, offf, t, C.N, TB);
            else
                body_upd<T, SB>(Fd.xa + offf, k > 0, B, kk, cx, offf, t, F.N, TB);
            __syncthreads();
        }
    }
    // coarsest level: exact solve
    {
        const TLev<T> &Cd = lev[L - 1];
        const size_t off = rhs * Cd.ld;
        const Cx<T> *b = (lt == L - 1 ? b_in : Cd.b) + off;
        Cx<T> *x = (lt == L - 1 ? x_out : Cd.xb) + off;
        body_coarse<T, TB>(minvT, nc, b, x, cpart);
        __syncthreads();
    }
    // up: interpolated correction and post-smoothing
    for (int l = L - 2; l >= lt; --l) {
        const TLev<T> &Fd = lev[l];
        const TLev<T> &Cd = lev[l + 1];
        const LvlK<T> F = tlvl(Fd, rhs), C = tlvl(Cd, rhs);
        const size_t offf = rhs * Fd.ld, offc = rhs * Cd.ld;
        const Cx<T> *b = (l == lt ? b_in : Fd.b) + offf;
        Cx<T> *x = (l == lt ? x_out : Fd.xb) + offf;
        const Cx<T> *xi = nu1 > 0 ? Fd.xa + offf : nullptr;
        const Cx<T> *ec = Cd.xb + offc;
        if (nu2 == 0) {
            body_prolong<T, DIM>(F, C, ec, xi, x, t, F.N, TB);
            __syncthreads();
            continue;
        }
        body_prc<T, DIM>(F, C, ec, xi, x, b, Fd.r + offf, t, F.N, TB);
        __syncthreads();
        Basis<T> B;
        for (int q = 0; q <= CSG_MAX_S; ++q) B.u[q] = Fd.u[q];
        B.u[0] = Fd.r;
        if (norm_from_sums<T>()) place(B, s, ((s - 1) & 1) ? Fd.w[1] : Fd.w[0]);
        for (int k = 0; k < nu2; ++k) {
            if (k > 0) {
                body_resid<T, DIM>(F, x, b, Fd.r + offf, t, F.N, TB);
                __syncthreads();
            }
            tail_steps<T, DIM, SB>(F, B, Fd.w[0], Fd.w[1], offf, s, tiny, &gs, sh, res, fold);
            Cx<T> cx[SB], cr[SB];
            const int kk = tail_close<T, SB>(&gs, s, Rs, ys, crs, ax, ar, &ks, fold, cx, cr);
            body_upd<T, SB>(x, 1, B, kk, cx, offf, t, F.N, TB);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// outer flexible GMRES passes (FP64)
//
// Orthogonalisation is classical Gram-Schmidt applied twice (CGS2): with a good
// preconditioner H z_j is close to v_j, the first projection cancels most of
// w, and a second round restores orthogonality to working precision.
// Inner products over many basis vectors are taken in groups of 8 so a thread
// holds 8 accumulators, re-reading its chunk of w from cache per group.
// ---------------------------------------------------------------------------

// Points a thread handles per iteration in the outer passes (loads of all of
// them issued before any use; indices clamped, stores masked).  Per-thread
// accumulation still visits points in increasing order.
constexpr int UO = 4;

// acc[q] += <v_{8g+q}, w> over points p0, p0+BLK, ... < p1 (q with 8g+q <= j)
__device__ __forceinline__ void dots8(const zc *w, const zc *V, size_t vstride, int g, int j, size_t off, unsigned p0,
                                      unsigned p1, zc (&acc)[8])
{
    if (p0 >= p1) return;
    const unsigned last = p1 - 1;
    for (unsigned p = p0; p < p1; p += UO * BLK) {
        zc wv[UO], vv[UO][8];
#pragma unroll
        for (int k = 0; k < UO; ++k) {
            const unsigned pk = min(p + k * BLK, last);
            wv[k] = w[off + pk];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (8 * g + q <= j) vv[k][q] = V[(8 * g + q) * vstride + off + pk];
        }
#pragma unroll
        for (int k = 0; k < UO; ++k) {
            if (p + k * BLK >= p1) break;
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (8 * g + q <= j) acc[q] = cjfma(vv[k][q], wv[k], acc[q]);
        }
    }
}

// block total of group g's accumulators into the partials of values 8g..8g+7
__device__ __forceinline__ void store_group(zc (&acc)[8], int g, int j, zc *pout, unsigned c, zc *sh, zc *res)
{
    block_sum<8>(acc, 8, sh, res);
    if (threadIdx.x < 8 && 8 * g + (int)threadIdx.x <= j) pout[(8 * g + threadIdx.x) * NBMAX + c] = res[threadIdx.x];
}

// w = H z and the first-round inner products <v_i, w>, i <= j: the first group
// of 8 is accumulated while w is formed, later groups re-read w.
template <typename TZ, int DIM>
__global__ __launch_bounds__(BLK) void k_hdot(LvlK<double> H, const Cx<TZ> *__restrict__ z, zc *__restrict__ w,
                                              const zc *__restrict__ V, size_t vstride, int j, size_t ld,
                                              zc *__restrict__ pout, unsigned chunk, int nb, const int *active)
{
    constexpr int UH = 2;
    __shared__ zc sh[(BLK / 64) * 8];
    __shared__ zc res[8];
    const int rhs = blockIdx.y;
    H = H.at(rhs);
    if (!active[rhs]) return;
    const size_t off = rhs * ld;
    zc *po = pout + (size_t)rhs * OVAL * NBMAX;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk + threadIdx.x, p1 = min(H.N, c * chunk + chunk);
    zc acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = mkc(0.0, 0.0);
    zc wn[1] = {mkc(0.0, 0.0)};
    if (p0 < p1) {
        const unsigned last = p1 - 1;
        for (unsigned p = p0; p < p1; p += UH * BLK) {
            zc wv[UH], vv[UH][8];
#pragma unroll
            for (int k = 0; k < UH; ++k) {
                const unsigned pk = min(p + k * BLK, last);
                unsigned i, jj, kk;
                decomp<DIM>(pk, H.nx, H.ny, i, jj, kk);
                wv[k] = apply_pt<double, DIM>(H, z + off, i, jj, kk, pk);
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (q <= j) vv[k][q] = V[q * vstride + off + pk];
            }
#pragma unroll
            for (int k = 0; k < UH; ++k) {
                if (p + k * BLK >= p1) break;
                w[off + p + k * BLK] = wv[k];
                wn[0].re += cabs2(wv[k]);
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (q <= j) acc[q] = cjfma(vv[k][q], wv[k], acc[q]);
            }
        }
    }
    store_group(acc, 0, j, po, c, sh, res);
    for (int g = 1; 8 * g <= j; ++g) {
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = mkc(0.0, 0.0);
        dots8(w, V, vstride, g, j, off, p0, p1, acc);
        store_group(acc, g, j, po, c, sh, res);
    }
    block_sum<1>(wn, 1, sh, res);
    if (threadIdx.x == 0) po[(j + 1) * NBMAX + c] = res[0];
}

// The later groups of 8 first-round inner products <v_{8g+q}, w> (8g+q <= j,
// g >= 1) after k_slab_hdot: w re-read over chunks of points, one partial per
// chunk in the partial slots of the slab blocks (as many chunks as slab
// blocks).
__global__ __launch_bounds__(BLK) void k_hdot_groups(const zc *__restrict__ w, const zc *__restrict__ V,
                                                     size_t vstride, int j, unsigned N, size_t ld,
                                                     zc *__restrict__ pout, unsigned chunk, int nb,
                                                     const int *active)
{
    __shared__ zc sh[(BLK / 64) * 8];
    __shared__ zc res[8];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const size_t off = rhs * ld;
    zc *po = pout + (size_t)rhs * OVAL * NBMAX;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk + threadIdx.x, p1 = min(N, c * chunk + chunk);
    for (int g = 1; 8 * g <= j; ++g) {
        zc acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = mkc(0.0, 0.0);
        dots8(w, V, vstride, g, j, off, p0, p1, acc);
        store_group(acc, g, j, po, c, sh, res);
    }
}

// Inner products <v_{8g+q}, w> (q < QN, 8g+q <= j) over a thread's tile points,
// w in its own shared-memory slots, PB points per batch of loads.
template <int PB, int QN>
__device__ __forceinline__ void tile_dots(const zc *lz, const zc *V, size_t vstride, size_t off,
                                          const size_t (&pq)[TILE_MAXE], int HN, int HX, int HY, int g, int j,
                                          zc (&acc)[8])
{
#pragma unroll
    for (int b0 = 0; b0 < TILE_MAXE; b0 += PB) {
        if (b0 * BLK >= HN) break;   // the same for every thread of the block
        zc vv[PB][QN], wv[PB];
        bool in[PB];
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int it = b0 + i;
            if (it >= TILE_MAXE) break;
            const int e = threadIdx.x + it * BLK;
            const int ey = e / HX, ex = e - ey * HX;
            in[i] = e < HN && ex >= 1 && ex <= HX - 2 && ey >= 1 && ey <= HY - 2;
            wv[i] = in[i] ? lz[e] : mkc(0.0, 0.0);
#pragma unroll
            for (int q = 0; q < QN; ++q)
                if (8 * g + q <= j) vv[i][q] = V[(8 * g + q) * vstride + off + pq[it]];
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            if (b0 + i >= TILE_MAXE) break;
            if (!in[i]) continue;
#pragma unroll
            for (int q = 0; q < QN; ++q)
                if (8 * g + q <= j) acc[q] = cjfma(vv[i][q], wv[i], acc[q]);
        }
    }
}

// k_hdot on one 2-D tile of the finest level (same partials, one per tile):
// z on the tile and its one-point halo is loaded in one batch (all of a
// thread's points at once) into shared memory with the tile's tables of H;
// the tile's points form w = H z from there, write it and ||w||^2, and keep
// w in their own shared-memory slots for the inner products <v_i, w> (groups
// of 8 basis vectors, four points per batch), so w is never read back from
// memory.
template <typename TZ>
__global__ __launch_bounds__(BLK) void k_hdot_tile(LvlK<double> H, const Cx<TZ> *__restrict__ z,
                                                   zc *__restrict__ w, const zc *__restrict__ V, size_t vstride,
                                                   int j, size_t ld, zc *__restrict__ pout, TileGeo tg, int ntile,
                                                   const int *active)
{
    __shared__ zc sh[(BLK / 64) * 8];
    __shared__ zc res[8];
    __shared__ zc lz[TILE_MAXN];
    __shared__ zc ltab[6 * TAB_MAXD];   // x lower, diag, upper; y lower, diag, upper
    const int rhs = blockIdx.y;
    H = H.at(rhs);
    if (!active[rhs]) return;
    const unsigned t = chunk_id(ntile);
    const unsigned tyi = t / tg.ntx, txi = t - tyi * tg.ntx;
    const int nx = (int)H.nx, ny = (int)H.ny;
    const int x0 = (int)(txi * tg.tx), y0 = (int)(tyi * tg.ty);
    const int TX = min(x0 + (int)tg.tx, nx) - x0, TY = min(y0 + (int)tg.ty, ny) - y0;
    const int HX = TX + 2, HY = TY + 2, HN = HX * HY;
    const size_t off = rhs * ld;
    const size_t pc = (size_t)y0 * nx + x0;   // a point of the level every clamped address goes to
    int tslot = -1;
    const zc *tsrc;
    {
        const int q = threadIdx.x;
        const bool xs = q < 3 * TX;
        const int qq = xs ? q : min(q - 3 * TX, 3 * TY - 1);
        const int c = qq / 3, a = qq - 3 * c;
        tsrc = (xs ? H.tab[0] + a * nx + x0 : H.tab[1] + a * ny + y0) + c;
        if (q < 3 * TX + 3 * TY) tslot = (xs ? a : 3 + a) * TAB_MAXD + c;
    }
    const double tre = tsrc->re, tim = tsrc->im;
    auto inner = [&](int e) {
        const int ey = e / HX, ex = e - ey * HX;
        return e < HN && ex >= 1 && ex <= HX - 2 && ey >= 1 && ey <= HY - 2;
    };
    Cx<TZ> zq[TILE_MAXE];
    double phq[TILE_MAXE];
    size_t pq[TILE_MAXE];
    bool okq[TILE_MAXE];
#pragma unroll
    for (int it = 0; it < TILE_MAXE; ++it) {
        const int e = threadIdx.x + it * BLK;
        const int ey = e / HX, ex = e - ey * HX;
        const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
        okq[it] = e < HN && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        pq[it] = okq[it] ? (size_t)gy * nx + gx : pc;
        zq[it] = z[off + pq[it]];
        phq[it] = H.phi[pq[it]];
    }
#pragma unroll
    for (int it = 0; it < TILE_MAXE; ++it) {
        const int e = threadIdx.x + it * BLK;
        if (e < HN) lz[e] = okq[it] ? cvt<double>(zq[it]) : mkc(0.0, 0.0);
    }
    if (tslot >= 0) ltab[tslot] = mkc(tre, tim);
    __syncthreads();
    zc wq[TILE_MAXE];
    zc wn[1] = {mkc(0.0, 0.0)};
#pragma unroll
    for (int it = 0; it < TILE_MAXE; ++it) {
        const int e = threadIdx.x + it * BLK;
        wq[it] = mkc(0.0, 0.0);
        if (!inner(e)) continue;
        const int ey = e / HX, ex = e - ey * HX;
        const int c = ex - 1, r = ey - 1;
        zc d = ltab[1 * TAB_MAXD + c] + ltab[4 * TAB_MAXD + r];
        d.re -= phq[it];
        zc a = d * lz[e];
        a = cfma(ltab[0 * TAB_MAXD + c], lz[e - 1], a);
        a = cfma(ltab[2 * TAB_MAXD + c], lz[e + 1], a);
        a = cfma(ltab[3 * TAB_MAXD + r], lz[e - HX], a);
        a = cfma(ltab[5 * TAB_MAXD + r], lz[e + HX], a);
        w[off + pq[it]] = a;
        wq[it] = a;
        wn[0].re += cabs2(a);
    }
    __syncthreads();   // every neighbour read of z is done
#pragma unroll
    for (int it = 0; it < TILE_MAXE; ++it) {
        const int e = threadIdx.x + it * BLK;
        if (inner(e)) lz[e] = wq[it];   // a thread reads back only its own slots
    }
    zc *po = pout + (size_t)rhs * OVAL * NBMAX;
    for (int g = 0; 8 * g <= j; ++g) {
        zc acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = mkc(0.0, 0.0);
        // a group of at most two vectors loads all of a thread's points at
        // once, larger ones four points per batch
        if (j - 8 * g < 2)
            tile_dots<TILE_MAXE, 2>(lz, V, vstride, off, pq, HN, HX, HY, g, j, acc);
        else
            tile_dots<4, 8>(lz, V, vstride, off, pq, HN, HX, HY, g, j, acc);
        store_group(acc, g, j, po, t, sh, res);
    }
    block_sum<1>(wn, 1, sh, res);
    if (threadIdx.x == 0) po[(j + 1) * NBMAX + t] = res[0];
}

// x(p) = w(p) - sum_{q <= j} a_q v_q(p) for the U points of one batch
__device__ __forceinline__ void proj_batch(const zc *w, const zc *V, size_t vstride, int j, size_t off, unsigned p,
                                           unsigned last, const zc *cc, zc (&x)[UO])
{
#pragma unroll
    for (int k = 0; k < UO; ++k) x[k] = w[off + min(p + k * BLK, last)];
#pragma unroll 2
    for (int q = 0; q <= j; ++q) {
        zc vq[UO];
        const zc a = cc[q];
#pragma unroll
        for (int k = 0; k < UO; ++k) vq[k] = V[q * vstride + off + min(p + k * BLK, last)];
#pragma unroll
        for (int k = 0; k < UO; ++k) x[k] = x[k] - a * vq[k];
    }
}

// v = w / h (scale from the FGMRES state), optional cycle-precision copy.
template <typename TB>
__global__ __launch_bounds__(BLK) void k_vnorm(const zc *w, zc *v, Cx<TB> *__restrict__ bc, unsigned N, size_t ld,
                                               const FState *fsb, unsigned chunk, int nb, const int *active)
{
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const double sc = fsb[rhs].inv_hn;
    const size_t off = rhs * ld;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk + threadIdx.x, p1 = min(N, c * chunk + chunk);
    if (p0 >= p1) return;
    const unsigned last = p1 - 1;
    for (unsigned p = p0; p < p1; p += UO * BLK) {
        zc x[UO];
#pragma unroll
        for (int k = 0; k < UO; ++k) x[k] = sc * w[off + min(p + k * BLK, last)];
#pragma unroll
        for (int k = 0; k < UO; ++k) {
            if (p + k * BLK >= p1) break;
            v[off + p + k * BLK] = x[k];
            if (bc) bc[off + p + k * BLK] = cvt<TB>(x[k]);
        }
    }
}

// r = chi - H u, partial ||r||^2 (value 0) and ||chi||^2 (value 1).
template <int DIM>
__global__ __launch_bounds__(BLK) void k_tres(LvlK<double> H, const zc *__restrict__ chi, const zc *__restrict__ u,
                                              zc *__restrict__ r, size_t ld, int with_chi, zc *__restrict__ pout,
                                              unsigned chunk, int nb, const int *active)
{
    __shared__ zc sh[(BLK / 64) * 2];
    __shared__ zc res[2];
    const int rhs = blockIdx.y;
    H = H.at(rhs);
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
    block_sum_last<2>(acc, nv, sh, res);
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
    const unsigned p0 = c * chunk + threadIdx.x, p1 = min(N, c * chunk + chunk);
    if (p0 >= p1) return;
    const unsigned last = p1 - 1;
    for (unsigned p = p0; p < p1; p += UO * BLK) {
        zc x[UO];
#pragma unroll
        for (int k = 0; k < UO; ++k) x[k] = u[off + min(p + k * BLK, last)];
        for (int q = 0; q < kc; ++q) {
            Cx<TZ> zq[UO];
#pragma unroll
            for (int k = 0; k < UO; ++k) zq[k] = Z[q * zstride + off + min(p + k * BLK, last)];
#pragma unroll
            for (int k = 0; k < UO; ++k) x[k] = cfma(yy[q], cvt<double>(zq[k]), x[k]);
        }
#pragma unroll
        for (int k = 0; k < UO; ++k) {
            if (p + k * BLK >= p1) break;
            u[off + p + k * BLK] = x[k];
        }
    }
}

constexpr int FT = 1024;   // threads of the finish kernel (restarts, least squares)
constexpr int FG = 32;     // lanes that reduce one value

// Sum of the partials of value q by FG consecutive lanes (independent loads,
// then a butterfly inside the lane group): deterministic, no block barrier.
__device__ __forceinline__ zc group_parts(const zc *pp, int nbin)
{
    // the lane's loads issued eight at a time (inside the row of NBMAX
    // partials), then summed in the order of b
    constexpr int K = NBMAX / FG, KB = 8;
    const int lane = threadIdx.x % FG;
    zc v = mkc(0.0, 0.0);
    for (int k0 = 0; k0 < K && k0 * FG < nbin; k0 += KB) {
        zc t[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) t[k] = pp[min(lane + (k0 + k) * FG, NBMAX - 1)];
#pragma unroll
        for (int k = 0; k < KB; ++k)
            if (lane + (k0 + k) * FG < nbin) v = v + t[k];
    }
#pragma unroll
    for (int off = FG / 2; off > 0; off >>= 1) {
        v.re += __shfl_xor(v.re, off, FG);
        v.im += __shfl_xor(v.im, off, FG);
    }
    return v;
}

// Column j of the Hessenberg matrix is complete (col[0..j] in shared memory,
// h_{j+1,j} = hn): apply the previous rotations (cs, sn staged in shared
// memory), form the new one, update g and the estimate.  One thread; the
// rotated column is left in col for the block to store.
// Also decides, as the host does on reading the report, whether the RHS stops
// iterating (non-finite estimate, tolerance reached, breakdown, iteration
// limit); stop (when given) is then cleared, so the iterations queued behind
// this one skip it.
__device__ void givens_column(FState *fs, Report *rp, int j, double hn, zc *col, const double *cs_s, const zc *sn_s,
                              int *stop)
{
    col[j + 1] = mkc(hn, 0.0);
    for (int q = 0; q < j; ++q) {
        const zc t1 = col[q], t2 = col[q + 1];
        col[q] = cs_s[q] * t1 + sn_s[q] * t2;
        col[q + 1] = cs_s[q] * t2 - mkc(sn_s[q].re, -sn_s[q].im) * t1;
    }
    double cs;
    zc sn;
    rot(col[j], col[j + 1], cs, sn);
    fs->cs[j] = cs;
    fs->sn[j] = sn;
    const zc t1 = col[j], t2 = col[j + 1];
    col[j] = cs * t1 + sn * t2;
    col[j + 1] = mkc(0.0, 0.0);
    const zc gj = fs->g[j];
    const zc g1 = mkc(0.0, 0.0) - mkc(sn.re, -sn.im) * gj;
    fs->g[j + 1] = g1;
    fs->g[j] = cs * gj;
    fs->hn = hn;
    fs->inv_hn = hn > 0.0 ? 1.0 / hn : 0.0;
    fs->kcols = j + 1;
    const double est = sqrt(cabs2(g1)) / fs->nchi;
    rp->est = est;
    rp->hn = hn;
    rp->finite = isfinite(est) && isfinite(hn);
    fs->it += 1;
    if (stop && (!rp->finite || est <= fs->tol || hn == 0.0 || fs->it >= fs->maxit)) *stop = 0;
}

// One block per RHS: finish an outer reduction and advance the small FGMRES
// state (Hessenberg column, Givens rotations, residual estimate, LS solve).
// The serial parts run on one thread over shared-memory copies of the state.
__global__ __launch_bounds__(FT) void k_fin(int mode, const zc *__restrict__ pin, int nbin, int j, FState *fsb,
                                            Report *rep, const int *active, int *stop)
{
    constexpr int M = CSG_MAX_RESTART;
    __shared__ zc val[2];
    const int rhs = blockIdx.x;
    if (!active[rhs]) return;
    FState *fs = fsb + rhs;
    const zc *pp = pin + (size_t)rhs * OVAL * NBMAX;
    if (mode == FIN_LS) {
        // back substitution R y = g on the k x k upper triangle (staged)
        __shared__ zc Rt[M * M];
        __shared__ zc gy[M];
        const int k = fs->kcols;
        for (int e = threadIdx.x; e < k * k; e += FT) {
            const int i = e / k, c = e % k;
            if (c >= i) Rt[i * M + c] = fs->R[i * M + c];
        }
        for (int i = threadIdx.x; i < k; i += FT) gy[i] = fs->g[i];
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = k - 1; i >= 0; --i) {
                zc acc = gy[i];
                for (int c = i + 1; c < k; ++c) acc = acc - Rt[i * M + c] * gy[c];
                const zc d = Rt[i * M + i];
                gy[i] = (1.0 / cabs2(d)) * (acc * mkc(d.re, -d.im));
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < k; i += FT) fs->y[i] = gy[i];
        return;
    }
    // values: FIN_BEGIN: 0, 1; FIN_BETA: 0
    const int nv = mode == FIN_BEGIN ? 2 : 1;
    const int grp = threadIdx.x / FG;
    for (int q = grp; q < nv; q += FT / FG) {
        const zc v = group_parts(pp + q * NBMAX, nbin);
        if (threadIdx.x % FG == 0) val[q] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    {
        // FIN_BEGIN / FIN_BETA: start of a restart cycle
        const double beta = sqrt(val[0].re);
        if (mode == FIN_BEGIN) fs->nchi = sqrt(val[1].re);
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
}

__global__ void k_copy_mask(const int *src, int *dst, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Third-order polynomial smoother (section 4): one sweep is three Richardson
// steps x <- x + w_i (b - A x), so the error is multiplied by
// p(A) = (1 - w1 A)(1 - w2 A)(1 - w3 A).  No inner products: nothing couples
// distant points, which is what lets the three steps run on a tile at once.
// ---------------------------------------------------------------------------

// One step on the plain chunked layout: xout = xin + w (b - A xin), xin null
// meaning zero (xout = w b); xout must not alias xin.
template <typename T, int DIM>
__global__ __launch_bounds__(BLK) void k_rich(LvlK<T> L, const Cx<T> *__restrict__ xin, const Cx<T> *__restrict__ b,
                                              Cx<T> *__restrict__ xout, Cx<T> w, size_t ld, unsigned chunk, int nb,
                                              const int *active)
{
    constexpr int U = Ubatch<T>::U;
    const int rhs = blockIdx.y;
    L = L.at(rhs);
    if (!active[rhs]) return;
    const size_t off = rhs * ld;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk + threadIdx.x, p1 = min(L.N, c * chunk + chunk);
    if (p0 >= p1) return;
    const unsigned last = p1 - 1;
    for (unsigned p = p0; p < p1; p += U * BLK) {
        Cx<T> v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const unsigned pk = min(p + k * BLK, last);
            const Cx<T> bv = b[off + pk];
            if (xin) {
                unsigned i, jj, kk;
                decomp<DIM>(pk, L.nx, L.ny, i, jj, kk);
                v[k] = xin[off + pk] + w * (bv - apply_pt<T, DIM>(L, xin + off, i, jj, kk, pk));
            } else {
                v[k] = w * bv;
            }
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (p + k * BLK >= p1) break;
            xout[off + p + k * BLK] = v[k];
        }
    }
}

// A whole sweep on one 2-D tile of PT x PT points: x is staged on the tile and
// a three-point halo in shared memory (zero outside the level); step i
// updates the points within 3 - i of the tile (each step's stencil reaches one
// point further than the next step needs), so after three steps the tile's
// points hold the sweep's result, with x, b and phi read from memory once per
// staged point.  With ec, the start value is xin + P ec (the interpolated
// coarse correction of the up path; xin may be null).  A thread owns the same
// points of the two-point-halo region in every step and keeps their b, phi
// and stencil rows in registers.  xout must not alias xin.
constexpr int PT = 32;                      // tile side
constexpr int PR = PT + 6;                  // staged region side
constexpr int PN = (PT + 4) * (PT + 4);     // points updated by step 1
constexpr int PE = (PN + BLK - 1) / BLK;    // of them per thread
template <typename T, bool ZERO, bool PROL>
__global__ __launch_bounds__(BLK) void k_poly_tile(LvlK<T> L, LvlK<T> C, const Cx<T> *__restrict__ ec,
                                                   const Cx<T> *__restrict__ xin, const Cx<T> *__restrict__ b,
                                                   Cx<T> *__restrict__ xout, Cx<T> w1, Cx<T> w2, Cx<T> w3,
                                                   size_t ld, size_t ldc, unsigned ntx, const int *active)
{
    __shared__ Cx<T> X[2][PR * PR];
    const int rhs = blockIdx.y;
    L = L.at(rhs);
    C = C.at(rhs);
    if (!active[rhs]) return;
    const size_t off = rhs * ld;
    const int nx = (int)L.nx, ny = (int)L.ny;
    const unsigned t = blockIdx.x, tyi = t / ntx, txi = t - tyi * ntx;
    const int x0 = (int)txi * PT, y0 = (int)tyi * PT;
    const int TX = min(PT, nx - x0), TY = min(PT, ny - y0);
    const int RX = TX + 6, RY = TY + 6;
    // stage the start value on the tile and its three-point halo
    if (!ZERO) {
        for (int e = threadIdx.x; e < RX * RY; e += BLK) {
            const int ey = e / RX, ex = e - ey * RX;
            const int gx = x0 - 3 + ex, gy = y0 - 3 + ey;
            Cx<T> v = mkc<T>(0, 0);
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                const unsigned gp = (unsigned)gy * nx + gx;
                if (xin) v = xin[off + gp];
                if (PROL) v = v + prolong_pt<T, 2>(ec + rhs * ldc, (unsigned)gx, (unsigned)gy, 0u, C.nx, C.ny, 1u);
            }
            X[0][e] = v;
        }
    }
    // owned points of the two-point-halo region: b, phi-shifted diagonal and
    // the four off-diagonal weights
    const int QX = TX + 4, QY = TY + 4;
    Cx<T> bq[PE], dq[PE], wxq[PE], exq[PE], wyq[PE], eyq[PE];
    int eq[PE], mq[PE];
#pragma unroll
    for (int k = 0; k < PE; ++k) {
        const int q = threadIdx.x + k * BLK;
        const int qy = q / QX, qx = q - qy * QX;
        const int gx = x0 - 2 + qx, gy = y0 - 2 + qy;
        const bool in = q < QX * QY && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        // distance of the point from the tile (0 on the tile), 9 when absent
        const int m = max(max(max(-gx + x0, gx - (x0 + TX - 1)), max(-gy + y0, gy - (y0 + TY - 1))), 0);
        mq[k] = in ? m : 9;
        eq[k] = (qy + 1) * RX + qx + 1;
        const int cx = in ? gx : 0, cy = in ? gy : 0;
        const unsigned gp = (unsigned)cy * nx + cx;
        bq[k] = b[off + gp];
        Cx<T> d = L.tab[0][nx + cx] + L.tab[1][ny + cy];
        sub_phi(d, L, L.phi[gp]);
        dq[k] = d;
        wxq[k] = L.tab[0][cx];
        exq[k] = L.tab[0][2 * nx + cx];
        wyq[k] = L.tab[1][cy];
        eyq[k] = L.tab[1][2 * ny + cy];
    }
    if (ZERO) {
        // the first step from x = 0 is x1 = w1 b: written straight into buffer 1,
        // zero where absent
        for (int e = threadIdx.x; e < RX * RY; e += BLK) X[1][e] = mkc<T>(0, 0);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PE; ++k)
            if (mq[k] <= 2) X[1][eq[k]] = w1 * bq[k];
    } else {
        for (int e = threadIdx.x; e < RX * RY; e += BLK) X[1][e] = mkc<T>(0, 0);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PE; ++k) {
            if (mq[k] > 2) continue;
            const Cx<T> *S = X[0];
            const int e = eq[k];
            Cx<T> a = dq[k] * S[e];
            a = cfma(wxq[k], S[e - 1], a);
            a = cfma(exq[k], S[e + 1], a);
            a = cfma(wyq[k], S[e - RX], a);
            a = cfma(eyq[k], S[e + RX], a);
            X[1][e] = S[e] + w1 * (bq[k] - a);
        }
    }
    __syncthreads();
    // step 2 into buffer 0 (points within one of the tile), step 3 from there
    Cx<T> res[PE];
#pragma unroll
    for (int k = 0; k < PE; ++k) {
        if (mq[k] > 1) continue;
        const Cx<T> *S = X[1];
        const int e = eq[k];
        Cx<T> a = dq[k] * S[e];
        a = cfma(wxq[k], S[e - 1], a);
        a = cfma(exq[k], S[e + 1], a);
        a = cfma(wyq[k], S[e - RX], a);
        a = cfma(eyq[k], S[e + RX], a);
        res[k] = S[e] + w2 * (bq[k] - a);
    }
    __syncthreads();   // every step-2 read of X[0]'s old contents is done
    // buffer 0 now: zero outside the level and on the ring the steps never reach
    for (int e = threadIdx.x; e < RX * RY; e += BLK) X[0][e] = mkc<T>(0, 0);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PE; ++k)
        if (mq[k] <= 1) X[0][eq[k]] = res[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PE; ++k) {
        if (mq[k] != 0) continue;
        const Cx<T> *S = X[0];
        const int e = eq[k];
        Cx<T> a = dq[k] * S[e];
        a = cfma(wxq[k], S[e - 1], a);
        a = cfma(exq[k], S[e + 1], a);
        a = cfma(wyq[k], S[e - RX], a);
        a = cfma(eyq[k], S[e + RX], a);
        const int q = threadIdx.x + k * BLK;
        const int qy = q / QX, qx = q - qy * QX;
        xout[off + (size_t)(y0 - 2 + qy) * nx + (x0 - 2 + qx)] = S[e] + w3 * (bq[k] - a);
    }
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
void launch_st0(const LvlK<T> &L, const Cx<T> *u0, Cx<T> *w, int wn, size_t ld, zc *pout, const Launch &g,
                const int *active)
{
    if (wn)
        hipLaunchKernelGGL((k_st0<T, DIM, 3>), grid(g), dim3(BLK), 0, g.st, L, u0, w, ld, pout, g.chunk, g.nb, active);
    else
        hipLaunchKernelGGL((k_st0<T, DIM, 2>), grid(g), dim3(BLK), 0, g.st, L, u0, w, ld, pout, g.chunk, g.nb, active);
}

template <typename T, int DIM>
void launch_stj(const LvlK<T> &L, const Basis<T> &B, Cx<T> *w, int j, int s, size_t ld, zc *pout, const Launch &g,
                const int *active)
{
    const int wn = norm_from_sums<T>() && j + 1 == s;
    if (s <= 3)
        hipLaunchKernelGGL((k_stj<T, DIM, 4>), grid(g), dim3(BLK), 0, g.st, L, B, w, j, wn, ld, pout, g.chunk, g.nb,
                           active);
    else
        hipLaunchKernelGGL((k_stj<T, DIM, NVAL - 1>), grid(g), dim3(BLK), 0, g.st, L, B, w, j, wn, ld, pout, g.chunk,
                           g.nb, active);
}

template <typename T, int DIM>
void launch_os(const LvlK<T> &L, const Basis<T> &B, const Cx<T> *win, Cx<T> *wout, int j, int s, size_t ld,
               const zc *pin, int nbin, zc *pout, GState *gs, double tiny, const Launch &g, const int *active)
{
    if (s <= 3)
        hipLaunchKernelGGL((k_os<T, DIM, 4>), grid(g), dim3(BLK), 0, g.st, L, B, win, wout, j, s, ld, pin, nbin, pout,
                           gs, tiny, g.chunk, g.nb, active);
    else
        hipLaunchKernelGGL((k_os<T, DIM, NVAL - 1>), grid(g), dim3(BLK), 0, g.st, L, B, win, wout, j, s, ld, pin, nbin,
                           pout, gs, tiny, g.chunk, g.nb, active);
}

template <typename T>
void launch_os_tile(const LvlK<T> &L, const Basis<T> &B, const Cx<T> *win, Cx<T> *wout, int j, int s, size_t ld,
                    const zc *pin, int nbin, zc *pout, GState *gs, double tiny, const TileGeo &tg, int nrhs,
                    hipStream_t st, const int *active)
{
    const int ntile = (int)(tg.ntx * tg.nty);
    if (j == 0)
        hipLaunchKernelGGL((k_os_tile<T, 4, 0>), dim3(ntile, nrhs), dim3(BLK), 0, st, L, B, win, wout, s, ld, pin,
                           nbin, pout, gs, tiny, tg, ntile, active);
    else
        hipLaunchKernelGGL((k_os_tile<T, 4, 1>), dim3(ntile, nrhs), dim3(BLK), 0, st, L, B, win, wout, s, ld, pin,
                           nbin, pout, gs, tiny, tg, ntile, active);
}

// Interpolated correction and the residual that opens the post-sweep on the
// z-marching slabs of a 3-D level (the transfer-pass analogue of k_slab): the
// coarse correction's window under the column (its x-y extent plus the
// interpolation stencil) is staged into a three-plane shared-memory ring of
// coarse planes, each loaded an iteration before it is first needed; for each
// plane every thread forms x = P ec (+ xin) from there at its column point and
// at one halo point of the 32 x 16 column into the three-plane ring of fine
// planes (zero outside the level), stores x at its own points, and from the
// ring planes around plane k forms r = b - A x there; xin of the plane after
// next, b and phi of the next plane are loaded while a plane's residual runs.
// x never goes back to memory for the residual's stencil, and the values
// equal k_prolong then k_resid bit for bit (the same formulas in the same
// order).
constexpr int CWX = SX / 2 + 3, CWY = SY / 2 + 3;   // coarse window of a column, halo included
static_assert(CWX * CWY <= BLK, "one coarse window point per thread");
template <typename T>
__global__ __launch_bounds__(BLK) void k_slab_pr(LvlK<T> F, LvlK<T> C, const Cx<T> *__restrict__ ec,
                                                 const Cx<T> *__restrict__ xin, Cx<T> *__restrict__ xout,
                                                 const Cx<T> *__restrict__ b, Cx<T> *__restrict__ r, size_t ldf,
                                                 size_t ldc, unsigned ntx, unsigned nty, unsigned nzc, unsigned zrun,
                                                 int nslab, const int *active)
{
    __shared__ Cx<T> ring[3][SHX * SHY];
    __shared__ Cx<T> cring[3][CWX * CWY];
    __shared__ Cx<T> ltab[3 * SX + 3 * SY];
    const int rhs = blockIdx.y;
    F = F.at(rhs);
    C = C.at(rhs);
    if (!active[rhs]) return;
    const unsigned slot = chunk_id(nslab);
    const unsigned col = slot / nzc, zci = slot - col * nzc;
    if (col >= ntx * nty) return;   // padding block
    const unsigned cyi = col / ntx, cxi = col - cyi * ntx;
    const int nx = (int)F.nx, ny = (int)F.ny, nz = (int)F.nz;
    const int x0 = (int)cxi * SX, y0 = (int)cyi * SY;
    const int TX = min(SX, nx - x0), TY = min(SY, ny - y0);
    const int z0 = (int)(zci * zrun), z1 = min(nz, z0 + (int)zrun);
    const int tx = threadIdx.x % SX, ty = threadIdx.x / SX;
    const bool own = tx < TX && ty < TY;
    const int eo = (ty + 1) * SHX + tx + 1;
    const int gxo = x0 + min(tx, TX - 1), gyo = y0 + min(ty, TY - 1);
    const unsigned po = (unsigned)gyo * nx + gxo;
    int er = -1, gxr = gxo, gyr = gyo;
    unsigned pr = po;
    bool rin = false;
    if ((int)threadIdx.x < 2 * (TX + 2) + 2 * TY) {
        int ex, ey;
        ring_pos(threadIdx.x, TX, TY, ex, ey);
        er = ey * SHX + ex;
        const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
        rin = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        if (rin) {
            pr = (unsigned)gy * nx + gx;
            gxr = gx;
            gyr = gy;
        }
    }
    for (int q = threadIdx.x; q < 3 * (TX + TY); q += BLK) {
        if (q < 3 * TX) {
            const int a = q / TX, c = q - a * TX;
            ltab[a * SX + c] = F.tab[0][a * nx + x0 + c];
        } else {
            const int qq = q - 3 * TX, a = qq / TY, c = qq - a * TY;
            ltab[3 * SX + a * SY + c] = F.tab[1][a * ny + y0 + c];
        }
    }
    const unsigned plane = (unsigned)nx * ny;
    const Cx<T> *e = ec + rhs * ldc;
    const Cx<T> *xi = xin ? xin + rhs * ldf : nullptr;
    const size_t off = rhs * ldf;
    // the coarse window: every coarse node the interpolation of a fine point
    // of the column or its halo inside the level reads (paxis of the extreme
    // fine coordinates), at most CWX x CWY of them
    const unsigned ncx = C.nx, ncy = C.ny, ncz = C.nz;
    const int gxa = max(x0 - 1, 0), gxb = min(x0 + TX, nx - 1);
    const int gya = max(y0 - 1, 0), gyb = min(y0 + TY, ny - 1);
    const unsigned cx0 = paxis((unsigned)gxa, ncx).idx[0], cx1 = paxis((unsigned)gxb, ncx).idx[1];
    const unsigned cy0 = paxis((unsigned)gya, ncy).idx[0], cy1 = paxis((unsigned)gyb, ncy).idx[1];
    const int cwx = (int)(cx1 - cx0) + 1, cwn = cwx * (int)(cy1 - cy0 + 1);
    const int cq = (int)threadIdx.x;
    const int cqy = cq / max(cwx, 1), cqx = cq - cqy * max(cwx, 1);
    const size_t cpt = (size_t)(cy0 + cqy) * ncx + cx0 + cqx;   // this thread's window node (cq < cwn)
    const int cslot = cqy * CWX + cqx;
    // the last coarse plane fine plane k reads (paxis(k).idx[1])
    auto chi = [&](int k) -> int { return (int)paxis((unsigned)max(0, min(k, nz - 1)), ncz).idx[1]; };
    auto cload = [&](int K) -> Cx<T> {
        return cq < cwn ? e[(size_t)K * ncx * ncy + cpt] : mkc<T>(0, 0);
    };
    auto cput = [&](int K, const Cx<T> &v) {
        if (cq < cwn) cring[K % 3][cslot] = v;
    };
    // x at a point of plane k (as k_prolong forms it, the coarse values from
    // the staged window)
    auto xat = [&](int k, int gx, int gy, const Cx<T> &xa) -> Cx<T> {
        const PAx ax = paxis((unsigned)gx, ncx), ay = paxis((unsigned)gy, ncy), az = paxis((unsigned)k, ncz);
        Cx<T> v = mkc<T>(0, 0);
#pragma unroll
        for (int cz = 0; cz < 2; ++cz)
#pragma unroll
            for (int bb = 0; bb < 2; ++bb)
#pragma unroll
                for (int a = 0; a < 2; ++a)
                    v = v + (T)(ax.w[a] * ay.w[bb] * az.w[cz]) *
                                cring[az.idx[cz] % 3][(ay.idx[bb] - cy0) * CWX + ax.idx[a] - cx0];
        if (xi) v = v + xa;
        return v;
    };
    auto load_xa = [&](int k, Cx<T> &xo, Cx<T> &xr) {
        if (!xi) return;
        const size_t kp = (size_t)max(0, min(k, nz - 1)) * plane;
        xo = xi[kp + po];
        if (er >= 0) xr = xi[kp + pr];
    };
    // plane k into ring slot k % 3 (zero outside the level); x of the run's own planes to memory
    auto stage = [&](int k, const Cx<T> &xao, const Cx<T> &xar) {
        Cx<T> *R = ring[(k + 3) % 3];
        const bool kin = k >= 0 && k < nz;
        if (er >= 0) R[er] = (kin && rin) ? xat(k, gxr, gyr, xar) : mkc<T>(0, 0);
        const Cx<T> xo = kin ? xat(k, gxo, gyo, xao) : mkc<T>(0, 0);
        R[eo] = (kin && own) ? xo : mkc<T>(0, 0);
        if (kin && own && k >= z0 && k < z1) xout[off + (size_t)k * plane + po] = xo;
    };
    // coarse planes read by the planes staged before the loop (at most three)
    const int klo = max(z0 - 1, 0);
    int cstaged = chi(z0 + 1);
    for (int K = (int)paxis((unsigned)min(klo, nz - 1), ncz).idx[0]; K <= cstaged; ++K) cput(K, cload(K));
    Cx<T> xao = mkc<T>(0, 0), xar = mkc<T>(0, 0);
    load_xa(z0 - 1, xao, xar);
    __syncthreads();
    stage(z0 - 1, xao, xar);
    load_xa(z0, xao, xar);
    stage(z0, xao, xar);
    load_xa(z0 + 1, xao, xar);
    // the coarse plane the loop's first iteration stages for the one after it
    int cnext = chi(z0 + 2);
    Cx<T> cv = cnext > cstaged ? cload(cnext) : mkc<T>(0, 0);
    Cx<T> bc = b[off + (size_t)z0 * plane + po];
    T phc = F.phi[(size_t)z0 * plane + po];
    for (int k = z0; k < z1; ++k) {
        stage(k + 1, xao, xar);
        if (cnext > cstaged) {
            cput(cnext, cv);
            cstaged = cnext;
        }
        load_xa(k + 2, xao, xar);
        cnext = chi(k + 3);
        if (cnext > cstaged) cv = cload(cnext);
        const int kn = min(k + 1, nz - 1);
        const Cx<T> bn = b[off + (size_t)kn * plane + po];
        const T phn = F.phi[(size_t)kn * plane + po];
        __syncthreads();
        if (own) {
            const Cx<T> *Rm = ring[(k + 2) % 3], *R0 = ring[k % 3], *Rp = ring[(k + 1) % 3];
            const Cx<T> *tz = F.tab[2];
            Cx<T> d = ltab[SX + tx] + ltab[3 * SX + SY + ty] + tz[nz + k];
            sub_phi(d, F, phc);
            Cx<T> a = d * R0[eo];
            a = cfma(ltab[tx], R0[eo - 1], a);
            a = cfma(ltab[2 * SX + tx], R0[eo + 1], a);
            a = cfma(ltab[3 * SX + ty], R0[eo - SHX], a);
            a = cfma(ltab[3 * SX + 2 * SY + ty], R0[eo + SHX], a);
            a = cfma(tz[k], Rm[eo], a);
            a = cfma(tz[2 * nz + k], Rp[eo], a);
            r[off + (size_t)k * plane + po] = bc - a;
        }
        __syncthreads();
        bc = bn;
        phc = phn;
    }
}

// Closing pass of a pre-sweep fused with the restriction on the z-marching
// slabs of a 3-D level: every block solves the sweep's small least squares
// (close_sweep, as k_upd_r), then for each plane every thread forms the
// Arnoldi residual r = sum_{i<=k} cr_i u_i at its column point and at one halo
// point into the three-plane shared-memory ring, updates x (+)= sum_{i<k} cx_i
// u_i at its own points, and after an odd plane the block forms the full
// weighting of r for the coarse points centred on that plane and in its
// column (16 x 8 of them).  r never goes to memory; the values equal k_upd_r
// then k_restrict bit for bit (the same formulas in the same order).
template <typename T, int SB>
__global__ __launch_bounds__(BLK) void k_slab_down(Cx<T> *__restrict__ x, int accumulate, Basis<T> B, int s,
                                                   LvlK<T> F, LvlK<T> C, Cx<T> *__restrict__ bc, size_t ldf,
                                                   size_t ldc, const zc *__restrict__ pin, int nbin, GState *gsb,
                                                   double tiny, unsigned ntx, unsigned nty, unsigned nzc,
                                                   unsigned zrun, int nslab, const int *active)
{
    __shared__ zc sh[(BLK / 64) * (SB + 1)];
    __shared__ zc res[SB + 1];
    __shared__ zc ax[CSG_MAX_S], ar[CSG_MAX_S + 1];
    __shared__ Cx<T> ring[3][SHX * SHY];
    const int rhs = blockIdx.y;
    F = F.at(rhs);
    C = C.at(rhs);
    if (!active[rhs]) return;
    const int kb = close_sweep<T, SB>(pin + (size_t)rhs * NVAL * NBMAX, nbin, gsb + rhs, s, tiny, sh, res, ax, ar);
    // the update and residual coefficients in the cycle's precision, read
    // from shared memory at their use (registers go to the loads in flight)
    __shared__ Cx<T> scx[SB], scr[SB];
    if ((int)threadIdx.x < SB) {
        const int q = threadIdx.x;
        if (q < kb) scx[q] = cvt<T>(ax[q]);
        if (q <= kb) scr[q] = cvt<T>(ar[q]);
    }
    __syncthreads();
    const unsigned slot = chunk_id(nslab);
    const unsigned col = slot / nzc, zci = slot - col * nzc;
    if (col >= ntx * nty) return;   // padding block
    const unsigned cyi = col / ntx, cxi = col - cyi * ntx;
    const int nx = (int)F.nx, ny = (int)F.ny, nz = (int)F.nz;
    const int x0 = (int)cxi * SX, y0 = (int)cyi * SY;
    const int TX = min(SX, nx - x0), TY = min(SY, ny - y0);
    const int z0 = (int)(zci * zrun), z1 = min(nz, z0 + (int)zrun);
    const int tx = threadIdx.x % SX, ty = threadIdx.x / SX;
    const bool own = tx < TX && ty < TY;
    const int eo = (ty + 1) * SHX + tx + 1;
    const unsigned po = (unsigned)(y0 + min(ty, TY - 1)) * nx + (x0 + min(tx, TX - 1));
    int er = -1;
    unsigned pr = po;
    bool rin = false;
    if ((int)threadIdx.x < 2 * (TX + 2) + 2 * TY) {
        int ex, ey;
        ring_pos(threadIdx.x, TX, TY, ex, ey);
        er = ey * SHX + ex;
        const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
        rin = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        if (rin) pr = (unsigned)gy * nx + gx;
    }
    const unsigned plane = (unsigned)nx * ny;
    const size_t off = rhs * ldf;
    // the values plane z's residual and update are formed from: u_0..u_kb at
    // the column point (and x there on the run's own planes when the update
    // accumulates) and at the halo point; loaded a plane ahead of their use
    struct Raw {
        Cx<T> u[SB];
        Cx<T> x;
    };
    const bool upd_own = own;
    auto load = [&](int z, Raw &o, Raw &h) {
        const size_t zp = off + (size_t)max(0, min(z, nz - 1)) * plane;
#pragma unroll
        for (int q = 0; q < SB; ++q)
            if (q <= kb) o.u[q] = B.u[q][zp + po];
        if (accumulate && upd_own && z >= z0 && z < z1) o.x = x[zp + po];
        if (er >= 0) {
#pragma unroll
            for (int q = 0; q < SB; ++q)
                if (q <= kb) h.u[q] = B.u[q][zp + pr];
        }
    };
    // r = sum_i cr_i u_i at a point
    auto rsum = [&](const Raw &v) -> Cx<T> {
        const int oz = opaque_zero();
        Cx<T> rr = mkc<T>(0, 0);
#pragma unroll
        for (int q = 0; q < SB; ++q)
            if (q <= kb) rr = cfma(scr[q + oz], v.u[q], rr);
        return rr;
    };
    // plane z into ring slot z % 3 (zero outside the level); on the run's own
    // planes also x (+)= sum_{i<kb} cx_i u_i at the column point
    auto stage = [&](int z, const Raw &o, const Raw &h) {
        Cx<T> *R = ring[(z + 3) % 3];
        const bool kin = z >= 0 && z < nz;
        if (er >= 0) R[er] = (kin && rin) ? rsum(h) : mkc<T>(0, 0);
        const Cx<T> ro = kin ? rsum(o) : mkc<T>(0, 0);
        if (kin && upd_own && z >= z0 && z < z1) {
            const int oz = opaque_zero();
            Cx<T> v = accumulate ? o.x : mkc<T>(0, 0);
#pragma unroll
            for (int q = 0; q < SB; ++q)
                if (q < kb) v = cfma(scx[q + oz], o.u[q], v);
            x[off + (size_t)z * plane + po] = v;
        }
        R[eo] = (kin && own) ? ro : mkc<T>(0, 0);
    };
    // this thread's coarse point of a plane (16 x 8 per column), if any
    const int lx = threadIdx.x % (SX / 2), ly = threadIdx.x / (SX / 2);
    const int Kx = x0 / 2 + lx, Ky = y0 / 2 + ly;
    const bool cown = ly < SY / 2 && 2 * Kx + 1 < x0 + TX && 2 * Ky + 1 < y0 + TY && Kx < (int)C.nx &&
                      Ky < (int)C.ny;
    const int ec0 = (2 * Ky + 1 - y0 + 1) * SHX + (2 * Kx + 1 - x0 + 1);   // ring index of the centre
    const T scale = (T)0.125;
    Raw o, h;
    load(z0 - 1, o, h);
    stage(z0 - 1, o, h);
    load(z0, o, h);
    stage(z0, o, h);
    load(z0 + 1, o, h);
    for (int z = z0; z < z1; ++z) {
        stage(z + 1, o, h);
        // the plane after next is in flight across the restriction
        if (z + 2 <= z1) load(z + 2, o, h);
        __syncthreads();
        const int Kz = (z - 1) / 2;
        if ((z & 1) && cown && Kz < (int)C.nz) {
            const Cx<T> *Rq[3] = {ring[(z + 2) % 3], ring[z % 3], ring[(z + 1) % 3]};
            Cx<T> acc = mkc<T>(0, 0);
            for (int qz = 0; qz < 3; ++qz)
                for (int qy = 0; qy < 3; ++qy)
                    for (int qx = 0; qx < 3; ++qx) {
                        T wgt = (T)(rw(qx) * rw(qy));
                        wgt *= (T)rw(qz);
                        acc = acc + wgt * Rq[qz][ec0 + (qy - 1) * SHX + (qx - 1)];
                    }
            bc[rhs * ldc + ((size_t)Kz * C.ny + Ky) * C.nx + Kx] = scale * acc;
        }
        __syncthreads();
    }
}

template <typename T>
void launch_slab(const LvlK<T> &L, const Basis<T> &B, const Cx<T> *win, Cx<T> *wout, int j, int s, size_t ld,
                 const zc *pin, int nbin, zc *pout, GState *gs, double tiny, bool wnorm, const SlabGeo &sg, int nrhs,
                 hipStream_t st, const int *active)
{
    const int nslab = (int)sg.npad;
    const dim3 gr(nslab, nrhs);
    if (j < 0)
        hipLaunchKernelGGL((k_slab<T, 4, -1>), gr, dim3(BLK), 0, st, L, B, win, wout, s, ld, pin, nbin, pout, gs, tiny,
                           sg.ntx, sg.nty, sg.nzc, sg.zrun, wnorm ? 1 : 0, nslab, active);
    else if (j == 0)
        hipLaunchKernelGGL((k_slab<T, 4, 0>), gr, dim3(BLK), 0, st, L, B, win, wout, s, ld, pin, nbin, pout, gs, tiny,
                           sg.ntx, sg.nty, sg.nzc, sg.zrun, wnorm ? 1 : 0, nslab, active);
    else
        hipLaunchKernelGGL((k_slab<T, 4, 1>), gr, dim3(BLK), 0, st, L, B, win, wout, s, ld, pin, nbin, pout, gs, tiny,
                           sg.ntx, sg.nty, sg.nzc, sg.zrun, wnorm ? 1 : 0, nslab, active);
}

template <typename T>
void launch_slab_down(Cx<T> *x, int accumulate, const Basis<T> &B, int s, const LvlK<T> &F, const LvlK<T> &C,
                      Cx<T> *bc, size_t ldf, size_t ldc, const zc *pin, int nbin, GState *gs, double tiny,
                      const SlabGeo &sg, int nrhs, hipStream_t st, const int *active)
{
    const int nslab = (int)sg.npad;
    hipLaunchKernelGGL((k_slab_down<T, 4>), dim3(nslab, nrhs), dim3(BLK), 0, st, x, accumulate, B, s, F, C, bc, ldf,
                       ldc, pin, nbin, gs, tiny, sg.ntx, sg.nty, sg.nzc, sg.zrun, nslab, active);
}

template <typename T>
void launch_slab_pr(const LvlK<T> &F, const LvlK<T> &C, const Cx<T> *ec, const Cx<T> *xin, Cx<T> *xout,
                    const Cx<T> *b, Cx<T> *r, size_t ldf, size_t ldc, const SlabGeo &sg, int nrhs, hipStream_t st,
                    const int *active)
{
    const int nslab = (int)sg.npad;
    hipLaunchKernelGGL((k_slab_pr<T>), dim3(nslab, nrhs), dim3(BLK), 0, st, F, C, ec, xin, xout, b, r, ldf, ldc,
                       sg.ntx, sg.nty, sg.nzc, sg.zrun, nslab, active);
}

template <typename T>
void launch_st0_tile(const LvlK<T> &L, const Cx<T> *u0, Cx<T> *w, size_t ld, bool wnorm, zc *pout, const TileGeo &tg,
                     int nrhs, hipStream_t st, const int *active)
{
    const int ntile = (int)(tg.ntx * tg.nty);
    if (wnorm)
        hipLaunchKernelGGL((k_st0_tile<T, 3>), dim3(ntile, nrhs), dim3(BLK), 0, st, L, u0, w, ld, pout, tg, ntile,
                           active);
    else
        hipLaunchKernelGGL((k_st0_tile<T, 2>), dim3(ntile, nrhs), dim3(BLK), 0, st, L, u0, w, ld, pout, tg, ntile,
                           active);
}

template <typename T>
void launch_down_tile(Cx<T> *x, int accumulate, const Basis<T> &B, int s, const LvlK<T> &F, const LvlK<T> &C,
                      Cx<T> *bc, Cx<T> *wc, size_t ldf, size_t ldc, const zc *pin, int nbin, GState *gs,
                      double tiny, bool st0, bool wnorm, zc *pout, const TileGeo &tc, int nrhs, hipStream_t st,
                      const int *active)
{
    const int ntile = (int)(tc.ntx * tc.nty);
    const dim3 grd(ntile, nrhs);
    if (!st0)
        hipLaunchKernelGGL((k_down_tile<T, 4, 0>), grd, dim3(BLK), 0, st, x, accumulate, B, s, F, C, bc, wc, ldf, ldc,
                           pin, nbin, gs, tiny, pout, tc, ntile, active);
    else if (wnorm)
        hipLaunchKernelGGL((k_down_tile<T, 4, 3>), grd, dim3(BLK), 0, st, x, accumulate, B, s, F, C, bc, wc, ldf, ldc,
                           pin, nbin, gs, tiny, pout, tc, ntile, active);
    else
        hipLaunchKernelGGL((k_down_tile<T, 4, 2>), grd, dim3(BLK), 0, st, x, accumulate, B, s, F, C, bc, wc, ldf, ldc,
                           pin, nbin, gs, tiny, pout, tc, ntile, active);
}

template <typename T>
void launch_up_tile(const LvlK<T> &F, const LvlK<T> &C, const Cx<T> *ec, const Cx<T> *xin, Cx<T> *xout,
                    const Cx<T> *b, Cx<T> *r, Cx<T> *w, size_t ldf, size_t ldc, bool wnorm, zc *pout,
                    const TileGeo &tg, int nrhs, hipStream_t st, const int *active, const UpClose<T> *fuse)
{
    const int ntile = (int)(tg.ntx * tg.nty);
    const dim3 grd(ntile, nrhs);
    const UpClose<T> uc = fuse ? *fuse : UpClose<T>{};
    if (fuse) {
        if (wnorm)
            hipLaunchKernelGGL((k_up_tile<T, 3, true>), grd, dim3(BLK), 0, st, F, C, ec, xin, xout, b, r, w, ldf, ldc,
                               pout, tg, ntile, uc, active);
        else
            hipLaunchKernelGGL((k_up_tile<T, 2, true>), grd, dim3(BLK), 0, st, F, C, ec, xin, xout, b, r, w, ldf, ldc,
                               pout, tg, ntile, uc, active);
    } else {
        if (wnorm)
            hipLaunchKernelGGL((k_up_tile<T, 3, false>), grd, dim3(BLK), 0, st, F, C, ec, xin, xout, b, r, w, ldf,
                               ldc, pout, tg, ntile, uc, active);
        else
            hipLaunchKernelGGL((k_up_tile<T, 2, false>), grd, dim3(BLK), 0, st, F, C, ec, xin, xout, b, r, w, ldf,
                               ldc, pout, tg, ntile, uc, active);
    }
}

template <typename T>
void launch_orthl(const Basis<T> &B, const Cx<T> *win, int j, int s, unsigned N, size_t ld, const zc *pin, int nbin,
                  zc *pout, GState *gs, double tiny, const Launch &g, const int *active)
{
    if (s <= 3)
        hipLaunchKernelGGL((k_orthl<T, 4>), grid(g), dim3(BLK), 0, g.st, B, win, j, s, N, ld, pin, nbin, pout, gs, tiny,
                           g.chunk, g.nb, active);
    else
        hipLaunchKernelGGL((k_orthl<T, NVAL - 1>), grid(g), dim3(BLK), 0, g.st, B, win, j, s, N, ld, pin, nbin, pout, gs,
                           tiny, g.chunk, g.nb, active);
}

template <typename T>
void launch_upd(Cx<T> *x, int accumulate, const Basis<T> &B, int s, unsigned N, size_t ld, const zc *pin, int nbin,
                GState *gs, double tiny, const Launch &g, const int *active)
{
    if (s <= 3)
        hipLaunchKernelGGL((k_upd<T, 4>), grid(g), dim3(BLK), 0, g.st, x, accumulate, B, s, N, ld, pin, nbin, gs, tiny,
                           g.chunk, g.nb, active);
    else
        hipLaunchKernelGGL((k_upd<T, NVAL - 1>), grid(g), dim3(BLK), 0, g.st, x, accumulate, B, s, N, ld, pin, nbin,
                           gs, tiny, g.chunk, g.nb, active);
}

template <typename T, int DIM>
void launch_upd_res(Cx<T> *x, int accumulate, const Basis<T> &B, int s, const LvlK<T> &F, const LvlK<T> &C,
                    Cx<T> *bc, size_t ldf, size_t ldc, const zc *pin, int nbin, GState *gs, double tiny,
                    const Launch &gc, const int *active)
{
    if (s <= 3)
        hipLaunchKernelGGL((k_upd_res<T, DIM, 4>), grid(gc), dim3(BLK), 0, gc.st, x, accumulate, B, s, F, C, bc, ldf,
                           ldc, pin, nbin, gs, tiny, gc.chunk, gc.nb, active);
    else
        hipLaunchKernelGGL((k_upd_res<T, DIM, NVAL - 1>), grid(gc), dim3(BLK), 0, gc.st, x, accumulate, B, s, F, C, bc,
                           ldf, ldc, pin, nbin, gs, tiny, gc.chunk, gc.nb, active);
}

template <typename T>
void launch_upd_r(Cx<T> *x, int accumulate, Cx<T> *r, const Basis<T> &B, int s, unsigned N, size_t ld, const zc *pin,
                  int nbin, GState *gs, double tiny, const Launch &g, const int *active)
{
    if (s <= 3)
        hipLaunchKernelGGL((k_upd_r<T, 4>), grid(g), dim3(BLK), 0, g.st, x, accumulate, r, B, s, N, ld, pin, nbin, gs,
                           tiny, g.chunk, g.nb, active);
    else
        hipLaunchKernelGGL((k_upd_r<T, NVAL - 1>), grid(g), dim3(BLK), 0, g.st, x, accumulate, r, B, s, N, ld, pin,
                           nbin, gs, tiny, g.chunk, g.nb, active);
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
                   const int *active, size_t mstride, unsigned rpp)
{
    hipLaunchKernelGGL((k_coarse<T>), dim3(1, nrhs), dim3(BLK), 0, st, minvT, n, b, x, ld, mstride, rpp, active);
}

// Shared start of the first-round kernels: sum the inner products of k_hdot
// (h_i = <v_i, w>, i <= j, and ||w||^2) from the RHS's partials pp into cc
// (group_parts: a fixed order, so every block gets the same bits) and take
// the block-uniform decision: twos = 1 when a second round is needed.
// Deferred second rounds (lazy): when column j - 1 took a second round, v_j
// holds its first-round form v~_j and the coefficients c~ and scale g of
// v_j = g (v~_j - sum_{i<j} c~_i v_i) sit in the FGMRES state (pends = 1,
// ccor, gps); <v_j, w> then follows from the inner products already formed.
// scs scales the first round's result into v_{j+1} (final column) or into the
// next first-round form v~_{j+1} (second round pending; any positive scale
// serves, 1/||w1|| when the estimate ||w||^2 - ||h||^2 is usable).  cx holds
// the coefficients of the vectors as stored (v~_j in place of v_j).
__device__ __forceinline__ void proj0_head(const FState *fs, int j, const zc *pp, int nbin, bool lazy, zc *cc,
                                           zc *cx, zc *ccor, double &scs, double &gps, int &twos, int &pends)
{
    const bool pend = lazy && j > 0 && fs->pend;
    for (int q = threadIdx.x / FG; q <= j + 1; q += BLK / FG) {
        const zc v = group_parts(pp + q * NBMAX, nbin);
        if (threadIdx.x % FG == 0) cc[q] = v;
    }
    if (pend)
        for (int q = threadIdx.x; q < j; q += BLK) ccor[q] = fs->corr[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        const double gp = pend ? fs->gpend : 0.0;
        if (pend) {
            zc t = mkc(0.0, 0.0);
            for (int q = 0; q < j; ++q) t = cjfma(ccor[q], cc[q], t);
            cc[j] = gp * (cc[j] - t);
        }
        const double w2 = cc[j + 1].re;
        double h2 = 0.0;
        for (int q = 0; q <= j; ++q) h2 += cabs2(cc[q]);
        const double w1 = w2 - h2;
        // Daniel-Gragg-Kaufman-Stewart criterion: one round is final when it
        // keeps at least 1/sqrt(2) of ||w||; a laxer bound lets the error of
        // the single round (ratio ||h|| / ||w1|| times the basis's own loss of
        // orthogonality) compound from column to column
        const int two = fs->force2 || !(w1 >= 0.5 * w2);   // force2: every column, for tests
        double sc;
        if (!two) sc = w1 > 0.0 ? 1.0 / sqrt(w1) : 0.0;
        else sc = w1 > 1e-8 * w2 ? 1.0 / sqrt(w1) : (w2 > 0.0 ? 1.0 / sqrt(w2) : 0.0);
        twos = two;
        scs = sc;
        gps = gp;
        pends = pend;
    }
    __syncthreads();
    // coefficients of the vectors as stored: w1 = w - sum_q cx_q u_q with u_j = v~_j
    // when pending, i.e. cx_q = h_q - h_j g c~_q (q < j) and cx_j = h_j g
    for (int q = threadIdx.x; q <= j; q += BLK) {
        zc v = cc[q];
        if (pend) v = q < j ? cc[q] - (gps * cc[j]) * ccor[q] : gps * cc[j];
        cx[q] = v;
    }
    __syncthreads();
}

// Shared end of the first-round kernels (block 0): the FGMRES state advances
// by the column h, the flag of the second round and, for a final column, the
// Givens step, the report and the stop test.
__device__ __forceinline__ void proj0_state(FState *fs, Report *rep, int *stop, int j, const zc *cc, bool two,
                                            double sc)
{
    constexpr int M = CSG_MAX_RESTART;
    __shared__ zc col[OVAL];
    __shared__ double cs_s[M];
    __shared__ zc sn_s[M];
    for (int q = threadIdx.x; q < j; q += BLK) {
        cs_s[q] = fs->cs[q];
        sn_s[q] = fs->sn[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q <= j; ++q) {
            col[q] = cc[q];
            fs->hcol[q] = cc[q];
        }
        const double w2 = cc[j + 1].re;
        double h2 = 0.0;
        for (int q = 0; q <= j; ++q) h2 += cabs2(cc[q]);
        fs->w2 = w2;
        fs->reorth = two;
        fs->sc1 = sc;
        if (!two) givens_column(fs, rep, j, sqrt(w2 - h2), col, cs_s, sn_s, stop);
    }
    __syncthreads();
    if (!two)
        for (int q = threadIdx.x; q <= j + 1; q += BLK) fs->R[q * M + j] = col[q];
}

// First round of column j, finished and applied in one launch.  Every block
// sums the inner products of k_hdot (proj0_head) and takes the same decision:
// with ||w1||^2 = ||w||^2 - ||h||^2 (w1 = w - V h, V orthonormal) the column is
// final when ||w1||^2 >= ||w||^2 / 2; then h_{j+1,j} = ||w1|| and the block
// writes its chunk of v_{j+1} = w1 / h_{j+1,j} and its optional
// cycle-precision copy.  Otherwise it writes the second round's partials into
// pout (a buffer apart from pin, which other blocks may still be reading):
// <v_i, w1> (values 0..j) and ||w1||^2 (value j + 1), and either keeps w1 in w
// for k_proj1 or (lazy) writes the first-round form v~_{j+1} = scs w1 into
// v_{j+1}'s place and the copy: the V-cycle takes v~_{j+1} (flexible GMRES
// accepts any preconditioner input), k_col finishes the column, and the next
// column's first projection, which reads the whole basis anyway, replaces
// v~_{j+1} by v_{j+1} (vfix = v_j's place; pending form, see proj0_head).
// Block 0 then advances the FGMRES state: the column h, the flag of the
// second round and, for a final column, the Givens step, the report and the
// stop test (stop clears the RHS in the mask; blocks that read the mask after
// that skip their chunk of a v_{j+1} that is never used).
template <typename TB, int JB>
__global__ __launch_bounds__(BLK) void k_proj0(zc *__restrict__ w, const zc *__restrict__ V, size_t vstride, int j,
                                               unsigned N, size_t ld, FState *fsb, Report *rep, int *stop,
                                               const zc *__restrict__ pin, int nbin, zc *__restrict__ pout,
                                               zc *__restrict__ vout, Cx<TB> *__restrict__ bc, zc *vfix, int lazy,
                                               unsigned chunk, int nb, const int *active)
{
    __shared__ zc sh[(BLK / 64) * 8];
    __shared__ zc res[8];
    __shared__ zc cc[OVAL];
    __shared__ zc cx[OVAL];
    __shared__ zc ccor[OVAL];
    __shared__ double scs, gps;
    __shared__ int twos, pends;
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    FState *fs = fsb + rhs;
    proj0_head(fs, j, pin + (size_t)rhs * OVAL * NBMAX, nbin, lazy != 0 && JB > 0, cc, cx, ccor, scs, gps, twos,
               pends);
    const bool two = twos != 0, pend = pends != 0;
    const double sc = scs, gp = gps;
    const size_t off = rhs * ld;
    zc acc[1] = {mkc(0.0, 0.0)};
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk + threadIdx.x, p1 = min(N, c * chunk + chunk);
    if (JB > 0) {
        // every basis value of a point held in registers: the pending
        // correction of v_j, the first projection and, for a second round, its
        // inner products <v_i, w1> in one pass over V (j + 1 <= JB)
        zc dots[JB > 0 ? JB : 1];
#pragma unroll
        for (int q = 0; q < JB; ++q) dots[q] = mkc(0.0, 0.0);
        for (unsigned p = p0; p < p1; p += BLK) {
            zc v[JB > 0 ? JB : 1];
#pragma unroll
            for (int q = 0; q < JB; ++q)
                if (q <= j) v[q] = pend && q == j ? vfix[off + p] : V[q * vstride + off + p];
            const int oz = opaque_zero();
            zc x = w[off + p];
#pragma unroll
            for (int q = 0; q < JB; ++q)
                if (q <= j) x = x - cx[q + oz] * v[q];
            if (pend) {
                // v_j = g (v~_j - sum_{q<j} c~_q v_q), stored and used by the second round
                zc t = mkc(0.0, 0.0);
#pragma unroll
                for (int q = 0; q < JB; ++q)
                    if (q < j) t = cfma(ccor[q + oz], v[q], t);
#pragma unroll
                for (int q = 0; q < JB; ++q)
                    if (q == j) {
                        v[q] = gp * (v[q] - t);
                        vfix[off + p] = v[q];
                    }
            }
            if (two) {
                if (lazy) {
                    const zc vn = sc * x;
                    vout[off + p] = vn;
                    if (bc) bc[off + p] = cvt<TB>(vn);
                } else {
                    w[off + p] = x;
                }
                acc[0].re += cabs2(x);
#pragma unroll
                for (int q = 0; q < JB; ++q)
                    if (q <= j) dots[q] = cjfma(v[q], x, dots[q]);
            } else {
                const zc vn = sc * x;
                vout[off + p] = vn;
                if (bc) bc[off + p] = cvt<TB>(vn);
            }
        }
        if (two) {
            zc *po = pout + (size_t)rhs * OVAL * NBMAX;
            block_sum<1>(acc, 1, sh, res);
            if (threadIdx.x == 0) po[(j + 1) * NBMAX + c] = res[0];
#pragma unroll
            for (int g = 0; g < (JB + 7) / 8; ++g) {
                if (8 * g > j) break;
                zc d8[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) d8[q] = 8 * g + q < JB ? dots[8 * g + q < JB ? 8 * g + q : 0] : mkc(0.0, 0.0);
                store_group(d8, g, j, po, c, sh, res);
            }
        }
    } else if (p0 < p1) {
        // (not lazy: the host keeps k_proj1 for this path)
        const unsigned last = p1 - 1;
        for (unsigned p = p0; p < p1; p += UO * BLK) {
            zc x[UO];
            proj_batch(w, V, vstride, j, off, p, last, cc, x);
#pragma unroll
            for (int k = 0; k < UO; ++k) {
                if (p + k * BLK >= p1) break;
                if (two) {
                    w[off + p + k * BLK] = x[k];
                    acc[0].re += cabs2(x[k]);
                } else {
                    const zc v = sc * x[k];
                    vout[off + p + k * BLK] = v;
                    if (bc) bc[off + p + k * BLK] = cvt<TB>(v);
                }
            }
        }
    }
    if (JB == 0 && two) {
        zc *po = pout + (size_t)rhs * OVAL * NBMAX;
        block_sum<1>(acc, 1, sh, res);
        if (threadIdx.x == 0) po[(j + 1) * NBMAX + c] = res[0];
        // second-round inner products <v_i, w_1> (values 0..j) over the same
        // chunk: each thread re-reads the w_1 points it has just written
        for (int g = 0; 8 * g <= j; ++g) {
            zc dots[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) dots[q] = mkc(0.0, 0.0);
            dots8(w, V, vstride, g, j, off, p0, p1, dots);
            store_group(dots, g, j, po, c, sh, res);
        }
    }
    if (blockIdx.x != 0) return;
    proj0_state(fs, rep + rhs, stop ? stop + rhs : nullptr, j, cc, two, sc);
}

// k_proj0 for columns of more than 16 basis vectors, reading V once: the
// basis is split over the block's wavefronts (wavefront wv holds v_q for
// q = wv, wv + NW, ..., QW of them at most) and every lane takes PU points per
// step, so a point's basis values sit in the registers of NW lanes.  Each
// wavefront forms its share of (sum_q cx_q u_q)(p) (the vectors as stored,
// proj0_head) and, for a pending v_j, of (sum_{i<j} c~_i v_i)(p), in
// ascending q; the shares meet in shared memory with w(p), and every
// wavefront sums them in wavefront order, so all form the same
// w1(p) = w(p) - sum.  The wavefront holding v~_j forms and stores
// v_j = g (v~_j - sum); wavefront 0 stores w1 (or v_{j+1}, v~_{j+1} and the
// copy), and for a second round each wavefront accumulates the inner products
// <v_q, w1> of its own vectors and wavefront 0 also ||w1||^2.  The shares are
// double-buffered, so one barrier per step suffices.
// one step's loads of the split first projection: this wavefront's basis
// values v_{wv + NW k} (slot kfix from the corrected copy) at the step's
// points, and in slot QW w there for the last wavefront
template <int QW, int PU, int NW>
__device__ __forceinline__ void proj0w_load(zc (&v)[PU][QW + 1], unsigned pb, unsigned b1, int lane, int wv, int nq,
                                            int kfix, const zc *__restrict__ V, size_t vstride, const zc *vfix,
                                            const zc *w, size_t off)
{
#pragma unroll
    for (int u = 0; u < PU; ++u) {
        const unsigned pc = min(pb + u * 64 + lane, b1 - 1);
#pragma unroll
        for (int k = 0; k < QW; ++k)
            if (k < nq) v[u][k] = k == kfix ? vfix[off + pc] : V[(wv + NW * k) * vstride + off + pc];
        if (wv == NW - 1) {
            const zc x = w[off + pc];
            v[u][QW] = mkc(x.re, x.im);
        }
    }
}

// (four vectors per wavefront, one group per step: registers capped for two
// workgroups per CU, which the form fits without spilling)
template <typename TB, int QW, int PU, bool PF>
__global__ __launch_bounds__(BLK, QW * PU <= 4 ? 4 : 2) void k_proj0w(zc *__restrict__ w, const zc *__restrict__ V, size_t vstride, int j,
                                                unsigned N, size_t ld, FState *fsb, Report *rep, int *stop,
                                                const zc *__restrict__ pin, int nbin, zc *__restrict__ pout,
                                                zc *__restrict__ vout, Cx<TB> *__restrict__ bc, zc *vfix, int lazy,
                                                unsigned chunk, int nb, const int *active)
{
    constexpr int NW = BLK / 64;
    constexpr int NV = QW + 1;                    // QW inner products and ||w1||^2
    constexpr int ND = pow2_at_least(2 * NV);
    constexpr int SH = ND == 2 ? 5 : ND == 4 ? 4 : ND == 8 ? 3 : ND == 16 ? 2 : ND == 32 ? 1 : 0;
    __shared__ zc cc[OVAL];
    __shared__ zc cx[OVAL];
    __shared__ zc ccor[OVAL];
    __shared__ double scs, gps;
    __shared__ int twos, pends;
    __shared__ zc shareH[2][NW][PU * 64];
    __shared__ zc shareC[2][NW][PU * 64];
    __shared__ zc wsh[2][PU * 64];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    FState *fs = fsb + rhs;
    proj0_head(fs, j, pin + (size_t)rhs * OVAL * NBMAX, nbin, lazy != 0, cc, cx, ccor, scs, gps, twos, pends);
    const bool two = twos != 0, pend = pends != 0;
    const double sc = scs, gp = gps;
    const size_t off = rhs * ld;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nq = (j + NW - wv) / NW;            // vectors wv, wv + NW, ... <= j
    const int wj = j % NW, kj = j / NW;           // the wavefront and slot holding v_j
    const unsigned c = chunk_id(nb);
    const unsigned b0 = c * chunk, b1 = min(N, b0 + chunk);
    zc dots[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) dots[k] = mkc(0.0, 0.0);
    // PF: each step's loads are issued one step ahead, while the previous
    // step finishes (otherwise nothing is in flight across a step's barrier);
    // the arithmetic and its order are the same
    zc vq[PU][QW + 1];
    const int kfix = pend && wv == wj ? kj : -1;
    if (PF && b0 < b1) proj0w_load<QW, PU, NW>(vq, b0, b1, lane, wv, nq, kfix, V, vstride, vfix, w, off);
    int buf = 0;
    for (unsigned pb = b0; pb < b1; pb += PU * 64, buf ^= 1) {
        zc v[PU][QW];
        if (PF) {
#pragma unroll
            for (int u = 0; u < PU; ++u) {
#pragma unroll
                for (int k = 0; k < QW; ++k)
                    if (k < nq) v[u][k] = vq[u][k];
                if (wv == NW - 1) wsh[buf][u * 64 + lane] = mkc(vq[u][QW].re, vq[u][QW].im);
            }
        } else {
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            const unsigned pc = min(pb + u * 64 + lane, b1 - 1);
#pragma unroll
            for (int k = 0; k < QW; ++k)
                if (k < nq) v[u][k] = pend && wv == wj && k == kj ? vfix[off + pc] : V[(wv + NW * k) * vstride + off + pc];
            if (wv == NW - 1) wsh[buf][u * 64 + lane] = w[off + pc];
        }
        }
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            zc a = mkc(0.0, 0.0), t = mkc(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < QW; ++k) {
                if (k >= nq) continue;
                a = a + cx[wv + NW * k] * v[u][k];
                if (pend && wv + NW * k < j) t = cfma(ccor[wv + NW * k], v[u][k], t);
            }
            shareH[buf][wv][u * 64 + lane] = a;
            if (pend) shareC[buf][wv][u * 64 + lane] = t;
        }
        __syncthreads();
        if (PF && pb + PU * 64 < b1)
            proj0w_load<QW, PU, NW>(vq, pb + PU * 64, b1, lane, wv, nq, kfix, V, vstride, vfix, w, off);
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            const unsigned p = pb + u * 64 + lane;
            const int e = u * 64 + lane;
            zc a = shareH[buf][0][e];
#pragma unroll
            for (int t = 1; t < NW; ++t) a = a + shareH[buf][t][e];
            const zc x = wsh[buf][e] - a;
            if (pend && wv == wj) {
                // the wavefront holding v~_j forms v_j = g (v~_j - sum_{q<j} c~_q v_q)
                zc cs = shareC[buf][0][e];
#pragma unroll
                for (int t = 1; t < NW; ++t) cs = cs + shareC[buf][t][e];
#pragma unroll
                for (int k = 0; k < QW; ++k)
                    if (k == kj) {
                        v[u][k] = gp * (v[u][k] - cs);
                        if (p < b1) vfix[off + p] = v[u][k];
                    }
            }
            if (p < b1) {
                if (two) {
                    if (wv == 0) {
                        if (lazy) {
                            const zc vn = sc * x;
                            vout[off + p] = vn;
                            if (bc) bc[off + p] = cvt<TB>(vn);
                        } else {
                            w[off + p] = x;
                        }
                        dots[QW].re += cabs2(x);
                    }
#pragma unroll
                    for (int k = 0; k < QW; ++k)
                        if (k < nq) dots[k] = cjfma(v[u][k], x, dots[k]);
                } else if (wv == 0) {
                    const zc vn = sc * x;
                    vout[off + p] = vn;
                    if (bc) bc[off + p] = cvt<TB>(vn);
                }
            }
        }
    }
    if (two) {
        // wavefront totals straight into the partials: value wv + NW k from
        // wavefront wv, ||w1||^2 (value j + 1) from wavefront 0
        double d[ND];
#pragma unroll
        for (int k = 0; k < ND / 2; ++k) {
            const zc x = dots[k < NV ? k : 0];
            d[2 * k] = k < NV ? x.re : 0.0;
            d[2 * k + 1] = k < NV ? x.im : 0.0;
        }
        const double t = wave_totals<ND>(d);
        const int idx = lane >> SH, k = idx >> 1;
        zc *po = pout + (size_t)rhs * OVAL * NBMAX;
        if ((lane & ((1 << SH) - 1)) == 0 && k < NV) {
            int q = -1;
            if (k < QW && k < nq) q = wv + NW * k;
            if (k == QW && wv == 0) q = j + 1;
            if (q >= 0) reinterpret_cast<double *>(po + (size_t)q * NBMAX + c)[idx & 1] = t;
        }
    }
    if (blockIdx.x != 0) return;
    proj0_state(fs, rep + rhs, stop ? stop + rhs : nullptr, j, cc, two, sc);
}

// Finish of column j when its second round is deferred (lazy): one block per
// RHS sums the second round's inner products c_i = <v_i, w1> (i <= j) and
// ||w1||^2 from k_proj0's partials, takes h_{j+1,j} = sqrt(||w1||^2 - ||c||^2)
// (0 at a breakdown), keeps c~ = scs c and g = 1 / (scs h_{j+1,j}) for the next
// first projection (v_{j+1} = g (v~_{j+1} - sum_i c~_i v_i)) and advances the
// FGMRES state: the column h + c, the Givens step, the report and the stop
// test, so a converged RHS takes no further V-cycle.  After a final column it
// only clears the pending flag.
__global__ __launch_bounds__(BLK) void k_col(int j, FState *fsb, Report *rep, int *stop, const zc *__restrict__ pin,
                                             int nbin, const int *active)
{
    constexpr int M = CSG_MAX_RESTART;
    __shared__ zc cc[OVAL];
    __shared__ zc col[OVAL];
    __shared__ double cs_s[M];
    __shared__ zc sn_s[M];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    FState *fs = fsb + rhs;
    if (!fs->reorth) {
        if (threadIdx.x == 0) fs->pend = 0;
        return;
    }
    const zc *pp = pin + (size_t)rhs * OVAL * NBMAX;
    for (int q = threadIdx.x / FG; q <= j + 1; q += BLK / FG) {
        const zc v = group_parts(pp + q * NBMAX, nbin);
        if (threadIdx.x % FG == 0) cc[q] = v;
    }
    for (int q = threadIdx.x; q < j; q += BLK) {
        cs_s[q] = fs->cs[q];
        sn_s[q] = fs->sn[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double sc = fs->sc1;
        double c2 = 0.0;
        for (int q = 0; q <= j; ++q) {
            c2 += cabs2(cc[q]);
            col[q] = fs->hcol[q] + cc[q];
            fs->hcol[q] = col[q];
            fs->corr[q] = sc * cc[q];
        }
        const double w2 = cc[j + 1].re, h2 = w2 - c2;
        const double hn = h2 > 1e-13 * w2 ? sqrt(h2) : 0.0;
        fs->gpend = hn > 0.0 && sc > 0.0 ? 1.0 / (sc * hn) : 0.0;
        fs->pend = 1;
        givens_column(fs, rep + rhs, j, hn, col, cs_s, sn_s, stop ? stop + rhs : nullptr);
    }
    __syncthreads();
    for (int q = threadIdx.x; q <= j + 1; q += BLK) fs->R[q * M + j] = col[q];
}

// Second round of column j, finished and applied in one launch (columns
// whose first round was final return at once).  Every block sums the
// second-round inner products c_i = <v_i, w1> (i <= j) and ||w1||^2 from their
// partials (group_parts, as in k_proj0); h_{j+1,j}^2 = ||w1||^2 -
// ||c||^2 is the norm of w1 - V c for orthonormal V (a difference at rounding
// level of ||w1||^2 means w1 lies in span(V): breakdown, h = 0), and the block
// writes its chunk of v_{j+1} = (w1 - V c) / h_{j+1,j} with the optional
// cycle-precision copy.  Block 0 then advances the FGMRES state: the column
// h + c, the Givens step, the report and the stop test.
template <typename TB>
__global__ __launch_bounds__(BLK) void k_proj1(const zc *__restrict__ w, const zc *__restrict__ V, size_t vstride,
                                               int j, unsigned N, size_t ld, FState *fsb, Report *rep, int *stop,
                                               const zc *__restrict__ pin, int nbin, zc *__restrict__ vout,
                                               Cx<TB> *__restrict__ bc, unsigned chunk, int nb, const int *active)
{
    constexpr int M = CSG_MAX_RESTART;
    __shared__ zc cc[OVAL];
    __shared__ double scs;
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    FState *fs = fsb + rhs;
    if (!fs->reorth) return;   // v_{j+1} already written by the first projection
    {
        const zc *pp = pin + (size_t)rhs * OVAL * NBMAX;
        for (int q = threadIdx.x / FG; q <= j + 1; q += BLK / FG) {
            const zc v = group_parts(pp + q * NBMAX, nbin);
            if (threadIdx.x % FG == 0) cc[q] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double c2 = 0.0;
        for (int q = 0; q <= j; ++q) c2 += cabs2(cc[q]);
        const double w2 = cc[j + 1].re, h2 = w2 - c2;
        const double hn = h2 > 1e-13 * w2 ? sqrt(h2) : 0.0;
        scs = hn > 0.0 ? 1.0 / hn : 0.0;
    }
    __syncthreads();
    const double sc = scs;
    const size_t off = rhs * ld;
    const unsigned c = chunk_id(nb);
    const unsigned p0 = c * chunk + threadIdx.x, p1 = min(N, c * chunk + chunk);
    if (p0 < p1) {
        const unsigned last = p1 - 1;
        for (unsigned p = p0; p < p1; p += UO * BLK) {
            zc x[UO];
            proj_batch(w, V, vstride, j, off, p, last, cc, x);
#pragma unroll
            for (int k = 0; k < UO; ++k) {
                if (p + k * BLK >= p1) break;
                const zc v = sc * x[k];
                vout[off + p + k * BLK] = v;
                if (bc) bc[off + p + k * BLK] = cvt<TB>(v);
            }
        }
    }
    if (blockIdx.x != 0) return;
    // the FGMRES state (block 0)
    __shared__ zc col[OVAL];
    __shared__ double cs_s[M];
    __shared__ zc sn_s[M];
    for (int q = threadIdx.x; q < j; q += BLK) {
        cs_s[q] = fs->cs[q];
        sn_s[q] = fs->sn[q];
    }
    for (int q = threadIdx.x; q <= j; q += BLK) {
        const zc h1 = fs->hcol[q];
        col[q] = h1;
        fs->corr[q] = cc[q];
        fs->hcol[q] = h1 + cc[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double c2 = 0.0;
        for (int q = 0; q <= j; ++q) {
            col[q] = col[q] + cc[q];
            c2 += cabs2(cc[q]);
        }
        const double w2 = cc[j + 1].re, h2 = w2 - c2;
        givens_column(fs, rep + rhs, j, h2 > 1e-13 * w2 ? sqrt(h2) : 0.0, col, cs_s, sn_s,
                      stop ? stop + rhs : nullptr);
    }
    __syncthreads();
    for (int q = threadIdx.x; q <= j + 1; q += BLK) fs->R[q * M + j] = col[q];
}

template <typename TZ, int DIM>
void launch_hdot(const LvlK<double> &H, const Cx<TZ> *z, zc *w, const zc *V, size_t vstride, int j, size_t ld,
                 zc *pout, const Launch &g, const int *active)
{
    hipLaunchKernelGGL((k_hdot<TZ, DIM>), grid(g), dim3(BLK), 0, g.st, H, z, w, V, vstride, j, ld, pout, g.chunk,
                       g.nb, active);
}

template <typename TZ>
void launch_slab_hdot(const LvlK<double> &H, const Cx<TZ> *z, zc *w, const zc *V, size_t vstride, int j, size_t ld,
                      zc *pout, const SlabGeo &sg, int nrhs, hipStream_t st, const int *active)
{
    const int nslab = (int)sg.npad;
    hipLaunchKernelGGL((k_slab_hdot<TZ>), dim3(nslab, nrhs), dim3(BLK), 0, st, H, z, w, V, vstride, j, ld, pout,
                       sg.ntx, sg.nty, sg.nzc, sg.zrun, nslab, active);
    if (j >= 8) {
        const unsigned chunk = (unsigned)((H.N + nslab - 1) / nslab);
        hipLaunchKernelGGL(k_hdot_groups, dim3(nslab, nrhs), dim3(BLK), 0, st, w, V, vstride, j, H.N, ld, pout, chunk,
                           nslab, active);
    }
}

template <typename TZ>
void launch_hdot_tile(const LvlK<double> &H, const Cx<TZ> *z, zc *w, const zc *V, size_t vstride, int j, size_t ld,
                      zc *pout, const TileGeo &tg, int nrhs, hipStream_t st, const int *active)
{
    const int ntile = (int)(tg.ntx * tg.nty);
    hipLaunchKernelGGL((k_hdot_tile<TZ>), dim3(ntile, nrhs), dim3(BLK), 0, st, H, z, w, V, vstride, j, ld, pout, tg,
                       ntile, active);
}

// the wavefront-split first round for columns of 17..64 vectors (CSG_PROJ0W=0:
// the two-pass k_proj0 instead, for comparisons)
static bool wide_proj0()
{
    static const bool on = [] {
        const char *e = getenv("CSG_PROJ0W");
        return !(e && atoi(e) == 0);
    }();
    return on;
}

// CSG_PROJ0W_GROUPS=1: steps of one group of points whatever the launch size
// (for tests on small grids)
static bool proj0w_one_group()
{
    static const bool on = [] {
        const char *e = getenv("CSG_PROJ0W_GROUPS");
        return e && atoi(e) == 1;
    }();
    return on;
}

// whether the split first projection loads a step ahead (CSG_PROJ0W_AHEAD=0:
// loads at the top of each step, for comparisons)
static bool proj0w_ahead()
{
    static const bool on = [] {
        const char *e = getenv("CSG_PROJ0W_AHEAD");
        return !(e && atoi(e) == 0);
    }();
    return on;
}

template <typename TB>
void launch_proj0(zc *w, const zc *V, size_t vstride, int j, unsigned N, size_t ld, FState *fs, Report *rep,
                  int *stop, const zc *pin, int nbin, zc *pout, zc *vout, Cx<TB> *bcast, zc *vfix, int lazy,
                  const Launch &g, const int *active)
{
    // columns of up to 16 basis vectors keep a point's whole basis in one
    // lane's registers (more would spill); longer ones split it over the
    // block's wavefronts, loading each step's values while the previous step
    // finishes (without that, a block has no loads in flight across each
    // step's barrier: a fifth more time in this pass on 16 right-hand sides
    // of 128^3, 6 % more whole-solve time on one right-hand side of 1024^2).
    // Launches of many workgroups take steps of one group of 64 points, whose
    // registers leave room for two workgroups per CU (6 % less time in this
    // pass on 16 right-hand sides of 128^3); with about one workgroup per CU
    // (one right-hand side) steps of two groups keep more loads in flight.
    const bool ahead = proj0w_ahead();
    const bool few = (long)g.nb * g.nrhs < 1024 && !proj0w_one_group();
    if (j + 1 <= 8)
        hipLaunchKernelGGL((k_proj0<TB, 8>), grid(g), dim3(BLK), 0, g.st, w, V, vstride, j, N, ld, fs, rep, stop, pin,
                           nbin, pout, vout, bcast, vfix, lazy, g.chunk, g.nb, active);
    else if (j + 1 <= 16)
        hipLaunchKernelGGL((k_proj0<TB, 16>), grid(g), dim3(BLK), 0, g.st, w, V, vstride, j, N, ld, fs, rep, stop, pin,
                           nbin, pout, vout, bcast, vfix, lazy, g.chunk, g.nb, active);
    else if (j + 1 <= 4 * (BLK / 64) && wide_proj0() && ahead && !few)
        hipLaunchKernelGGL((k_proj0w<TB, 4, 1, true>), grid(g), dim3(BLK), 0, g.st, w, V, vstride, j, N, ld, fs, rep,
                           stop, pin, nbin, pout, vout, bcast, vfix, lazy, g.chunk, g.nb, active);
    else if (j + 1 <= 4 * (BLK / 64) && wide_proj0() && ahead)
        hipLaunchKernelGGL((k_proj0w<TB, 4, 2, true>), grid(g), dim3(BLK), 0, g.st, w, V, vstride, j, N, ld, fs, rep,
                           stop, pin, nbin, pout, vout, bcast, vfix, lazy, g.chunk, g.nb, active);
    else if (j + 1 <= 4 * (BLK / 64) && wide_proj0())
        hipLaunchKernelGGL((k_proj0w<TB, 4, 2, false>), grid(g), dim3(BLK), 0, g.st, w, V, vstride, j, N, ld, fs, rep,
                           stop, pin, nbin, pout, vout, bcast, vfix, lazy, g.chunk, g.nb, active);
    else if (j + 1 <= 8 * (BLK / 64) && wide_proj0() && ahead)
        hipLaunchKernelGGL((k_proj0w<TB, 8, 1, true>), grid(g), dim3(BLK), 0, g.st, w, V, vstride, j, N, ld, fs, rep,
                           stop, pin, nbin, pout, vout, bcast, vfix, lazy, g.chunk, g.nb, active);
    else if (j + 1 <= 8 * (BLK / 64) && wide_proj0())
        hipLaunchKernelGGL((k_proj0w<TB, 8, 1, false>), grid(g), dim3(BLK), 0, g.st, w, V, vstride, j, N, ld, fs, rep,
                           stop, pin, nbin, pout, vout, bcast, vfix, lazy, g.chunk, g.nb, active);
    else
        hipLaunchKernelGGL((k_proj0<TB, 0>), grid(g), dim3(BLK), 0, g.st, w, V, vstride, j, N, ld, fs, rep, stop, pin,
                           nbin, pout, vout, bcast, vfix, lazy, g.chunk, g.nb, active);
}

void launch_col(int j, FState *fs, Report *rep, int *stop, const zc *pin, int nbin, int nrhs, hipStream_t st,
                const int *active)
{
    hipLaunchKernelGGL(k_col, dim3(1, nrhs), dim3(BLK), 0, st, j, fs, rep, stop, pin, nbin, active);
}

template <typename TB>
void launch_proj1(const zc *w, const zc *V, size_t vstride, int j, unsigned N, size_t ld, FState *fs, Report *rep,
                  int *stop, const zc *pin, int nbin, zc *vout, Cx<TB> *bcast, const Launch &g, const int *active)
{
    hipLaunchKernelGGL((k_proj1<TB>), grid(g), dim3(BLK), 0, g.st, w, V, vstride, j, N, ld, fs, rep, stop, pin, nbin,
                       vout, bcast, g.chunk, g.nb, active);
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
                const int *active, int *stop)
{
    hipLaunchKernelGGL(k_fin, dim3(nrhs), dim3(FT), 0, st, mode, pin, nbin, j, fs, rep, active, stop);
}

__global__ void k_fs_params(FState *fs, double tol, int maxit, int force2, int nrhs)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nrhs) {
        fs[r].tol = tol;
        fs[r].maxit = maxit;
        fs[r].it = 0;
        fs[r].force2 = force2;
    }
}

void launch_fs_params(FState *fs, double tol, int maxit, int force2, int nrhs, hipStream_t st)
{
    hipLaunchKernelGGL(k_fs_params, dim3((nrhs + 63) / 64), dim3(64), 0, st, fs, tol, maxit, force2, nrhs);
}

template <typename T, int DIM>
size_t tail_lds_bytes(const unsigned *N, int lt, int L, int s)
{
    if (N[lt] > (unsigned)(tail_mp<T>() * TB)) return ~(size_t)0;   // more points per thread than the register stencils
    size_t n = 0;
    for (int l = lt; l < L - 1; ++l) n += (size_t)tail_vectors<T>(s) * N[l];
    n += 2 * (size_t)N[L - 1];
    if (lt == L - 1 || (size_t)(tail_vectors<T>(s) - 2) * N[lt] < TB) n += TB;   // coarse-solve partials
    return n * sizeof(Cx<T>);
}

template <typename T, int DIM>
bool tail_lds_prepare(size_t bytes, int s)
{
    const void *f = s <= 3 ? (const void *)k_tail_lds<T, DIM, 4> : (const void *)k_tail_lds<T, DIM, NVAL - 1>;
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess;
}

template <typename T, int DIM>
void launch_tail(const TLev<T> *lev, int lt, int L, const Cx<T> *b_in, Cx<T> *x_out, const Cx<T> *minvT, int nc,
                 int s, int nu1, int nu2, double tiny, int nrhs, size_t lds, hipStream_t st, const int *active,
                 size_t mstride)
{
    if (lds) {
        if (s <= 3)
            hipLaunchKernelGGL((k_tail_lds<T, DIM, 4>), dim3(nrhs), dim3(TB), lds, st, lev, lt, L, b_in, x_out, minvT,
                               nc, s, nu1, nu2, tiny, mstride, active);
        else
            hipLaunchKernelGGL((k_tail_lds<T, DIM, NVAL - 1>), dim3(nrhs), dim3(TB), lds, st, lev, lt, L, b_in, x_out,
                               minvT, nc, s, nu1, nu2, tiny, mstride, active);
        return;
    }
    if (s <= 3)
        hipLaunchKernelGGL((k_tail<T, DIM, 4>), dim3(nrhs), dim3(TB), 0, st, lev, lt, L, b_in, x_out, minvT, nc, s, nu1,
                           nu2, tiny, mstride, active);
    else
        hipLaunchKernelGGL((k_tail<T, DIM, NVAL - 1>), dim3(nrhs), dim3(TB), 0, st, lev, lt, L, b_in, x_out, minvT, nc,
                           s, nu1, nu2, tiny, mstride, active);
}

template <typename T, int DIM>
void launch_rich(const LvlK<T> &L, const Cx<T> *xin, const Cx<T> *b, Cx<T> *xout, Cx<T> w, size_t ld, const Launch &g,
                 const int *active)
{
    hipLaunchKernelGGL((k_rich<T, DIM>), grid(g), dim3(BLK), 0, g.st, L, xin, b, xout, w, ld, g.chunk, g.nb, active);
}

unsigned poly_tiles(unsigned nx, unsigned ny) { return ((nx + PT - 1) / PT) * ((ny + PT - 1) / PT); }

template <typename T>
void launch_poly_tile(const LvlK<T> &L, const LvlK<T> &C, const Cx<T> *ec, const Cx<T> *xin, const Cx<T> *b,
                      Cx<T> *xout, const Cx<T> (&w)[3], size_t ld, size_t ldc, int nrhs, hipStream_t st,
                      const int *active)
{
    const unsigned ntx = (L.nx + PT - 1) / PT;
    const dim3 gr(poly_tiles(L.nx, L.ny), nrhs);
    if (ec)
        hipLaunchKernelGGL((k_poly_tile<T, false, true>), gr, dim3(BLK), 0, st, L, C, ec, xin, b, xout, w[0], w[1], w[2],
                           ld, ldc, ntx, active);
    else if (xin)
        hipLaunchKernelGGL((k_poly_tile<T, false, false>), gr, dim3(BLK), 0, st, L, C, ec, xin, b, xout, w[0], w[1],
                           w[2], ld, ldc, ntx, active);
    else
        hipLaunchKernelGGL((k_poly_tile<T, true, false>), gr, dim3(BLK), 0, st, L, C, ec, xin, b, xout, w[0], w[1],
                           w[2], ld, ldc, ntx, active);
}

void launch_copy_mask(const int *src, int *dst, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy_mask, dim3((n + 255) / 256), dim3(256), 0, st, src, dst, n);
}

// n 16-byte words set to zero with vector stores (a kernel, not a memset node,
// so the clear also behaves inside captured graphs)
__global__ void k_zero16(uint4 *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

void launch_zero16(void *p, size_t bytes, hipStream_t st)
{
    const size_t n = bytes / 16;
    if (n == 0) return;
    const unsigned nb = (unsigned)std::min<size_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(k_zero16, dim3(nb), dim3(256), 0, st, (uint4 *)p, n);
}

// ---------------------------------------------------------------------------
// explicit instantiations
// ---------------------------------------------------------------------------

#define INST_TD(T, D)                                                                                               \
    template void launch_apply<T, D>(const LvlK<T> &, const void *, void *, size_t, const Launch &, const int *);  \
    template void launch_rich<T, D>(const LvlK<T> &, const Cx<T> *, const Cx<T> *, Cx<T> *, Cx<T>, size_t,         \
                                    const Launch &, const int *);                                                  \
    template void launch_st0<T, D>(const LvlK<T> &, const Cx<T> *, Cx<T> *, int, size_t, zc *, const Launch &,     \
                                   const int *);                                                                   \
    template void launch_stj<T, D>(const LvlK<T> &, const Basis<T> &, Cx<T> *, int, int, size_t, zc *,             \
                                   const Launch &, const int *);                                                   \
    template void launch_os<T, D>(const LvlK<T> &, const Basis<T> &, const Cx<T> *, Cx<T> *, int, int, size_t,     \
                                  const zc *, int, zc *, GState *, double, const Launch &, const int *);           \
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
    template void launch_hdot<T, D>(const LvlK<double> &, const Cx<T> *, zc *, const zc *, size_t, int, size_t,    \
                                    zc *, const Launch &, const int *);                                            \
    template void launch_tail<T, D>(const TLev<T> *, int, int, const Cx<T> *, Cx<T> *, const Cx<T> *, int, int,     \
                                    int, int, double, int, size_t, hipStream_t, const int *, size_t);              \
    template size_t tail_lds_bytes<T, D>(const unsigned *, int, int, int);                                         \
    template bool tail_lds_prepare<T, D>(size_t, int);

INST_TD(double, 2)
INST_TD(double, 3)
INST_TD(float, 2)
INST_TD(float, 3)

template void launch_slab_hdot<double>(const LvlK<double> &, const Cx<double> *, zc *, const zc *, size_t, int,
                                       size_t, zc *, const SlabGeo &, int, hipStream_t, const int *);
template void launch_slab_hdot<float>(const LvlK<double> &, const Cx<float> *, zc *, const zc *, size_t, int, size_t,
                                      zc *, const SlabGeo &, int, hipStream_t, const int *);
template void launch_hdot_tile<double>(const LvlK<double> &, const Cx<double> *, zc *, const zc *, size_t, int,
                                       size_t, zc *, const TileGeo &, int, hipStream_t, const int *);
template void launch_hdot_tile<float>(const LvlK<double> &, const Cx<float> *, zc *, const zc *, size_t, int,
                                      size_t, zc *, const TileGeo &, int, hipStream_t, const int *);

#define INST_T(T)                                                                                                  \
    template void launch_st0_tile<T>(const LvlK<T> &, const Cx<T> *, Cx<T> *, size_t, bool, zc *, const TileGeo &,  \
                                     int, hipStream_t, const int *);                                               \
    template void launch_down_tile<T>(Cx<T> *, int, const Basis<T> &, int, const LvlK<T> &, const LvlK<T> &,       \
                                      Cx<T> *, Cx<T> *, size_t, size_t, const zc *, int, GState *, double, bool,   \
                                      bool, zc *, const TileGeo &, int, hipStream_t, const int *);                 \
    template void launch_up_tile<T>(const LvlK<T> &, const LvlK<T> &, const Cx<T> *, const Cx<T> *, Cx<T> *,      \
                                    const Cx<T> *, Cx<T> *, Cx<T> *, size_t, size_t, bool, zc *, const TileGeo &,  \
                                    int, hipStream_t, const int *, const UpClose<T> *);                            \
    template void launch_orthl<T>(const Basis<T> &, const Cx<T> *, int, int, unsigned, size_t, const zc *, int,    \
                                  zc *, GState *, double, const Launch &, const int *);                            \
    template void launch_upd<T>(Cx<T> *, int, const Basis<T> &, int, unsigned, size_t, const zc *, int, GState *, \
                                double, const Launch &, const int *);                                              \
    template void launch_upd_r<T>(Cx<T> *, int, Cx<T> *, const Basis<T> &, int, unsigned, size_t, const zc *, int, \
                                  GState *, double, const Launch &, const int *);                                  \
    template void launch_os_tile<T>(const LvlK<T> &, const Basis<T> &, const Cx<T> *, Cx<T> *, int, int, size_t,   \
                                    const zc *, int, zc *, GState *, double, const TileGeo &, int, hipStream_t,    \
                                    const int *);                                                                  \
    template void launch_coarse<T>(const Cx<T> *, int, const Cx<T> *, Cx<T> *, size_t, int, hipStream_t,          \
                                   const int *, size_t, unsigned);                                                 \
    template void launch_vnorm<T>(const zc *, zc *, Cx<T> *, unsigned, size_t, const FState *, const Launch &,     \
                                  const int *);                                                                    \
    template void launch_proj1<T>(const zc *, const zc *, size_t, int, unsigned, size_t, FState *, Report *,       \
                                  int *, const zc *, int, zc *, Cx<T> *, const Launch &, const int *);             \
    template void launch_proj0<T>(zc *, const zc *, size_t, int, unsigned, size_t, FState *, Report *, int *,      \
                                  const zc *, int, zc *, zc *, Cx<T> *, zc *, int, const Launch &, const int *);   \
    template void launch_uupd<T>(zc *, const Cx<T> *, size_t, unsigned, size_t, const FState *, const Launch &,    \
                                 const int *);                                                                     \
    template void launch_slab<T>(const LvlK<T> &, const Basis<T> &, const Cx<T> *, Cx<T> *, int, int, size_t,     \
                                 const zc *, int, zc *, GState *, double, bool, const SlabGeo &, int, hipStream_t, \
                                 const int *);                                                                     \
    template void launch_slab_down<T>(Cx<T> *, int, const Basis<T> &, int, const LvlK<T> &, const LvlK<T> &,      \
                                      Cx<T> *, size_t, size_t, const zc *, int, GState *, double, const SlabGeo &, \
                                      int, hipStream_t, const int *);                                              \
    template void launch_slab_pr<T>(const LvlK<T> &, const LvlK<T> &, const Cx<T> *, const Cx<T> *, Cx<T> *,      \
                                    const Cx<T> *, Cx<T> *, size_t, size_t, const SlabGeo &, int, hipStream_t,    \
                                    const int *);                                                                  \
    template void launch_poly_tile<T>(const LvlK<T> &, const LvlK<T> &, const Cx<T> *, const Cx<T> *,            \
                                      const Cx<T> *, Cx<T> *, const Cx<T>(&)[3], size_t, size_t, int, hipStream_t, \
                                      const int *);

INST_T(double)
INST_T(float)

template void launch_tres<2>(const LvlK<double> &, const zc *, const zc *, zc *, size_t, int, zc *, const Launch &,
                             const int *);
template void launch_tres<3>(const LvlK<double> &, const zc *, const zc *, zc *, size_t, int, zc *, const Launch &,
                             const int *);

}  // namespace csg
