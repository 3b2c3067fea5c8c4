// kernels.h -- host-side launchers of the gfx950 kernels of libcsg.
#pragma once

#include "csg_internal.h"

namespace csg {

// Geometry of one level as seen by a kernel (tables and phi in precision T).
template <typename T>
struct LvlK {
    const Cx<T> *tab[3];   // per axis [west | centre | east], boundary weights zeroed
    const T *phi;
    unsigned nx, ny, nz, N;
    // A batch of problems of one size class (same grid, levels and cycle)
    // side by side: right-hand side r belongs to problem r / rpp, whose
    // tables and phi sit tstride[a] and pstride elements after the previous
    // problem's (rpp = 0: one problem).
    unsigned rpp;
    unsigned tstride[3];
    size_t pstride;
    // complex factor s of phi in the operator's diagonal (sum of the axes'
    // centre weights - s phi): 1 for H and the CSG preconditioner, 1 + i eps
    // for the complex shifted Laplacian
    double sre = 1.0, sim = 0.0;
    // Galerkin levels: 3^d coefficients per point, [offset][point] (offset
    // index sum_a (o_a + 1) 3^a), zero towards neighbours outside the grid;
    // gstride elements between problems.  Null: the Kronecker-sum form above.
    const Cx<T> *gst = nullptr;
    size_t gstride = 0;
    // the geometry as right-hand side rhs sees it
    __host__ __device__ __forceinline__ LvlK at(int rhs) const
    {
        LvlK r = *this;
        if (rpp) {
            const unsigned q = (unsigned)rhs / rpp;
            for (int a = 0; a < 3; ++a)
                if (r.tab[a]) r.tab[a] += (size_t)q * tstride[a];
            r.phi += q * pstride;
            if (r.gst) r.gst += q * gstride;
        }
        return r;
    }
};

// Up to CSG_MAX_S+1 basis vector pointers (u_0..u_s) of one level.
template <typename T>
struct Basis {
    Cx<T> *u[CSG_MAX_S + 1];
};

// Device-resident description of one level for the coarse-tail kernel.
template <typename T>
struct TLev {
    const Cx<T> *tab[3];
    const T *phi;
    Cx<T> *b, *xa, *xb, *r;
    Cx<T> *u[CSG_MAX_S + 1];
    Cx<T> *w[2];
    unsigned nx, ny, nz, N;
    size_t ld;
    // batches (see LvlK): problem stride of the tables and phi, RHS per problem
    unsigned rpp;
    unsigned tstride[3];
    size_t pstride;
    double sre = 1.0, sim = 0.0;   // factor of phi (see LvlK)
};

struct Launch {
    int nb;            // blocks along x (chunked passes: <= NBCH)
    unsigned chunk;    // points per block
    int nrhs;
    hipStream_t st;
};

// ---- smoother / cycle passes (T = float or double, DIM = 2 or 3) ----------
template <typename T, int DIM>
void launch_apply(const LvlK<T> &L, const void *x, void *y, size_t ld, const Launch &g, const int *active);

// GMRES(s) Arnoldi passes on the raw basis (see kernels.hip): pass 0, fused
// Gram-Schmidt + stencil passes j = 0..s-2; the last of them also sums
// ||w_{s-1}||^2 (wn) so the closing pass needs no further Gram-Schmidt pass.
template <typename T, int DIM>
void launch_st0(const LvlK<T> &L, const Cx<T> *u0, Cx<T> *w, int wn, size_t ld, zc *pout, const Launch &g,
                const int *active);

// unfused pass: w = A u_j, <u_i, w> (i <= j) and ||u_j||^2 (and ||w||^2 when j = s-1)
template <typename T, int DIM>
void launch_stj(const LvlK<T> &L, const Basis<T> &B, Cx<T> *w, int j, int s, size_t ld, zc *pout, const Launch &g,
                const int *active);

template <typename T, int DIM>
void launch_os(const LvlK<T> &L, const Basis<T> &B, const Cx<T> *win, Cx<T> *wout, int j, int s, size_t ld,
               const zc *pin, int nbin, zc *pout, GState *gs, double tiny, const Launch &g, const int *active);

// Fused pass j+1 on 2-D tiles (s <= 3): u_{j+1} is formed once per point of
// the tile and its one-point halo into shared memory, then w_{j+1} = A u_{j+1}
// is taken from there; same outputs as launch_os, partials by tile.
template <typename T>
void launch_os_tile(const LvlK<T> &L, const Basis<T> &B, const Cx<T> *win, Cx<T> *wout, int j, int s, size_t ld,
                    const zc *pin, int nbin, zc *pout, GState *gs, double tiny, const TileGeo &tg, int nrhs,
                    hipStream_t st, const int *active);

// Interpolated correction, the residual that opens the post-sweep and that
// sweep's pass 0 on 2-D tiles: xout = xin + P ec (xin may be null, never
// xout), r = b - A xout, w = A r with <r, w>, ||r||^2 (and ||w||^2 when
// wnorm) per tile into pout.  Same outputs as launch_prolong, launch_resid and
// launch_st0 in turn, partials by tile.
// With fuse: ec is not read; the pass first applies the coarse level's
// post-sweep closing update (x_c = fuse->xb + sum_{i<k} cx_i u_i, s <= 3) on
// the coarse nodes its interpolation reads, so that update needs no pass of
// its own and x_c is never stored.
template <typename T>
struct UpClose {
    Basis<T> B;        // the coarse sweep's closing basis
    const Cx<T> *xb;   // coarse x before the update
    const zc *pin;     // partials of the coarse sweep's last pass
    int nbin;
    GState *gs;        // the coarse sweep's state [rhs]
    int s;
    double tiny;
};
template <typename T>
void launch_up_tile(const LvlK<T> &F, const LvlK<T> &C, const Cx<T> *ec, const Cx<T> *xin, Cx<T> *xout,
                    const Cx<T> *b, Cx<T> *r, Cx<T> *w, size_t ldf, size_t ldc, bool wnorm, zc *pout,
                    const TileGeo &tg, int nrhs, hipStream_t st, const int *active,
                    const UpClose<T> *fuse = nullptr);

// Arnoldi pass on 3-D z-marching slabs: j = -1 is pass 0 (w_0 = A u_0, like
// launch_st0), j >= 0 the fused pass j+1 (like launch_os); s <= 3; one partial
// per slab run.
template <typename T>
void launch_slab(const LvlK<T> &L, const Basis<T> &B, const Cx<T> *win, Cx<T> *wout, int j, int s, size_t ld,
                 const zc *pin, int nbin, zc *pout, GState *gs, double tiny, bool wnorm, const SlabGeo &sg, int nrhs,
                 hipStream_t st, const int *active);
// closing update of a pre-sweep and the restriction of its Arnoldi residual on the slabs of a 3-D level
template <typename T>
void launch_slab_down(Cx<T> *x, int accumulate, const Basis<T> &B, int s, const LvlK<T> &F, const LvlK<T> &C,
                      Cx<T> *bc, size_t ldf, size_t ldc, const zc *pin, int nbin, GState *gs, double tiny,
                      const SlabGeo &sg, int nrhs, hipStream_t st, const int *active);
// interpolated correction and the residual opening the post-sweep on the slabs of a 3-D level
template <typename T>
void launch_slab_pr(const LvlK<T> &F, const LvlK<T> &C, const Cx<T> *ec, const Cx<T> *xin, Cx<T> *xout,
                    const Cx<T> *b, Cx<T> *r, size_t ldf, size_t ldc, const SlabGeo &sg, int nrhs, hipStream_t st,
                    const int *active);

// Pass 0 of a sweep on 2-D tiles: w = A u0 with <u0, w>, ||u0||^2 (and
// ||w||^2 when wnorm) per tile into pout; same outputs as launch_st0,
// partials by tile.
template <typename T>
void launch_st0_tile(const LvlK<T> &L, const Cx<T> *u0, Cx<T> *w, size_t ld, bool wnorm, zc *pout, const TileGeo &tg,
                     int nrhs, hipStream_t st, const int *active);

// Closing pass of the last pre-sweep on a 2-D level, the restriction and
// (st0) pass 0 of the coarse level's first sweep, on tiles tc of the coarse
// level: x (+)= sum cx_i u_i, bc = 2^-d P^T r with the Arnoldi residual
// r = sum cr_i u_i, and with st0 wc = A_c bc with <bc, wc>, ||bc||^2 (and
// ||wc||^2 when wnorm) per coarse tile into pout.  Same outputs as
// launch_upd_r, launch_restrict and launch_st0 in turn (r itself is not
// stored), partials by coarse tile.  Requires F.nx <= 2 C.nx + 1 and
// F.ny <= 2 C.ny + 1 (every fine point lies under the coarse grid).
template <typename T>
void launch_down_tile(Cx<T> *x, int accumulate, const Basis<T> &B, int s, const LvlK<T> &F, const LvlK<T> &C,
                      Cx<T> *bc, Cx<T> *wc, size_t ldf, size_t ldc, const zc *pin, int nbin, GState *gs,
                      double tiny, bool st0, bool wnorm, zc *pout, const TileGeo &tc, int nrhs, hipStream_t st,
                      const int *active);

template <typename T>
void launch_orthl(const Basis<T> &B, const Cx<T> *win, int j, int s, unsigned N, size_t ld, const zc *pin, int nbin,
                  zc *pout, GState *gs, double tiny, const Launch &g, const int *active);

template <typename T>
void launch_upd(Cx<T> *x, int accumulate, const Basis<T> &B, int s, unsigned N, size_t ld, const zc *pin,
                int nbin, GState *gs, double tiny, const Launch &g, const int *active);

// x (+)= V y and r = V (beta e1 - Hbar y) on the fine grid (closing pass of a sweep)
template <typename T>
void launch_upd_r(Cx<T> *x, int accumulate, Cx<T> *r, const Basis<T> &B, int s, unsigned N, size_t ld, const zc *pin,
                  int nbin, GState *gs, double tiny, const Launch &g, const int *active);

template <typename T, int DIM>
void launch_upd_res(Cx<T> *x, int accumulate, const Basis<T> &B, int s, const LvlK<T> &F, const LvlK<T> &C,
                    Cx<T> *bc, size_t ldf, size_t ldc, const zc *pin, int nbin, GState *gs, double tiny,
                    const Launch &gc, const int *active);

template <typename T, int DIM>
void launch_resid(const LvlK<T> &L, const Cx<T> *x, const Cx<T> *b, Cx<T> *r, size_t ld, const Launch &g,
                  const int *active);

template <typename T, int DIM>
void launch_restrict(const LvlK<T> &F, const LvlK<T> &C, const Cx<T> *x, const Cx<T> *b, Cx<T> *bc,
                     size_t ldf, size_t ldc, const Launch &gc, const int *active);

template <typename T, int DIM>
void launch_prolong(const LvlK<T> &F, const LvlK<T> &C, const Cx<T> *ec, const Cx<T> *xin, Cx<T> *xout,
                    size_t ldf, size_t ldc, const Launch &g, const int *active);

template <typename T, int DIM>
void launch_prc(const LvlK<T> &F, const LvlK<T> &C, const Cx<T> *ec, const Cx<T> *xin, Cx<T> *xout,
                const Cx<T> *b, Cx<T> *r, size_t ldf, size_t ldc, const Launch &g, const int *active);

// mstride, rpp: batches (see LvlK): elements between the problems' inverses
template <typename T>
void launch_coarse(const Cx<T> *minvT, int n, const Cx<T> *b, Cx<T> *x, size_t ld, int nrhs, hipStream_t st,
                   const int *active, size_t mstride = 0, unsigned rpp = 0);

// One workgroup per RHS runs levels lt..L-1 of the V-cycle (input b at level lt,
// output x at level lt).
template <typename T, int DIM>
void launch_tail(const TLev<T> *lev, int lt, int L, const Cx<T> *b_in, Cx<T> *x_out, const Cx<T> *minvT, int nc,
                 int s, int nu1, int nu2, double tiny, int nrhs, size_t lds, hipStream_t st, const int *active,
                 size_t mstride = 0);

// Shared-memory bytes of the tail's vectors from level lt down (N[l] unknowns
// per level), and the one-time launch attribute that allows them (false: the
// tail runs from global memory).
template <typename T, int DIM>
size_t tail_lds_bytes(const unsigned *N, int lt, int L, int s);
template <typename T, int DIM>
bool tail_lds_prepare(size_t bytes, int s);
constexpr size_t TAIL_LDS_MAX = 156 * 1024;   // of the 160 KB per workgroup, the rest static

// ---- outer FGMRES passes (FP64 arithmetic; TZ = cycle precision) ----------
// w = H z and <v_i, w> (i <= j)
template <typename TZ, int DIM>
void launch_hdot(const LvlK<double> &H, const Cx<TZ> *z, zc *w, const zc *V, size_t vstride, int j, size_t ld,
                 zc *pout, const Launch &g, const int *active);

// the same on the finest level's 3-D z-marching slabs (one partial per slab
// block, sg.npad of them)
template <typename TZ>
void launch_slab_hdot(const LvlK<double> &H, const Cx<TZ> *z, zc *w, const zc *V, size_t vstride, int j, size_t ld,
                      zc *pout, const SlabGeo &sg, int nrhs, hipStream_t st, const int *active);

// the same on the finest level's 2-D tiles (one partial per tile)
template <typename TZ>
void launch_hdot_tile(const LvlK<double> &H, const Cx<TZ> *z, zc *w, const zc *V, size_t vstride, int j, size_t ld,
                      zc *pout, const TileGeo &tg, int nrhs, hipStream_t st, const int *active);

// first round of column j: the inner products of k_hdot summed from their
// partials (pin) in every block, w1 = w - V h kept in w with the second
// round's partials (pout) when the column takes the second round, else
// written normalised as v_{j+1}; block 0 advances the FGMRES state (Givens
// step, report, stop test clearing stop[rhs]) for a final column
template <typename TB>
void launch_proj0(zc *w, const zc *V, size_t vstride, int j, unsigned N, size_t ld, FState *fs, Report *rep,
                  int *stop, const zc *pin, int nbin, zc *pout, zc *vout, Cx<TB> *bcast, zc *vfix, int lazy,
                  const Launch &g, const int *active);
// finish of a column whose second Gram-Schmidt round is deferred (lazy)
void launch_col(int j, FState *fs, Report *rep, int *stop, const zc *pin, int nbin, int nrhs, hipStream_t st,
                const int *active);

// second round of column j (columns that take it): the second-round inner
// products summed from their partials (pin) in every block, v_{j+1} = (w1 -
// V c) / h_{j+1,j} with its optional cycle-precision copy; block 0 advances
// the FGMRES state (report, stop test clearing stop[rhs])
template <typename TB>
void launch_proj1(const zc *w, const zc *V, size_t vstride, int j, unsigned N, size_t ld, FState *fs, Report *rep,
                  int *stop, const zc *pin, int nbin, zc *vout, Cx<TB> *bcast, const Launch &g, const int *active);

// v = w * scale (scale = fs->inv_hn), optional cycle-precision copy (cast).
template <typename TB>
void launch_vnorm(const zc *w, zc *v, Cx<TB> *bcast, unsigned N, size_t ld, const FState *fs, const Launch &g,
                  const int *active);

template <int DIM>
void launch_tres(const LvlK<double> &H, const zc *chi, const zc *u, zc *r, size_t ld, int with_chi, zc *pout,
                 const Launch &g, const int *active);

template <typename TZ>
void launch_uupd(zc *u, const Cx<TZ> *Z, size_t zstride, unsigned N, size_t ld, const FState *fs, const Launch &g,
                 const int *active);

// finish kernel (start of a restart cycle, least squares): one block per RHS
enum FinMode { FIN_BEGIN = 3, FIN_BETA = 4, FIN_LS = 5 };
void launch_fin(int mode, const zc *pin, int nbin, int j, FState *fs, Report *rep, int nrhs, hipStream_t st,
                const int *active, int *stop = nullptr);

// Stopping parameters of a solve into every RHS's state (iteration count
// reset; force2: every column takes the second Gram-Schmidt round).
void launch_fs_params(FState *fs, double tol, int maxit, int force2, int nrhs, hipStream_t st);

void launch_copy_mask(const int *src, int *dst, int n, hipStream_t st);

// ---- third-order polynomial smoother (section 4) ---------------------------
// one Richardson step xout = xin + w (b - A xin) (xin null: zero; xout must
// not alias xin)
template <typename T, int DIM>
void launch_rich(const LvlK<T> &L, const Cx<T> *xin, const Cx<T> *b, Cx<T> *xout, Cx<T> w, size_t ld, const Launch &g,
                 const int *active);
// a whole sweep (three steps with weights w[0..2]) on 32 x 32 tiles of a 2-D
// level, from xin (null: zero) or, with ec, from xin + P ec; xout must not
// alias xin
template <typename T>
void launch_poly_tile(const LvlK<T> &L, const LvlK<T> &C, const Cx<T> *ec, const Cx<T> *xin, const Cx<T> *b,
                      Cx<T> *xout, const Cx<T> (&w)[3], size_t ld, size_t ldc, int nrhs, hipStream_t st,
                      const int *active);

// bytes (a multiple of 16, 16-byte aligned) of device memory set to zero
void launch_zero16(void *p, size_t bytes, hipStream_t st);

}  // namespace csg
