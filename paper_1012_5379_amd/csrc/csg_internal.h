// csg_internal.h -- internal structures of libcsg (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstddef>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "csg.h"
#include "cx.h"

namespace csg {

using cd = std::complex<double>;

constexpr int BLK = 512;                    // threads per block of every level pass
constexpr int NBMAX = 1024;                 // max blocks of a reducing pass (partials per value)
constexpr int NBCH = 256;                   // blocks of a chunked (untiled) level pass
constexpr int NVAL = CSG_MAX_S + 2;         // partial values per smoother pass
constexpr int OVAL = CSG_MAX_RESTART + 1;   // partial values per outer pass
constexpr int MAXC = 4096;                  // max coarsest unknowns
#define CSG_MAX_RHS_HOST CSG_MAX_RHS

// ---------------------------------------------------------------------------
// Device-resident small state
// ---------------------------------------------------------------------------

// GMRES(s) smoother state of one (level, right-hand side).  The Krylov basis is
// stored unnormalised (u_i) with v_i = sig[i] * u_i; H holds the Arnoldi
// coefficients h_ij of the normalised basis, row-major (s+1) x s.
struct GState {
    double sig[CSG_MAX_S + 2];
    zc H[(CSG_MAX_S + 1) * CSG_MAX_S];
    zc y[CSG_MAX_S];
    double beta0;
    int k;
    int pad;
};

// Flexible GMRES state of one right-hand side.
struct FState {
    zc R[(CSG_MAX_RESTART + 1) * CSG_MAX_RESTART];  // rotated Hessenberg, row-major ld = MAXR
    double cs[CSG_MAX_RESTART];
    zc sn[CSG_MAX_RESTART];
    zc g[CSG_MAX_RESTART + 1];
    zc hcol[CSG_MAX_RESTART + 1];   // current column (first + second CGS round)
    zc corr[CSG_MAX_RESTART + 1];   // second-round coefficients of the current column (lazy: scaled by sc1)
    zc y[CSG_MAX_RESTART];
    double beta;       // norm of the current restart residual
    double nchi;       // ||chi||
    double hn;         // h_{j+1,j} of the current column
    double inv_hn;     // scale applied to form v_{j+1}
    double w2;         // ||H z_j||^2 of the current column
    double tol;        // stopping tolerance of the solve
    int kcols;         // columns of the current restart cycle used by the update
    int reorth;        // the current column takes the second Gram-Schmidt round
    int it;            // outer iterations done by this RHS in the solve
    int maxit;         // iteration limit of the solve
    int force2;        // every column takes the second Gram-Schmidt round (experiments, tests)
    int pad;
    // deferred second rounds: scale of the first-round form v~_{j+1} = sc1 w1,
    // and, when pend, v_j = gpend (v~_j - sum_{i<j} corr_i v_i)
    double sc1;
    double gpend;
    int pend;
    int pad2;
};

// Outer iterations a solve keeps queued ahead of the host's reading of their
// reports (the device itself clears a RHS's iteration mask when it stops),
// captured GCOLS columns to a graph (fewer graph boundaries, each of which
// costs a launch gap on the device).
constexpr int GCOLS = 3;
constexpr int LOOKAHEAD = 2 * GCOLS;

// Host-visible per-RHS report (copied back after every outer iteration).
struct Report {
    double est;        // |g_{j+1}| / ||chi||  (or true relres after a restart)
    double hn;
    int finite;
    int pad;
};

// ---------------------------------------------------------------------------
// Host hierarchy (FP64), built by setup.cpp
// ---------------------------------------------------------------------------

struct HostLevel {
    int nint[3] = {0, 0, 0};   // intervals per axis
    int nu[3] = {1, 1, 1};     // unknowns per axis (1 on unused axes)
    long N = 0;
    std::vector<cd> z[3];      // nested complex node coordinates of M's grid
    std::vector<cd> tab[3];    // Shortley-Weller rows of M: [west | centre | east]
    std::vector<double> phi;
    // Galerkin coarse operator R M_{l-1} P (coarse_op = 1, levels >= 1): 3^d
    // coefficients per unknown, [offset][unknown], offset index
    // sum_a (o_a + 1) 3^a over the used axes; 0 towards neighbours outside the grid
    std::vector<cd> gst;
    // third-order polynomial smoother of this level (section 4)
    double varphi = 0.0;
    cd omega[3];
    int conds = 2;
};

struct HostHier {
    int dim = 2, L = 0;
    HostLevel lev[CSG_MAX_LEVELS];
    std::vector<cd> tabH[3];   // finest-level Shortley-Weller rows of H (theta = 0)
    std::vector<cd> minvT;     // coarsest M^{-1}, transposed (column j contiguous)
    int nc = 0;
};

int plan_levels(const csg_params &p, int &L, int nint[CSG_MAX_LEVELS][3], std::string &err);
// the factor s of phi in the preconditioner (1 when the parameters leave it at 0)
cd phi_shift(const csg_params &p);
int build_hierarchy(const csg_params &p, const double *phi, HostHier &hh, std::string &err);

// ---------------------------------------------------------------------------
// Device hierarchy carved from the caller's workspace
// ---------------------------------------------------------------------------

// 2-D tiling of a level for the LDS-staged fused pass: ntx x nty tiles of
// tx x ty points (the last ones ragged); partial sums indexed by tile.
struct TileGeo {
    unsigned ntx, nty, tx, ty;
};
// 3-D z-marching slabs of the Arnoldi passes: ntx x nty columns of 32 x 16
// x-y points, each split into nzc runs of zrun planes (one partial per run);
// launched as npad >= ntx * nty * nzc blocks, a multiple of 8 (the extra ones
// only write zero partials) so every XCD receives a contiguous range of
// columns and shares their halos in its L2.
struct SlabGeo {
    unsigned ntx, nty, nzc, zrun, npad;
};
constexpr int TILE_MAXE = 10;                 // halo-tile points per thread
constexpr int TILE_PRE = 2;                   // of them loaded before the pass's reduction
constexpr int TILE_PB = 4;                    // points per thread whose loads are issued together
constexpr int TILE_MAXN = TILE_MAXE * BLK;    // halo-tile points per block
constexpr int TAB_MAXD = 80;                  // tile columns / rows whose stencil tables are staged
// Whether a tiling exists, its halo tile fits the shared-memory buffer and
// the stencil tables of its columns and rows can be staged (one per thread).
inline bool tile_fits(const TileGeo &t)
{
    return t.ntx > 0 && (t.tx + 2) * (t.ty + 2) <= (unsigned)TILE_MAXN && t.tx <= (unsigned)TAB_MAXD &&
           t.ty <= (unsigned)TAB_MAXD && 3 * (t.tx + t.ty) <= (unsigned)BLK;
}
// The up-path tile pass (interpolation, residual and pass 0 of the post-sweep)
// stages the tile with a two-point halo.
constexpr int UP_MAXE = 11;                   // two-point-halo tile points per thread
constexpr int UP_MAXN = UP_MAXE * BLK;
// Coarse window of an up-path pass that applies the coarse closing update:
// at most UPC_E points per thread.
constexpr int UPC_E = 4;
constexpr int UPC_MAXN = UPC_E * BLK;
inline bool upc_fits(const TileGeo &t) { return (t.tx / 2 + 4) * (t.ty / 2 + 4) <= (unsigned)UPC_MAXN; }
inline bool up_fits(const TileGeo &t)
{
    return tile_fits(t) && (t.tx + 4) * (t.ty + 4) <= (unsigned)UP_MAXN && t.tx + 2 <= (unsigned)TAB_MAXD &&
           t.ty + 2 <= (unsigned)TAB_MAXD && 3 * (t.tx + t.ty + 4) <= (unsigned)BLK;
}
// The down-path tile pass (closing of the last pre-sweep, restriction and pass
// 0 of the next level) runs on tiles of the coarse level: it stages the fine
// points under the tile and its one-point halo, and the coarse tile with halo.
constexpr int DN_MAXE = 4;                    // coarse halo-tile points per thread
constexpr int DN_MAXB = DN_MAXE * BLK;
inline bool down_fits(const TileGeo &tc)
{
    return tc.ntx > 0 && (int)(tc.ntx * tc.nty) <= NBMAX && (2 * tc.tx + 5) * (2 * tc.ty + 5) <= (unsigned)UP_MAXN &&
           (tc.tx + 2) * (tc.ty + 2) <= (unsigned)DN_MAXB && tc.tx <= (unsigned)TAB_MAXD &&
           tc.ty <= (unsigned)TAB_MAXD && 3 * (tc.tx + tc.ty) <= (unsigned)BLK;
}

struct DevLevel {
    unsigned nu[3];
    unsigned N;
    size_t ld;                 // elements between consecutive RHS vectors
    const void *tab[3];        // cycle-precision complex tables (boundary weights zeroed)
    const void *phi;           // cycle-precision real phi
    const void *gst;           // Galerkin levels: cycle-precision 3^d-point stencil per problem (else null)
    void *b, *xa, *xb, *r;     // cycle-precision vectors [max_rhs][ld]
    void *u[CSG_MAX_S + 1];    // u[1..s]; u[0] aliases b or r
    void *w[2];                // stencil outputs of the Arnoldi passes (ping-pong)
    zc *part[2];               // reduction partials [max_rhs][NVAL][NBMAX]
    GState *gs;                // [max_rhs]
    int nb;                    // blocks of a reducing pass
    unsigned chunk;            // points per block of a reducing pass
    TileGeo tile;              // 2-D tiling of the LDS-staged fused pass (ntx = 0: none)
    TileGeo dtile;             // tiling of the down-path pass that restricts onto this level
    SlabGeo slab;              // 3-D slabs of the Arnoldi passes (nzc = 0: none)
    double varphi;             // polynomial smoother: p(t0) = e^{i varphi}
    cd omega[3];               // ... its Richardson weights, in the order they are applied
    int conds;                 // ... which necessary stability conditions varphi meets
};

// Instantiated graphs of one FGMRES iteration (V-cycle + outer passes), per
// right-hand-side count and Arnoldi column, captured on a private stream.
struct GraphCache {
    std::map<int, std::vector<hipGraphExec_t>> it;   // by nrhs and cycle length: graphs by first column
    hipStream_t cap = nullptr;
    bool enabled = true;
};

// Event-pair instrumentation of one pass kind (benchmarks only).
struct Prof {
    int kind = 0;
    int cap = 0;
    int n = 0;
    std::vector<hipEvent_t> ev;   // 2 * cap events: start, stop
    std::vector<double> bytes;    // per timed launch
    std::vector<long> col;        // per timed launch: FGMRES column number (-1: outside columns)
    long cur = -1;                // column being enqueued
    long next = 0;                // first column number of the next cycle
    std::vector<std::pair<long, long>> skipped;   // [first, last) columns queued after a halt
};

}  // namespace csg

struct csg_operator {
    csg_params p;                     // (a batch: max_rhs is the total over its problems)
    int nprob;                        // problems side by side (csg_batch_create), 1 otherwise
    int rpp;                          // right-hand sides per problem (rhs r belongs to problem r / rpp)
    int L;
    int csize;                        // bytes of one cycle complex (8 or 16)
    csg::DevLevel lev[CSG_MAX_LEVELS];
    const void *tabH[3];              // FP64 H tables
    const double *phiH;               // FP64 phi on the finest level
    const void *minvT;                // coarsest inverse (cycle precision), transposed
    int nc;
    void *tlev;                       // device level descriptors of the coarse tail
    int lt;                           // first level handled by the coarse-tail kernel
    size_t tail_lds;                  // shared-memory bytes of the tail's vectors (0: tail in global memory)
    long fuse_max;                    // levels up to this size use the fused Arnoldi passes
    bool tiles;                       // 2-D levels whose tiles fit use the LDS-staged fused pass
    bool hdot_tiles;                  // w = H z and its inner products on the finest level's tiles
    bool up_tiles;                    // ... and the LDS-staged interpolation + residual + pass 0
    bool down_tiles;                  // ... and the LDS-staged closing + restriction + next pass 0
    bool fuse_upd;                    // coarse post-sweep updates applied by the finer up-path pass
    bool force_cgs2;                  // every outer column takes the second Gram-Schmidt round
    bool lazy;                        // second rounds deferred into the next first projection
    bool slab_pr;                     // 3-D slab levels: interpolation and residual in one slab pass
    bool slab_down;                   // 3-D slab levels: closing update and restriction in one slab pass
    bool poly_tiles;                  // polynomial sweeps of 2-D levels run as one tiled launch
    long slab_min;                    // 3-D levels from this size run the Arnoldi passes on z-marching slabs
    // outer FGMRES storage
    csg::zc *V;                       // (m+1) x max_rhs x ld0
    void *Z;                          // m x max_rhs x ld0, cycle precision
    csg::zc *w;                       // max_rhs x ld0
    void *b0;                         // cycle-precision copy of v_j (mixed mode)
    csg::zc *opart;                   // [max_rhs][OVAL][NBMAX]
    csg::zc *opart2;                  // second-round partials of the first projection, same layout
    csg::FState *fs;                  // [max_rhs]
    int *active;                      // [max_rhs] device mask of RHS still iterating
    int *ones;                        // [max_rhs] device all-ones mask
    csg::Report *rep_host;            // pinned host reports: LOOKAHEAD + 1 slots of max_rhs, written by k_proj0/k_proj1 and k_fin
    csg::Report *rep_dev;             // the same memory as the device addresses it
    hipEvent_t evq[csg::LOOKAHEAD + 1];   // one per report slot (the last: cycle begin / end)
    size_t ws_used;
    int busy;                         // a csg_solve is in flight
    csg::Prof *prof;                  // instrumentation, or null
    csg::GraphCache *gc;              // captured FGMRES iterations
};
