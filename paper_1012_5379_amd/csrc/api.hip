// api.hip -- C ABI of libcsg: workspace layout, operator construction, the
// V-cycle sequence (section 3.1) and the flexible GMRES driver (section 5).
#include <dlfcn.h>

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "kernels.h"

using namespace csg;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(x)                                                                               \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess) return fail(CSG_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// Scratch of csg_smooth_static (callers that cannot allocate device memory):
// one array per GPU, created with the code object and held until the process
// ends.  Host code never passes `scratch` itself (in host code the name is a
// stand-in, not a device address): it uses the address hipGetSymbolAddress
// returned for the device, kept in scratch_dev.
// ---------------------------------------------------------------------------
constexpr size_t SCRATCH_BYTES = (size_t)128 << 20;
static __device__ __align__(256) char scratch[SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEV = 64;
std::mutex g_scratch_mu;
char *g_scratch_dev[SCRATCH_MAX_DEV];   // device address of `scratch` per device (null: not looked up yet)

// The current device's address of `scratch`, looked up once per device with
// that device current; null (with the error in g_err) on failure.
char *scratch_dev()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SCRATCH_MAX_DEV) {
        g_err = "no current HIP device for the static scratch";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            g_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_scratch_dev[dev] = (char *)ptr;
    }
    return g_scratch_dev[dev];
}

// Bump allocator over the caller's workspace (base == nullptr: size only).
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base((char *)b) {}
    void *take(size_t bytes)
    {
        off = (off + 255) & ~(size_t)255;
        void *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
};

// Blocks and points per block of a pass over n points.
void geometry(unsigned n, int &nb, unsigned &chunk)
{
    long want = ((long)n + BLK - 1) / BLK;
    if (want < 1) want = 1;
    nb = (int)std::min<long>(NBCH, want);
    if (nb >= 8) nb &= ~7;
    long per = ((long)n + nb - 1) / nb;
    chunk = (unsigned)(((per + BLK - 1) / BLK) * BLK);
}

// Tiles of a 2-D level for the LDS-staged fused pass: as many as the chunked
// passes have blocks (nb), tile rows in multiples of 8 when nb is, so the
// XCD-aware block order hands each XCD a band of rows as in the chunked passes;
// where such tiles overflow the shared-memory buffer, 2, 4 ... times as many
// (at most NBMAX partials per value).
TileGeo tiling_n(unsigned nx, unsigned ny, int nb);
TileGeo tiling(unsigned nx, unsigned ny, int nb)
{
    for (int k = nb; k >= 1 && k <= NBMAX; k *= 2) {
        const TileGeo t = tiling_n(nx, ny, k);
        if (t.ntx) return t;
    }
    return TileGeo{0, 0, 0, 0};
}
TileGeo tiling_n(unsigned nx, unsigned ny, int nb)
{
    TileGeo t{0, 0, 0, 0};
    if (nb < 1) return t;
    unsigned nty;
    if (nb >= 64 && nb % 8 == 0) {
        const unsigned k = std::max(1u, (unsigned)std::lround(std::sqrt((double)nb) / 8.0));
        nty = 8 * k;
    } else {
        nty = std::max(1u, (unsigned)std::lround(std::sqrt((double)nb)));
    }
    nty = std::min(nty, ny);
    unsigned ntx = std::max(1u, std::min((unsigned)nb / nty, nx));
    t.tx = (nx + ntx - 1) / ntx;
    t.ty = (ny + nty - 1) / nty;
    // no empty tile rows or columns
    t.ntx = (nx + t.tx - 1) / t.tx;
    t.nty = (ny + t.ty - 1) / t.ty;
    if (!tile_fits(t) || (int)(t.ntx * t.nty) > NBMAX) t.ntx = 0;
    return t;
}

// Tiling of the down-path pass onto a coarse level: small tiles whose fine
// footprint each thread covers with one batch of loads, when they number at
// most NBCH; else the level's own tiling.
TileGeo down_tiling(unsigned nx, unsigned ny, const TileGeo &dflt)
{
    constexpr unsigned D = 20;   // (2 D + 5)^2 <= TILE_PB * BLK
    static_assert((2 * D + 5) * (2 * D + 5) <= (unsigned)(TILE_PB * BLK), "one batch per thread");
    TileGeo t;
    t.tx = std::min(D, nx);
    t.ty = std::min(D, ny);
    t.ntx = (nx + t.tx - 1) / t.tx;
    t.nty = (ny + t.ty - 1) / t.ty;
    if (down_fits(t) && (int)(t.ntx * t.nty) <= NBCH) return t;
    return dflt;
}

// z-marching slabs of a 3-D level: columns of 32 x 16 points; enough runs of
// planes for about 128 blocks per right-hand side (runs of at least 4 planes,
// at most NBMAX partials).  The geometry depends on the level alone, so a
// right-hand side's result is the same whatever else shares its launches.
SlabGeo slab_geo(unsigned nx, unsigned ny, unsigned nz, int blocks)
{
    SlabGeo g{0, 0, 0, 0, 0};
    g.ntx = (nx + 31) / 32;
    g.nty = (ny + 15) / 16;
    const unsigned cols = g.ntx * g.nty;
    if (cols == 0 || cols + 8 > (unsigned)NBMAX) return SlabGeo{0, 0, 0, 0, 0};
    unsigned target = 128u;
    if (const char *e = getenv("CSG_SLAB_BLOCKS")) target = (unsigned)std::max(1, atoi(e));
    if (blocks > 0) target = (unsigned)blocks;
    unsigned want = (target + cols - 1) / cols;
    want = std::max(1u, std::min({want, (unsigned)(NBMAX - 8) / cols, std::max(1u, nz / 4)}));
    g.zrun = (nz + want - 1) / want;
    g.nzc = (nz + g.zrun - 1) / g.zrun;
    g.npad = (g.ntx * g.nty * g.nzc + 7) / 8 * 8;
    return g;
}

// The layout of every buffer in the workspace; `op` may be a dry-run object.
void carve(csg_operator &op, const int nint[CSG_MAX_LEVELS][3], Carver &cv)
{
    const csg_params &p = op.p;
    const int R = p.max_rhs;
    const size_t cz = op.csize, cr = cz / 2;
    for (int l = 0; l < op.L; ++l) {
        DevLevel &lv = op.lev[l];
        lv.N = 1;
        for (int a = 0; a < 3; ++a) {
            lv.nu[a] = a < p.dim ? (unsigned)(nint[l][a] - 1) : 1u;
            lv.N *= lv.nu[a];
        }
        lv.ld = lv.N;
        geometry(lv.N, lv.nb, lv.chunk);
        lv.tile = p.dim == 2 ? tiling(lv.nu[0], lv.nu[1], lv.nb * std::max(1, p.tile_mult)) : TileGeo{0, 0, 0, 0};
        lv.dtile = p.dim == 2 ? down_tiling(lv.nu[0], lv.nu[1], lv.tile) : TileGeo{0, 0, 0, 0};
        lv.slab = p.dim == 3 ? slab_geo(lv.nu[0], lv.nu[1], lv.nu[2], p.slab_blocks) : SlabGeo{0, 0, 0, 0, 0};
        for (int a = 0; a < p.dim; ++a) lv.tab[a] = cv.take((size_t)op.nprob * 3 * lv.nu[a] * cz);
        for (int a = p.dim; a < 3; ++a) lv.tab[a] = nullptr;
        lv.phi = cv.take((size_t)op.nprob * lv.N * cr);
        lv.gst = p.coarse_op == 1 && l > 0 ? cv.take((size_t)op.nprob * (p.dim == 2 ? 9 : 27) * lv.N * cz) : nullptr;
        const size_t vb = (size_t)R * lv.N * cz;
        lv.b = cv.take(vb);
        lv.xa = cv.take(vb);
        lv.xb = cv.take(vb);
        lv.r = cv.take(vb);
        lv.u[0] = nullptr;
        for (int i = 1; i <= CSG_MAX_S; ++i) lv.u[i] = i <= p.s ? cv.take(vb) : nullptr;
        lv.w[0] = cv.take(vb);
        lv.w[1] = cv.take(vb);
        for (int k = 0; k < 2; ++k) lv.part[k] = (zc *)cv.take((size_t)R * NVAL * NBMAX * sizeof(zc));
        lv.gs = (GState *)cv.take((size_t)R * sizeof(GState));
    }
    const DevLevel &f = op.lev[0];
    for (int a = 0; a < p.dim; ++a) op.tabH[a] = cv.take((size_t)op.nprob * 3 * f.nu[a] * sizeof(zc));
    for (int a = p.dim; a < 3; ++a) op.tabH[a] = nullptr;
    op.phiH = (const double *)cv.take((size_t)op.nprob * f.N * sizeof(double));
    const DevLevel &c = op.lev[op.L - 1];
    op.nc = (int)c.N;
    op.minvT = cv.take((size_t)op.nprob * op.nc * op.nc * cz);
    op.tlev = cv.take((size_t)op.L * sizeof(TLev<double>));
    const size_t n0 = (size_t)R * f.N;
    op.V = (zc *)cv.take((size_t)(p.restart + 1) * n0 * sizeof(zc));
    op.Z = cv.take((size_t)p.restart * n0 * cz);
    op.w = (zc *)cv.take(n0 * sizeof(zc));
    op.b0 = p.cycle_prec ? cv.take(n0 * cz) : nullptr;
    op.opart = (zc *)cv.take((size_t)R * OVAL * NBMAX * sizeof(zc));
    op.opart2 = (zc *)cv.take((size_t)R * OVAL * NBMAX * sizeof(zc));
    op.fs = (FState *)cv.take((size_t)R * sizeof(FState));
    op.active = (int *)cv.take((size_t)3 * R * sizeof(int));
    op.ones = op.active ? op.active + 2 * R : nullptr;   // (no arithmetic on the dry run's null)
}

int cyc_mask_offset(const csg_operator *op) { return op->p.max_rhs; }

// problem strides of a level's tables and phi (batched operators)
template <typename T>
void batch_strides(const csg_operator *op, const DevLevel &d, LvlK<T> &L)
{
    L.rpp = op->nprob > 1 ? (unsigned)op->rpp : 0u;
    for (int a = 0; a < 3; ++a) L.tstride[a] = 3 * d.nu[a];
    L.pstride = d.N;
}

template <typename T>
LvlK<T> lvl(const csg_operator *op, int l)
{
    const DevLevel &d = op->lev[l];
    LvlK<T> L;
    for (int a = 0; a < 3; ++a) L.tab[a] = (const Cx<T> *)d.tab[a];
    L.phi = (const T *)d.phi;
    L.nx = d.nu[0];
    L.ny = d.nu[1];
    L.nz = d.nu[2];
    L.N = d.N;
    batch_strides<T>(op, d, L);
    const cd sh = phi_shift(op->p);
    L.sre = sh.real();
    L.sim = sh.imag();
    L.gst = (const Cx<T> *)d.gst;
    L.gstride = (size_t)(op->p.dim == 2 ? 9 : 27) * d.N;
    return L;
}

LvlK<double> lvlH(const csg_operator *op)
{
    const DevLevel &d = op->lev[0];
    LvlK<double> L;
    for (int a = 0; a < 3; ++a) L.tab[a] = (const zc *)op->tabH[a];
    L.phi = op->phiH;
    L.nx = d.nu[0];
    L.ny = d.nu[1];
    L.nz = d.nu[2];
    L.N = d.N;
    batch_strides<double>(op, d, L);
    return L;
}

// elements between the coarsest inverses of consecutive problems, and RHS per problem
size_t minv_stride(const csg_operator *op) { return (size_t)op->nc * op->nc; }
unsigned batch_rpp(const csg_operator *op) { return op->nprob > 1 ? (unsigned)op->rpp : 0u; }

Launch lch(const csg_operator *op, int l, int nrhs, hipStream_t st)
{
    Launch g;
    g.nb = op->lev[l].nb;
    g.chunk = op->lev[l].chunk;
    g.nrhs = nrhs;
    g.st = st;
    return g;
}

template <typename T>
double tiny_of() { return 10.0 * (sizeof(T) == 8 ? DBL_EPSILON : (double)FLT_EPSILON); }

// ---------------------------------------------------------------------------
// benchmark instrumentation: event pairs around the launches of one pass kind
// ---------------------------------------------------------------------------
// roctx ranges around the host's enqueue of every level visit of the V-cycle
// and every outer pass (CSG_ROCTX=1), for rocprofv3 --marker-trace: with
// eager launches (CSG_GRAPHS=0) each range holds the launches of its passes,
// which trace_summary's `ranges` attributes kernel time to.  The marker
// library is opened on first use, so libcsg has no link dependency on it.
struct Roctx {
    int (*push)(const char *) = nullptr;
    int (*pop)() = nullptr;
    bool on = false;
};

const Roctx &roctx()
{
    static const Roctx r = [] {
        Roctx x;
        const char *e = getenv("CSG_ROCTX");
        if (!e || atoi(e) == 0) return x;
        void *h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_GLOBAL);
        if (!h) h = dlopen("libroctx64.so.4", RTLD_NOW | RTLD_GLOBAL);
        if (!h) return x;
        x.push = reinterpret_cast<int (*)(const char *)>(dlsym(h, "roctxRangePushA"));
        x.pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
        x.on = x.push && x.pop;
        return x;
    }();
    return r;
}

struct Range {
    bool on;
    explicit Range(const char *name, int a = -1) : on(roctx().on)
    {
        if (!on) return;
        char buf[80];
        if (a >= 0) snprintf(buf, sizeof buf, name, a);
        else snprintf(buf, sizeof buf, "%s", name);
        roctx().push(buf);
    }
    ~Range()
    {
        if (on) roctx().pop();
    }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

struct ProfScope {
    Prof *pr = nullptr;
    hipStream_t st = nullptr;
    bool on = false;
    ProfScope(const csg_operator *op, int kind, hipStream_t s, double bytes)
    {
        pr = op->prof;
        on = pr && pr->kind == kind && pr->n < pr->cap;
        if (on) {
            st = s;
            hipEventRecord(pr->ev[2 * pr->n], s);
            pr->bytes[pr->n] = bytes;
            pr->col[pr->n] = pr->cur;
        }
    }
    ~ProfScope()
    {
        if (on) {
            hipEventRecord(pr->ev[2 * pr->n + 1], st);
            pr->n++;
        }
    }
};

// Algorithmic bytes of the passes (each input vector read once, each output
// written once; phi and tables counted once per launch).
struct Bytes {
    double z, p;   // bytes of one cycle complex / real
    int R;         // right-hand sides
    double st(int j, double N) const { return R * (j + 2) * z * N + p * N; }
    double orth(int j, double N) const { return R * (j + 3) * z * N; }
    // fused pass j+1: reads w_j, u_0..u_j, phi; writes u_{j+1}, w_{j+1}
    double os(int j, double N) const { return R * (j + 4) * z * N + p * N; }
    double upd(int k, bool acc, double N) const { return R * (k + 1 + (acc ? 1 : 0)) * z * N; }
    double upd_r(int s, bool acc, double N) const { return R * (s + 1 + (acc ? 1 : 0) + 2) * z * N; }
    double upd_res(int s, bool acc, double N, double Nc) const
    {
        return R * ((s + 2 + (acc ? 1 : 0)) * z * N + z * Nc);
    }
    double resid(double N) const { return R * 3 * z * N + p * N; }
    double restrict_b(double N, double Nc) const { return R * z * (N + Nc); }
    double prc(bool xin, double N, double Nc) const { return R * z * ((xin ? N : 0) + Nc + 3 * N) + p * N; }
    double prolong(bool xin, double N, double Nc) const { return R * z * ((xin ? N : 0) + Nc + N); }
    // closing + restriction (+ the coarse pass 0): reads u_0..u_s (and x), writes x, bc (and w_0, phi_c read)
    double down(int s, bool acc, double N, double Nc, bool st0) const
    {
        return R * z * ((s + 2 + (acc ? 1 : 0)) * N + Nc + (st0 ? Nc : 0)) + (st0 ? p * Nc : 0);
    }
    // interpolation + residual + pass 0: reads xin, ec, b, phi; writes x, r, w_0
    double up(bool xin, double N, double Nc) const { return R * z * ((xin ? N : 0) + Nc + 4 * N) + p * N; }
    double coarse(double n) const { return n * n * z + R * 2 * n * z; }
};

Bytes bytes_of(const csg_operator *op, int nrhs)
{
    Bytes b;
    b.z = op->csize;
    b.p = op->csize / 2;
    b.R = nrhs;
    return b;
}

double vcycle_bytes(const csg_operator *op, int nrhs)
{
    const Bytes b = bytes_of(op, nrhs);
    if (op->p.smoother == 1) {
        // polynomial smoother: a tiled 2-D sweep reads x, b, phi and writes x
        // once (3z + p; 2z + p from zero), the untiled one does so per step
        const bool tl = op->p.dim == 2 && op->poly_tiles;
        const double sz = b.z * b.R, sp = b.p;
        double tot = b.coarse(op->nc);
        for (int l = 0; l + 1 < op->L; ++l) {
            const double N = op->lev[l].N, Nc = op->lev[l + 1].N;
            const double sweep0 = tl ? N * (2 * sz + sp) : N * (2 * sz + sp + 2 * (3 * sz + sp));
            const double sweep1 = tl ? N * (3 * sz + sp) : 3 * N * (3 * sz + sp);
            const int nu1 = op->p.nu1, nu2 = op->p.nu2;
            if (nu1 > 0) tot += sweep0 + (nu1 - 1) * sweep1;
            tot += N * ((nu1 > 0 ? 2 : 1) * sz + (nu1 > 0 ? sp : 0)) + Nc * sz;   // restriction (of the residual)
            if (nu2 > 0) tot += nu2 * sweep1 + Nc * sz + (tl ? 0.0 : 2 * N * sz);   // interpolated start
            else tot += b.prolong(nu1 > 0, N, Nc);
        }
        return tot;
    }
    const int s = op->p.s, nu1 = op->p.nu1, nu2 = op->p.nu2;
    double tot = b.coarse(op->nc);
    for (int l = 0; l + 1 < op->L; ++l) {
        const double N = op->lev[l].N, Nc = op->lev[l + 1].N;
        // Arnoldi passes of one sweep: pass 0 and the fused passes (FP64: h_{s,s-1}
        // from the last pass's sums, the closing pass combines w_{s-1} in place of
        // u_s; complex64: a last Gram-Schmidt pass forms u_s)
        double steps = b.st(0, N) + (op->p.cycle_prec ? b.orth(s - 1, N) : 0.0);
        for (int j = 0; j + 1 < s; ++j) steps += b.os(j, N);
        if (nu1 == 0) tot += b.restrict_b(N, Nc);
        for (int k = 0; k < nu1; ++k) {
            tot += (k ? b.resid(N) : 0) + steps;
            tot += (k == nu1 - 1) ? b.upd_res(s, k > 0, N, Nc) : b.upd(s, k > 0, N);
        }
        if (nu2 == 0) {
            tot += b.prolong(nu1 > 0, N, Nc);
        } else {
            tot += b.prc(nu1 > 0, N, Nc);
            for (int k = 0; k < nu2; ++k) tot += (k ? b.resid(N) : 0) + steps + b.upd(s, true, N);
        }
    }
    return tot;
}

// Arnoldi passes of one GMRES(s) sweep on level l with u_0 = B.u[0]: pass 0 and
// s-1 fused Gram-Schmidt + stencil passes (large levels: a stencil pass and a
// Gram-Schmidt pass per step).  The last pass also sums ||w_{s-1}||^2, from
// which the closing pass takes h_{s,s-1}; w_{s-1} stays in lv.w[(s-1) % 2].
// The fused passes write partials to part[k % 2] for pass k; the closing pass
// reads close_part().
template <typename T, int DIM>
bool tiled(const csg_operator *op, int l)
{
    return DIM == 2 && op->tiles && op->p.s <= 3 && tile_fits(op->lev[l].tile);
}

// Whether level l's Arnoldi passes run on 3-D z-marching slabs.
template <typename T, int DIM>
bool slabbed(const csg_operator *op, int l)
{
    return DIM == 3 && op->p.s <= 3 && op->lev[l].slab.nzc > 0 && (long)op->lev[l].N >= op->slab_min;
}

// w = H z and its inner products on the finest level's tiles (the tiles of the
// fused pass, which share the grid of H)
template <int DIM>
bool hdot_tiled(const csg_operator *op)
{
    const TileGeo &t = op->lev[0].tile;
    return DIM == 2 && op->hdot_tiles && tile_fits(t) && (int)(t.ntx * t.nty) <= NBMAX;
}

// the same on the finest level's slabs, when its Arnoldi passes take them
template <int DIM>
bool hdot_slabbed(const csg_operator *op)
{
    return DIM == 3 && op->hdot_tiles && slabbed<double, DIM>(op, 0);
}

// how many per-block partials w = H z leaves for the first projection
template <int DIM>
int hdot_parts(const csg_operator *op)
{
    const DevLevel &f = op->lev[0];
    if (hdot_tiled<DIM>(op)) return (int)(f.tile.ntx * f.tile.nty);
    if (hdot_slabbed<DIM>(op)) return (int)f.slab.npad;
    return f.nb;
}

// Whether the up path of level l runs as one tiled pass (interpolation,
// residual and pass 0 of the post-sweep).
template <typename T, int DIM>
bool up_tiled(const csg_operator *op, int l)
{
    return tiled<T, DIM>(op, l) && op->up_tiles && up_fits(op->lev[l].tile);
}

// Whether level l's (l >= 1) last post-sweep closing update is applied by
// level l-1's up-path pass instead of a pass of its own.
template <typename T, int DIM>
bool fuse_up(const csg_operator *op, int l)
{
    return l >= 1 && op->fuse_upd && op->p.s <= 3 && op->p.nu1 > 0 && up_tiled<T, DIM>(op, l - 1) &&
           upc_fits(op->lev[l - 1].tile);
}

// `first` > 0: pass 0 already ran (fused into the up-path pass), leaving
// `first` partials in part[0].
template <typename T, int DIM>
int arnoldi_passes(const csg_operator *op, int l, const Basis<T> &B, int nrhs, hipStream_t st, const int *active,
                   int first = 0)
{
    const DevLevel &lv = op->lev[l];
    const int s = op->p.s;
    const LvlK<T> L = lvl<T>(op, l);
    const Launch g = lch(op, l, nrhs, st);
    const double tiny = tiny_of<T>();
    const Bytes by = bytes_of(op, nrhs);
    Cx<T> *W[2] = {(Cx<T> *)lv.w[0], (Cx<T> *)lv.w[1]};
    const bool sums = sizeof(T) == 8;   // FP64: h_{s,s-1} from the last pass's sums
    const bool tl = tiled<T, DIM>(op, l);
    if (slabbed<T, DIM>(op, l)) {
        // 3-D: pass 0 and the fused passes on z-marching slabs
        const SlabGeo &sg = lv.slab;
        const int nslab = (int)sg.npad;
        {
            ProfScope ps(op, l == 0 ? CSG_PROF_STENCIL_DOTS : -1, st, by.st(0, lv.N));
            launch_slab<T>(L, B, nullptr, W[0], -1, s, lv.ld, nullptr, 0, lv.part[0], lv.gs, tiny, sums && s == 1, sg,
                           nrhs, st, active);
        }
        for (int j = 0; j + 1 < s; ++j) {
            ProfScope ps(op, l == 0 ? CSG_PROF_FUSED : -1, st, by.os(j, lv.N));
            launch_slab<T>(L, B, W[j & 1], W[(j + 1) & 1], j, s, lv.ld, lv.part[j & 1], nslab, lv.part[(j + 1) & 1],
                           lv.gs, tiny, sums && j + 2 == s, sg, nrhs, st, active);
        }
        if (!sums) {
            ProfScope ps(op, l == 0 ? CSG_PROF_ORTH : -1, st, by.orth(s - 1, lv.N));
            launch_orthl<T>(B, W[(s - 1) & 1], s - 1, s, lv.N, lv.ld, lv.part[(s - 1) & 1], nslab, lv.part[s & 1],
                            lv.gs, tiny, g, active);
            return lv.nb;
        }
        return nslab;
    }
    if (!tl && lv.N > op->fuse_max) {
        // large level: stencil pass then Gram-Schmidt pass per step (fewer loads per point)
        for (int j = 0; j < s; ++j) {
            {
                ProfScope ps(op, l == 0 ? CSG_PROF_STENCIL_DOTS : -1, st, by.st(j, lv.N));
                launch_stj<T, DIM>(L, B, W[j & 1], j, s, lv.ld, lv.part[0], g, active);
            }
            if (sums && j + 1 == s) break;
            ProfScope ps(op, l == 0 ? CSG_PROF_ORTH : -1, st, by.orth(j, lv.N));
            launch_orthl<T>(B, W[j & 1], j, s, lv.N, lv.ld, lv.part[0], lv.nb, lv.part[1], lv.gs, tiny, g, active);
        }
        return lv.nb;
    }
    const int ntile = tl ? (int)(lv.tile.ntx * lv.tile.nty) : lv.nb;
    int nlast = first;   // partials written by the last pass
    if (first == 0) {
        ProfScope ps(op, l == 0 ? CSG_PROF_STENCIL_DOTS : -1, st, by.st(0, lv.N));
        if (tl) {
            launch_st0_tile<T>(L, B.u[0], W[0], lv.ld, sums && s == 1, lv.part[0], lv.tile, nrhs, st, active);
            nlast = ntile;
        } else {
            launch_st0<T, DIM>(L, B.u[0], W[0], sums && s == 1, lv.ld, lv.part[0], g, active);
            nlast = lv.nb;
        }
    }
    for (int j = 0; j + 1 < s; ++j) {
        ProfScope ps(op, l == 0 ? CSG_PROF_FUSED : -1, st, by.os(j, lv.N));
        if (tl) {
            launch_os_tile<T>(L, B, W[j & 1], W[(j + 1) & 1], j, s, lv.ld, lv.part[j & 1], nlast,
                              lv.part[(j + 1) & 1], lv.gs, tiny, lv.tile, nrhs, st, active);
            nlast = ntile;
        } else {
            launch_os<T, DIM>(L, B, W[j & 1], W[(j + 1) & 1], j, s, lv.ld, lv.part[j & 1], lv.nb,
                              lv.part[(j + 1) & 1], lv.gs, tiny, g, active);
        }
    }
    if (!sums) {
        // complex64: the last Gram-Schmidt pass forms u_s and its norm
        ProfScope ps(op, l == 0 ? CSG_PROF_ORTH : -1, st, by.orth(s - 1, lv.N));
        launch_orthl<T>(B, W[(s - 1) & 1], s - 1, s, lv.N, lv.ld, lv.part[(s - 1) & 1], nlast, lv.part[s & 1], lv.gs,
                        tiny, g, active);
        nlast = lv.nb;
    }
    return nlast;
}

// Partials buffer the closing pass of a sweep on level l reads (written by the
// last Arnoldi pass).
template <typename T, int DIM>
zc *close_part(const csg_operator *op, int l)
{
    const DevLevel &lv = op->lev[l];
    const int s = op->p.s;
    const bool unfused = !tiled<T, DIM>(op, l) && !slabbed<T, DIM>(op, l) && lv.N > op->fuse_max;
    if (sizeof(T) == 8) return unfused ? lv.part[0] : lv.part[(s - 1) & 1];
    return unfused ? lv.part[1] : lv.part[s & 1];
}

// Basis the closing pass combines: u_0..u_{s-1} and, in place of u_s, w_{s-1}
// (FP64; complex64 sweeps form u_s).
template <typename T>
Basis<T> closing_basis(const csg_operator *op, int l, Basis<T> B)
{
    if (sizeof(T) == 8) B.u[op->p.s] = (Cx<T> *)op->lev[l].w[(op->p.s - 1) & 1];
    return B;
}

// Whether the closing pass of level l's last pre-sweep runs fused with the
// restriction on tiles of level l+1; with st0 also level l+1's pass 0.
template <typename T, int DIM>
bool down_tiled(const csg_operator *op, int l)
{
    if (DIM != 2 || !op->tiles || !op->down_tiles || op->p.s > 3 || l + 1 >= op->L) return false;
    const DevLevel &f = op->lev[l], &c = op->lev[l + 1];
    return down_fits(c.dtile) && f.nu[0] <= 2 * c.nu[0] + 1 && f.nu[1] <= 2 * c.nu[1] + 1;
}
template <typename T, int DIM>
bool down_st0(const csg_operator *op, int l)
{
    return l + 1 < op->lt && op->p.nu1 > 0 && tiled<T, DIM>(op, l + 1);
}

// One GMRES(s) sweep on level l: Arnoldi passes on u_0 (= b when x == 0, else
// the residual in lv.r), then the closing pass: the plain update
// (x (+)= V y) or, before the restriction, the update plus the Arnoldi residual.
// `first`: pass 0 already ran (see arnoldi_passes).  Returns the `first` of
// level l+1's first sweep: its partial count when the closing pass also ran
// that sweep's pass 0, else 0.
template <typename T, int DIM>
int sweep(const csg_operator *op, int l, const Cx<T> *b, Cx<T> *x, bool from_zero, bool restrict_after, int nrhs,
          hipStream_t st, const int *active, int first = 0)
{
    const DevLevel &lv = op->lev[l];
    const int s = op->p.s;
    const LvlK<T> L = lvl<T>(op, l);
    const Launch g = lch(op, l, nrhs, st);
    const double tiny = tiny_of<T>();
    Basis<T> B;
    for (int i = 0; i <= CSG_MAX_S; ++i) B.u[i] = (Cx<T> *)lv.u[i];
    if (from_zero) {
        B.u[0] = const_cast<Cx<T> *>(b);
    } else {
        launch_resid<T, DIM>(L, x, b, (Cx<T> *)lv.r, lv.ld, g, active);
        B.u[0] = (Cx<T> *)lv.r;
    }
    const int nclose = arnoldi_passes<T, DIM>(op, l, B, nrhs, st, active, first);
    B = closing_basis<T>(op, l, B);
    const Bytes by = bytes_of(op, nrhs);
    const int k0 = l == 0 ? 0 : -1;   // instrumented kinds exist for the finest level only
    zc *pclose = close_part<T, DIM>(op, l);
    if (restrict_after && down_tiled<T, DIM>(op, l)) {
        // closing update, restriction of the Arnoldi residual and (when level
        // l+1 sweeps next) its pass 0, per coarse tile
        const DevLevel &cl = op->lev[l + 1];
        const bool st0 = down_st0<T, DIM>(op, l);
        ProfScope ps(op, k0 ? -1 : CSG_PROF_UPD_RESTRICT, st, by.down(s, !from_zero, lv.N, cl.N, st0));
        launch_down_tile<T>(x, from_zero ? 0 : 1, B, s, L, lvl<T>(op, l + 1), (Cx<T> *)cl.b, (Cx<T> *)cl.w[0],
                            lv.ld, cl.ld, pclose, nclose, lv.gs, tiny, st0, sizeof(T) == 8 && s == 1, cl.part[0],
                            cl.dtile, nrhs, st, active);
        return st0 ? (int)(cl.dtile.ntx * cl.dtile.nty) : 0;
    }
    if (restrict_after && slabbed<T, DIM>(op, l) && op->slab_down) {
        // closing update and full weighting of the Arnoldi residual in one slab pass
        const DevLevel &cl = op->lev[l + 1];
        ProfScope ps(op, k0 ? -1 : CSG_PROF_UPD_RESTRICT, st, by.upd_res(s, !from_zero, lv.N, cl.N));
        launch_slab_down<T>(x, from_zero ? 0 : 1, B, s, L, lvl<T>(op, l + 1), (Cx<T> *)cl.b, lv.ld, cl.ld, pclose,
                            nclose, lv.gs, tiny, lv.slab, nrhs, st, active);
    } else if (restrict_after) {
        // closing update writes x and the Arnoldi residual r; full weighting of r
        const DevLevel &cl = op->lev[l + 1];
        ProfScope ps(op, k0 ? -1 : CSG_PROF_UPD_RESTRICT, st,
                     by.upd_r(s, !from_zero, lv.N) + by.restrict_b(lv.N, cl.N));
        launch_upd_r<T>(x, from_zero ? 0 : 1, (Cx<T> *)lv.r, B, s, lv.N, lv.ld, pclose, nclose, lv.gs, tiny, g,
                        active);
        launch_restrict<T, DIM>(L, lvl<T>(op, l + 1), nullptr, (const Cx<T> *)lv.r, (Cx<T> *)cl.b, lv.ld, cl.ld,
                                lch(op, l + 1, nrhs, st), active);
    } else {
        ProfScope ps(op, k0 ? -1 : CSG_PROF_UPDATE, st, by.upd(s, !from_zero, lv.N));
        launch_upd<T>(x, from_zero ? 0 : 1, B, s, lv.N, lv.ld, pclose, nclose, lv.gs, tiny, g, active);
    }
    return 0;
}

// x = V_{nu1,nu2}(0; b) on level l downwards (section 3.1).
template <typename T, int DIM>
void vcycle_impl(const csg_operator *op, const Cx<T> *b0, Cx<T> *x0, int nrhs, hipStream_t st, const int *active)
{
    const int L = op->L;
    const int lt = op->lt;
    const int nu1 = op->p.nu1, nu2 = op->p.nu2;
    int first = 0;   // pass 0 of this level's first sweep already ran
    for (int l = 0; l < lt; ++l) {
        const Range rg("V-cycle down L%d", l);
        const DevLevel &lv = op->lev[l];
        const DevLevel &cl = op->lev[l + 1];
        const Cx<T> *b = l == 0 ? b0 : (const Cx<T> *)lv.b;
        Cx<T> *xa = (Cx<T> *)lv.xa;
        if (nu1 == 0) {
            launch_restrict<T, DIM>(lvl<T>(op, l), lvl<T>(op, l + 1), nullptr, b, (Cx<T> *)cl.b, lv.ld, cl.ld,
                                    lch(op, l + 1, nrhs, st), active);
        } else {
            int next = 0;
            for (int k = 0; k < nu1; ++k)
                next = sweep<T, DIM>(op, l, b, xa, k == 0, k == nu1 - 1, nrhs, st, active, k == 0 ? first : 0);
            first = next;
        }
    }
    {
        // levels lt..L-1 (coarsest solve included) in one workgroup per RHS
        const Range rg("V-cycle coarse tail from L%d", lt);
        const Cx<T> *bt = lt == 0 ? b0 : (const Cx<T> *)op->lev[lt].b;
        Cx<T> *xt = lt == 0 ? x0 : (Cx<T> *)op->lev[lt].xb;
        launch_tail<T, DIM>((const TLev<T> *)op->tlev, lt, L, bt, xt, (const Cx<T> *)op->minvT, op->nc, op->p.s, nu1,
                            nu2, tiny_of<T>(), nrhs, op->tail_lds, st, active, minv_stride(op));
    }
    // A level's post-sweep closing update is deferred to the next finer
    // level's up-path pass when that pass is tiled (fuse_up): x_c then exists
    // only on the tiles' coarse windows.
    UpClose<T> pend{};
    bool have_pend = false;
    for (int l = lt - 1; l >= 0; --l) {
        const Range rg("V-cycle up L%d", l);
        const DevLevel &lv = op->lev[l];
        const DevLevel &cl = op->lev[l + 1];
        const Cx<T> *b = l == 0 ? b0 : (const Cx<T> *)lv.b;
        Cx<T> *xo = l == 0 ? x0 : (Cx<T> *)lv.xb;
        const Cx<T> *xi = nu1 > 0 ? (const Cx<T> *)lv.xa : nullptr;
        const Launch g = lch(op, l, nrhs, st);
        if (nu2 == 0) {
            launch_prolong<T, DIM>(lvl<T>(op, l), lvl<T>(op, l + 1), (const Cx<T> *)cl.xb, xi, xo, lv.ld, cl.ld, g,
                                   active);
        } else {
            const bool ut = up_tiled<T, DIM>(op, l) && xi != xo;
            const int ntile = (int)(lv.tile.ntx * lv.tile.nty);
            if (ut) {
                // interpolated correction (after the coarse level's deferred
                // closing update), residual and the post-sweep's pass 0 per tile
                const Bytes by = bytes_of(op, nrhs);
                ProfScope ps(op, l == 0 ? CSG_PROF_PROLONG_RESID : -1, st,
                             by.up(xi != nullptr, lv.N, cl.N) + (have_pend ? by.upd(op->p.s, true, cl.N) : 0.0));
                launch_up_tile<T>(lvl<T>(op, l), lvl<T>(op, l + 1), (const Cx<T> *)cl.xb, xi, xo, b,
                                  (Cx<T> *)lv.r, (Cx<T> *)lv.w[0], lv.ld, cl.ld, sizeof(T) == 8 && op->p.s == 1,
                                  lv.part[0], lv.tile, nrhs, st, active, have_pend ? &pend : nullptr);
            } else if (slabbed<T, DIM>(op, l) && op->slab_pr) {
                // interpolated correction and the residual that opens the post-sweep in one slab pass
                const Bytes by = bytes_of(op, nrhs);
                ProfScope ps(op, l == 0 ? CSG_PROF_PROLONG_RESID : -1, st, by.prc(xi != nullptr, lv.N, cl.N));
                launch_slab_pr<T>(lvl<T>(op, l), lvl<T>(op, l + 1), (const Cx<T> *)cl.xb, xi, xo, b, (Cx<T> *)lv.r,
                                  lv.ld, cl.ld, lv.slab, nrhs, st, active);
            } else {
                // interpolated correction, then the residual that opens the post-sweep
                const Bytes by = bytes_of(op, nrhs);
                ProfScope ps(op, l == 0 ? CSG_PROF_PROLONG_RESID : -1, st,
                             by.prolong(xi != nullptr, lv.N, cl.N) + by.resid(lv.N));
                launch_prolong<T, DIM>(lvl<T>(op, l), lvl<T>(op, l + 1), (const Cx<T> *)cl.xb, xi, xo, lv.ld, cl.ld,
                                       g, active);
                launch_resid<T, DIM>(lvl<T>(op, l), xo, b, (Cx<T> *)lv.r, lv.ld, g, active);
            }
            have_pend = false;
            for (int k = 0; k < nu2; ++k) {
                // the first post-sweep starts from the residual already in lv.r
                const DevLevel &d = op->lev[l];
                const int s = op->p.s;
                const LvlK<T> Lk = lvl<T>(op, l);
                const double tiny = tiny_of<T>();
                Basis<T> B;
                for (int i = 0; i <= CSG_MAX_S; ++i) B.u[i] = (Cx<T> *)d.u[i];
                if (k > 0) launch_resid<T, DIM>(Lk, xo, b, (Cx<T> *)d.r, d.ld, g, active);
                B.u[0] = (Cx<T> *)d.r;
                const int nclose = arnoldi_passes<T, DIM>(op, l, B, nrhs, st, active, ut && k == 0 ? ntile : 0);
                B = closing_basis<T>(op, l, B);
                if (k + 1 == nu2 && fuse_up<T, DIM>(op, l)) {
                    pend = UpClose<T>{B, xo, close_part<T, DIM>(op, l), nclose, d.gs, s, tiny};
                    have_pend = true;
                    continue;
                }
                ProfScope ps(op, l == 0 ? CSG_PROF_UPDATE : -1, st, bytes_of(op, nrhs).upd(s, true, d.N));
                launch_upd<T>(xo, 1, B, s, d.N, d.ld, close_part<T, DIM>(op, l), nclose, d.gs, tiny, g, active);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Third-order polynomial smoother (section 4)
// ---------------------------------------------------------------------------

template <typename T>
void poly_weights(const DevLevel &lv, Cx<T> (&w)[3])
{
    for (int i = 0; i < 3; ++i) w[i] = mkc<T>((T)lv.omega[i].real(), (T)lv.omega[i].imag());
}

// `sweeps` polynomial sweeps on level l from the start value xi + P ec (either
// may be null: zero, no correction) into out, which aliases neither xi nor the
// level's r, w[0], w[1] (its temporaries).  2-D levels run a whole sweep per
// tiled launch (the tile kernel cannot update in place, so a chain of sweeps
// alternates between out and r, ending in out); otherwise each sweep is three
// Richardson passes through w[0] and w[1].
template <typename T, int DIM>
void poly_smooth(const csg_operator *op, int l, const Cx<T> *b, const Cx<T> *xi, const Cx<T> *ec, Cx<T> *out,
                 int sweeps, int nrhs, hipStream_t st, const int *active)
{
    const DevLevel &lv = op->lev[l];
    Cx<T> w[3];
    poly_weights<T>(lv, w);
    const LvlK<T> L = lvl<T>(op, l);
    const LvlK<T> C = l + 1 < op->L ? lvl<T>(op, l + 1) : L;
    const size_t ldc = l + 1 < op->L ? op->lev[l + 1].ld : 0;
    Cx<T> *tmp = (Cx<T> *)lv.r;
    if (DIM == 2 && op->poly_tiles) {
        const Cx<T> *src = xi;
        for (int k = 0; k < sweeps; ++k) {
            Cx<T> *dst = ((sweeps - 1 - k) % 2 == 0) ? out : tmp;
            launch_poly_tile<T>(L, C, k == 0 ? ec : nullptr, src, b, dst, w, lv.ld, ldc, nrhs, st, active);
            src = dst;
        }
        return;
    }
    const Launch g = lch(op, l, nrhs, st);
    const Cx<T> *src = xi;
    if (ec) {
        launch_prolong<T, DIM>(L, C, ec, xi, tmp, lv.ld, ldc, g, active);
        src = tmp;
    }
    Cx<T> *W0 = (Cx<T> *)lv.w[0], *W1 = (Cx<T> *)lv.w[1];
    for (int k = 0; k < sweeps; ++k) {
        launch_rich<T, DIM>(L, src, b, W0, w[0], lv.ld, g, active);
        launch_rich<T, DIM>(L, W0, b, W1, w[1], lv.ld, g, active);
        launch_rich<T, DIM>(L, W1, b, out, w[2], lv.ld, g, active);
        src = out;
    }
}

// x = V_{nu1,nu2}(0; b) with the polynomial smoother on every non-coarsest
// level: pre-sweeps from zero, restriction of the residual, recursion,
// interpolated correction feeding the post-sweeps; dense coarsest solve.
template <typename T, int DIM>
void vcycle_poly(const csg_operator *op, const Cx<T> *b0, Cx<T> *x0, int nrhs, hipStream_t st, const int *active)
{
    const int L = op->L;
    const int nu1 = op->p.nu1, nu2 = op->p.nu2;
    for (int l = 0; l + 1 < L; ++l) {
        const DevLevel &lv = op->lev[l];
        const DevLevel &cl = op->lev[l + 1];
        const Cx<T> *b = l == 0 ? b0 : (const Cx<T> *)lv.b;
        Cx<T> *xa = nu1 > 0 ? (Cx<T> *)lv.xa : nullptr;
        if (nu1 > 0) poly_smooth<T, DIM>(op, l, b, nullptr, nullptr, xa, nu1, nrhs, st, active);
        launch_restrict<T, DIM>(lvl<T>(op, l), lvl<T>(op, l + 1), xa, b, (Cx<T> *)cl.b, lv.ld, cl.ld,
                                lch(op, l + 1, nrhs, st), active);
    }
    const Cx<T> *bL = L == 1 ? b0 : (const Cx<T> *)op->lev[L - 1].b;
    Cx<T> *xL = L == 1 ? x0 : (Cx<T> *)op->lev[L - 1].xb;
    launch_coarse<T>((const Cx<T> *)op->minvT, op->nc, bL, xL, op->lev[L - 1].ld, nrhs, st, active, minv_stride(op),
                     batch_rpp(op));
    for (int l = L - 2; l >= 0; --l) {
        const DevLevel &lv = op->lev[l];
        const DevLevel &cl = op->lev[l + 1];
        const Cx<T> *b = l == 0 ? b0 : (const Cx<T> *)lv.b;
        Cx<T> *xo = l == 0 ? x0 : (Cx<T> *)lv.xb;
        const Cx<T> *xi = nu1 > 0 ? (const Cx<T> *)lv.xa : nullptr;
        if (nu2 == 0)
            launch_prolong<T, DIM>(lvl<T>(op, l), lvl<T>(op, l + 1), (const Cx<T> *)cl.xb, xi, xo, lv.ld, cl.ld,
                                   lch(op, l, nrhs, st), active);
        else
            poly_smooth<T, DIM>(op, l, b, xi, (const Cx<T> *)cl.xb, xo, nu2, nrhs, st, active);
    }
}

// One smoothing sweep of csg_smooth on level l (x in place): GMRES(s), or a
// polynomial sweep into the level's xb, copied back (the polynomial kernels
// never update in place).
template <typename T, int DIM>
void smooth_inplace(const csg_operator *op, int level, const Cx<T> *b, Cx<T> *x, int nrhs, hipStream_t st,
                    const int *active)
{
    if (op->p.smoother != 1) {
        sweep<T, DIM>(op, level, b, x, false, false, nrhs, st, active);
        return;
    }
    const DevLevel &lv = op->lev[level];
    Cx<T> *tmp = (Cx<T> *)lv.xb;
    poly_smooth<T, DIM>(op, level, b, x, nullptr, tmp, 1, nrhs, st, active);
    hipMemcpyAsync(x, tmp, (size_t)nrhs * lv.ld * sizeof(Cx<T>), hipMemcpyDeviceToDevice, st);
}

template <typename T>
void vcycle_dispatch(const csg_operator *op, const void *b, void *x, int nrhs, hipStream_t st, const int *active)
{
    if (op->p.smoother == 1) {
        if (op->p.dim == 2)
            vcycle_poly<T, 2>(op, (const Cx<T> *)b, (Cx<T> *)x, nrhs, st, active);
        else
            vcycle_poly<T, 3>(op, (const Cx<T> *)b, (Cx<T> *)x, nrhs, st, active);
        return;
    }
    if (op->p.dim == 2)
        vcycle_impl<T, 2>(op, (const Cx<T> *)b, (Cx<T> *)x, nrhs, st, active);
    else
        vcycle_impl<T, 3>(op, (const Cx<T> *)b, (Cx<T> *)x, nrhs, st, active);
}

void run_vcycle(const csg_operator *op, const void *b, void *x, int nrhs, hipStream_t st, const int *active)
{
    const Range rg("V-cycle");
    ProfScope ps(op, CSG_PROF_VCYCLE, st, vcycle_bytes(op, nrhs));
    if (op->p.cycle_prec)
        vcycle_dispatch<float>(op, b, x, nrhs, st, active);
    else
        vcycle_dispatch<double>(op, b, x, nrhs, st, active);
}

int check_op(const csg_operator *op, int nrhs)
{
    if (!op) return fail(CSG_EINVAL, "null operator");
    if (nrhs < 0 || nrhs > op->p.max_rhs) return fail(CSG_EINVAL, "nrhs out of range 0..max_rhs");
    return CSG_OK;
}

int last_launch_error()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CSG_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return CSG_OK;
}

}  // namespace

// ===========================================================================
// FGMRES driver (section 5): a small host state machine over device passes.
// ===========================================================================

struct csg_solve {
    csg_operator *op;
    const zc *chi;
    zc *u;
    int nrhs, m, maxit, use_x0;
    double tol;
    hipStream_t st;
    enum { INIT, WAIT_BEGIN, CYCLE, CYCLE_END, WAIT_END, FINISHED } phase;
    int j;            // columns of the current cycle whose reports the host has read
    int jq;           // columns of the current cycle queued (j <= jq <= j + LOOKAHEAD)
    bool halt;        // no RHS iterates any more in this cycle: queue no further column
    long col0;        // profiling: number of the cycle's first column
    int rc;
    int it[CSG_MAX_RHS_HOST];
    int done[CSG_MAX_RHS_HOST], conv[CSG_MAX_RHS_HOST], act[CSG_MAX_RHS_HOST], restarts[CSG_MAX_RHS_HOST];
    double est[CSG_MAX_RHS_HOST], truer[CSG_MAX_RHS_HOST];
    int *mask_host;   // pinned: [active | cyc]
    std::chrono::steady_clock::time_point t0;
    double seconds;
};

namespace {

// Device address of report slot `slot` in pinned host memory.
Report *report_slot(const csg_operator *op, int slot) { return op->rep_dev + (size_t)slot * op->p.max_rhs; }

template <int DIM>
void enqueue_begin(csg_solve *sv, bool with_chi_norm)
{
    csg_operator *op = sv->op;
    const DevLevel &f = op->lev[0];
    const Launch g = lch(op, 0, sv->nrhs, sv->st);
    const int *mask = op->active + cyc_mask_offset(op);
    launch_tres<DIM>(lvlH(op), sv->chi, sv->u, op->V, f.ld, with_chi_norm ? 1 : 0, op->opart, g, mask);
    launch_fin(with_chi_norm ? FIN_BEGIN : FIN_BETA, op->opart, f.nb, 0, op->fs, report_slot(op, LOOKAHEAD), sv->nrhs,
               sv->st, mask);
    ProfScope ps(op, CSG_PROF_OUTER_NORM, sv->st, sv->nrhs * f.N * (32.0 + (op->p.cycle_prec ? 8.0 : 0.0)));
    if (op->p.cycle_prec)
        launch_vnorm<float>(op->V, op->V, (cf *)op->b0, f.N, f.ld, op->fs, g, mask);
    else
        launch_vnorm<double>(op->V, op->V, (zc *)nullptr, f.N, f.ld, op->fs, g, mask);
}

// One FGMRES iteration (section 5): z_j = V(v_j), w = H z_j, classical
// Gram-Schmidt against v_0..v_j with ||w||^2 summed alongside, so
// h_{j+1,j}^2 = ||w||^2 - ||h||^2 is known before the projection.  When the
// projection keeps at least 1/sqrt(2) of ||w|| one round is final and the
// first projection writes v_{j+1}; otherwise a second round (its inner
// products formed by the first projection, h_{j+1,j} from ||w1||^2 - ||c||^2)
// restores orthogonality.  Lazy (default): the first projection writes the
// first-round form v~_{j+1}, which the next V-cycle takes as its input, k_col
// finishes the column, and the next first projection replaces v~_{j+1} by
// v_{j+1} while it reads the basis anyway, so a second round costs no pass
// over V of its own.  Otherwise k_proj1 applies the second round at once.
// Givens update on the device either way.
template <typename TZ, int DIM>
void iter_body(csg_solve *sv, int j, hipStream_t st)
{
    csg_operator *op = sv->op;
    const DevLevel &f = op->lev[0];
    const size_t vstride = (size_t)op->p.max_rhs * f.N;
    const Launch g = lch(op, 0, sv->nrhs, st);
    const int *mask = op->active;
    const void *b = op->p.cycle_prec ? op->b0 : (const void *)(op->V + j * vstride);
    Cx<TZ> *z = (Cx<TZ> *)op->Z + j * vstride;
    const Range rg("FGMRES column %d", j);
    run_vcycle(op, b, z, sv->nrhs, st, mask);
    const double N = f.N, R = sv->nrhs;
    {
        const Range rh("outer w = H z");
        ProfScope ps(op, CSG_PROF_OUTER_H, st, R * N * (sizeof(Cx<TZ>) + 16.0 * (j + 2)) + 8.0 * N);
        if (hdot_tiled<DIM>(op))
            launch_hdot_tile<TZ>(lvlH(op), z, op->w, op->V, vstride, j, f.ld, op->opart, f.tile, sv->nrhs, st, mask);
        else if (hdot_slabbed<DIM>(op))
            launch_slab_hdot<TZ>(lvlH(op), z, op->w, op->V, vstride, j, f.ld, op->opart, f.slab, sv->nrhs, st, mask);
        else
            launch_hdot<TZ, DIM>(lvlH(op), z, op->w, op->V, vstride, j, f.ld, op->opart, g, mask);
    }
    {
        // first round finished and applied: writes v_{j+1} (and advances the
        // FGMRES state) when the first round is final, and the second-round
        // passes below then return at once; otherwise keeps w_1 and forms the
        // second round's inner products in the same launch
        const Range rp("outer first projection");
        ProfScope ps(op, CSG_PROF_OUTER_CGS1, st,
                     R * N * (16.0 * (j + 3) + (op->p.cycle_prec ? 8.0 : 0.0) + (op->lazy && j > 0 ? 16.0 : 0.0)));
        launch_proj0<TZ>(op->w, op->V, vstride, j, f.N, f.ld, op->fs, report_slot(op, j % LOOKAHEAD), op->active,
                         op->opart, hdot_parts<DIM>(op), op->opart2, op->V + (j + 1) * vstride,
                         op->p.cycle_prec ? (Cx<TZ> *)op->b0 : nullptr, op->V + j * vstride, op->lazy ? 1 : 0, g,
                         mask);
    }
    if (op->lazy) {
        // the column's finish (its second round's vector update waits for the next first projection)
        const Range rc("outer column finish");
        ProfScope ps(op, CSG_PROF_OUTER_PROJ2, st, 0.0);
        launch_col(j, op->fs, report_slot(op, j % LOOKAHEAD), op->active, op->opart2, f.nb, sv->nrhs, st, mask);
        return;
    }
    const Range r2("outer second projection");
    ProfScope ps(op, CSG_PROF_OUTER_PROJ2, st, R * N * (16.0 * (j + 3) + (op->p.cycle_prec ? 8.0 : 0.0)));
    launch_proj1<TZ>(op->w, op->V, vstride, j, f.N, f.ld, op->fs, report_slot(op, j % LOOKAHEAD), op->active,
                     op->opart2, f.nb, op->V + (j + 1) * vstride, op->p.cycle_prec ? (Cx<TZ> *)op->b0 : nullptr, g,
                     mask);
}

// Destroys every cached graph.
void drop_graphs(csg_operator *op)
{
    GraphCache *gc = op->gc;
    if (!gc) return;
    for (auto &kv : gc->it)
        for (hipGraphExec_t g : kv.second)
            if (g) hipGraphExecDestroy(g);
    gc->it.clear();
}

// Replays the captured graph of columns j .. j+g-1 (capturing it on first use;
// groups start at multiples of GCOLS); eager launches when graphs are disabled
// or a pass is being instrumented.
template <typename TZ, int DIM>
void enqueue_iters(csg_solve *sv, int j, int g)
{
    csg_operator *op = sv->op;
    GraphCache *gc = op->gc;
    if (!gc || !gc->enabled || op->prof) {
        // eager: graphs disabled, or launches being timed (this HIP cannot time
        // events recorded inside a graph)
        for (int c = j; c < j + g; ++c) {
            if (op->prof) op->prof->cur = sv->col0 + c;
            iter_body<TZ, DIM>(sv, c, sv->st);
        }
        if (op->prof) op->prof->cur = -1;
        return;
    }
    // a graph holds the columns of its group, which depend on the cycle length m
    std::vector<hipGraphExec_t> &v = gc->it[sv->nrhs * (CSG_MAX_RESTART + 1) + sv->m];
    if ((int)v.size() < op->p.restart) v.resize(op->p.restart, nullptr);
    if (!v[j]) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        bool ok = hipStreamBeginCapture(gc->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            for (int c = j; c < j + g; ++c) iter_body<TZ, DIM>(sv, c, gc->cap);
            ok = hipStreamEndCapture(gc->cap, &graph) == hipSuccess && graph;
        }
        ok = ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) hipGraphDestroy(graph);
        if (!ok) {
            hipGetLastError();
            drop_graphs(op);
            gc->enabled = false;   // capture unsupported here: stay eager
            for (int c = j; c < j + g; ++c) iter_body<TZ, DIM>(sv, c, sv->st);
            return;
        }
        v[j] = exec;
    }
    hipGraphLaunch(v[j], sv->st);
}

template <typename TZ, int DIM>
void enqueue_end(csg_solve *sv)
{
    csg_operator *op = sv->op;
    const DevLevel &f = op->lev[0];
    const size_t vstride = (size_t)op->p.max_rhs * f.N;
    const Launch g = lch(op, 0, sv->nrhs, sv->st);
    const int *mask = op->active + cyc_mask_offset(op);
    launch_fin(FIN_LS, op->opart, f.nb, 0, op->fs, report_slot(op, LOOKAHEAD), sv->nrhs, sv->st, mask);
    launch_uupd<TZ>(sv->u, (const Cx<TZ> *)op->Z, vstride, f.N, f.ld, op->fs, g, mask);
    enqueue_begin<DIM>(sv, false);
}

void upload_masks(csg_solve *sv)
{
    csg_operator *op = sv->op;
    const int R = op->p.max_rhs;
    for (int r = 0; r < R; ++r) {
        const bool in = r < sv->nrhs && !sv->done[r];
        sv->mask_host[r] = in && sv->act[r];
        sv->mask_host[R + r] = in;
    }
    hipMemcpyAsync(op->active, sv->mask_host, 2 * R * sizeof(int), hipMemcpyHostToDevice, sv->st);
}

// The event of report slot `slot` (column j of a cycle: j % LOOKAHEAD; cycle
// begin / end: LOOKAHEAD), whose reports the projection passes (or, at a restart, k_fin) wrote to pinned host memory.
void enqueue_report(csg_solve *sv, int slot) { hipEventRecord(sv->op->evq[slot], sv->st); }

// The event of the report the host reads next, or null when none is queued.
hipEvent_t pending_event(const csg_solve *sv)
{
    switch (sv->phase) {
    case csg_solve::WAIT_BEGIN:
    case csg_solve::WAIT_END:
        return sv->op->evq[LOOKAHEAD];
    case csg_solve::CYCLE:
        return sv->j < sv->jq ? sv->op->evq[sv->j % LOOKAHEAD] : nullptr;
    default:
        return nullptr;
    }
}

int solve_step(csg_solve *sv)
{
    csg_operator *op = sv->op;
    const bool mixed = op->p.cycle_prec != 0;
    const bool d3 = op->p.dim == 3;
    switch (sv->phase) {
    case csg_solve::INIT:
        upload_masks(sv);
        launch_fs_params(op->fs, sv->tol, sv->maxit, op->force_cgs2 ? 1 : 0, sv->nrhs, sv->st);
        if (d3) enqueue_begin<3>(sv, true); else enqueue_begin<2>(sv, true);
        enqueue_report(sv, LOOKAHEAD);
        sv->phase = csg_solve::WAIT_BEGIN;
        break;
    case csg_solve::CYCLE:
        // queue groups of GCOLS columns (one graph each) up to LOOKAHEAD columns
        // ahead of the reports read; each RHS's iteration mask is cleared by
        // the device when it stops.  Instrumented solves queue single columns
        // as far ahead (the GPU never waits for the host, as in a plain
        // solve); launches of columns queued after the halt are dropped from
        // the timings.
        if (sv->jq == 0) upload_masks(sv);
        for (;;) {
            const int g = op->prof ? 1 : std::min(GCOLS, sv->m - sv->jq);
            if (sv->halt || sv->jq >= sv->m || sv->jq + g - sv->j > LOOKAHEAD) break;
            if (mixed) { if (d3) enqueue_iters<float, 3>(sv, sv->jq, g); else enqueue_iters<float, 2>(sv, sv->jq, g); }
            else { if (d3) enqueue_iters<double, 3>(sv, sv->jq, g); else enqueue_iters<double, 2>(sv, sv->jq, g); }
            for (int c = 0; c < g; ++c) enqueue_report(sv, (sv->jq + c) % LOOKAHEAD);
            sv->jq += g;
        }
        break;
    case csg_solve::CYCLE_END:
        upload_masks(sv);
        if (mixed) { if (d3) enqueue_end<float, 3>(sv); else enqueue_end<float, 2>(sv); }
        else { if (d3) enqueue_end<double, 3>(sv); else enqueue_end<double, 2>(sv); }
        enqueue_report(sv, LOOKAHEAD);
        sv->phase = csg_solve::WAIT_END;
        break;
    default:
        return CSG_OK;   // waiting or finished: nothing to enqueue
    }
    return last_launch_error();
}

// Host decisions after a report has landed.
void solve_advance(csg_solve *sv)
{
    csg_operator *op = sv->op;
    const int R = op->p.max_rhs;
    const Report *rp = op->rep_host + (size_t)(sv->phase == csg_solve::CYCLE ? sv->j % LOOKAHEAD : LOOKAHEAD) * R;
    bool any = false;
    switch (sv->phase) {
    case csg_solve::WAIT_BEGIN:
    case csg_solve::WAIT_END:
        for (int r = 0; r < sv->nrhs; ++r) {
            if (sv->done[r]) continue;
            if (sv->phase == csg_solve::WAIT_END) sv->restarts[r]++;
            const double nchi = (sv->phase == csg_solve::WAIT_BEGIN) ? rp[r].hn : 1.0;
            if (!rp[r].finite) { sv->done[r] = 1; sv->rc = CSG_ENUMERIC; continue; }
            if (sv->phase == csg_solve::WAIT_BEGIN && nchi == 0.0) {
                // zero source: the solution is zero
                hipMemsetAsync(sv->u + (size_t)r * op->lev[0].ld, 0, op->lev[0].N * sizeof(zc), sv->st);
                sv->done[r] = sv->conv[r] = 1;
                sv->truer[r] = sv->est[r] = 0.0;
                continue;
            }
            sv->truer[r] = rp[r].est;
            if (sv->phase == csg_solve::WAIT_BEGIN) sv->est[r] = rp[r].est;
            if (rp[r].est <= sv->tol) { sv->done[r] = sv->conv[r] = 1; continue; }
            if (sv->it[r] >= sv->maxit) { sv->done[r] = 1; continue; }
            sv->act[r] = 1;
            any = true;
        }
        sv->j = sv->jq = 0;
        sv->halt = false;
        if (op->prof) {
            sv->col0 = op->prof->next;
            op->prof->next += sv->m;
        }
        sv->phase = any ? csg_solve::CYCLE : csg_solve::FINISHED;
        break;
    case csg_solve::CYCLE: {
        bool still = false;
        for (int r = 0; r < sv->nrhs; ++r) {
            if (sv->done[r] || !sv->act[r]) continue;
            sv->it[r]++;
            sv->est[r] = rp[r].est;
            if (!rp[r].finite) { sv->act[r] = 0; sv->rc = CSG_ENUMERIC; sv->done[r] = 1; continue; }
            if (rp[r].est <= sv->tol || rp[r].hn == 0.0 || sv->it[r] >= sv->maxit) { sv->act[r] = 0; continue; }
            still = true;
        }
        sv->j++;
        if (!still) {
            sv->halt = true;   // the columns queued behind this one are no-ops
            if (op->prof && sv->jq > sv->j) op->prof->skipped.push_back({sv->col0 + sv->j, sv->col0 + sv->jq});
        }
        if (sv->j == sv->jq && (sv->halt || sv->j == sv->m)) sv->phase = csg_solve::CYCLE_END;
        break;
    }
    default:
        break;
    }
}

}  // namespace

// ===========================================================================
// exported entry points
// ===========================================================================

extern "C" {

const char *csg_last_error(void) { return g_err.c_str(); }

int csg_plan_levels(const csg_params *p, int *levels, int dims[][3])
{
    if (!p) return fail(CSG_EINVAL, "null params");
    int nint[CSG_MAX_LEVELS][3];
    int L = 0;
    std::string err;
    int st = plan_levels(*p, L, nint, err);
    if (st) return fail(st, err);
    if (levels) *levels = L;
    if (dims)
        for (int l = 0; l < L; ++l)
            for (int a = 0; a < 3; ++a) dims[l][a] = a < p->dim ? nint[l][a] - 1 : 1;
    return CSG_OK;
}

}  // extern "C"

namespace {

// Fields a batch's problems must share (one size class): the grid shape,
// level count, cycle and solver sizes; h, beta, gamma and phi may differ.
bool same_class(const csg_params &a, const csg_params &b)
{
    bool eq = a.dim == b.dim && a.levels == b.levels && a.s == b.s && a.nu1 == b.nu1 && a.nu2 == b.nu2 &&
              a.cycle_prec == b.cycle_prec && a.max_rhs == b.max_rhs && a.restart == b.restart &&
              a.tail_max == b.tail_max && a.fuse_max == b.fuse_max && a.graphs == b.graphs &&
              a.smoother == b.smoother && a.slab_blocks == b.slab_blocks && a.tile_mult == b.tile_mult &&
              a.slab_min == b.slab_min && phi_shift(a) == phi_shift(b) && a.coarse_op == b.coarse_op;
    for (int d = 0; d < a.dim; ++d)
        eq = eq && a.n[d] == b.n[d] && a.layer_lo[d] == b.layer_lo[d] && a.layer_hi[d] == b.layer_hi[d];
    return eq;
}

int batch_bytes(const csg_params *p, int nprob, size_t *bytes)
{
    if (!p || !bytes) return fail(CSG_EINVAL, "null argument");
    if (nprob < 1 || (long)nprob * p->max_rhs > CSG_MAX_RHS)
        return fail(CSG_EINVAL, "nprob * max_rhs must be in 1..CSG_MAX_RHS");
    if (nprob > 1 && p->smoother != 0) return fail(CSG_EINVAL, "batched operators take the GMRES(s) smoother");
    int nint[CSG_MAX_LEVELS][3];
    int L = 0;
    std::string err;
    int st = plan_levels(*p, L, nint, err);
    if (st) return fail(st, err);
    csg_operator dry;
    memset(&dry, 0, sizeof(dry));
    dry.p = *p;
    dry.p.max_rhs = nprob * p->max_rhs;
    dry.nprob = nprob;
    dry.rpp = p->max_rhs;
    dry.L = L;
    dry.csize = p->cycle_prec ? 8 : 16;
    Carver cv(nullptr);
    carve(dry, nint, cv);
    *bytes = (cv.off + 255) & ~(size_t)255;
    return CSG_OK;
}

int create_impl(const csg_params *const *ps, const double *const *phis, int P, void *ws_dev, size_t ws_bytes,
                void *stream, csg_operator **out);

}  // namespace

extern "C" {

int csg_workspace_bytes(const csg_params *p, size_t *bytes) { return batch_bytes(p, 1, bytes); }

int csg_batch_workspace_bytes(const csg_params *p, int nprob, size_t *bytes) { return batch_bytes(p, nprob, bytes); }

int csg_operator_create(const csg_params *p, const double *phi_host, void *ws_dev, size_t ws_bytes, void *stream,
                        csg_operator **out)
{
    if (!p || !phi_host || !out) return fail(CSG_EINVAL, "null argument");
    return create_impl(&p, &phi_host, 1, ws_dev, ws_bytes, stream, out);
}

int csg_batch_create(const csg_params *const *p, int nprob, const double *const *phi_host, void *ws_dev,
                     size_t ws_bytes, void *stream, csg_operator **out)
{
    if (!p || !phi_host || !out || nprob < 1) return fail(CSG_EINVAL, "null argument or nprob < 1");
    for (int q = 0; q < nprob; ++q) {
        if (!p[q] || !phi_host[q]) return fail(CSG_EINVAL, "null params or phi");
        if (!same_class(*p[0], *p[q])) return fail(CSG_EINVAL, "batched problems must share one size class");
    }
    return create_impl(p, phi_host, nprob, ws_dev, ws_bytes, stream, out);
}

}  // extern "C"

namespace {

int create_impl(const csg_params *const *ps, const double *const *phis, int P, void *ws_dev, size_t ws_bytes,
                void *stream, csg_operator **out)
{
    const csg_params *p = ps[0];
    *out = nullptr;
    if (((uintptr_t)ws_dev & 255) != 0) return fail(CSG_EINVAL, "workspace must be 256-byte aligned");
    size_t need = 0;
    int st = batch_bytes(p, P, &need);
    if (st) return st;
    if (!ws_dev || ws_bytes < need) return fail(CSG_ENOMEM, "workspace too small");
    std::vector<HostHier> hhs(P);
    std::string err;
    for (int q = 0; q < P; ++q) {
        st = build_hierarchy(*ps[q], phis[q], hhs[q], err);
        if (st) return fail(st, P > 1 ? "problem " + std::to_string(q) + ": " + err : err);
    }
    const HostHier &hh = hhs[0];
    // the static scratch's address on this device, once per device (a failure
    // only disables csg_smooth_static, which reports it)
    if (!scratch_dev()) g_err = "no error";

    csg_operator *op = new csg_operator;
    memset(op, 0, sizeof(*op));
    op->p = *p;
    op->p.max_rhs = P * p->max_rhs;
    op->nprob = P;
    op->rpp = p->max_rhs;
    op->L = hh.L;
    op->csize = p->cycle_prec ? 8 : 16;
    int nint[CSG_MAX_LEVELS][3];
    for (int l = 0; l < hh.L; ++l)
        for (int a = 0; a < 3; ++a) nint[l][a] = hh.lev[l].nint[a];
    Carver cv(ws_dev);
    carve(*op, nint, cv);
    op->ws_used = cv.off;
    hipStream_t s = (hipStream_t)stream;
    const bool mixed = p->cycle_prec != 0;

    // tables with zeroed boundary weights (west of the first, east of the last unknown)
    std::vector<char> buf;
    auto put_tab = [&](const std::vector<cd> &t, int nu, const void *dst, bool dbl) -> hipError_t {
        const size_t esz = dbl ? 16 : 8;
        buf.assign(3 * (size_t)nu * esz, 0);
        for (int q = 0; q < 3 * nu; ++q) {
            cd v = t[q];
            if (q == 0 || q == 3 * nu - 1) v = 0.0;   // west[0], east[nu-1]
            if (dbl) {
                double *d = (double *)buf.data() + 2 * q;
                d[0] = v.real();
                d[1] = v.imag();
            } else {
                float *d = (float *)buf.data() + 2 * q;
                d[0] = (float)v.real();
                d[1] = (float)v.imag();
            }
        }
        return hipMemcpyAsync((void *)dst, buf.data(), buf.size(), hipMemcpyHostToDevice, s);
    };
    int rc = CSG_OK;
    std::vector<std::vector<char>> keep;   // host staging kept alive until the sync below
    const int R = op->p.max_rhs;   // every problem's right-hand sides
    const size_t cz = op->csize;
    for (int l = 0; l < hh.L && rc == CSG_OK; ++l) {
        for (int q = 0; q < P; ++q) {
            // problem q's tables and phi follow problem q-1's (strides of the kernels' LvlK)
            const HostLevel &hl = hhs[q].lev[l];
            for (int a = 0; a < p->dim; ++a) {
                const char *dst = (const char *)op->lev[l].tab[a] + (size_t)q * 3 * hl.nu[a] * cz;
                if (put_tab(hl.tab[a], hl.nu[a], dst, !mixed) != hipSuccess) rc = CSG_EDEVICE;
                hipStreamSynchronize(s);
            }
            std::vector<char> ph(hl.N * (mixed ? 4 : 8));
            for (long k = 0; k < hl.N; ++k) {
                if (mixed) ((float *)ph.data())[k] = (float)hl.phi[k];
                else ((double *)ph.data())[k] = hl.phi[k];
            }
            if (hipMemcpyAsync((char *)op->lev[l].phi + (size_t)q * ph.size(), ph.data(), ph.size(),
                               hipMemcpyHostToDevice, s) != hipSuccess)
                rc = CSG_EDEVICE;
            keep.push_back(std::move(ph));
            if (op->lev[l].gst) {
                // Galerkin stencil in the cycle precision, problem q after problem q-1
                std::vector<char> gs(hl.gst.size() * cz);
                for (size_t k = 0; k < hl.gst.size(); ++k) {
                    if (mixed) {
                        ((float *)gs.data())[2 * k] = (float)hl.gst[k].real();
                        ((float *)gs.data())[2 * k + 1] = (float)hl.gst[k].imag();
                    } else {
                        ((double *)gs.data())[2 * k] = hl.gst[k].real();
                        ((double *)gs.data())[2 * k + 1] = hl.gst[k].imag();
                    }
                }
                if (hipMemcpyAsync((char *)op->lev[l].gst + (size_t)q * gs.size(), gs.data(), gs.size(),
                                   hipMemcpyHostToDevice, s) != hipSuccess)
                    rc = CSG_EDEVICE;
                keep.push_back(std::move(gs));
            }
        }
        if (hipMemsetAsync(op->lev[l].gs, 0, R * sizeof(GState), s) != hipSuccess) rc = CSG_EDEVICE;
        for (int k = 0; k < 2; ++k)
            if (hipMemsetAsync(op->lev[l].part[k], 0, (size_t)R * NVAL * NBMAX * sizeof(zc), s) != hipSuccess)
                rc = CSG_EDEVICE;
    }
    for (int q = 0; q < P; ++q)
        for (int a = 0; a < p->dim && rc == CSG_OK; ++a) {
            const char *dst = (const char *)op->tabH[a] + (size_t)q * 3 * hh.lev[0].nu[a] * sizeof(zc);
            if (put_tab(hhs[q].tabH[a], hh.lev[0].nu[a], dst, true) != hipSuccess) rc = CSG_EDEVICE;
            hipStreamSynchronize(s);
        }
    {
        // the coarse tail starts at the first level small enough for one workgroup
        // execution tuning: parameter, else environment (experiments), else default
        long tail_max = 1200;
        if (const char *e = getenv("CSG_TAIL_MAX")) tail_max = atol(e);
        if (p->tail_max) tail_max = p->tail_max < 0 ? 0 : p->tail_max;
        op->fuse_max = 300000;
        if (const char *e = getenv("CSG_FUSE_MAX")) op->fuse_max = atol(e);
        if (p->fuse_max) op->fuse_max = p->fuse_max < 0 ? 0 : p->fuse_max;
        op->tiles = true;
        if (const char *e = getenv("CSG_TILES")) op->tiles = atoi(e) != 0;
        op->hdot_tiles = true;
        if (const char *e = getenv("CSG_HDOT_TILES")) op->hdot_tiles = atoi(e) != 0;
        op->up_tiles = true;
        if (const char *e = getenv("CSG_UP_TILES")) op->up_tiles = atoi(e) != 0;
        op->down_tiles = true;
        if (const char *e = getenv("CSG_DOWN_TILES")) op->down_tiles = atoi(e) != 0;
        op->fuse_upd = true;
        if (const char *e = getenv("CSG_FUSE_UPD")) op->fuse_upd = atoi(e) != 0;
        op->force_cgs2 = false;
        if (const char *e = getenv("CSG_FORCE_CGS2")) op->force_cgs2 = atoi(e) != 0;
        // deferred second rounds need the register or wavefront-split first
        // projection (CSG_PROJ0W=0 selects the two-pass one for long columns)
        op->lazy = true;
        if (const char *e = getenv("CSG_LAZY")) op->lazy = atoi(e) != 0;
        op->slab_pr = true;
        if (const char *e = getenv("CSG_SLAB_PR")) op->slab_pr = atoi(e) != 0;
        op->slab_down = true;
        if (const char *e = getenv("CSG_SLAB_DOWN")) op->slab_down = atoi(e) != 0;
        if (const char *e = getenv("CSG_PROJ0W"))
            if (atoi(e) == 0) op->lazy = false;
        op->poly_tiles = true;
        if (const char *e = getenv("CSG_POLY_TILES")) op->poly_tiles = atoi(e) != 0;
        op->slab_min = 100000;
        if (const char *e = getenv("CSG_SLAB_MIN")) op->slab_min = atol(e);
        if (const char *e = getenv("CSG_SLABS"))
            if (atoi(e) == 0) op->slab_min = -1;
        if (p->slab_min) op->slab_min = p->slab_min;
        if (op->slab_min < 0) op->slab_min = (long)1 << 62;
        if (p->coarse_op == 1) {
            // Galerkin levels: only the multi-block passes take a stored stencil
            op->tiles = false;
            op->slab_min = (long)1 << 62;
            op->fuse_max = 0;
            tail_max = 0;
        }
        for (int l = 0; l < op->L; ++l) {
            op->lev[l].varphi = hh.lev[l].varphi;
            op->lev[l].conds = hh.lev[l].conds;
            for (int i = 0; i < 3; ++i) op->lev[l].omega[i] = hh.lev[l].omega[i];
        }
        op->lt = op->L - 1;
        for (int l = 0; l < op->L; ++l)
            if ((long)op->lev[l].N <= tail_max) { op->lt = l; break; }
        // the tail keeps its vectors in shared memory when they fit
        op->tail_lds = 0;
        bool lds_on = true;
        if (const char *e = getenv("CSG_TAIL_LDS")) lds_on = atoi(e) != 0;
        if (lds_on) {
            unsigned Ns[CSG_MAX_LEVELS];
            for (int l = 0; l < op->L; ++l) Ns[l] = op->lev[l].N;
            const bool c64 = p->cycle_prec != 0, d3 = p->dim == 3;
            const size_t need = c64 ? (d3 ? tail_lds_bytes<float, 3>(Ns, op->lt, op->L, p->s)
                                          : tail_lds_bytes<float, 2>(Ns, op->lt, op->L, p->s))
                                    : (d3 ? tail_lds_bytes<double, 3>(Ns, op->lt, op->L, p->s)
                                          : tail_lds_bytes<double, 2>(Ns, op->lt, op->L, p->s));
            const bool ok = need <= TAIL_LDS_MAX &&
                            (c64 ? (d3 ? tail_lds_prepare<float, 3>(need, p->s) : tail_lds_prepare<float, 2>(need, p->s))
                                 : (d3 ? tail_lds_prepare<double, 3>(need, p->s)
                                       : tail_lds_prepare<double, 2>(need, p->s)));
            if (ok) op->tail_lds = need;
            hipGetLastError();
        }
        std::vector<TLev<double>> tl(op->L);
        for (int l = 0; l < op->L; ++l) {
            const DevLevel &d = op->lev[l];
            TLev<double> &t = tl[l];
            for (int a = 0; a < 3; ++a) t.tab[a] = (const zc *)d.tab[a];
            t.phi = (const double *)d.phi;
            t.b = (zc *)d.b;
            t.xa = (zc *)d.xa;
            t.xb = (zc *)d.xb;
            t.r = (zc *)d.r;
            for (int q = 0; q <= CSG_MAX_S; ++q) t.u[q] = (zc *)d.u[q];
            t.w[0] = (zc *)d.w[0];
            t.w[1] = (zc *)d.w[1];
            t.nx = d.nu[0];
            t.ny = d.nu[1];
            t.nz = d.nu[2];
            t.N = d.N;
            t.ld = d.ld;
            t.rpp = op->nprob > 1 ? (unsigned)op->rpp : 0u;
            for (int a = 0; a < 3; ++a) t.tstride[a] = 3 * d.nu[a];
            t.pstride = d.N;
            const cd sh = phi_shift(op->p);
            t.sre = sh.real();
            t.sim = sh.imag();
        }
        // the descriptor holds only pointers and sizes: identical layout for both precisions
        if (rc == CSG_OK && hipMemcpyAsync(op->tlev, tl.data(), tl.size() * sizeof(TLev<double>),
                                           hipMemcpyHostToDevice, s) != hipSuccess)
            rc = CSG_EDEVICE;
        hipStreamSynchronize(s);
    }
    for (int q = 0; q < P && rc == CSG_OK; ++q) {
        const HostHier &hq = hhs[q];
        if (hipMemcpyAsync((double *)op->phiH + (size_t)q * hh.lev[0].N, hq.lev[0].phi.data(),
                           hh.lev[0].N * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
            rc = CSG_EDEVICE;
        std::vector<char> mi((size_t)op->nc * op->nc * op->csize);
        for (size_t k = 0; k < (size_t)op->nc * op->nc; ++k) {
            if (mixed) {
                ((float *)mi.data())[2 * k] = (float)hq.minvT[k].real();
                ((float *)mi.data())[2 * k + 1] = (float)hq.minvT[k].imag();
            } else {
                ((double *)mi.data())[2 * k] = hq.minvT[k].real();
                ((double *)mi.data())[2 * k + 1] = hq.minvT[k].imag();
            }
        }
        if (hipMemcpyAsync((char *)op->minvT + (size_t)q * mi.size(), mi.data(), mi.size(), hipMemcpyHostToDevice,
                           s) != hipSuccess)
            rc = CSG_EDEVICE;
        keep.push_back(std::move(mi));
    }
    if (rc == CSG_OK) {
        std::vector<int> ones(3 * (size_t)R, 1);
        if (hipMemcpyAsync(op->active, ones.data(), ones.size() * sizeof(int), hipMemcpyHostToDevice, s) !=
            hipSuccess)
            rc = CSG_EDEVICE;
        if (hipMemsetAsync(op->fs, 0, R * sizeof(FState), s) != hipSuccess) rc = CSG_EDEVICE;
        if (hipStreamSynchronize(s) != hipSuccess) rc = CSG_EDEVICE;
    }
    if (rc == CSG_OK) {
        if (hipHostMalloc((void **)&op->rep_host, (LOOKAHEAD + 1) * (size_t)R * sizeof(Report),
                          hipHostMallocDefault) != hipSuccess ||
            hipHostGetDevicePointer((void **)&op->rep_dev, op->rep_host, 0) != hipSuccess)
            rc = CSG_EDEVICE;
        for (int q = 0; q <= LOOKAHEAD; ++q)
            if (hipEventCreateWithFlags(&op->evq[q], hipEventDisableTiming) != hipSuccess) rc = CSG_EDEVICE;
        op->gc = new GraphCache;
        if (const char *e = getenv("CSG_GRAPHS")) op->gc->enabled = atoi(e) != 0;
        if (p->graphs) op->gc->enabled = p->graphs > 0;
        if (hipStreamCreateWithFlags(&op->gc->cap, hipStreamNonBlocking) != hipSuccess) rc = CSG_EDEVICE;
    }
    if (rc != CSG_OK) {
        hipError_t e = hipGetLastError();
        if (op->rep_host) hipHostFree(op->rep_host);
        for (int q = 0; q <= LOOKAHEAD; ++q)
            if (op->evq[q]) hipEventDestroy(op->evq[q]);
        if (op->gc) {
            if (op->gc->cap) hipStreamDestroy(op->gc->cap);
            delete op->gc;
        }
        delete op;
        return fail(rc, std::string("device setup failed: ") + hipGetErrorString(e));
    }
    *out = op;
    return CSG_OK;
}

}  // namespace

extern "C" {

int csg_profile(csg_operator *op, int kind, int cap)
{
    if (!op) return fail(CSG_EINVAL, "null operator");
    if (kind < 0 || kind >= CSG_PROF_KINDS || cap < 0 || cap > (1 << 20)) return fail(CSG_EINVAL, "bad profile kind/cap");
    hipDeviceSynchronize();
    if (op->prof) {
        for (hipEvent_t e : op->prof->ev) hipEventDestroy(e);
        delete op->prof;
        op->prof = nullptr;
    }
    if (kind == CSG_PROF_OFF || cap == 0) return CSG_OK;
    Prof *pr = new Prof;
    pr->kind = kind;
    pr->cap = cap;
    pr->ev.resize(2 * (size_t)cap);
    pr->bytes.assign((size_t)cap, 0.0);
    pr->col.assign((size_t)cap, -1);
    // timing-only events: no system-scope fence (cache write-back and
    // invalidation) around the timed launches
    for (auto &e : pr->ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
            delete pr;
            return fail(CSG_EDEVICE, "event creation failed");
        }
    op->prof = pr;
    return CSG_OK;
}

int csg_profile_read(csg_operator *op, double *ms, long *launches, double *bytes)
{
    if (!op) return fail(CSG_EINVAL, "null operator");
    double tot = 0.0;
    long n = 0;
    double by = 0.0;
    if (op->prof && op->prof->n > 0) {
        Prof *pr = op->prof;
        if (hipEventSynchronize(pr->ev[2 * (pr->n - 1) + 1]) != hipSuccess) return fail(CSG_EDEVICE, "event wait");
        for (int i = 0; i < pr->n; ++i) {
            bool skip = false;
            for (const auto &r : pr->skipped) skip = skip || (pr->col[i] >= r.first && pr->col[i] < r.second);
            if (skip) continue;
            float t = 0.f;
            if (hipEventElapsedTime(&t, pr->ev[2 * i], pr->ev[2 * i + 1]) != hipSuccess)
                return fail(CSG_EDEVICE, "event elapsed time");
            tot += t;
            by += pr->bytes[i];
            ++n;
        }
    }

    if (ms) *ms = tot;
    if (launches) *launches = n;
    if (bytes) *bytes = by;
    return CSG_OK;
}

int csg_graphs_active(const csg_operator *op)
{
    if (!op) return fail(CSG_EINVAL, "null operator");
    return op->gc && op->gc->enabled ? 1 : 0;
}

int csg_operator_destroy(csg_operator *op)
{
    if (!op) return CSG_OK;
    if (op->prof) csg_profile(op, CSG_PROF_OFF, 0);
    if (op->gc) {
        // a solve's graphs finished when csg_solve_end synchronised its stream;
        // captures run on the private stream only
        if (op->gc->cap) hipStreamSynchronize(op->gc->cap);
        drop_graphs(op);
        if (op->gc->cap) hipStreamDestroy(op->gc->cap);
        delete op->gc;
    }
    for (int q = 0; q <= LOOKAHEAD; ++q)
        if (op->evq[q]) hipEventDestroy(op->evq[q]);
    if (op->rep_host) hipHostFree(op->rep_host);
    delete op;
    return CSG_OK;
}

int csg_operator_info(const csg_operator *op, int *levels, int dims[][3])
{
    if (!op) return fail(CSG_EINVAL, "null operator");
    if (levels) *levels = op->L;
    if (dims)
        for (int l = 0; l < op->L; ++l)
            for (int a = 0; a < 3; ++a) dims[l][a] = (int)op->lev[l].nu[a];
    return CSG_OK;
}

int csg_stencil_apply(const csg_operator *op, int which, int level, const void *x, void *y, int nrhs, void *stream)
{
    int st = check_op(op, nrhs);
    if (st) return st;
    if (which != 0 && which != 1) return fail(CSG_EINVAL, "which must be 0 (H) or 1 (M)");
    if (level < 0 || level >= op->L || (which == 0 && level != 0)) return fail(CSG_EINVAL, "bad level");
    if (nrhs == 0) return CSG_OK;
    if (!x || !y) return fail(CSG_EINVAL, "null vector");
    const Launch g = lch(op, level, nrhs, (hipStream_t)stream);
    const size_t ld = op->lev[level].ld;
    const bool d3 = op->p.dim == 3;
    if (which == 0) {
        if (d3) launch_apply<double, 3>(lvlH(op), x, y, ld, g, op->ones);
        else launch_apply<double, 2>(lvlH(op), x, y, ld, g, op->ones);
    } else if (op->p.cycle_prec) {
        if (d3) launch_apply<float, 3>(lvl<float>(op, level), x, y, ld, g, op->ones);
        else launch_apply<float, 2>(lvl<float>(op, level), x, y, ld, g, op->ones);
    } else {
        if (d3) launch_apply<double, 3>(lvl<double>(op, level), x, y, ld, g, op->ones);
        else launch_apply<double, 2>(lvl<double>(op, level), x, y, ld, g, op->ones);
    }
    return last_launch_error();
}

int csg_vcycle(const csg_operator *op, const void *b, void *x, int nrhs, void *stream)
{
    int st = check_op(op, nrhs);
    if (st) return st;
    if (nrhs == 0) return CSG_OK;
    if (!b || !x) return fail(CSG_EINVAL, "null vector");
    run_vcycle(op, b, x, nrhs, (hipStream_t)stream, op->ones);
    return last_launch_error();
}

int csg_smooth(const csg_operator *op, int level, const void *b, void *x, int nrhs, void *stream)
{
    int st = check_op(op, nrhs);
    if (st) return st;
    if (level < 0 || level >= op->L) return fail(CSG_EINVAL, "bad level");
    if (nrhs == 0) return CSG_OK;
    if (!b || !x) return fail(CSG_EINVAL, "null vector");
    hipStream_t s = (hipStream_t)stream;
    if (op->p.cycle_prec) {
        if (op->p.dim == 3) smooth_inplace<float, 3>(op, level, (const cf *)b, (cf *)x, nrhs, s, op->ones);
        else smooth_inplace<float, 2>(op, level, (const cf *)b, (cf *)x, nrhs, s, op->ones);
    } else {
        if (op->p.dim == 3) smooth_inplace<double, 3>(op, level, (const zc *)b, (zc *)x, nrhs, s, op->ones);
        else smooth_inplace<double, 2>(op, level, (const zc *)b, (zc *)x, nrhs, s, op->ones);
    }
    return last_launch_error();
}

int csg_poly_info(const csg_operator *op, int level, double *varphi, double omega[6], int *conds)
{
    if (!op) return fail(CSG_EINVAL, "null operator");
    if (level < 0 || level >= op->L) return fail(CSG_EINVAL, "bad level");
    const DevLevel &lv = op->lev[level];
    if (varphi) *varphi = lv.varphi;
    if (omega)
        for (int i = 0; i < 3; ++i) {
            omega[2 * i] = lv.omega[i].real();
            omega[2 * i + 1] = lv.omega[i].imag();
        }
    if (conds) *conds = lv.conds;
    return CSG_OK;
}

int csg_smooth_static(const csg_operator *op, int level, const void *b, void *x, int nrhs, void *stream)
{
    int st = check_op(op, nrhs);
    if (st) return st;
    if (level < 0 || level >= op->L) return fail(CSG_EINVAL, "bad level");
    if (nrhs == 0) return CSG_OK;
    if (!b || !x) return fail(CSG_EINVAL, "null vector");
    char *base = scratch_dev();
    if (!base) return fail(CSG_EDEVICE, g_err);
    // the sweep's own vectors (residual, u_1..u_s, w_0, w_1), reduction
    // partials and smoother states, carved from the scratch as from a workspace
    csg_operator tmp = *op;
    tmp.prof = nullptr;
    DevLevel &lv = tmp.lev[level];
    Carver cv(base);
    const size_t vb = (size_t)nrhs * lv.ld * op->csize;
    lv.r = cv.take(vb);
    for (int i = 1; i <= op->p.s; ++i) lv.u[i] = cv.take(vb);
    lv.w[0] = cv.take(vb);
    lv.w[1] = cv.take(vb);
    if (op->p.smoother == 1) lv.xb = cv.take(vb);   // the polynomial sweep's result before the copy back
    const size_t cleared = cv.off;
    const size_t pb = (size_t)nrhs * NVAL * NBMAX * sizeof(zc);
    lv.part[0] = (zc *)cv.take(pb);
    lv.part[1] = (zc *)cv.take(pb);
    lv.gs = (GState *)cv.take((size_t)nrhs * sizeof(GState));
    const size_t end = (cv.off + 255) & ~(size_t)255;
    if (end > SCRATCH_BYTES)
        return fail(CSG_ENOMEM, "csg_smooth_static: the sweep needs " + std::to_string(end) +
                                    " bytes of scratch, more than the " + std::to_string(SCRATCH_BYTES) + " it has");
    hipStream_t s = (hipStream_t)stream;
    // partials and states start at zero on every call (the array keeps the last call's contents)
    const size_t z0 = (cleared + 255) & ~(size_t)255;
    launch_zero16(base + z0, end - z0, s);
    if (op->p.cycle_prec) {
        if (op->p.dim == 3) smooth_inplace<float, 3>(&tmp, level, (const cf *)b, (cf *)x, nrhs, s, op->ones);
        else smooth_inplace<float, 2>(&tmp, level, (const cf *)b, (cf *)x, nrhs, s, op->ones);
    } else {
        if (op->p.dim == 3) smooth_inplace<double, 3>(&tmp, level, (const zc *)b, (zc *)x, nrhs, s, op->ones);
        else smooth_inplace<double, 2>(&tmp, level, (const zc *)b, (zc *)x, nrhs, s, op->ones);
    }
    return last_launch_error();
}

int csg_residual_restrict(const csg_operator *op, int level, const void *b, const void *x, void *bc, int nrhs,
                          void *stream)
{
    int st = check_op(op, nrhs);
    if (st) return st;
    if (level < 0 || level >= op->L - 1) return fail(CSG_EINVAL, "bad level (needs a coarser level)");
    if (nrhs == 0) return CSG_OK;
    if (!b || !bc) return fail(CSG_EINVAL, "null vector");
    const Launch g = lch(op, level + 1, nrhs, (hipStream_t)stream);
    const size_t ldf = op->lev[level].ld, ldc = op->lev[level + 1].ld;
    if (op->p.cycle_prec) {
        if (op->p.dim == 3)
            launch_restrict<float, 3>(lvl<float>(op, level), lvl<float>(op, level + 1), (const cf *)x, (const cf *)b,
                                      (cf *)bc, ldf, ldc, g, op->ones);
        else
            launch_restrict<float, 2>(lvl<float>(op, level), lvl<float>(op, level + 1), (const cf *)x, (const cf *)b,
                                      (cf *)bc, ldf, ldc, g, op->ones);
    } else {
        if (op->p.dim == 3)
            launch_restrict<double, 3>(lvl<double>(op, level), lvl<double>(op, level + 1), (const zc *)x,
                                       (const zc *)b, (zc *)bc, ldf, ldc, g, op->ones);
        else
            launch_restrict<double, 2>(lvl<double>(op, level), lvl<double>(op, level + 1), (const zc *)x,
                                       (const zc *)b, (zc *)bc, ldf, ldc, g, op->ones);
    }
    return last_launch_error();
}

int csg_prolong_correct(const csg_operator *op, int level, const void *ec, void *x, int nrhs, void *stream)
{
    int st = check_op(op, nrhs);
    if (st) return st;
    if (level < 0 || level >= op->L - 1) return fail(CSG_EINVAL, "bad level (needs a coarser level)");
    if (nrhs == 0) return CSG_OK;
    if (!ec || !x) return fail(CSG_EINVAL, "null vector");
    const Launch g = lch(op, level, nrhs, (hipStream_t)stream);
    const size_t ldf = op->lev[level].ld, ldc = op->lev[level + 1].ld;
    if (op->p.cycle_prec) {
        if (op->p.dim == 3)
            launch_prolong<float, 3>(lvl<float>(op, level), lvl<float>(op, level + 1), (const cf *)ec, (const cf *)x,
                                     (cf *)x, ldf, ldc, g, op->ones);
        else
            launch_prolong<float, 2>(lvl<float>(op, level), lvl<float>(op, level + 1), (const cf *)ec, (const cf *)x,
                                     (cf *)x, ldf, ldc, g, op->ones);
    } else {
        if (op->p.dim == 3)
            launch_prolong<double, 3>(lvl<double>(op, level), lvl<double>(op, level + 1), (const zc *)ec,
                                      (const zc *)x, (zc *)x, ldf, ldc, g, op->ones);
        else
            launch_prolong<double, 2>(lvl<double>(op, level), lvl<double>(op, level + 1), (const zc *)ec,
                                      (const zc *)x, (zc *)x, ldf, ldc, g, op->ones);
    }
    return last_launch_error();
}

int csg_coarse_solve(const csg_operator *op, const void *b, void *x, int nrhs, void *stream)
{
    int st = check_op(op, nrhs);
    if (st) return st;
    if (nrhs == 0) return CSG_OK;
    if (!b || !x) return fail(CSG_EINVAL, "null vector");
    const size_t ld = op->lev[op->L - 1].ld;
    if (op->p.cycle_prec)
        launch_coarse<float>((const cf *)op->minvT, op->nc, (const cf *)b, (cf *)x, ld, nrhs, (hipStream_t)stream,
                             op->ones, minv_stride(op), batch_rpp(op));
    else
        launch_coarse<double>((const zc *)op->minvT, op->nc, (const zc *)b, (zc *)x, ld, nrhs, (hipStream_t)stream,
                              op->ones, minv_stride(op), batch_rpp(op));
    return last_launch_error();
}

int csg_solve_begin(const csg_operator *opc, const void *chi, void *u, int nrhs, double tol, int restart, int maxit,
                    int use_initial_guess, void *stream, csg_solve **out)
{
    csg_operator *op = const_cast<csg_operator *>(opc);
    if (!out) return fail(CSG_EINVAL, "null output");
    *out = nullptr;
    int st = check_op(op, nrhs);
    if (st) return st;
    if (nrhs < 1) return fail(CSG_EINVAL, "nrhs must be >= 1");
    if (!chi || !u) return fail(CSG_EINVAL, "null vector");
    if (restart < 1 || restart > op->p.restart) return fail(CSG_EINVAL, "restart exceeds the workspace's restart");
    if (maxit < 0) return fail(CSG_EINVAL, "maxit must be >= 0");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(CSG_EINVAL, "tol must be finite and >= 0");
    if (op->busy) return fail(CSG_EINVAL, "a solve is already in flight on this operator");
    csg_solve *sv = new csg_solve();
    sv->op = op;
    sv->chi = (const zc *)chi;
    sv->u = (zc *)u;
    sv->nrhs = nrhs;
    sv->m = restart;
    sv->maxit = maxit;
    sv->use_x0 = use_initial_guess;
    sv->tol = tol;
    sv->st = (hipStream_t)stream;
    sv->phase = csg_solve::INIT;
    sv->rc = CSG_OK;
    if (hipHostMalloc((void **)&sv->mask_host, 2 * op->p.max_rhs * sizeof(int), hipHostMallocDefault) != hipSuccess) {
        delete sv;
        return fail(CSG_EDEVICE, "pinned host allocation failed");
    }
    sv->t0 = std::chrono::steady_clock::now();
    if (!use_initial_guess) {
        if (hipMemsetAsync(sv->u, 0, (size_t)nrhs * op->lev[0].ld * sizeof(zc), sv->st) != hipSuccess) {
            hipHostFree(sv->mask_host);
            delete sv;
            return fail(CSG_EDEVICE, "memset of the initial guess failed");
        }
    }
    op->busy = 1;
    *out = sv;
    return solve_step(sv);
}

int csg_solve_step(csg_solve *sv)
{
    if (!sv) return fail(CSG_EINVAL, "null solve");
    return solve_step(sv);
}

int csg_solve_poll(csg_solve *sv, int *done)
{
    if (!sv) return fail(CSG_EINVAL, "null solve");
    if (done) *done = sv->phase == csg_solve::FINISHED;
    if (sv->phase == csg_solve::FINISHED) return 1;
    hipEvent_t ev = pending_event(sv);
    if (!ev) return 1;   // no report in flight: the caller should step
    hipError_t e = hipEventQuery(ev);
    if (e == hipErrorNotReady) return 0;
    if (e != hipSuccess) return fail(CSG_EDEVICE, std::string("solve: ") + hipGetErrorString(e));
    solve_advance(sv);
    if (done) *done = sv->phase == csg_solve::FINISHED;
    return 1;
}

int csg_solve_end(csg_solve *sv, csg_solve_info *info)
{
    if (!sv) return fail(CSG_EINVAL, "null solve");
    hipError_t e = hipStreamSynchronize(sv->st);
    sv->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - sv->t0).count();
    int rc = sv->rc;
    if (e != hipSuccess) rc = fail(CSG_EDEVICE, std::string("solve: ") + hipGetErrorString(e));
    bool all = true;
    for (int r = 0; r < sv->nrhs; ++r) {
        all = all && sv->conv[r];
        if (info) {
            info[r].iterations = sv->it[r];
            info[r].restarts = sv->restarts[r];
            info[r].vcycles = sv->it[r];
            info[r].converged = sv->conv[r];
            info[r].relres_true = sv->truer[r];
            info[r].relres_est = sv->est[r];
            info[r].seconds = sv->seconds;
        }
    }
    if (rc == CSG_OK && !all) rc = fail(CSG_ENOCONV, "maxit reached before the tolerance");
    if (rc == CSG_ENUMERIC) fail(CSG_ENUMERIC, "non-finite residual norm");
    sv->op->busy = 0;
    hipHostFree(sv->mask_host);
    delete sv;
    return rc;
}

int helm_step_batch(csg_solve *sv, int *done)
{
    if (!sv) return fail(CSG_EINVAL, "null solve");
    int d = sv->phase == csg_solve::FINISHED;
    if (!d) {
        hipEvent_t ev = pending_event(sv);
        if (ev && hipEventSynchronize(ev) != hipSuccess) return fail(CSG_EDEVICE, "event wait failed");
        const int pr = csg_solve_poll(sv, &d);
        if (pr < 0) return pr;
        if (!d) {
            const int st = csg_solve_step(sv);
            if (st) return st;
        }
    }
    if (done) *done = d;
    return CSG_OK;
}

int helm_solve(const csg_operator *op, const void *chi, void *u, int nrhs, double tol, int restart, int maxit,
               int use_initial_guess, csg_solve_info *info, void *stream)
{
    int st = check_op(op, nrhs);
    if (st) return st;
    if (nrhs == 0) return CSG_OK;
    csg_solve *sv = nullptr;
    st = csg_solve_begin(op, chi, u, nrhs, tol, restart, maxit, use_initial_guess, stream, &sv);
    if (!sv) return st;
    while (st == CSG_OK && sv->phase != csg_solve::FINISHED) {
        hipEvent_t ev = pending_event(sv);
        if (ev && hipEventSynchronize(ev) != hipSuccess) { st = fail(CSG_EDEVICE, "event wait failed"); break; }
        int done = 0;
        int pr = csg_solve_poll(sv, &done);
        if (pr < 0) { st = pr; break; }
        if (done) break;
        st = csg_solve_step(sv);
    }
    const std::string first = g_err;
    int rc = csg_solve_end(sv, info);
    if (st != CSG_OK) {
        g_err = first;   // report the failure that stopped the loop
        return st;
    }
    return rc;
}

}  // extern "C"
