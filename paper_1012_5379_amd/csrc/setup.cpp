// setup.cpp -- host construction of the multigrid hierarchy in FP64.
//
// Section 2 (eq. csggrid): each axis is a complex grid of layer_lo intervals of
// h e^{i gamma}, n interior intervals of h e^{i theta} and layer_hi intervals of
// h e^{i gamma}; theta = 0 gives the ECS grid of H, theta = beta the stretched
// grid of the preconditioner M.  The operator is the Shortley-Weller 3-point
// discretisation of the negative second derivative per axis, summed over axes
// (Kronecker sum), minus phi.  Section 3.1: coarse operators are obtained by
// rediscretising on the coarser complex grid; here each coarse grid takes every
// other node of the finer one (the last node always kept, so an odd interval
// count leaves one single interval at the high end) and phi is injected.
#include <cmath>
#include <cstring>

#include "csg_internal.h"

namespace csg {

int plan_levels(const csg_params &p, int &L, int nint[CSG_MAX_LEVELS][3], std::string &err)
{
    if (p.dim != 2 && p.dim != 3) { err = "dim must be 2 or 3"; return CSG_EINVAL; }
    if (!(p.h > 0.0) || !std::isfinite(p.h)) { err = "h must be positive and finite"; return CSG_EINVAL; }
    if (!(p.gamma > 0.0 && p.gamma < M_PI / 4)) { err = "need 0 < gamma < pi/4"; return CSG_EINVAL; }
    if (!(p.beta >= 0.0 && p.beta < p.gamma)) { err = "need 0 <= beta < gamma"; return CSG_EINVAL; }
    if (p.s < 1 || p.s > CSG_MAX_S) { err = "s out of range 1..CSG_MAX_S"; return CSG_EINVAL; }
    if (p.nu1 < 0 || p.nu2 < 0) { err = "nu1, nu2 must be >= 0"; return CSG_EINVAL; }
    if (p.levels < 0 || p.levels > CSG_MAX_LEVELS) { err = "levels out of range"; return CSG_EINVAL; }
    if (p.cycle_prec != 0 && p.cycle_prec != 1) { err = "cycle_prec must be 0 or 1"; return CSG_EINVAL; }
    if (p.max_rhs < 1 || p.max_rhs > CSG_MAX_RHS) { err = "max_rhs out of range 1..CSG_MAX_RHS"; return CSG_EINVAL; }
    if (p.restart < 1 || p.restart > CSG_MAX_RESTART) { err = "restart out of range"; return CSG_EINVAL; }
    int cur[3] = {0, 0, 0};
    for (int a = 0; a < p.dim; ++a) {
        if (p.n[a] < 1 || p.layer_lo[a] < 0 || p.layer_hi[a] < 0) {
            err = "n >= 1 and layers >= 0 required";
            return CSG_EINVAL;
        }
        long tot = (long)p.n[a] + p.layer_lo[a] + p.layer_hi[a];
        if (tot < 2 || tot > (1L << 20)) { err = "interval count per axis out of range"; return CSG_EINVAL; }
        cur[a] = (int)tot;
    }
    long total = 1;
    for (int a = 0; a < p.dim; ++a) total *= (cur[a] - 1);
    if (total >= (1L << 31)) { err = "too many unknowns per right-hand side"; return CSG_EINVAL; }
    L = 0;
    for (;;) {
        for (int a = 0; a < 3; ++a) nint[L][a] = a < p.dim ? cur[a] : 0;
        ++L;
        bool more;
        if (p.levels > 0) {
            more = L < p.levels;
        } else {
            more = false;
            for (int a = 0; a < p.dim; ++a) more = more || cur[a] > 9;
        }
        if (!more) break;
        if (L >= CSG_MAX_LEVELS) { err = "too many levels"; return CSG_EINVAL; }
        for (int a = 0; a < p.dim; ++a) {
            cur[a] = (cur[a] + 1) / 2;
            if (cur[a] < 2) { err = "a level would have fewer than 2 intervals on an axis"; return CSG_EINVAL; }
        }
    }
    long nc = 1;
    for (int a = 0; a < p.dim; ++a) nc *= nint[L - 1][a] - 1;
    if (nc > MAXC) { err = "coarsest level has more than 4096 unknowns; add levels"; return CSG_EINVAL; }
    return CSG_OK;
}

namespace {

void fine_nodes(const csg_params &p, int a, double theta, std::vector<cd> &z)
{
    const cd hg = std::polar(p.h, p.gamma);
    const cd hb = std::polar(p.h, theta);
    const int nint = p.layer_lo[a] + p.n[a] + p.layer_hi[a];
    z.assign(nint + 1, cd(0.0));
    for (int j = 0; j < nint; ++j) {
        const bool layer = j < p.layer_lo[a] || j >= p.layer_lo[a] + p.n[a];
        z[j + 1] = z[j] + (layer ? hg : hb);
    }
}

// Shortley-Weller rows for the unknown nodes 1..nint-1:
//   west = -2 / (hm (hm + hp)), centre = 2 / (hm hp), east = -2 / (hp (hm + hp)).
void sw_rows(const std::vector<cd> &z, std::vector<cd> &tab)
{
    const int nu = (int)z.size() - 2;
    tab.assign(3 * (size_t)nu, cd(0.0));
    for (int q = 0; q < nu; ++q) {
        const cd hm = z[q + 1] - z[q];
        const cd hp = z[q + 2] - z[q + 1];
        tab[q] = -2.0 / (hm * (hm + hp));
        tab[nu + q] = 2.0 / (hm * hp);
        tab[2 * nu + q] = -2.0 / (hp * (hm + hp));
    }
}

// Gauss-Jordan inversion with partial pivoting of the dense coarsest matrix.
int invert(std::vector<cd> &A, int n, std::vector<cd> &inv)
{
    inv.assign((size_t)n * n, cd(0.0));
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        double best = std::abs(A[(size_t)c * n + c]);
        for (int r = c + 1; r < n; ++r) {
            double v = std::abs(A[(size_t)r * n + c]);
            if (v > best) { best = v; piv = r; }
        }
        if (!(best > 0.0)) return -1;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                std::swap(A[(size_t)c * n + k], A[(size_t)piv * n + k]);
                std::swap(inv[(size_t)c * n + k], inv[(size_t)piv * n + k]);
            }
        }
        const cd d = 1.0 / A[(size_t)c * n + c];
        for (int k = 0; k < n; ++k) {
            A[(size_t)c * n + k] *= d;
            inv[(size_t)c * n + k] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const cd f = A[(size_t)r * n + c];
            if (f == cd(0.0)) continue;
            for (int k = 0; k < n; ++k) {
                A[(size_t)r * n + k] -= f * A[(size_t)c * n + k];
                inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
            }
        }
    }
    return 0;
}

}  // namespace

int build_hierarchy(const csg_params &p, const double *phi, HostHier &hh, std::string &err)
{
    int nint[CSG_MAX_LEVELS][3];
    int L = 0;
    int st = plan_levels(p, L, nint, err);
    if (st) return st;
    hh.dim = p.dim;
    hh.L = L;
    for (int l = 0; l < L; ++l) {
        HostLevel &lv = hh.lev[l];
        lv.N = 1;
        for (int a = 0; a < 3; ++a) {
            lv.nint[a] = nint[l][a];
            lv.nu[a] = a < p.dim ? nint[l][a] - 1 : 1;
            lv.N *= lv.nu[a];
        }
        for (int a = 0; a < p.dim; ++a) {
            if (l == 0) {
                fine_nodes(p, a, p.beta, lv.z[a]);
            } else {
                const std::vector<cd> &zf = hh.lev[l - 1].z[a];
                const int nc = lv.nint[a];
                lv.z[a].resize(nc + 1);
                for (int J = 0; J < nc; ++J) lv.z[a][J] = zf[2 * (size_t)J];
                lv.z[a][nc] = zf.back();
            }
            sw_rows(lv.z[a], lv.tab[a]);
        }
        lv.phi.resize(lv.N);
        if (l == 0) {
            for (long q = 0; q < lv.N; ++q) {
                if (!std::isfinite(phi[q])) { err = "phi has a non-finite value"; return CSG_EINVAL; }
                lv.phi[q] = phi[q];
            }
        } else {
            // coarse unknown J sits on fine node 2(J+1), i.e. fine unknown 2J+1
            const HostLevel &F = hh.lev[l - 1];
            for (int K = 0; K < lv.nu[2]; ++K)
                for (int J = 0; J < lv.nu[1]; ++J)
                    for (int I = 0; I < lv.nu[0]; ++I) {
                        const long fi = 2L * I + 1;
                        const long fj = p.dim > 1 ? 2L * J + 1 : 0;
                        const long fk = p.dim > 2 ? 2L * K + 1 : 0;
                        lv.phi[I + (long)lv.nu[0] * (J + (long)lv.nu[1] * K)] =
                            F.phi[fi + (long)F.nu[0] * (fj + (long)F.nu[1] * fk)];
                    }
        }
    }
    for (int a = 0; a < p.dim; ++a) {
        std::vector<cd> zH;
        fine_nodes(p, a, 0.0, zH);
        sw_rows(zH, hh.tabH[a]);
    }
    // dense coarsest matrix, assembled row by row from the tables
    const HostLevel &C = hh.lev[L - 1];
    const int n = (int)C.N;
    hh.nc = n;
    std::vector<cd> A((size_t)n * n, cd(0.0));
    const int nx = C.nu[0], ny = C.nu[1], nz = C.nu[2];
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const long r = i + (long)nx * (j + (long)ny * k);
                cd diag = C.tab[0][nx + i] - C.phi[r];
                if (i > 0) A[r * n + r - 1] += C.tab[0][i];
                if (i < nx - 1) A[r * n + r + 1] += C.tab[0][2 * nx + i];
                if (p.dim > 1) {
                    diag += C.tab[1][ny + j];
                    if (j > 0) A[r * n + r - nx] += C.tab[1][j];
                    if (j < ny - 1) A[r * n + r + nx] += C.tab[1][2 * ny + j];
                }
                if (p.dim > 2) {
                    diag += C.tab[2][nz + k];
                    if (k > 0) A[r * n + r - (long)nx * ny] += C.tab[2][k];
                    if (k < nz - 1) A[r * n + r + (long)nx * ny] += C.tab[2][2 * nz + k];
                }
                A[r * n + r] += diag;
            }
    std::vector<cd> inv;
    if (invert(A, n, inv)) { err = "coarsest operator is singular"; return CSG_ENUMERIC; }
    hh.minvT.resize((size_t)n * n);
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) hh.minvT[(size_t)c * n + r] = inv[(size_t)r * n + c];
    return CSG_OK;
}

}  // namespace csg
