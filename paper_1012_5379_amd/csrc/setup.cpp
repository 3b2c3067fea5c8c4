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
#include <algorithm>
#include <cmath>
#include <cstring>

#include "csg_internal.h"

namespace csg {

std::complex<double> phi_shift(const csg_params &p)
{
    if (p.shift_re == 0.0 && p.shift_im == 0.0) return 1.0;
    return {p.shift_re, p.shift_im};
}

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
    if (p.smoother != 0 && p.smoother != 1) { err = "smoother must be 0 (GMRES) or 1 (polynomial)"; return CSG_EINVAL; }
    if (!(p.poly_k2 >= 0.0) || !std::isfinite(p.poly_k2)) { err = "poly_k2 must be finite and >= 0"; return CSG_EINVAL; }
    if (p.slab_blocks < 0 || p.slab_blocks > 4096) { err = "slab_blocks out of range 0..4096"; return CSG_EINVAL; }
    if (p.tile_mult < 0 || p.tile_mult > 64 || (p.tile_mult & (p.tile_mult - 1))) {
        err = "tile_mult must be 0 or a power of two <= 64";
        return CSG_EINVAL;
    }
    if (p.slab_min < -1) { err = "slab_min must be >= -1"; return CSG_EINVAL; }
    if (!std::isfinite(p.shift_re) || !std::isfinite(p.shift_im)) { err = "shift must be finite"; return CSG_EINVAL; }
    if (p.coarse_op != 0 && p.coarse_op != 1) { err = "coarse_op must be 0 (rediscretised) or 1 (Galerkin)"; return CSG_EINVAL; }
    if (p.smoother == 1 && p.coarse_op != 0) {
        err = "the polynomial smoother takes rediscretised coarse operators";
        return CSG_EINVAL;
    }
    if (p.smoother == 1 && !(p.shift_re == 0.0 && p.shift_im == 0.0) && !(p.shift_re == 1.0 && p.shift_im == 0.0)) {
        err = "the polynomial smoother takes the unshifted preconditioner (shift 1)";
        return CSG_EINVAL;
    }
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

// ---------------------------------------------------------------------------
// Third-order polynomial smoother (section 4)
// ---------------------------------------------------------------------------

// Monomial coefficients (g0, g1, g2) of the quadratic through (x_r, y_r),
// r = 0, 1, 2, from its Newton form.
void quad_through(const cd x[3], const cd y[3], cd g[3])
{
    const cd d01 = (y[1] - y[0]) / (x[1] - x[0]);
    const cd d12 = (y[2] - y[1]) / (x[2] - x[1]);
    const cd d012 = (d12 - d01) / (x[2] - x[0]);
    g[2] = d012;
    g[1] = d01 - d012 * (x[0] + x[1]);
    g[0] = y[0] - d01 * x[0] + d012 * x[0] * x[1];
}

// Angles v with |a| cos(v - arg a) < g, as [centre - half, centre + half];
// returns 1 for every angle, 0 for an arc, -1 for none.
int arc_of(cd a, double g, double &centre, double &half)
{
    const double m = std::abs(a);
    centre = std::arg(a) + M_PI;
    if (g >= m) { half = M_PI; return 1; }
    if (-g >= m) { half = 0.0; return -1; }
    half = M_PI - std::acos(g / m);
    return 0;
}

// The level's polynomial: triangle t0 = -k^2, t1 = -k^2 + 4d/(H e^{i beta})^2,
// t2 = -k^2 + 4d/(H e^{i gamma})^2 (Prop. 3.1, H = 2^l h).  Writing
// p(t) = c0 + (t - t0) g(t - t0) with g quadratic, p(0) = 1 and p(t1) = p(t2)
// = 0 fix g at the three nodes x = -t0, t1 - t0, t2 - t0 (eq.
// coefficients_system): g(x_r) = b_r / x_r with b = (1 - c0, -c0, -c0), so
// g = E - c0 F with E, F interpolating (1/x0, 0, 0) and (1/x0, 1/x1, 1/x2)
// (eq. coefficients_solution: c_j = e_j - e^{i varphi} f_j).  Along the top
// edge t0 + rho w, w = e^{-2i beta}, |p|^2 = 1 + 2 rho Fo + rho^2 So + ...:
//   Fo(v) = Re(e^{-iv} E0 w) - Re(F0 w)                        (first order)
//   So(v) = |E0|^2 + |F0|^2 - 2 Re(F1 w^2) + Re(e^{-iv} Z),
//   Z = 2 (E1 w^2 - E0 conj(F0))                               (second order)
// varphi is the midpoint of the angles where both are negative (or of those
// where the first is, when no angle meets both).
void poly_level(int dim, double beta, double gamma, double k2, double H, HostLevel &lv)
{
    const cd hb = std::polar(H, beta), hg = std::polar(H, gamma);
    const cd t0 = -k2, t1 = t0 + 4.0 * dim / (hb * hb), t2 = t0 + 4.0 * dim / (hg * hg);
    const cd x[3] = {-t0, t1 - t0, t2 - t0};
    const cd ye[3] = {1.0 / x[0], 0.0, 0.0};
    const cd yf[3] = {1.0 / x[0], 1.0 / x[1], 1.0 / x[2]};
    cd E[3], F[3];
    quad_through(x, ye, E);
    quad_through(x, yf, F);
    const cd w = std::polar(1.0, -2.0 * beta);
    double cA, hA, cB, hB;
    const int kA = arc_of(E[0] * w, (F[0] * w).real(), cA, hA);
    const double K = std::norm(E[0]) + std::norm(F[0]) - 2.0 * (F[1] * w * w).real();
    const int kB = arc_of(2.0 * (E[1] * w * w - E[0] * std::conj(F[0])), -K, cB, hB);
    double v = 0.0;
    int conds = 2;
    if (kA >= 0 && kB >= 0) {
        conds = 0;
        if (kA == 1 && kB == 1) v = 0.0;
        else if (kA == 1) v = cB;
        else if (kB == 1) v = cA;
        else {
            // overlap of [-hA, hA] with arc B shifted about arc A's centre
            const double d = std::remainder(cB - cA, 2.0 * M_PI);
            double len = 0.0, mid = 0.0;
            for (int q = -1; q <= 1; ++q) {
                const double lo = std::max(-hA, d + q * 2.0 * M_PI - hB);
                const double hi = std::min(hA, d + q * 2.0 * M_PI + hB);
                if (hi - lo > len) { len = hi - lo; mid = 0.5 * (lo + hi); }
            }
            if (len > 0.0) v = cA + mid;
            else { v = cA; conds = 1; }
        }
    } else if (kA >= 0) {
        v = kA == 1 ? 0.0 : cA;
        conds = 1;
    }
    v = std::remainder(v, 2.0 * M_PI);
    if (v < 0.0) v += 2.0 * M_PI;
    const cd c0 = std::polar(1.0, v);
    const cd c3 = E[2] - c0 * F[2];
    lv.varphi = v;
    lv.conds = conds;
    // roots 1/w: t1, t2 by construction, and the third from p(0) = 1 with
    // leading coefficient c3: p(t) = c3 (t - t1)(t - t2)(t - t3)
    lv.omega[0] = 1.0 / t1;
    lv.omega[1] = 1.0 / t2;
    lv.omega[2] = -c3 * t1 * t2;
}

}  // namespace

// ---------------------------------------------------------------------------
// Galerkin coarse operators (section 5 remark)

namespace {

// Entry (p, p + o) of level F's operator, o in {-1, 0, 1}^d (0 when p + o lies
// outside the grid): the Kronecker-sum rows with s phi on the diagonal, or a
// Galerkin level's stored stencil.
cd op_entry(const HostLevel &F, int dim, cd shift, const int i[3], const int o[3])
{
    for (int a = 0; a < 3; ++a)
        if (i[a] + o[a] < 0 || i[a] + o[a] >= F.nu[a]) return 0.0;
    const long p = i[0] + (long)F.nu[0] * (i[1] + (long)F.nu[1] * i[2]);
    if (!F.gst.empty()) {
        int oi = 0, m = 1;
        for (int a = 0; a < dim; ++a, m *= 3) oi += (o[a] + 1) * m;
        return F.gst[(size_t)oi * F.N + p];
    }
    int moved = 0, ax = 0;
    for (int a = 0; a < dim; ++a)
        if (o[a]) { ++moved; ax = a; }
    if (moved > 1) return 0.0;
    if (moved == 0) {
        cd d = -shift * F.phi[p];
        for (int a = 0; a < dim; ++a) d += F.tab[a][F.nu[a] + i[a]];
        return d;
    }
    const int n = F.nu[ax];
    return o[ax] < 0 ? F.tab[ax][i[ax]] : F.tab[ax][2 * n + i[ax]];
}

// Linear interpolation weight of coarse unknown J at fine unknown f on one
// axis: coarse unknown J is fine unknown 2J + 1 (weight 1), its fine
// neighbours take 1/2.
double lin_w(int f, int J)
{
    const int c = 2 * J + 1;
    return f == c ? 1.0 : (f == c - 1 || f == c + 1) ? 0.5 : 0.0;
}

// C.gst = R M_F P, entry by entry: for coarse unknown K and each fine unknown i
// that R_K weighs (2^{-d} times the interpolation weights), each fine neighbour
// i' of i in M_F, and each coarse unknown J within one of K that P spreads onto
// i', accumulate R_{K,i} (M_F)_{i,i'} P_{i',J} into offset J - K.
void galerkin_level(const HostLevel &F, HostLevel &C, int dim, cd shift)
{
    const int np = dim == 2 ? 9 : 27;
    C.gst.assign((size_t)np * C.N, cd(0.0));
    const double rs = std::ldexp(1.0, -dim);
    const int r1[3] = {1, dim > 1 ? 1 : 0, dim > 2 ? 1 : 0};   // offset range per axis
    for (int K2 = 0; K2 < C.nu[2]; ++K2)
        for (int K1 = 0; K1 < C.nu[1]; ++K1)
            for (int K0 = 0; K0 < C.nu[0]; ++K0) {
                const int K[3] = {K0, K1, K2};
                const long pk = K0 + (long)C.nu[0] * (K1 + (long)C.nu[1] * K2);
                int i[3], o[3], jj[3], ip[3];
                for (i[2] = 2 * K[2] + 1 - r1[2]; i[2] <= 2 * K[2] + 1 + r1[2]; ++i[2])
                    for (i[1] = 2 * K[1] + 1 - r1[1]; i[1] <= 2 * K[1] + 1 + r1[1]; ++i[1])
                        for (i[0] = 2 * K[0] + 1 - 1; i[0] <= 2 * K[0] + 1 + 1; ++i[0]) {
                            const int fi[3] = {i[0], dim > 1 ? i[1] : 0, dim > 2 ? i[2] : 0};
                            bool in = true;
                            double r = rs;
                            for (int a = 0; a < dim; ++a) {
                                in = in && fi[a] >= 0 && fi[a] < F.nu[a];
                                r *= lin_w(fi[a], K[a]);
                            }
                            if (!in || r == 0.0) continue;
                            for (o[2] = -r1[2]; o[2] <= r1[2]; ++o[2])
                                for (o[1] = -r1[1]; o[1] <= r1[1]; ++o[1])
                                    for (o[0] = -1; o[0] <= 1; ++o[0]) {
                                        const cd aij = op_entry(F, dim, shift, fi, o);
                                        if (aij == cd(0.0)) continue;
                                        for (int a = 0; a < 3; ++a) ip[a] = fi[a] + o[a];
                                        for (jj[2] = -r1[2]; jj[2] <= r1[2]; ++jj[2])
                                            for (jj[1] = -r1[1]; jj[1] <= r1[1]; ++jj[1])
                                                for (jj[0] = -1; jj[0] <= 1; ++jj[0]) {
                                                    double w = 1.0;
                                                    int oi = 0, m = 1;
                                                    for (int a = 0; a < dim; ++a, m *= 3) {
                                                        const int J = K[a] + jj[a];
                                                        w *= (J >= 0 && J < C.nu[a]) ? lin_w(ip[a], J) : 0.0;
                                                        oi += (jj[a] + 1) * m;
                                                    }
                                                    if (w != 0.0) C.gst[(size_t)oi * C.N + pk] += r * aij * w;
                                                }
                                    }
                        }
            }
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
    if (p.coarse_op == 1)
        for (int l = 1; l < L; ++l) galerkin_level(hh.lev[l - 1], hh.lev[l], p.dim, phi_shift(p));
    {
        // polynomial smoothers; k^2 of the vertex t0: given, else the mean of phi
        double k2 = p.poly_k2;
        if (k2 == 0.0) {
            const HostLevel &F0 = hh.lev[0];
            double acc = 0.0;
            for (long q = 0; q < F0.N; ++q) acc += F0.phi[q];
            k2 = acc / (double)F0.N;
        }
        for (int l = 0; l < L; ++l) poly_level(p.dim, p.beta, p.gamma, k2, std::ldexp(p.h, l), hh.lev[l]);
    }
    // dense coarsest matrix, assembled row by row from the tables
    const HostLevel &C = hh.lev[L - 1];
    const cd shift = phi_shift(p);
    const int n = (int)C.N;
    hh.nc = n;
    std::vector<cd> A((size_t)n * n, cd(0.0));
    const int nx = C.nu[0], ny = C.nu[1], nz = C.nu[2];
    if (!C.gst.empty()) {
        // Galerkin: row r from the stored stencil
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    const int ii[3] = {i, j, k};
                    const long r = i + (long)nx * (j + (long)ny * k);
                    int o[3];
                    for (o[2] = p.dim > 2 ? -1 : 0; o[2] <= (p.dim > 2 ? 1 : 0); ++o[2])
                        for (o[1] = -1; o[1] <= 1; ++o[1])
                            for (o[0] = -1; o[0] <= 1; ++o[0]) {
                                const cd v = op_entry(C, p.dim, shift, ii, o);
                                if (v != cd(0.0)) A[r * n + r + o[0] + (long)nx * (o[1] + (long)ny * o[2])] += v;
                            }
                }
    }
    for (int k = 0; k < nz && C.gst.empty(); ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const long r = i + (long)nx * (j + (long)ny * k);
                cd diag = C.tab[0][nx + i] - shift * C.phi[r];
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
