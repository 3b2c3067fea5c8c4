/*
 * csg_oracle.c -- plain FP64 CPU oracle (test infrastructure; see csg_oracle.h).
 *
 * Each function states the passage of the paper it follows.  Nothing here is
 * blocked, fused or reordered beyond what the definition needs; OpenMP only
 * splits independent per-point loops, and inner products are summed in fixed
 * 4096-element chunks in chunk order so results do not depend on thread count.
 */
#include "csg_oracle.h"

#include <float.h>
#include <math.h>
#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define CHUNK 4096L

typedef double complex cplx;

typedef struct ora_level {
    int nint[3];   /* intervals per axis */
    int nu[3];     /* unknowns per axis = nint - 1 (1 for unused axes) */
    long N;        /* unknowns */
    cplx *zM[3];   /* node coordinates of the CSG grid (theta = beta) */
    cplx *swM[3];  /* Shortley-Weller coefficients of M: west | centre | east */
    double *phi;   /* injected phi */
    cplx *gal;     /* Galerkin levels: 3^d-point stencil, [offset][unknown] */
} ora_level;

struct ora_hier {
    ora_params p;
    int L;
    ora_level lev[ORA_MAXL];
    cplx *zH[3];   /* node coordinates of the ECS grid (theta = 0), finest level */
    cplx *swH[3];  /* Shortley-Weller coefficients of H on the finest level */
    int nc;        /* coarsest unknowns */
    cplx *lu;      /* LU factors of the dense coarsest M, row-major nc x nc */
    int *piv;      /* row permutation of the partial pivoting */
};

/* ---------------------------------------------------------------------------
 * Vector helpers
 * ------------------------------------------------------------------------- */

cplx ora_dot(long n, const cplx *x, const cplx *y)
{
    long nchunks = (n + CHUNK - 1) / CHUNK;
    if (nchunks == 0) return 0.0;
    cplx *part = (cplx *)malloc(sizeof(cplx) * (size_t)nchunks);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < nchunks; ++c) {
        long lo = c * CHUNK, hi = lo + CHUNK < n ? lo + CHUNK : n;
        cplx acc = 0.0;
        for (long i = lo; i < hi; ++i) acc += conj(x[i]) * y[i];
        part[c] = acc;
    }
    cplx s = 0.0;
    for (long c = 0; c < nchunks; ++c) s += part[c];
    free(part);
    return s;
}

int ora_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static double nrm2(long n, const cplx *x) { return sqrt(creal(ora_dot(n, x, x))); }

/* y += a x */
static void axpy(long n, cplx a, const cplx *x, cplx *y)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) y[i] += a * x[i];
}

static cplx *cvec(long n) { return (cplx *)calloc((size_t)(n > 0 ? n : 1), sizeof(cplx)); }

/* ---------------------------------------------------------------------------
 * Grid and discretisation (section 2, eq. csggrid; Shortley-Weller scheme)
 * ------------------------------------------------------------------------- */

/* Finest-level node coordinates of one axis: layer_lo intervals of h e^{i gamma},
 * n intervals of h e^{i theta}, layer_hi intervals of h e^{i gamma}; z_0 = 0. */
static void axis_nodes_fine(const ora_params *p, int a, double theta, cplx *z)
{
    int mlo = p->layer_lo[a], n = p->n[a], mhi = p->layer_hi[a];
    cplx hg = p->h * cexp(I * p->gamma);
    cplx hb = p->h * cexp(I * theta);
    z[0] = 0.0;
    int j = 0;
    for (int k = 0; k < mlo; ++k, ++j) z[j + 1] = z[j] + hg;
    for (int k = 0; k < n; ++k, ++j) z[j + 1] = z[j] + hb;
    for (int k = 0; k < mhi; ++k, ++j) z[j + 1] = z[j] + hg;
}

/* Nested coarse nodes: coarse node J is fine node 2J for J < Nc, and the last
 * coarse node is the last fine node (ceil-halving of the interval count). */
static void axis_nodes_coarsen(int nf, const cplx *zf, int nc, cplx *zc)
{
    for (int J = 0; J < nc; ++J) zc[J] = zf[2 * J];
    zc[nc] = zf[nf];
}

/* Shortley-Weller 3-point formula for -u'' on a non-uniform (complex) grid:
 * with h- = z_j - z_{j-1}, h+ = z_{j+1} - z_j,
 *   -u''(z_j) ~ -2/(h-(h- + h+)) u_{j-1} + 2/(h- h+) u_j - 2/(h+(h- + h+)) u_{j+1}. */
static void axis_sw(int nint, const cplx *z, cplx *sw)
{
    int nu = nint - 1;
    for (int j = 1; j <= nu; ++j) {
        cplx hm = z[j] - z[j - 1], hp = z[j + 1] - z[j];
        sw[j - 1] = -2.0 / (hm * (hm + hp));
        sw[nu + j - 1] = 2.0 / (hm * hp);
        sw[2 * nu + j - 1] = -2.0 / (hp * (hm + hp));
    }
}

/* d-dimensional operator as a Kronecker sum of the 1-D operators, minus s phi
 * (eq. csg_dis with the sign of eq. helm and Lemma 2.1; s = 1 but for the
 * shifted preconditioner):
 *   (A u)_p = sum_a (w_a u_{p-e_a} + e_a u_{p+e_a}) + (sum_a c_a - s phi_p) u_p,
 * with values beyond the unknown range equal to zero (Dirichlet). */
static void apply_tables(const ora_level *lv, cplx *const sw[3], cplx s, const cplx *x, cplx *y)
{
    const int n0 = lv->nu[0], n1 = lv->nu[1], n2 = lv->nu[2];
    const long s1 = n0, s2 = (long)n0 * n1;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n2; ++k) {
        for (int j = 0; j < n1; ++j) {
            for (int i = 0; i < n0; ++i) {
                long p = i + s1 * j + s2 * k;
                cplx diag = -s * lv->phi[p];
                cplx acc = 0.0;
                /* axis 0 */
                diag += sw[0][n0 + i];
                if (i > 0) acc += sw[0][i] * x[p - 1];
                if (i < n0 - 1) acc += sw[0][2 * n0 + i] * x[p + 1];
                if (sw[1]) {
                    diag += sw[1][n1 + j];
                    if (j > 0) acc += sw[1][j] * x[p - s1];
                    if (j < n1 - 1) acc += sw[1][2 * n1 + j] * x[p + s1];
                }
                if (sw[2]) {
                    diag += sw[2][n2 + k];
                    if (k > 0) acc += sw[2][k] * x[p - s2];
                    if (k < n2 - 1) acc += sw[2][2 * n2 + k] * x[p + s2];
                }
                y[p] = acc + diag * x[p];
            }
        }
    }
}

/* the factor s of phi in M */
static cplx shift_of(const ora_params *p)
{
    if (p->shift_re == 0.0 && p->shift_im == 0.0) return 1.0;
    return p->shift_re + I * p->shift_im;
}

/* offsets of a 3^d-point stencil: index sum_a (o_a + 1) 3^a over the used axes */
static int stencil_points(int d)
{
    return d == 1 ? 3 : d == 2 ? 9 : 27;
}

/* y = A x for a stored 3^d-point stencil (Galerkin levels) */
static void apply_stencil(const ora_level *lv, int d, const cplx *st, const cplx *x, cplx *y)
{
    const int n0 = lv->nu[0], n1 = lv->nu[1], n2 = lv->nu[2];
    const long N = lv->N;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n2; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n0; ++i) {
                const long p = i + (long)n0 * (j + (long)n1 * k);
                cplx acc = 0.0;
                for (int o2 = (d > 2 ? -1 : 0); o2 <= (d > 2 ? 1 : 0); ++o2)
                    for (int o1 = (d > 1 ? -1 : 0); o1 <= (d > 1 ? 1 : 0); ++o1)
                        for (int o0 = -1; o0 <= 1; ++o0) {
                            const long kk = k + o2;
                            const int jj = j + o1, ii = i + o0;
                            if (ii < 0 || ii >= n0 || jj < 0 || jj >= n1 || kk < 0 || kk >= n2) continue;
                            const int oi = (o0 + 1) + 3 * (o1 + 1) * (d > 1) + 9 * (o2 + 1) * (d > 2);
                            acc += st[oi * N + p] * x[ii + (long)n0 * (jj + (long)n1 * kk)];
                        }
                y[p] = acc;
            }
}

static void applyM(const ora_hier *hh, int l, const cplx *x, cplx *y)
{
    const ora_level *lv = &hh->lev[l];
    if (lv->gal) apply_stencil(lv, hh->p.dim, lv->gal, x, y);
    else apply_tables(lv, (cplx *const *)lv->swM, shift_of(&hh->p), x, y);
}

/* ---------------------------------------------------------------------------
 * Inter-grid transfers (standard multigrid components, section 3)
 * ------------------------------------------------------------------------- */

/* 1-D linear interpolation weight of coarse unknown J (0-based, node J+1) at
 * fine unknown i (0-based, node i+1): fine node i+1 even -> coarse node
 * (i+1)/2 with weight 1; odd -> coarse nodes (i)/2 and (i+2)/2 with 1/2. */
static double pw(int i, int J)
{
    int f = i + 1, c = J + 1;
    if (f % 2 == 0) return (f / 2 == c) ? 1.0 : 0.0;
    return (c == (f - 1) / 2 || c == (f + 1) / 2) ? 0.5 : 0.0;
}

/* x_f += P e_c, tensor-product linear interpolation, coarse Dirichlet nodes 0 */
int ora_prolong_add(const ora_hier *hh, int l, const cplx *ec, cplx *x)
{
    if (!hh || l < 0 || l >= hh->L - 1) return -1;
    const ora_level *F = &hh->lev[l], *C = &hh->lev[l + 1];
    const int d = hh->p.dim;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < F->nu[2]; ++k) {
        for (int j = 0; j < F->nu[1]; ++j) {
            for (int i = 0; i < F->nu[0]; ++i) {
                /* coarse candidates per axis: floor((f-1)/2) .. ceil((f+1)/2) */
                int lo[3], hi[3], fi[3] = {i, j, (int)k};
                for (int a = 0; a < 3; ++a) {
                    if (a >= d) { lo[a] = hi[a] = 0; continue; }
                    int f = fi[a] + 1;
                    lo[a] = (f - 1) / 2 - 1;  /* 0-based coarse unknown of node (f-1)/2 */
                    hi[a] = (f + 1) / 2 - 1;
                    if (lo[a] < 0) lo[a] = 0;
                    if (hi[a] > C->nu[a] - 1) hi[a] = C->nu[a] - 1;
                }
                cplx acc = 0.0;
                for (int K = lo[2]; K <= hi[2]; ++K)
                    for (int J = lo[1]; J <= hi[1]; ++J)
                        for (int Ii = lo[0]; Ii <= hi[0]; ++Ii) {
                            double w = pw(i, Ii);
                            if (d > 1) w *= pw(j, J);
                            if (d > 2) w *= pw((int)k, K);
                            if (w != 0.0)
                                acc += w * ec[Ii + (long)C->nu[0] * (J + (long)C->nu[1] * K)];
                        }
                x[i + (long)F->nu[0] * (j + (long)F->nu[1] * k)] += acc;
            }
        }
    }
    return 0;
}

/* b_c = R r with R = 2^{-d} P^T (full weighting: 1/4, 1/2, 1/4 per axis) */
int ora_restrict(const ora_hier *hh, int l, const cplx *r, cplx *bc)
{
    if (!hh || l < 0 || l >= hh->L - 1) return -1;
    const ora_level *F = &hh->lev[l], *C = &hh->lev[l + 1];
    const int d = hh->p.dim;
    const double scale = ldexp(1.0, -d);
#pragma omp parallel for schedule(static)
    for (long K = 0; K < C->nu[2]; ++K) {
        for (int J = 0; J < C->nu[1]; ++J) {
            for (int Ii = 0; Ii < C->nu[0]; ++Ii) {
                int cJ[3] = {Ii, J, (int)K};
                int lo[3], hi[3];
                for (int a = 0; a < 3; ++a) {
                    if (a >= d) { lo[a] = hi[a] = 0; continue; }
                    int c = cJ[a] + 1;           /* coarse node */
                    lo[a] = 2 * c - 1 - 1;       /* fine unknown of node 2c-1 */
                    hi[a] = 2 * c + 1 - 1;
                    if (lo[a] < 0) lo[a] = 0;
                    if (hi[a] > F->nu[a] - 1) hi[a] = F->nu[a] - 1;
                }
                cplx acc = 0.0;
                for (int k = lo[2]; k <= hi[2]; ++k)
                    for (int j = lo[1]; j <= hi[1]; ++j)
                        for (int i = lo[0]; i <= hi[0]; ++i) {
                            double w = pw(i, Ii);
                            if (d > 1) w *= pw(j, J);
                            if (d > 2) w *= pw(k, (int)K);
                            if (w != 0.0)
                                acc += w * r[i + (long)F->nu[0] * (j + (long)F->nu[1] * k)];
                        }
                bc[Ii + (long)C->nu[0] * (J + (long)C->nu[1] * K)] = scale * acc;
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Coarsest level: dense matrix, Gaussian elimination with partial pivoting
 * ------------------------------------------------------------------------- */

static int coarse_factor(ora_hier *hh)
{
    const ora_level *C = &hh->lev[hh->L - 1];
    int n = (int)C->N;
    hh->nc = n;
    hh->lu = cvec((long)n * n);
    hh->piv = (int *)calloc((size_t)n, sizeof(int));
    cplx *e = cvec(n), *col = cvec(n);
    /* assemble column by column: column c = M e_c */
    for (int c = 0; c < n; ++c) {
        memset(e, 0, sizeof(cplx) * (size_t)n);
        e[c] = 1.0;
        applyM(hh, hh->L - 1, e, col);
        for (int r = 0; r < n; ++r) hh->lu[(long)r * n + c] = col[r];
    }
    free(e);
    free(col);
    cplx *A = hh->lu;
    for (int k = 0; k < n; ++k) {
        int pr = k;
        double best = cabs(A[(long)k * n + k]);
        for (int r = k + 1; r < n; ++r) {
            double v = cabs(A[(long)r * n + k]);
            if (v > best) { best = v; pr = r; }
        }
        if (best == 0.0) return -5;
        hh->piv[k] = pr;
        if (pr != k)
            for (int c = 0; c < n; ++c) {
                cplx t = A[(long)k * n + c];
                A[(long)k * n + c] = A[(long)pr * n + c];
                A[(long)pr * n + c] = t;
            }
        for (int r = k + 1; r < n; ++r) {
            cplx f = A[(long)r * n + k] / A[(long)k * n + k];
            A[(long)r * n + k] = f;
            for (int c = k + 1; c < n; ++c) A[(long)r * n + c] -= f * A[(long)k * n + c];
        }
    }
    return 0;
}

int ora_coarse_solve(const ora_hier *hh, const cplx *b, cplx *x)
{
    if (!hh) return -1;
    int n = hh->nc;
    const cplx *A = hh->lu;
    cplx *y = cvec(n);
    memcpy(y, b, sizeof(cplx) * (size_t)n);
    for (int k = 0; k < n; ++k) {
        int pr = hh->piv[k];
        if (pr != k) { cplx t = y[k]; y[k] = y[pr]; y[pr] = t; }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < r; ++c) y[r] -= A[(long)r * n + c] * y[c];
    for (int r = n - 1; r >= 0; --r) {
        for (int c = r + 1; c < n; ++c) y[r] -= A[(long)r * n + c] * y[c];
        y[r] /= A[(long)r * n + r];
    }
    memcpy(x, y, sizeof(cplx) * (size_t)n);
    free(y);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Hierarchy (section 3: coarse operators by rediscretisation on the coarser
 * complex grid; phi injected)
 * ------------------------------------------------------------------------- */

/* Galerkin coarse operator of level l from level l - 1 (its Kronecker-sum
 * tables or its own stencil): M_l = R M_{l-1} P.  Column J of M_l has its
 * nonzeros at |K_a - J_a| <= 1 (P e_J spans fine unknowns 2J .. 2J+2 per axis,
 * M_{l-1} widens that by one, R reaches back to coarse unknowns within one),
 * so the columns whose indices agree mod 3 on every axis have disjoint
 * supports: each of the 3^d colour classes is applied at once,
 * y = R M_{l-1} P (sum of e_J over the class), and entry (K, K + o) is y_K for
 * the class of K + o. */
static void galerkin_level(ora_hier *hh, int l)
{
    ora_level *C = &hh->lev[l];
    const ora_level *F = &hh->lev[l - 1];
    const int d = hh->p.dim, np = stencil_points(d);
    const long N = C->N;
    C->gal = cvec(np * N);
    cplx *xc = cvec(N), *y = cvec(N), *f = cvec(F->N), *g = cvec(F->N);
    for (int col = 0; col < np; ++col) {
        const int c0 = col % 3, c1 = (col / 3) % 3, c2 = col / 9;
        for (long K = 0; K < C->nu[2]; ++K)
            for (int J = 0; J < C->nu[1]; ++J)
                for (int Ii = 0; Ii < C->nu[0]; ++Ii) {
                    const int on = Ii % 3 == c0 && (d < 2 || J % 3 == c1) && (d < 3 || K % 3 == c2);
                    xc[Ii + (long)C->nu[0] * (J + (long)C->nu[1] * K)] = on ? 1.0 : 0.0;
                }
        memset(f, 0, sizeof(cplx) * (size_t)F->N);
        ora_prolong_add(hh, l - 1, xc, f);
        applyM(hh, l - 1, f, g);
        ora_restrict(hh, l - 1, g, y);
        for (long K = 0; K < C->nu[2]; ++K)
            for (int J = 0; J < C->nu[1]; ++J)
                for (int Ii = 0; Ii < C->nu[0]; ++Ii) {
                    const long p = Ii + (long)C->nu[0] * (J + (long)C->nu[1] * K);
                    for (int o2 = (d > 2 ? -1 : 0); o2 <= (d > 2 ? 1 : 0); ++o2)
                        for (int o1 = (d > 1 ? -1 : 0); o1 <= (d > 1 ? 1 : 0); ++o1)
                            for (int o0 = -1; o0 <= 1; ++o0) {
                                const long kk = K + o2;
                                const int jj = J + o1, ii = Ii + o0;
                                if (ii < 0 || ii >= C->nu[0] || jj < 0 || jj >= C->nu[1] || kk < 0 ||
                                    kk >= C->nu[2])
                                    continue;
                                const int in = ii % 3 == c0 && (d < 2 || jj % 3 == c1) && (d < 3 || kk % 3 == c2);
                                if (!in) continue;
                                const int oi = (o0 + 1) + 3 * (o1 + 1) * (d > 1) + 9 * (o2 + 1) * (d > 2);
                                C->gal[oi * N + p] = y[p];
                            }
                }
    }
    free(xc);
    free(y);
    free(f);
    free(g);
}

int ora_galerkin_stencil(const ora_hier *hh, int l, cplx *out)
{
    if (!hh || l < 0 || l >= hh->L || !hh->lev[l].gal) return -1;
    memcpy(out, hh->lev[l].gal, sizeof(cplx) * (size_t)stencil_points(hh->p.dim) * (size_t)hh->lev[l].N);
    return 0;
}

static int validate(const ora_params *p)
{
    if (p->dim < 1 || p->dim > 3) return -1;
    if (!(p->h > 0.0) || !isfinite(p->h)) return -1;
    if (!(p->gamma > 0.0 && p->gamma < atan(1.0))) return -1; /* gamma < pi/4 */
    if (!(p->beta >= 0.0 && p->beta < p->gamma)) return -1;
    if (p->s < 1 || p->nu1 < 0 || p->nu2 < 0 || p->levels < 0 || p->levels > ORA_MAXL) return -1;
    if (p->smoother < 0 || p->smoother > 1 || !(p->poly_k2 >= 0.0) || !isfinite(p->poly_k2)) return -1;
    if (!isfinite(p->shift_re) || !isfinite(p->shift_im) || p->coarse_op < 0 || p->coarse_op > 1) return -1;
    /* the polynomial smoother's triangle is that of the rediscretised CSG operator */
    if (p->smoother == 1 && (p->coarse_op != 0 || shift_of(p) != 1.0)) return -1;
    for (int a = 0; a < p->dim; ++a) {
        if (p->n[a] < 1 || p->layer_lo[a] < 0 || p->layer_hi[a] < 0) return -1;
        if (p->n[a] + p->layer_lo[a] + p->layer_hi[a] < 2) return -1;
    }
    return 0;
}

ora_hier *ora_build(const ora_params *p, const double *phi, int *status)
{
    int st = validate(p);
    if (st) { if (status) *status = st; return NULL; }
    ora_hier *hh = (ora_hier *)calloc(1, sizeof(ora_hier));
    hh->p = *p;
    const int d = p->dim;
    int nint[3] = {2, 2, 2};
    for (int a = 0; a < d; ++a) nint[a] = p->n[a] + p->layer_lo[a] + p->layer_hi[a];

    /* level count: requested, or coarsen until every axis has <= 9 intervals */
    int L = 1;
    {
        int cur[3] = {nint[0], nint[1], nint[2]};
        for (;;) {
            if (p->levels > 0) { if (L >= p->levels) break; }
            else {
                int big = 0;
                for (int a = 0; a < d; ++a) if (cur[a] > 9) big = 1;
                if (!big || L >= ORA_MAXL) break;
            }
            for (int a = 0; a < d; ++a) cur[a] = (cur[a] + 1) / 2;
            for (int a = 0; a < d; ++a) if (cur[a] < 2) { free(hh); if (status) *status = -1; return NULL; }
            ++L;
        }
    }
    hh->L = L;

    for (int l = 0; l < L; ++l) {
        ora_level *lv = &hh->lev[l];
        lv->N = 1;
        for (int a = 0; a < 3; ++a) {
            if (a < d) {
                lv->nint[a] = (l == 0) ? nint[a] : (hh->lev[l - 1].nint[a] + 1) / 2;
                lv->nu[a] = lv->nint[a] - 1;
            } else {
                lv->nint[a] = 0;
                lv->nu[a] = 1;
            }
            lv->N *= lv->nu[a];
        }
        for (int a = 0; a < d; ++a) {
            lv->zM[a] = cvec(lv->nint[a] + 1);
            if (l == 0) axis_nodes_fine(p, a, p->beta, lv->zM[a]);
            else axis_nodes_coarsen(hh->lev[l - 1].nint[a], hh->lev[l - 1].zM[a], lv->nint[a], lv->zM[a]);
            lv->swM[a] = cvec(3L * lv->nu[a]);
            axis_sw(lv->nint[a], lv->zM[a], lv->swM[a]);
        }
        lv->phi = (double *)calloc((size_t)lv->N, sizeof(double));
        if (l == 0) {
            memcpy(lv->phi, phi, sizeof(double) * (size_t)lv->N);
        } else {
            /* injection: coarse unknown J (node J+1) takes fine node 2(J+1), i.e.
             * fine unknown 2J+1 */
            const ora_level *F = &hh->lev[l - 1];
            for (long K = 0; K < lv->nu[2]; ++K)
                for (int J = 0; J < lv->nu[1]; ++J)
                    for (int Ii = 0; Ii < lv->nu[0]; ++Ii) {
                        long fi = 2L * Ii + 1, fj = d > 1 ? 2L * J + 1 : 0, fk = d > 2 ? 2L * K + 1 : 0;
                        lv->phi[Ii + (long)lv->nu[0] * (J + (long)lv->nu[1] * K)] =
                            F->phi[fi + (long)F->nu[0] * (fj + (long)F->nu[1] * fk)];
                    }
        }
    }
    for (int a = 0; a < d; ++a) {
        hh->zH[a] = cvec(nint[a] + 1);
        axis_nodes_fine(p, a, 0.0, hh->zH[a]);
        hh->swH[a] = cvec(3L * (nint[a] - 1));
        axis_sw(nint[a], hh->zH[a], hh->swH[a]);
    }
    if (p->coarse_op == 1)
        for (int l = 1; l < L; ++l) galerkin_level(hh, l);
    st = coarse_factor(hh);
    if (st) { ora_free(hh); if (status) *status = st; return NULL; }
    if (status) *status = 0;
    return hh;
}

void ora_free(ora_hier *hh)
{
    if (!hh) return;
    for (int l = 0; l < hh->L; ++l) {
        for (int a = 0; a < 3; ++a) { free(hh->lev[l].zM[a]); free(hh->lev[l].swM[a]); }
        free(hh->lev[l].phi);
        free(hh->lev[l].gal);
    }
    for (int a = 0; a < 3; ++a) { free(hh->zH[a]); free(hh->swH[a]); }
    free(hh->lu);
    free(hh->piv);
    free(hh);
}

int ora_levels(const ora_hier *hh) { return hh ? hh->L : -1; }

void ora_level_dims(const ora_hier *hh, int l, int dims[3])
{
    for (int a = 0; a < 3; ++a) dims[a] = (hh && l >= 0 && l < hh->L) ? hh->lev[l].nu[a] : 0;
}

int ora_axis_nodes(const ora_hier *hh, int which, int l, int a, cplx *out)
{
    if (!hh || l < 0 || l >= hh->L || a < 0 || a >= hh->p.dim) return -1;
    if (which == 0 && l != 0) return -1;
    const cplx *z = which == 0 ? hh->zH[a] : hh->lev[l].zM[a];
    memcpy(out, z, sizeof(cplx) * (size_t)(hh->lev[l].nint[a] + 1));
    return 0;
}

int ora_axis_sw(const ora_hier *hh, int which, int l, int a, cplx *out)
{
    if (!hh || l < 0 || l >= hh->L || a < 0 || a >= hh->p.dim) return -1;
    if (which == 0 && l != 0) return -1;
    const cplx *sw = which == 0 ? hh->swH[a] : hh->lev[l].swM[a];
    memcpy(out, sw, sizeof(cplx) * 3 * (size_t)hh->lev[l].nu[a]);
    return 0;
}

int ora_level_phi(const ora_hier *hh, int l, double *out)
{
    if (!hh || l < 0 || l >= hh->L) return -1;
    memcpy(out, hh->lev[l].phi, sizeof(double) * (size_t)hh->lev[l].N);
    return 0;
}

int ora_apply(const ora_hier *hh, int which, int l, const cplx *x, cplx *y)
{
    if (!hh || l < 0 || l >= hh->L) return -1;
    if (which == 0) {
        if (l != 0) return -1;
        apply_tables(&hh->lev[0], (cplx *const *)hh->swH, 1.0, x, y);
        return 0;
    }
    if (which != 1) return -1;
    applyM(hh, l, x, y);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Small dense helpers: complex Givens rotation and back substitution
 * ------------------------------------------------------------------------- */

/* Rotation [c s; -conj(s) c] with real c mapping (a, b) to (r, 0). */
static void givens(cplx a, cplx b, double *c, cplx *s)
{
    double aa = cabs(a), bb = cabs(b);
    if (bb == 0.0) { *c = 1.0; *s = 0.0; return; }
    if (aa == 0.0) { *c = 0.0; *s = conj(b) / bb; return; }
    double nu = hypot(aa, bb);
    *c = aa / nu;
    *s = (a / aa) * conj(b) / nu;
}

/* Solve the k x k upper-triangular system R y = g, R stored with leading
 * dimension ld (R[i][j] = R[i*ld + j]). */
static void back_solve(int k, const cplx *R, int ld, const cplx *g, cplx *y)
{
    for (int i = k - 1; i >= 0; --i) {
        cplx acc = g[i];
        for (int j = i + 1; j < k; ++j) acc -= R[i * ld + j] * y[j];
        y[i] = acc / R[i * ld + i];
    }
}

/* ---------------------------------------------------------------------------
 * GMRES(s) smoothing sweep (section 3.1: a GMRES solve on the error stopped
 * after s iterations; minimal residual over the degree-s Krylov polynomials,
 * section 4).  Textbook Arnoldi with modified Gram-Schmidt and Givens.
 * ------------------------------------------------------------------------- */

int ora_gmres_sweep(const ora_hier *hh, int l, int s, const cplx *b, cplx *x, int x_is_zero)
{
    if (!hh || l < 0 || l >= hh->L || s < 1) return -1;
    const long N = hh->lev[l].N;
    cplx **V = (cplx **)calloc((size_t)s + 1, sizeof(cplx *));
    for (int i = 0; i <= s; ++i) V[i] = cvec(N);
    cplx *w = cvec(N);
    cplx *Hm = (cplx *)calloc((size_t)(s + 1) * s, sizeof(cplx)); /* (s+1) x s, row-major ld s */
    cplx *g = (cplx *)calloc((size_t)s + 1, sizeof(cplx));
    double *cs = (double *)calloc((size_t)s, sizeof(double));
    cplx *sn = (cplx *)calloc((size_t)s, sizeof(cplx));
    cplx *y = (cplx *)calloc((size_t)s, sizeof(cplx));

    /* r = b - A x */
    if (x_is_zero) {
        memcpy(V[0], b, sizeof(cplx) * (size_t)N);
    } else {
        applyM(hh, l, x, w);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i) V[0][i] = b[i] - w[i];
    }
    double beta0 = nrm2(N, V[0]);
    int k = 0;
    if (beta0 > 0.0) {
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i) V[0][i] /= beta0;
        g[0] = beta0;
        const double tiny = 10.0 * DBL_EPSILON * beta0;
        for (int j = 0; j < s; ++j) {
            applyM(hh, l, V[j], w);
            for (int i = 0; i <= j; ++i) {
                cplx hij = ora_dot(N, V[i], w);
                Hm[i * s + j] = hij;
                axpy(N, -hij, V[i], w);
            }
            double hn = nrm2(N, w);
            Hm[(j + 1) * s + j] = hn;
            for (int i = 0; i < j; ++i) {
                cplx t1 = Hm[i * s + j], t2 = Hm[(i + 1) * s + j];
                Hm[i * s + j] = cs[i] * t1 + sn[i] * t2;
                Hm[(i + 1) * s + j] = -conj(sn[i]) * t1 + cs[i] * t2;
            }
            givens(Hm[j * s + j], Hm[(j + 1) * s + j], &cs[j], &sn[j]);
            {
                cplx t1 = Hm[j * s + j], t2 = Hm[(j + 1) * s + j];
                Hm[j * s + j] = cs[j] * t1 + sn[j] * t2;
                Hm[(j + 1) * s + j] = 0.0;
                g[j + 1] = -conj(sn[j]) * g[j];
                g[j] = cs[j] * g[j];
            }
            k = j + 1;
            if (hn <= tiny) break;
#pragma omp parallel for schedule(static)
            for (long i = 0; i < N; ++i) V[j + 1][i] = w[i] / hn;
        }
        back_solve(k, Hm, s, g, y);
        for (int i = 0; i < k; ++i) axpy(N, y[i], V[i], x);
    }
    for (int i = 0; i <= s; ++i) free(V[i]);
    free(V); free(w); free(Hm); free(g); free(cs); free(sn); free(y);
    return k;
}

/* ---------------------------------------------------------------------------
 * Third-order polynomial smoother (section 4)
 * ------------------------------------------------------------------------- */

/* Vertices of the bounding triangle of Prop. 3.1 for spacing H:
 * t0 = -k^2, t1 = -k^2 + 4d/(H e^{i beta})^2, t2 = -k^2 + 4d/(H e^{i gamma})^2. */
static void poly_triangle(double k2, double H, int dim, double beta, double gamma, cplx t[3])
{
    cplx hb = H * cexp(I * beta), hg = H * cexp(I * gamma);
    t[0] = -k2;
    t[1] = -k2 + 4.0 * dim / (hb * hb);
    t[2] = -k2 + 4.0 * dim / (hg * hg);
}

/* Solve the 3x3 system A x = b by Gaussian elimination with partial pivoting. */
static void solve3(cplx A[3][3], const cplx b[3], cplx x[3])
{
    cplx M[3][4];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) M[r][c] = A[r][c];
        M[r][3] = b[r];
    }
    for (int k = 0; k < 3; ++k) {
        int pr = k;
        for (int r = k + 1; r < 3; ++r) if (cabs(M[r][k]) > cabs(M[pr][k])) pr = r;
        for (int c = 0; c < 4; ++c) { cplx t = M[k][c]; M[k][c] = M[pr][c]; M[pr][c] = t; }
        for (int r = k + 1; r < 3; ++r) {
            cplx f = M[r][k] / M[k][k];
            for (int c = k; c < 4; ++c) M[r][c] -= f * M[k][c];
        }
    }
    for (int r = 2; r >= 0; --r) {
        cplx acc = M[r][3];
        for (int c = r + 1; c < 3; ++c) acc -= M[r][c] * x[c];
        x[r] = acc / M[r][r];
    }
}

/* e and f of eq. coefficients_solution: the system of eq. coefficients_system
 * (rows: p(0) = 1, p(t1) = 0, p(t2) = 0 written for c_1..c_3 around t0) solved
 * for the right-hand sides (1,0,0) and (1,1,1). */
static void poly_ef(const cplx t[3], cplx e[3], cplx f[3])
{
    cplx A[3][3];
    const cplx x[3] = {-t[0], t[1] - t[0], t[2] - t[0]};
    for (int r = 0; r < 3; ++r) {
        A[r][0] = x[r];
        A[r][1] = x[r] * x[r];
        A[r][2] = x[r] * x[r] * x[r];
    }
    const cplx b100[3] = {1.0, 0.0, 0.0}, b111[3] = {1.0, 1.0, 1.0};
    solve3(A, b100, e);
    solve3(A, b111, f);
}

/* First- and second-order coefficients of |p|^2 along the edge t0 + rho w,
 * w = e^{-2 i beta}, with c_0 = e^{i varphi}, c_j = e_j - e^{i varphi} f_j:
 * |p|^2 = 1 + 2 rho Re(conj(c0) c1 w) + rho^2 (|c1|^2 + 2 Re(conj(c0) c2 w^2)) + O(rho^3). */
static void poly_FS(const cplx e[3], const cplx f[3], double beta, double varphi, double *F, double *S)
{
    cplx w = cexp(-2.0 * I * beta), c0 = cexp(I * varphi);
    cplx c1 = e[0] - c0 * f[0], c2 = e[1] - c0 * f[1];
    *F = creal(conj(c0) * c1 * w);
    *S = cabs(c1) * cabs(c1) + 2.0 * creal(conj(c0) * c2 * w * w);
}

int ora_poly_conditions(double k2, double H, int dim, double beta, double gamma, double varphi, double *F,
                        double *S)
{
    if (!(H > 0.0) || dim < 1 || dim > 3 || !F || !S) return -1;
    cplx t[3], e[3], f[3];
    poly_triangle(k2, H, dim, beta, gamma, t);
    poly_ef(t, e, f);
    poly_FS(e, f, beta, varphi, F, S);
    return 0;
}

/* The set {varphi : |a| cos(varphi - arg a) < g} as an arc: centre and half
 * width in [0, pi]; *all / *none flag the whole circle / the empty set. */
static void arc_below(cplx a, double g, double *centre, double *half, int *all, int *none)
{
    double m = cabs(a);
    *all = *none = 0;
    *centre = carg(a) + M_PI;
    *half = 0.0;
    if (m <= g) { *all = 1; *half = M_PI; return; }      /* cos < g/|a| with g/|a| >= 1 */
    if (m <= -g) { *none = 1; return; }                  /* g/|a| <= -1 */
    *half = M_PI - acos(g / m);
}

int ora_poly_level(const ora_hier *hh, int l, ora_poly *out)
{
    if (!hh || l < 0 || l >= hh->L || !out) return -1;
    const ora_params *p = &hh->p;
    double k2 = p->poly_k2;
    if (k2 == 0.0) {
        /* reading: the mean of phi over the finest unknowns (the paper's k is constant) */
        const ora_level *F0 = &hh->lev[0];
        double acc = 0.0;
        for (long i = 0; i < F0->N; ++i) acc += F0->phi[i];
        k2 = acc / (double)F0->N;
    }
    out->k2 = k2;
    out->H = ldexp(p->h, l);
    poly_triangle(k2, out->H, p->dim, p->beta, p->gamma, out->t);
    poly_ef(out->t, out->e, out->f);
    const cplx *e = out->e, *f = out->f;
    /* F(varphi) = Re(e^{-i varphi} e1 w) - Re(f1 w) < 0 and
     * S(varphi) = K + Re(e^{-i varphi} Z) < 0, with w = e^{-2i beta},
     * K = |e1|^2 + |f1|^2 - 2 Re(f2 w^2), Z = 2 (e2 w^2 - e1 conj(f1)) */
    const cplx w = cexp(-2.0 * I * p->beta);
    double cA, rA, cB, rB;
    int allA, noneA, allB, noneB;
    arc_below(e[0] * w, creal(f[0] * w), &cA, &rA, &allA, &noneA);
    const double K = cabs(e[0]) * cabs(e[0]) + cabs(f[0]) * cabs(f[0]) - 2.0 * creal(f[1] * w * w);
    arc_below(2.0 * (e[1] * w * w - e[0] * conj(f[0])), -K, &cB, &rB, &allB, &noneB);
    double varphi = 0.0;
    int conds = 2;
    if (!noneA && !noneB) {
        if (allA && allB) { varphi = 0.0; conds = 0; }
        else if (allA) { varphi = cB; conds = 0; }
        else if (allB) { varphi = cA; conds = 0; }
        else {
            /* arc B around arc A's centre: offsets d - 2pi, d, d + 2pi; the
             * longest overlap's midpoint */
            double d = remainder(cB - cA, 2.0 * M_PI), best = 0.0, mid = 0.0;
            for (int q = -1; q <= 1; ++q) {
                double lo = fmax(-rA, d + 2.0 * M_PI * q - rB), hi = fmin(rA, d + 2.0 * M_PI * q + rB);
                if (hi - lo > best) { best = hi - lo; mid = 0.5 * (lo + hi); }
            }
            if (best > 0.0) { varphi = cA + mid; conds = 0; }
            else { varphi = cA; conds = 1; }
        }
    } else if (!noneA) {
        varphi = allA ? 0.0 : cA;
        conds = 1;
    }
    varphi = remainder(varphi, 2.0 * M_PI);
    if (varphi < 0.0) varphi += 2.0 * M_PI;
    out->varphi = varphi;
    out->conds = conds;
    const cplx c0 = cexp(I * varphi);
    out->c[0] = c0;
    for (int j = 0; j < 3; ++j) out->c[j + 1] = e[j] - c0 * f[j];
    /* roots: t1 and t2 by construction; the third from the leading coefficient
     * (p(t) = c3 (t - t1)(t - t2)(t - t3) and p(0) = 1) */
    out->omega[0] = 1.0 / out->t[1];
    out->omega[1] = 1.0 / out->t[2];
    out->omega[2] = -out->c[3] * out->t[1] * out->t[2];
    return 0;
}

int ora_poly_sweep(const ora_hier *hh, int l, const cplx *b, cplx *x, int x_is_zero)
{
    if (!hh || l < 0 || l >= hh->L) return -1;
    ora_poly pl;
    ora_poly_level(hh, l, &pl);
    const long N = hh->lev[l].N;
    cplx *r = cvec(N);
    for (int i = 0; i < 3; ++i) {
        /* x <- x + omega_i (b - M x): the error is multiplied by (1 - omega_i M) */
        if (x_is_zero && i == 0) {
            memcpy(r, b, sizeof(cplx) * (size_t)N);
        } else {
            applyM(hh, l, x, r);
#pragma omp parallel for schedule(static)
            for (long q = 0; q < N; ++q) r[q] = b[q] - r[q];
        }
        if (x_is_zero && i == 0) memset(x, 0, sizeof(cplx) * (size_t)N);
        axpy(N, pl.omega[i], r, x);
    }
    free(r);
    return 3;
}

/* ---------------------------------------------------------------------------
 * V(nu1, nu2)-cycle (section 3.1): nu1 GMRES(s) pre-sweeps from a zero guess,
 * restriction of the residual, recursion, interpolated correction, nu2
 * post-sweeps; exact solve on the coarsest level.
 * ------------------------------------------------------------------------- */

int ora_vcycle_level(const ora_hier *hh, int l, const cplx *b, cplx *x)
{
    if (!hh || l < 0 || l >= hh->L) return -1;
    const long N = hh->lev[l].N;
    if (l == hh->L - 1) return ora_coarse_solve(hh, b, x);
    memset(x, 0, sizeof(cplx) * (size_t)N);
    int zero = 1;
    for (int k = 0; k < hh->p.nu1; ++k) {
        if (hh->p.smoother == 1) ora_poly_sweep(hh, l, b, x, zero);
        else ora_gmres_sweep(hh, l, hh->p.s, b, x, zero);
        zero = 0;
    }
    cplx *r = cvec(N);
    if (zero) {
        memcpy(r, b, sizeof(cplx) * (size_t)N);
    } else {
        applyM(hh, l, x, r);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i) r[i] = b[i] - r[i];
    }
    const long Nc = hh->lev[l + 1].N;
    cplx *bc = cvec(Nc), *ec = cvec(Nc);
    ora_restrict(hh, l, r, bc);
    ora_vcycle_level(hh, l + 1, bc, ec);
    ora_prolong_add(hh, l, ec, x);
    for (int k = 0; k < hh->p.nu2; ++k) {
        if (hh->p.smoother == 1) ora_poly_sweep(hh, l, b, x, 0);
        else ora_gmres_sweep(hh, l, hh->p.s, b, x, 0);
    }
    free(r); free(bc); free(ec);
    return 0;
}

int ora_vcycle(const ora_hier *hh, const cplx *b, cplx *x) { return ora_vcycle_level(hh, 0, b, x); }

/* ---------------------------------------------------------------------------
 * Flexible GMRES(m) (section 5, the outer Krylov method; right preconditioning
 * because the GMRES-smoothed cycle changes from step to step).
 * ------------------------------------------------------------------------- */

int ora_fgmres(const ora_hier *hh, const cplx *chi, cplx *u, double tol, int m, int maxit,
               int use_x0, ora_info *info, double *hist, int hist_len)
{
    if (!hh || m < 1 || maxit < 0) return -1;
    const long N = hh->lev[0].N;
    ora_info inf;
    memset(&inf, 0, sizeof(inf));
    const double nchi = nrm2(N, chi);
    if (!use_x0) memset(u, 0, sizeof(cplx) * (size_t)N);
    if (nchi == 0.0) {
        memset(u, 0, sizeof(cplx) * (size_t)N);
        inf.converged = 1;
        if (info) *info = inf;
        return 0;
    }
    cplx **V = (cplx **)calloc((size_t)m + 1, sizeof(cplx *));
    cplx **Z = (cplx **)calloc((size_t)m, sizeof(cplx *));
    for (int i = 0; i <= m; ++i) V[i] = cvec(N);
    for (int i = 0; i < m; ++i) Z[i] = cvec(N);
    cplx *w = cvec(N), *r = cvec(N);
    cplx *Hm = (cplx *)calloc((size_t)(m + 1) * m, sizeof(cplx));
    cplx *g = (cplx *)calloc((size_t)m + 1, sizeof(cplx));
    double *cs = (double *)calloc((size_t)m, sizeof(double));
    cplx *sn = (cplx *)calloc((size_t)m, sizeof(cplx));
    cplx *y = (cplx *)calloc((size_t)m, sizeof(cplx));

    int rc = 0;
    ora_apply(hh, 0, 0, u, w);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) r[i] = chi[i] - w[i];
    double beta = nrm2(N, r);
    inf.relres_est = beta / nchi;
    for (;;) {
        if (!isfinite(beta)) { rc = -5; break; }
        if (beta / nchi <= tol) break;
        if (inf.iterations >= maxit) break;
        memset(Hm, 0, sizeof(cplx) * (size_t)(m + 1) * m);
        memset(g, 0, sizeof(cplx) * (size_t)(m + 1));
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i) V[0][i] = r[i] / beta;
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            ora_vcycle(hh, V[j], Z[j]);
            inf.vcycles++;
            ora_apply(hh, 0, 0, Z[j], w);
            for (int i = 0; i <= j; ++i) {
                cplx hij = ora_dot(N, V[i], w);
                Hm[i * m + j] = hij;
                axpy(N, -hij, V[i], w);
            }
            double hn = nrm2(N, w);
            Hm[(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                cplx t1 = Hm[i * m + j], t2 = Hm[(i + 1) * m + j];
                Hm[i * m + j] = cs[i] * t1 + sn[i] * t2;
                Hm[(i + 1) * m + j] = -conj(sn[i]) * t1 + cs[i] * t2;
            }
            givens(Hm[j * m + j], Hm[(j + 1) * m + j], &cs[j], &sn[j]);
            {
                cplx t1 = Hm[j * m + j], t2 = Hm[(j + 1) * m + j];
                Hm[j * m + j] = cs[j] * t1 + sn[j] * t2;
                Hm[(j + 1) * m + j] = 0.0;
                g[j + 1] = -conj(sn[j]) * g[j];
                g[j] = cs[j] * g[j];
            }
            inf.iterations++;
            k = j + 1;
            double est = cabs(g[j + 1]) / nchi;
            inf.relres_est = est;
            if (hist && inf.iterations <= hist_len) hist[inf.iterations - 1] = est;
            if (!isfinite(est)) { rc = -5; break; }
            if (est <= tol || hn == 0.0 || inf.iterations >= maxit) break;
#pragma omp parallel for schedule(static)
            for (long i = 0; i < N; ++i) V[j + 1][i] = w[i] / hn;
        }
        if (rc) break;
        back_solve(k, Hm, m, g, y);
        for (int i = 0; i < k; ++i) axpy(N, y[i], Z[i], u);
        ora_apply(hh, 0, 0, u, w);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i) r[i] = chi[i] - w[i];
        beta = nrm2(N, r);
        inf.restarts++;
    }
    inf.relres_true = beta / nchi;
    inf.converged = (rc == 0 && beta / nchi <= tol);
    if (rc == 0 && !inf.converged) rc = 1;
    if (info) *info = inf;
    for (int i = 0; i <= m; ++i) free(V[i]);
    for (int i = 0; i < m; ++i) free(Z[i]);
    free(V); free(Z); free(w); free(r); free(Hm); free(g); free(cs); free(sn); free(y);
    return rc;
}
