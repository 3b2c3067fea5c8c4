/*
 * Drives the CPU oracle through every entry point on small problems, built
 * with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_host_sanitize.py: any out-of-bounds access, use after free,
 * leak or undefined operation ends the run with a non-zero status.
 */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "csg_oracle.h"

static double complex *cv(long n)
{
    double complex *v = (double complex *)calloc((size_t)(n > 0 ? n : 1), sizeof(double complex));
    for (long i = 0; i < n; ++i) v[i] = sin(0.37 * (double)i) + I * cos(0.11 * (double)i);
    return v;
}

static int run(const ora_params *p)
{
    long N = 1;
    int nu[3];
    for (int a = 0; a < 3; ++a) {
        nu[a] = a < p->dim ? p->n[a] + p->layer_lo[a] + p->layer_hi[a] - 1 : 1;
        N *= nu[a];
    }
    double *phi = (double *)malloc(sizeof(double) * (size_t)N);
    for (long i = 0; i < N; ++i) phi[i] = 150.0 * (1.0 + 0.2 * sin(0.05 * (double)i));
    int st = 0;
    ora_hier *hh = ora_build(p, phi, &st);
    if (!hh) { free(phi); return st == 0 ? 1 : 0; }   /* rejected parameters are fine */
    const int L = ora_levels(hh);
    for (int l = 0; l < L; ++l) {
        int d[3];
        ora_level_dims(hh, l, d);
        const long n = (long)d[0] * d[1] * d[2];
        double complex *x = cv(n), *y = cv(n), *b = cv(n);
        double *ph = (double *)malloc(sizeof(double) * (size_t)n);
        ora_level_phi(hh, l, ph);
        ora_apply(hh, 1, l, x, y);
        if (l == 0) ora_apply(hh, 0, 0, x, y);
        ora_gmres_sweep(hh, l, p->s, b, x, 0);
        ora_gmres_sweep(hh, l, p->s, b, y, 1);
        for (int a = 0; a < p->dim; ++a) {
            double complex *z = cv(3L * d[a] + 3);
            ora_axis_nodes(hh, 1, l, a, z);
            ora_axis_sw(hh, 1, l, a, z);
            free(z);
        }
        if (p->coarse_op == 1 && l > 0) {
            const int np = p->dim == 1 ? 3 : p->dim == 2 ? 9 : 27;
            double complex *g = cv((long)np * n);
            ora_galerkin_stencil(hh, l, g);
            free(g);
        }
        if (p->smoother == 1 && l + 1 < L) {
            ora_poly pl;
            ora_poly_level(hh, l, &pl);
            ora_poly_sweep(hh, l, b, x, 0);
        }
        if (l + 1 < L) {
            int dc[3];
            ora_level_dims(hh, l + 1, dc);
            const long nc = (long)dc[0] * dc[1] * dc[2];
            double complex *c = cv(nc);
            ora_restrict(hh, l, x, c);
            ora_prolong_add(hh, l, c, y);
            ora_vcycle_level(hh, l, b, x);
            free(c);
        } else {
            ora_coarse_solve(hh, b, x);
        }
        free(x); free(y); free(b); free(ph);
    }
    double complex *chi = cv(N), *u = cv(N);
    ora_info info;
    double hist[64];
    ora_fgmres(hh, chi, u, 1e-6, 8, 20, 0, &info, hist, 64);
    ora_fgmres(hh, chi, u, 1e-6, 8, 10, 1, &info, NULL, 0);
    (void)ora_dot(N, chi, u);
    free(chi); free(u);
    ora_free(hh);
    free(phi);
    return 0;
}

int main(void)
{
    int bad = 0;
    const double pi6 = 0.5235987755982988;
    ora_params base;
    memset(&base, 0, sizeof base);
    base.h = 1.0 / 16;
    base.gamma = pi6;
    base.beta = 0.35;
    base.s = 3;
    base.nu1 = base.nu2 = 1;
    for (int dim = 1; dim <= 3; ++dim)
        for (int var = 0; var < 6; ++var) {
            ora_params p = base;
            p.dim = dim;
            for (int a = 0; a < dim; ++a) {
                p.n[a] = dim == 3 ? 9 + a : 17 + 2 * a;
                p.layer_lo[a] = var == 5 ? 0 : 3;
                p.layer_hi[a] = 2 + a;
            }
            if (var == 1) p.smoother = 1;
            if (var == 2) { p.coarse_op = 1; p.shift_re = 1.0; p.shift_im = 0.5; }
            if (var == 3) { p.levels = 2; p.s = 4; p.nu1 = 2; p.nu2 = 0; }
            if (var == 4) { p.beta = 0.9; }   /* invalid: beta >= gamma */
            bad |= run(&p);
        }
    printf("oracle driver: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
