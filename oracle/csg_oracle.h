/*
 * csg_oracle.h -- FP64 CPU oracle for the GMRES-smoothed complex-stretched-grid
 * multigrid preconditioner and the outer flexible GMRES solve of the ECS
 * Helmholtz problem (Reps, Vanroose, bin Zubair, "GMRES-based multigrid for the
 * complex scaled preconditioner for the indefinite Helmholtz equation").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against the paper.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares no
 * source, header, table or helper with the GPU library.
 *
 * Conventions (all readings of the paper are listed in the design notes):
 *  - complex values are C99 `double complex` (interleaved re,im in memory);
 *  - unknowns of one grid are stored x fastest: idx = i0 + n0*(i1 + n1*i2);
 *  - L is the NEGATIVE discrete Laplacian; H = L(theta=0) - diag(phi) and
 *    M = L(theta=beta) - diag(phi)  (problem statement, eq. helm; Lemma 2.1);
 *  - interior spacing h*exp(i*theta), ECS layer spacing h*exp(i*gamma) on both
 *    sides of every axis (eq. csggrid and the remark on two-sided layers);
 *  - homogeneous Dirichlet at the far end of each layer.
 */
#ifndef CSG_ORACLE_H
#define CSG_ORACLE_H

#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORA_MAXL 16

typedef struct ora_params {
    int dim;            /* 1, 2 or 3 */
    int n[3];           /* interior intervals per axis */
    double h;           /* real mesh width of the interior */
    int layer_lo[3];    /* ECS layer intervals on the low side of each axis */
    int layer_hi[3];    /* ECS layer intervals on the high side of each axis */
    double gamma;       /* ECS rotation angle (radians) */
    double beta;        /* CSG rotation angle of the preconditioner interior (radians) */
    int levels;         /* multigrid levels; 0 = coarsen until <= 9 intervals per axis */
    int s;              /* GMRES(s) smoother length */
    int nu1, nu2;       /* pre- and post-smoothing sweeps */
    int smoother;       /* 0 = GMRES(s) (section 3.1), 1 = third-order polynomial (section 4) */
    double poly_k2;     /* k^2 of the polynomial's vertex t0 = -k^2; 0 = mean of phi on the finest level */
    /* complex factor s of phi in the preconditioner, M = L(theta = beta) - s phi
     * on every level (0 + 0i means s = 1, the CSG preconditioner).  beta = 0 and
     * s = 1 + i eps is the complex shifted Laplacian (section 1, section 2). */
    double shift_re, shift_im;
    /* coarse operators: 0 = rediscretisation on the coarser complex grid
     * (section 3), 1 = Galerkin products M_{l+1} = R M_l P (section 5 remark on
     * the bound states), stored as 3^d-point stencils */
    int coarse_op;
} ora_params;

typedef struct ora_info {
    int iterations;     /* preconditioner applications (outer FGMRES steps) */
    int restarts;       /* completed restart cycles */
    int vcycles;        /* V-cycles applied */
    int converged;      /* 1 if the true relative residual is <= tol */
    double relres_true; /* ||chi - H u|| / ||chi|| recomputed at exit */
    double relres_est;  /* last Arnoldi estimate |g_{j+1}| / ||chi|| */
} ora_info;

typedef struct ora_hier ora_hier;

/* Build the hierarchy.  phi is real FP64 on the finest unknown grid.  Returns
 * NULL and sets *status < 0 on invalid parameters. */
ora_hier *ora_build(const ora_params *p, const double *phi, int *status);
void ora_free(ora_hier *hh);

int ora_levels(const ora_hier *hh);
/* unknowns per axis on level l (unused axes report 1) */
void ora_level_dims(const ora_hier *hh, int l, int dims[3]);
/* complex node coordinates of axis a on level l: nint+1 values.
 * which = 0 -> ECS grid of H (theta = 0), 1 -> CSG grid of M (theta = beta). */
int ora_axis_nodes(const ora_hier *hh, int which, int l, int a, double complex *out);
/* Shortley-Weller west/centre/east of axis a, level l: 3*(unknowns) values,
 * laid out [west..., centre..., east...] */
int ora_axis_sw(const ora_hier *hh, int which, int l, int a, double complex *out);
/* phi injected onto level l */
int ora_level_phi(const ora_hier *hh, int l, double *out);

/* y = A x; which = 0 -> H (finest only), 1 -> M on level l */
int ora_apply(const ora_hier *hh, int which, int l, const double complex *x, double complex *y);
/* bc = R r: full weighting from level l to l+1 */
int ora_restrict(const ora_hier *hh, int l, const double complex *r, double complex *bc);
/* x += P ec: linear interpolation from level l+1 to level l */
int ora_prolong_add(const ora_hier *hh, int l, const double complex *ec, double complex *x);
/* x = M_L^{-1} b on the coarsest level */
int ora_coarse_solve(const ora_hier *hh, const double complex *b, double complex *x);
/* One GMRES(s) sweep on M_l for M_l x = b, updating x in place.  x_is_zero
 * selects r = b without a matrix-vector product.  Returns steps taken. */
int ora_gmres_sweep(const ora_hier *hh, int l, int s, const double complex *b,
                    double complex *x, int x_is_zero);
/* x = V_{nu1,nu2}(0; b) on level l (l = 0 is the finest level) */
int ora_vcycle_level(const ora_hier *hh, int l, const double complex *b, double complex *x);
int ora_vcycle(const ora_hier *hh, const double complex *b, double complex *x);
/* Flexible GMRES(m) on H, right-preconditioned by one V-cycle per step.
 * hist (may be NULL) receives the Arnoldi estimate per iteration (hist_len max).
 * Returns 0 on convergence, 1 when maxit is reached, <0 on error. */
int ora_fgmres(const ora_hier *hh, const double complex *chi, double complex *u,
               double tol, int m, int maxit, int use_x0, ora_info *info,
               double *hist, int hist_len);

/* Third-order polynomial smoother of section 4 on one level.  The bounding
 * triangle of Prop. 3.1 has vertices t0 = -k^2, t1 = -k^2 + 4d/(H e^{i beta})^2,
 * t2 = -k^2 + 4d/(H e^{i gamma})^2 with H = 2^l h the level's spacing.  p is
 * fixed by p(0) = 1, p(t1) = p(t2) = 0, p(t0) = e^{i varphi} (eq.
 * coefficients_system, coefficients_solution); varphi is the midpoint of the
 * angles meeting both necessary stability conditions (first-order and
 * second-order along the edge t0 t1), see ora_poly_conditions. */
typedef struct ora_poly {
    double k2;          /* k^2 of t0 */
    double H;           /* the level's spacing 2^l h */
    double complex t[3];      /* t0, t1, t2 */
    double complex e[3], f[3];/* eq. coefficients_system solved for b = (1,0,0) and (1,1,1) */
    double varphi;      /* p(t0) = e^{i varphi} */
    double complex c[4];      /* p(t) = sum_j c_j (t - t0)^j */
    double complex omega[3];  /* p(t) = (1 - omega_1 t)(1 - omega_2 t)(1 - omega_3 t) */
    int conds;          /* 0: both conditions met; 1: only the first-order one; 2: neither */
} ora_poly;
int ora_poly_level(const ora_hier *hh, int l, ora_poly *out);
/* Coefficients of |p(t0 + rho e^{-2i beta})|^2 = 1 + 2 rho F + rho^2 S + O(rho^3)
 * along the top edge of the triangle for the polynomial of varphi: F < 0 is
 * the first-order condition (eq. firstorder_varphi), S < 0 the second-order one
 * (eq. secondorder_varphi).  k2, H, dim, beta, gamma define the triangle. */
int ora_poly_conditions(double k2, double H, int dim, double beta, double gamma, double varphi,
                        double *F, double *S);
/* One polynomial smoothing sweep on M_l: x <- x + omega_i (b - M_l x) for
 * i = 1, 2, 3, so the error is multiplied by p(M_l).  x_is_zero: x = 0 on entry. */
int ora_poly_sweep(const ora_hier *hh, int l, const double complex *b, double complex *x, int x_is_zero);

/* Galerkin coarse operator of level l >= 1 (coarse_op = 1): 3^d coefficients
 * per unknown, laid out [offset][unknown] with the offset index
 * sum_a (o_a + 1) 3^a over the used axes, o_a in {-1, 0, 1} (entries whose
 * neighbour lies outside the grid are 0). */
int ora_galerkin_stencil(const ora_hier *hh, int l, double complex *out);

/* Deterministic Hermitian inner product sum conj(x) y in fixed 4096-element
 * chunks, summed in chunk order (independent of the thread count). */
double complex ora_dot(long n, const double complex *x, const double complex *y);

/* OpenMP threads the oracle's parallel loops use (1 without OpenMP). */
int ora_threads(void);

#ifdef __cplusplus
}
#endif
#endif
