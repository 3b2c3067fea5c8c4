/*
 * csg.h -- C ABI of libcsg: an MI355X (gfx950) solver for the indefinite
 * Helmholtz problem  H u = -(Laplace + phi) u = chi  discretised on a grid with
 * exterior-complex-scaled (ECS) absorbing layers, by flexible GMRES
 * preconditioned with one multigrid V-cycle on the complex-stretched-grid (CSG)
 * operator M, with GMRES(s) as the smoother on every level.
 *
 * Paper: B. Reps, W. Vanroose, H. bin Zubair, "GMRES-based multigrid for the
 * complex scaled preconditioner for the indefinite Helmholtz equation".
 *   - problem statement ........................ section 1, eq. (helm)
 *   - ECS / CSG complex grids ................... section 2, eq. (csggrid)
 *   - Shortley-Weller discretisation, Kronecker
 *     sums, preconditioned system ............... section 2, eq. (csg_dis)
 *   - GMRES(s) smoother, V(nu1,nu2)-cycle,
 *     coarse operators by rediscretisation ...... section 3.1
 *   - flexible GMRES outer solve ................ section 5
 *
 * Conventions shared by every entry point
 *  - Grid: per axis a there are layer_lo[a] + n[a] + layer_hi[a] intervals of
 *    mesh width h; interior intervals have complex length h e^{i beta} (M) or h
 *    (H), layer intervals h e^{i gamma}.  Unknowns are the interior nodes
 *    1..N_a-1 of each axis (homogeneous Dirichlet at the far layer ends).
 *  - Vectors are interleaved complex (re, im), x fastest, laid out
 *    [rhs][z][y][x] over the unknowns only; consecutive right-hand sides are
 *    contiguous (stride = unknowns of the level).  complex128 = 2 doubles,
 *    complex64 = 2 floats.
 *  - All pointers named *_dev are device pointers (hipMalloc'ed or torch CUDA
 *    tensors); *_host are host pointers.  The caller owns every buffer.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Every call
 *    only enqueues work on that stream, except csg_operator_create (copies
 *    the setup tables and waits for them) and helm_solve (reads back one small
 *    residual estimate per iteration and waits for it).
 *  - Return value: CSG_OK or a negative status; csg_last_error() returns a
 *    thread-local message describing the last failure.  Nothing throws or
 *    aborts across this ABI.
 */
#ifndef CSG_H
#define CSG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CSG_OK = 0,
    CSG_EINVAL = -1,   /* invalid argument or parameter combination */
    CSG_ENOMEM = -2,   /* workspace too small */
    CSG_EDEVICE = -3,  /* HIP runtime error */
    CSG_ENOCONV = -4,  /* maxit reached before the tolerance */
    CSG_ENUMERIC = -5  /* non-finite residual norm */
};

#define CSG_MAX_LEVELS 16
#define CSG_MAX_S 8
#define CSG_MAX_RESTART 64
#define CSG_MAX_RHS 64

/* Problem and preconditioner parameters (section 1 problem statement; section 2
 * grid; section 3.1 cycle).  Unused axes (dim = 2: index 2) are ignored. */
typedef struct csg_params {
    int dim;            /* 2 (5-point stencil) or 3 (7-point stencil) */
    int n[3];           /* interior intervals per axis, >= 1 */
    double h;           /* real mesh width, > 0 */
    int layer_lo[3];    /* ECS layer intervals on the low side of each axis, >= 0 */
    int layer_hi[3];    /* ECS layer intervals on the high side of each axis, >= 0 */
    double gamma;       /* ECS rotation angle theta_gamma, 0 < gamma < pi/4 (radians) */
    double beta;        /* CSG rotation angle theta_beta of M's interior, 0 <= beta < gamma */
    int levels;         /* multigrid levels; 0 = ceil-halve until <= 9 intervals per axis */
    int s;              /* GMRES(s) smoother length, 1..CSG_MAX_S */
    int nu1, nu2;       /* pre-/post-smoothing sweeps, >= 0 */
    int cycle_prec;     /* 0 = complex128 V-cycle, 1 = complex64 V-cycle (mixed) */
    int max_rhs;        /* right-hand sides solved together, 1..CSG_MAX_RHS */
    int restart;        /* FGMRES restart length m the workspace is sized for, 1..CSG_MAX_RESTART */
    /* execution tuning (0 = library default; results are unaffected beyond rounding):
     *   tail_max  levels with at most this many unknowns run in the one-workgroup
     *             coarse-tail kernel (-1: only the coarsest level)
     *   fuse_max  levels with at most this many unknowns use the fused
     *             Gram-Schmidt + stencil Arnoldi passes (-1: never)
     *   graphs    1 (default) replay FGMRES iterations from captured HIP graphs,
     *             -1 launch eagerly */
    int tail_max;
    int fuse_max;
    int graphs;
    /* smoother of every non-coarsest level (section 4 compares the two):
     *   0  GMRES(s) sweeps (section 3.1)
     *   1  the third-order polynomial smoother of section 4: per level
     *      p(t) = (1 - w1 t)(1 - w2 t)(1 - w3 t) with p(0) = 1, p(t1) = p(t2) = 0
     *      and p(t0) = e^{i varphi} on the bounding triangle t0 = -k^2,
     *      t1 = -k^2 + 4d/(2^l h e^{i beta})^2, t2 = -k^2 + 4d/(2^l h e^{i gamma})^2
     *      (Prop. 3.1), varphi the midpoint of the angles meeting the first-
     *      and second-order stability conditions (eq. firstorder_varphi,
     *      eq. secondorder_varphi); one sweep = three Richardson steps
     *      x += w_i (b - M x), no inner products
     * poly_k2: k^2 of t0 (0 = the mean of phi over the finest unknowns). */
    int smoother;
    double poly_k2;
    /* more execution tuning (0 = library default; results are unaffected
     * beyond rounding), the knobs the autotuner searches:
     *   slab_blocks  3-D levels: workgroups per right-hand side the z-marching
     *                slab passes aim for (default 128; fewer runs of planes
     *                re-read fewer halo planes, more fill more CUs), 1..4096
     *   tile_mult    2-D levels: LDS tiles of the fused passes per chunked-pass
     *                block, a power of two 1..64 (default 1)
     *   slab_min     3-D levels with at least this many unknowns run the slab
     *                passes (default 100000; -1: never) */
    int slab_blocks;
    int tile_mult;
    int slab_min;
    /* complex factor s of phi in the preconditioner on every level,
     * M = L(theta_beta) - s phi (0 + 0i means s = 1, the CSG preconditioner).
     * beta = 0 and s = 1 + i eps is the complex shifted Laplacian the paper
     * compares with (section 1, section 2: (1 + eps i) k^2); on a grid without
     * ECS layers the CSG preconditioner equals e^{-2i beta} times the one with
     * beta = 0 and s = e^{2i beta}.  H is never shifted.  Takes the GMRES(s)
     * smoother (smoother = 0). */
    double shift_re, shift_im;
    /* coarse operators: 0 = rediscretisation on the coarser complex grid
     * (section 3.1), 1 = Galerkin products M_{l+1} = R M_l P with the
     * transfers of csg_residual_restrict / csg_prolong_correct (the section 5
     * remark reports similar convergence), stored as 9- or 27-point stencils.
     * Galerkin operators run every level on the unfused multi-block passes
     * (no LDS tiles, slabs or coarse tail) and take the GMRES(s) smoother. */
    int coarse_op;
} csg_params;

typedef struct csg_operator csg_operator;

typedef struct csg_solve_info {
    int iterations;     /* outer FGMRES iterations = V-cycles applied */
    int restarts;       /* completed restart cycles */
    int vcycles;        /* V-cycles applied */
    int converged;      /* 1 if the true relative residual is <= tol */
    double relres_true; /* ||chi - H u||_2 / ||chi||_2, recomputed in FP64 at exit */
    double relres_est;  /* last Arnoldi estimate |g_{j+1}| / ||chi|| */
    double seconds;     /* host wall time of the solve */
} csg_solve_info;

/* Thread-local description of the last error (never NULL). */
const char *csg_last_error(void);

/* Exact device workspace bytes for these parameters: hierarchy tables, phi on
 * every level, V-cycle vectors and FGMRES bases for max_rhs right-hand sides.
 * Returns CSG_EINVAL on invalid parameters (see csg_operator_create). */
int csg_workspace_bytes(const csg_params *p, size_t *bytes);

/* Level count and unknowns per axis per level (dims[l][0..2], unused axes 1)
 * that csg_operator_create would build; host-only, no device work. */
int csg_plan_levels(const csg_params *p, int *levels, int dims[][3]);

/* Build the multigrid hierarchy (section 3.1: coarse operators by
 * rediscretisation on the nested complex grid, phi injected) and the FGMRES
 * state inside the caller's workspace.
 *   phi_host : real FP64 wavenumber field phi on the finest unknowns, one
 *              grid (layers included).  Copied; the caller may free it.
 *   ws_dev   : device workspace of ws_bytes >= csg_workspace_bytes(); must
 *              stay allocated until csg_operator_destroy.  256-byte aligned.
 * Errors: CSG_EINVAL (bad parameters: dim not 2/3, n < 1, negative layers,
 * not 0 <= beta < gamma < pi/4, s not in 1..CSG_MAX_S, nu < 0, a level with < 2
 * intervals on an axis, more than 4096 coarsest unknowns, non-finite phi),
 * CSG_ENOMEM (ws_bytes too small), CSG_EDEVICE (HIP failure). */
int csg_operator_create(const csg_params *p, const double *phi_host, void *ws_dev,
                        size_t ws_bytes, void *stream, csg_operator **out);

int csg_operator_destroy(csg_operator *op);

/* Level count and unknowns per axis of each level of a built operator. */
int csg_operator_info(const csg_operator *op, int *levels, int dims[][3]);

/* y = A x on one level (section 2, eq. csg_dis, negative Laplacian minus phi):
 * which = 0 -> H (ECS grid, theta = 0; level 0 only, complex128 in and out),
 * which = 1 -> M on `level` in the cycle precision (complex128 or complex64).
 * x_dev, y_dev: nrhs vectors of that level, must not overlap. */
int csg_stencil_apply(const csg_operator *op, int which, int level, const void *x_dev,
                      void *y_dev, int nrhs, void *stream);

/* x = V_{nu1,nu2}(0; b): one V-cycle on M with GMRES(s) smoothing from a zero
 * initial guess (section 3.1), exact dense solve on the coarsest level.  b_dev,
 * x_dev: nrhs finest-level vectors in the cycle precision; must not overlap. */
int csg_vcycle(const csg_operator *op, const void *b_dev, void *x_dev, int nrhs, void *stream);

/* One smoothing sweep on M_level for M x = b, x updated in place: GMRES(s)
 * (section 3.1: a GMRES solve on the error stopped after s iterations) or,
 * with csg_params.smoother = 1, the polynomial sweep of section 4. */
int csg_smooth(const csg_operator *op, int level, const void *b_dev, void *x_dev, int nrhs,
               void *stream);

/* csg_smooth for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same sweep, same results, with its own vectors (residual, u_1..u_s, w_0,
 * w_1), reduction partials and smoother states in a static device array of
 * 128 MiB per GPU instead of the operator's workspace.  The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine); the array is
 * created with the library's code object on each GPU it runs on and held until
 * the process ends.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller; partials and states are cleared on every call.
 * Errors: CSG_ENOMEM when the sweep needs more than 128 MiB, i.e.
 * (s + 3) * nrhs * unknowns(level) * (16 or 8 bytes) (s + 4 with the
 * polynomial smoother) plus about 330 KB per RHS of partials and states;
 * CSG_EDEVICE if the array's device address cannot be obtained; otherwise as
 * csg_smooth. */
int csg_smooth_static(const csg_operator *op, int level, const void *b_dev, void *x_dev, int nrhs,
                      void *stream);

/* The polynomial smoother of `level` (section 4; built for every level at
 * create whatever csg_params.smoother says): varphi, the three Richardson
 * weights omega[0..5] = (re, im) of w1, w2, w3 in the order the sweep applies
 * them, and conds = 0 when varphi meets both necessary stability conditions,
 * 1 when only the first-order one can be met, 2 when neither. */
int csg_poly_info(const csg_operator *op, int level, double *varphi, double omega[6], int *conds);

/* bc = R (b - M_level x): residual restricted by full weighting R = 2^-d P^T
 * to level+1. */
int csg_residual_restrict(const csg_operator *op, int level, const void *b_dev,
                          const void *x_dev, void *bc_dev, int nrhs, void *stream);

/* x += P ec: bi/trilinear interpolation from level+1 to level. */
int csg_prolong_correct(const csg_operator *op, int level, const void *ec_dev, void *x_dev,
                        int nrhs, void *stream);

/* x = M_L^{-1} b on the coarsest level (dense inverse built at create). */
int csg_coarse_solve(const csg_operator *op, const void *b_dev, void *x_dev, int nrhs,
                     void *stream);

/* Flexible GMRES(restart) on H, right-preconditioned by one V-cycle per
 * iteration (section 5), all outer arithmetic in FP64.
 *   chi_dev : nrhs complex128 sources;  u_dev: nrhs complex128 solutions (in:
 *             initial guess if use_initial_guess, out: result).
 *   tol     : stop when ||chi - H u|| / ||chi|| <= tol (true FP64 residual).
 *   restart : <= params.restart;  maxit: iteration budget per right-hand side.
 *   info    : host array of nrhs entries (may be NULL).
 * Returns CSG_OK when every RHS converged, CSG_ENOCONV if maxit was reached
 * (u holds the last iterate, info filled), CSG_ENUMERIC on a non-finite norm.
 * A zero source gives u = 0 and iterations = 0.  Synchronises the stream. */
int helm_solve(const csg_operator *op, const void *chi_dev, void *u_dev, int nrhs, double tol,
               int restart, int maxit, int use_initial_guess, csg_solve_info *info,
               void *stream);

/* Incremental form of helm_solve for a serving loop that interleaves several
 * solves on several streams.  begin enqueues the initial residual; step
 * enqueues one FGMRES iteration (or the restart/true-residual work when due)
 * and an asynchronous copy of the residual estimate; poll returns 1 when that
 * copy has landed and the solve state has been advanced on the host, 0 if it
 * is still in flight; *done becomes 1 when every RHS has converged or maxit is
 * reached.  end writes info and returns the helm_solve status.  One solve per
 * operator at a time. */
typedef struct csg_solve csg_solve;
int csg_solve_begin(const csg_operator *op, const void *chi_dev, void *u_dev, int nrhs,
                    double tol, int restart, int maxit, int use_initial_guess, void *stream,
                    csg_solve **out);
int csg_solve_step(csg_solve *sv);
int csg_solve_poll(csg_solve *sv, int *done);
int csg_solve_end(csg_solve *sv, csg_solve_info *info);

/* Batches: several problems of one size class in one operator, so their
 * solves advance in the same launches (section 5's FGMRES and section 3.1's
 * V-cycle, right-hand sides of every problem on the grid's second dimension).
 * Problems share the grid shape (dim, n, layers, levels), s, nu1, nu2,
 * cycle_prec, max_rhs (per problem), restart and the tuning fields; h, beta,
 * gamma and phi may differ.  Only the GMRES(s) smoother is batched
 * (smoother = 0).  The batched operator has nprob * max_rhs right-hand sides:
 * problem q owns RHS q*max_rhs .. (q+1)*max_rhs - 1 of every vector (give
 * unused ones a zero source: they finish at once with u = 0).  Every other
 * entry point (stencil, V-cycle, helm_solve, csg_solve_*) works on it as on a
 * single operator; results of each problem equal its solve alone.
 *   csg_batch_workspace_bytes: exact workspace of nprob problems of class p
 *   (CSG_EINVAL if nprob * max_rhs > CSG_MAX_RHS or smoother != 0).
 *   csg_batch_create: p[q], phi_host[q] for q < nprob; errors as
 *   csg_operator_create, CSG_EINVAL when the classes differ.
 *   helm_step_batch: one step of a (batched) solve begun by csg_solve_begin:
 *   waits for the oldest report in flight, applies the stop and restart
 *   decisions of every problem's RHS and enqueues the next iterations (one
 *   launch sequence for all problems); *done = 1 when every RHS has stopped
 *   (then call csg_solve_end). */
int csg_batch_workspace_bytes(const csg_params *p, int nprob, size_t *bytes);
int csg_batch_create(const csg_params *const *p, int nprob, const double *const *phi_host, void *ws_dev,
                     size_t ws_bytes, void *stream, csg_operator **out);
int helm_step_batch(csg_solve *sv, int *done);

/* Benchmark instrumentation (not needed to solve).  csg_profile(op, kind, cap)
 * makes the library record a pair of HIP events around every launch of one
 * pass kind, on the stream that launch uses, for up to `cap` launches, and sum
 * the algorithmic bytes those launches move (the minimal traffic of the pass:
 * each input vector read once, each output written once).  kind 0 disables it.
 * csg_profile_read waits for the last recorded event and returns the summed
 * kernel time (ms), the number of launches timed and the summed algorithmic
 * bytes.  The events are timing-only (no system-scope fence), so recording
 * them leaves the caches of the timed launches alone.  Kinds: */
enum {
    CSG_PROF_OFF = 0,
    CSG_PROF_VCYCLE = 1,        /* one whole V-cycle (every level)            */
    CSG_PROF_STENCIL_DOTS = 2,  /* finest-level Arnoldi stencil + dot pass    */
    CSG_PROF_ORTH = 3,          /* finest-level Gram-Schmidt + norm pass      */
    CSG_PROF_UPD_RESTRICT = 4,  /* finest-level update + restriction pass     */
    CSG_PROF_PROLONG_RESID = 5, /* finest-level correction + residual pass    */
    CSG_PROF_UPDATE = 6,        /* finest-level post-smoother update pass     */
    CSG_PROF_OUTER_H = 7,       /* FGMRES: w = H z + first-round dots         */
    CSG_PROF_OUTER_CGS1 = 8,    /* FGMRES: first projection + ||w1||^2        */
    CSG_PROF_OUTER_CGS2 = 9,    /* (unused: the second-round dots run inside the first projection) */
    CSG_PROF_OUTER_NORM = 10,   /* FGMRES: v_1 = r / beta at a cycle start    */
    CSG_PROF_OUTER_PROJ2 = 11,  /* FGMRES: second projection, scale, cast     */
    CSG_PROF_FUSED = 12,        /* finest-level fused Gram-Schmidt + stencil  */
    CSG_PROF_KINDS = 13
};
int csg_profile(csg_operator *op, int kind, int cap);
int csg_profile_read(csg_operator *op, double *ms, long *launches, double *bytes);

/* 1 when uninstrumented FGMRES iterations replay captured HIP graphs (the
 * default), 0 when they run as individual launches (graphs disabled by
 * csg_params.graphs, or capture unavailable).  While a pass kind is being
 * timed (csg_profile) iterations always run as individual launches: events
 * recorded inside a graph cannot be timed on this HIP. */
int csg_graphs_active(const csg_operator *op);

#ifdef __cplusplus
}
#endif
#endif
