/*
 * gp2s.h -- C ABI of the MI355X (gfx950) implementation of the gp2Scale hot path
 * (arXiv 2512.06143): assemble the sparse covariance of a compactly supported,
 * non-stationary kernel, multiply with it, solve with it, and evaluate the log
 * marginal likelihood (LML) and its gradient with respect to the hyperparameters.
 *
 * Problem statement (Sec. 3, first displayed equation; Sec. 4.6):
 *   data x_1..x_N in R^d (d = 2 or 3), targets y, zero prior mean, noise
 *   variance sigma_n^2 on the diagonal;
 *   K_ij = g(x_i) g(x_j) W(||x_i - x_j|| / r) + sigma_n^2 [i == j]
 *   with W(rho) = (1 - rho)^4 (4 rho + 1) for rho < 1, else 0 (a C^2 member of the
 *   Wendland family of Sec. 4.1, Eq. wendland), and the bump mask
 *   g(x) = sum_k a_k exp(1 - 1 / (1 - ||x - c_k||^2 / w^2)) inside ||x - c_k|| < w
 *   (Sec. 4.3, Eq. bump with shape parameter 1, amplitudes a_k = the bump weights,
 *   g a sum of P bumps; the product g g W is a valid kernel by Theorem 1, App. A);
 *   LML = -1/2 y^T K^{-1} y - 1/2 ln|K| - N/2 ln(2 pi).
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers unless the comment says HOST.
 *   - Vectors are float64 and in USER order (the order of the rows of x); the
 *     library reorders internally and undoes it on output.
 *   - All device work is ordered on the context's stream. Calls that return
 *     values to the host (report, gradient, nnz) synchronise that stream.
 *   - The return value is a gp2s_status. No entry point aborts, throws or prints.
 *     gp2s_last_error() gives a one-line description of the last failure. On
 *     failure, outputs are unspecified; handles stay valid and must still be freed.
 *   - Scalar arguments are validated on the host before any GPU call, so invalid
 *     arguments are reported even on a machine without a GPU.
 *   - A context is not thread-safe; use one context per host thread and stream.
 */
#ifndef GP2S_H
#define GP2S_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GP2S_ABI_VERSION 2

typedef int32_t gp2s_status;
#define GP2S_OK           0
#define GP2S_E_INVALID    1  /* an argument is out of range, null, or inconsistent   */
#define GP2S_E_HIP        2  /* a HIP runtime call or kernel launch failed            */
#define GP2S_E_OOM        3  /* the allocator returned NULL                            */
#define GP2S_E_CAPACITY   4  /* a preplanned capacity (batched mode) was exceeded     */
#define GP2S_E_NOT_SPD    5  /* CG met p^T K p <= 0: the matrix is not positive definite */
#define GP2S_E_NOCONV     6  /* max_iter reached; outputs hold the last iterate        */
#define GP2S_E_NONFINITE  7  /* a NaN or infinity in x, y, or the hyperparameters     */

typedef int32_t gp2s_precision;
#define GP2S_FP64   0  /* kernel evaluation, stored K and all vectors in float64        */
#define GP2S_MIXED  1  /* kernel evaluation and stored K in float32 (distances in
                          float64 so that 1 - rho^2 is accurate); CG dot products,
                          solution and residual vectors, refinement and the
                          log-determinant accumulate in float64                       */

typedef struct gp2s_ctx_s* gp2s_ctx;
typedef struct gp2s_matrix_s* gp2s_matrix;

/* Device memory callbacks. alloc returns a device pointer (NULL on failure) aligned
 * to at least 256 bytes; free releases it. Both are called on the host from within
 * library calls, with the context's stream as the stream of use. Passing NULL for
 * both makes the library use hipMalloc / hipFree. */
typedef void* (*gp2s_alloc_fn)(size_t bytes, void* user);
typedef void (*gp2s_free_fn)(void* ptr, void* user);

/* Kernel hyperparameters theta = (r, a_1..a_P, sigma_n^2) plus the fixed bump
 * geometry (centres and width are not differentiated).
 *
 * K_ij = g_i g_j W(rho_ij) + sigma_n^2 [i == j], g the bump mask (Sec. 4.3). With
 * radii == NULL and ls_weights == NULL (zero-initialised params) the kernel is the
 * stationary product construction of Sec. 4.1, rho = ||x_i - x_j|| / r. Otherwise it
 * is the non-stationary convolution form of Eq. wendconv (Sec. 4.2) with
 * S(x) = diag(r_1^2..r_d^2) l(x)^2 and signal deviation g:
 *   l(x) = exp(sum_q c_q bhat_q(x))  (bhat_q the unweighted bumps; l = 1 without ls_weights),
 *   m_ij = (l_i^2 + l_j^2) / 2,  Q_ij = sum_k ((x_ik - x_jk) / r_k)^2 / m_ij,
 *   K_ij = g_i g_j (l_i l_j / m_ij)^{d/2} W(sqrt(Q_ij)),  stored where Q_ij < 1,
 * r_k = radii[k], or r for every axis without radii. The gradient then holds
 * (r or r_1..r_d, a_1..a_P, [c_1..c_P when ls_weights is given], sigma_n^2). This
 * construction is not positive semi-definite for every choice of the parameters (the
 * argument for it assumes a Gaussian scale mixture, which a Wendland function is
 * not); solves report GP2S_E_NOT_SPD when K is not positive definite. */
typedef struct {
  int32_t dim;            /* 2 or 3                                                  */
  int32_t n_bumps;        /* P, 1..256                                               */
  double radius;          /* Wendland support radius r > 0 (Sec. 4.1, r_0)           */
  double bump_width;      /* bump radius w > 0 (Sec. 4.3, r in Eq. bump)             */
  double noise_var;       /* sigma_n^2 >= 0, added on the diagonal (Sec. 3, V)       */
  const double* centers;  /* HOST [n_bumps * dim], row-major bump centres c_k        */
  const double* weights;  /* HOST [n_bumps], bump amplitudes a_k                     */
  int32_t kernel;         /* Wendland member W (Sec. 4.1): GP2S_WENDLAND_C2 (0) is
                             (1-rho)^4 (4 rho + 1); GP2S_WENDLAND_C6 (1) is Eq. wendland
                             as printed, (1-rho)^8 (32 rho^3 + 25 rho^2 + 8 rho + 1).
                             Zero-initialised params select C2.                      */
  const double* radii;    /* HOST [dim] per-axis support radii r_k > 0 (axis-anisotropic
                             W), or NULL: every axis uses radius                     */
  const double* ls_weights; /* HOST [n_bumps] c_q of the length-scale field l(x), or
                             NULL: l = 1. |c_q| <= 20.                               */
  const int32_t* ff_groups; /* HOST [n_bumps] group u in [0, 16) of each bump for the
                             far-field bump kernel, or NULL (see below)              */
} gp2s_params;
/* Far-field bump kernel (Sec. 4.3, Eq. bump_kernel with the core kernel 1), selected by
 * ff_groups != NULL (radii and ls_weights must then be NULL):
 *   K_ij = sum_u g_u(x_i) g_u(x_j) + W(||x_i - x_j|| / r) + sigma_n^2 [i == j],
 *   g_u = sum over the bumps p with ff_groups[p] == u of weights[p] bhat_p,
 * W without a bump mask. The bump term couples points at any distance; it has rank U
 * (the number of groups) and is applied as G (G^T v), never stored as a matrix: the
 * handle's CSR (gp2s_matrix_export) holds K_loc = W + sigma_n^2 I only, while every
 * solve, product (gp2s_spmv), log-determinant, gradient and prediction uses the full K.
 * The gradient keeps the order (r, a_1..a_P, sigma_n^2). */
#define GP2S_WENDLAND_C2 0
#define GP2S_WENDLAND_C6 1

/* Solver options. gp2s_default_opts() fills the defaults given in brackets. */
typedef struct {
  int32_t n_probes;       /* S in [0, 64] Rademacher probes for ln|K| and the trace
                             term of the gradient [64]                               */
  int32_t max_iter;       /* CG iteration cap per solve [20000]                       */
  int32_t max_ir;         /* iterative-refinement restarts of the y solve [4]         */
  int32_t check_every;    /* host convergence poll interval in iterations [16]        */
  uint64_t seed;          /* probe seed [0]                                           */
  double tol;             /* target ||y - K a|| / ||y|| (K as stored) [1e-8]          */
  double probe_tol;       /* per-probe relative CG residual target [1e-5]             */
  int32_t precond;        /* preconditioner M of every CG solve [GP2S_PRECOND_BLOCK]:
                             GP2S_PRECOND_JACOBI (0): M = diag(K);
                             GP2S_PRECOND_BLOCK (1): M = the block diagonal of K over
                             runs of 128 consecutive points of the handle's internal
                             order (the bin order of an assembled handle, the given
                             order of an imported one; the last run holds the
                             remainder), factored M = L L^T blockwise by Cholesky;
                             GP2S_PRECOND_BLOCK64 (2): the same over runs of 64 points
                             (cheaper per iteration; on strongly clustered clouds it
                             converges in as few iterations).
                             The log-determinant estimate is ln|M| + the Lanczos
                             estimate of ln|L^-1 K L^-T| on right-hand sides L z_s; the
                             gradient's trace uses q_s = K^-1 L z_s and w_s = L^-T z_s.
                             Either choice leaves E[ln|K| estimate] = ln|K| (the
                             same-probe value depends on it). The factor is computed on
                             the first solve that needs it and kept with the handle
                             (gp2s_matrix_refill drops it); a block that is not
                             positive definite fails with GP2S_E_NOT_SPD. The batched
                             path (gp2s_batch_*) takes its blocks from each instance's
                             own bin order (its 64-row workgroup blocks) and factors
                             them on every run.                                     */
} gp2s_solve_opts;
#define GP2S_PRECOND_JACOBI 0
#define GP2S_PRECOND_BLOCK 1
#define GP2S_PRECOND_BLOCK64 2

/* Filled on return (HOST struct). */
typedef struct {
  double lml;             /* LML estimate (same-probe log-determinant)              */
  double logdet;          /* ln|K| estimate                                          */
  double yTa;             /* y^T a                                                    */
  double resid;           /* ||y - K a|| / ||y|| recomputed in float64 at the end    */
  double logdet_stderr;   /* standard error of the probe average                     */
  int32_t iters;          /* CG iterations of the y solve, all restarts included     */
  int32_t probe_iters;    /* CG iterations of the probe block (longest column)       */
  int32_t ir_steps;       /* refinement restarts used                                */
  int32_t n_probes;       /* probes used                                             */
} gp2s_report;

/* Per-kernel timing (HIP events on the context's stream), for measurement tools.
 * Index into gp2s_stats.ms / .count: */
#define GP2S_T_ASM_PREP          0  /* bounding box, bump mask, binning sort, gathers   */
#define GP2S_T_ASM_COUNT         1  /* assembly count pass                               */
#define GP2S_T_ASM_FILL          2  /* assembly fill pass (evaluation + compaction)      */
#define GP2S_T_CG_MATVEC1        3  /* CG product, single right-hand side (+ p^T q)      */
#define GP2S_T_CG_MATVEC_BLOCK   4  /* CG product, probe block (+ p^T q per column)      */
#define GP2S_T_CG_UPDATE1        5  /* CG solution/residual update, single RHS (+ dots)  */
#define GP2S_T_CG_PUPDATE1       6  /* CG direction update, single RHS                   */
#define GP2S_T_SPMV              7  /* standalone single-RHS product (residual checks)   */
#define GP2S_T_SPMM              8  /* standalone multi-RHS product                      */
#define GP2S_T_SLQ               9  /* Lanczos quadrature                                */
#define GP2S_T_BACKWARD         10  /* gradient row contraction                          */
#define GP2S_T_GRAD_REDUCE      11  /* gradient per-point reduction                      */
#define GP2S_T_CG_UPDATE_BLOCK  12  /* CG solution/residual update, probe block          */
#define GP2S_T_CG_PUPDATE_BLOCK 13  /* CG direction update, probe block                  */
#define GP2S_NUM_TIMERS         16
typedef struct {
  double ms[GP2S_NUM_TIMERS];     /* summed device time per category, milliseconds */
  int64_t count[GP2S_NUM_TIMERS]; /* number of timed launches per category         */
} gp2s_stats;

/* ---- version and options ------------------------------------------------------ */
int32_t gp2s_abi_version(void);
void gp2s_default_opts(gp2s_solve_opts* opts);     /* HOST struct; no-op on NULL    */
const char* gp2s_status_string(gp2s_status s);     /* static string                 */

/* ---- context --------------------------------------------------------------------
 * stream: a hipStream_t (NULL = the default stream). No GPU call is made here; the
 * device is the one current when the first compute call is made. */
gp2s_status gp2s_create(gp2s_ctx* out, void* stream, gp2s_alloc_fn alloc, gp2s_free_fn free_fn,
                        void* user);
gp2s_status gp2s_destroy(gp2s_ctx ctx);
const char* gp2s_last_error(gp2s_ctx ctx);         /* valid until the next call on ctx */

/* Enable (1) or disable (0) per-kernel event timing on ctx; either call resets the
 * totals. Timing adds two event records per timed launch. */
gp2s_status gp2s_set_timing(gp2s_ctx ctx, int32_t enable);
/* Time only the categories whose bits are set in mask (bit k = GP2S_T_* value k; 0 turns
 * timing off; bits past GP2S_NUM_TIMERS are ignored), so that a measurement of one
 * kernel does not pay the event records of every launch. Resets the totals. */
gp2s_status gp2s_set_timing_mask(gp2s_ctx ctx, uint32_t mask);
/* Totals since the last gp2s_set_timing (HOST struct); waits for the stream. */
gp2s_status gp2s_get_stats(gp2s_ctx ctx, gp2s_stats* out);

/* Optional progress callback, called on the host at every convergence poll of a CG
 * solve with the solve's label ("y solve", "refinement solve", "probe block"), the
 * iterations done, the number of unfinished columns and the largest relative residual
 * of the recurrence among them. NULL disables it. */
typedef void (*gp2s_progress_fn)(const char* label, int32_t iters, int32_t open_cols, double max_rel_resid,
                                 void* user);
gp2s_status gp2s_set_progress(gp2s_ctx ctx, gp2s_progress_fn fn, void* user);

/* Validate n and params on the host only (what gp2s_assemble checks first). */
gp2s_status gp2s_check_params(gp2s_ctx ctx, int64_t n, const gp2s_params* params);

/* ---- assembly (Sec. 4.6 covariance computation; App. B.7 pipeline) ---------------
 * Builds K for points x (DEVICE [n * dim] float64, row-major, user order) as CSR in
 * an internal, spatially sorted order. Only pairs within the kernel's support are
 * evaluated: points are binned on a grid of side >= r, each row tests the points
 * of its neighbouring bins, and survivors are compacted straight into CSR.
 * Stored pattern: the diagonal plus every pair with ||x_i - x_j|| < r whose two
 * points both lie strictly inside some bump (entries may be explicit zeros).
 * The handle keeps a float copy of x, g, the permutation and the CSR; it is owned
 * by the caller and released with gp2s_matrix_free. Non-finite coordinates give
 * GP2S_E_NONFINITE. */
gp2s_status gp2s_assemble(gp2s_ctx ctx, int64_t n, const double* x, const gp2s_params* params,
                          gp2s_precision precision, gp2s_matrix* out);

gp2s_status gp2s_matrix_info(gp2s_matrix m, int64_t* n, int64_t* nnz, gp2s_precision* precision);

/* Copy the CSR out (DEVICE, caller-allocated): row_ptr [n+1] int64, col [nnz] int32,
 * val [nnz] float32 (GP2S_MIXED) or float64 (GP2S_FP64), perm [n] int32 with
 * perm[internal row] = user row. Rows and columns are in internal order, columns
 * ascending within a row. Any output pointer may be NULL to skip it. */
gp2s_status gp2s_matrix_export(gp2s_ctx ctx, gp2s_matrix m, int64_t* row_ptr, int32_t* col,
                               void* val, int32_t* perm);

/* Wrap a caller's CSR (DEVICE; user order, columns ascending, diagonal present and
 * positive) in a handle that gp2s_spmv / gp2s_solve / gp2s_lml accept. The data are
 * copied. gp2s_lml_grad rejects imported handles: it needs the points and the
 * hyperparameters to differentiate K. */
gp2s_status gp2s_matrix_import(gp2s_ctx ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                               const int32_t* col, const void* val, gp2s_precision precision,
                               gp2s_matrix* out);

gp2s_status gp2s_matrix_free(gp2s_matrix m);

/* New hyperparameters on an assembled handle that keep its stored pattern: the bump
 * weights, the noise variance and the Wendland member may change; the dimension,
 * radius, bump count, centres and width must equal the handle's (the pattern depends
 * only on them), else GP2S_E_INVALID. Recomputes g and every stored value in place
 * (no count pass, no allocation of the CSR): the step a sampler takes when a move
 * leaves r and the bump geometry unchanged (Sec. 4.6 and App. D, block-MCMC). The result equals a
 * fresh gp2s_assemble with the same parameters, bit for bit. */
gp2s_status gp2s_matrix_refill(gp2s_ctx ctx, gp2s_matrix m, const gp2s_params* params);

/* Block-product kernel used for `nrhs` columns (2..64) of this matrix, in CG probe
 * blocks and gp2s_spmv: 0 one lane per column (any nrhs), 1 a 16-byte column slice
 * per lane, 2 the same with the rows of X that a tile of bin-sorted rows references
 * staged in LDS (assembled handles only), 3 rows grouped by 4 with the union of their
 * columns (each row of X gathered once per group; nrhs 32 or 64; the grouped copy is
 * built on first use and kept with the handle), 5 the block split K = B + R (B the dense
 * 64 x 64 diagonal blocks of K over runs of 64 rows, multiplied on the float64 matrix
 * cores; R the other entries, gathered by column slices; nrhs 8, 16, 32 or 64; B is
 * built on first use and kept with the handle, 64 values per row), 6 the column slices of
 * variant 1 in two launches, each over half of every XCD's rows (nrhs 8, 16, 32 or 64),
 * 4 / 8 / 16 that many lanes splitting
 * each row's stored entries (1, 2, 4, 8 and 16 need nrhs in {8, 16, 32, 64}, and
 * G <= nrhs),
 * -1 (the default) times the candidates on the first CG block product and keeps the
 * fastest. The context remembers that choice for the handle's shape (N, nnz, precision,
 * nrhs and direction type); a later handle of the same shape in the same context takes
 * it without timing, unless -1 is set on that handle explicitly, which times afresh and
 * replaces the remembered choice. A variant that does not apply gives GP2S_E_INVALID. All variants give the
 * same products up to the order of float64 summation. */
gp2s_status gp2s_matrix_set_block_product(gp2s_matrix m, int32_t nrhs, int32_t variant);
/* The variant in use for `nrhs` columns (HOST output), -1 while not yet chosen. */
gp2s_status gp2s_matrix_get_block_product(gp2s_matrix m, int32_t nrhs, int32_t* variant);

/* ---- products and solves ------------------------------------------------------------
 * Y = K X for nrhs in [1, 64] right-hand sides; X and Y are DEVICE [n * nrhs] float64,
 * row-major (row i holds the nrhs values of point i). The CSR SpMV that drives the
 * solve (Sec. 4.6; App. B.6 "MINRES"): products of stored values with float64
 * vectors accumulate in float64. */
gp2s_status gp2s_spmv(gp2s_ctx ctx, gp2s_matrix m, int32_t nrhs, const double* X, double* Y);
/* (n * nrhs, and n * n_probes below, must stay below 2^31.) */

/* gp2s_spmv without any device allocation, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc). Same
 * arguments, layout and result as gp2s_spmv (up to the order of float64 summation); its
 * workspace is a fixed array of 2 x 2^22 float64 values (64 MiB) that the library holds
 * on every GPU it runs on until the process ends, so n * nrhs must be at most 2^22
 * (else GP2S_E_INVALID). Handles with the far-field term are rejected (GP2S_E_INVALID).
 * Block-product structures that a handle would build on first use are not built here:
 * the call then uses the default kernel. All calls on one GPU share the workspace:
 * calls that overlap on one GPU (other streams, other threads, other contexts) race
 * and must be serialised by the caller. Synchronises the context's stream. */
gp2s_status gp2s_spmv_noalloc(gp2s_ctx ctx, gp2s_matrix m, int32_t nrhs, const double* X, double* Y);

/* a = K^{-1} y (DEVICE [n] float64 each) by preconditioned CG (opts->precond) with float64
 * vectors and dot products, restarted from the recomputed residual (iterative
 * refinement) until ||y - K a|| <= tol ||y||. The paper's host solver is MINRES
 * (App. B.6); K is symmetric positive definite here, so CG reaches the same
 * solution. report may be NULL. */
gp2s_status gp2s_solve(gp2s_ctx ctx, gp2s_matrix m, const double* y, double* a,
                       const gp2s_solve_opts* opts, gp2s_report* report);

/* LML (Sec. 3): solves K a = y as gp2s_solve does, then estimates ln|K| from
 * opts->n_probes Rademacher probes z_s (SplitMix64 signs, counter s * 2^40 + user
 * index): ln|K| ~ ln|M| + (1/S) sum_s z_s^T ln(Khat) z_s, Khat = L^-1 K L^-T with
 * M = L L^T the preconditioner of opts->precond, each quadratic form by Lanczos
 * quadrature from the preconditioned-CG coefficients of the solve K q_s = L z_s.
 * report is required (HOST). a may be NULL. */
gp2s_status gp2s_lml(gp2s_ctx ctx, gp2s_matrix m, const double* y, const gp2s_solve_opts* opts,
                     double* a, gp2s_report* report);

/* gp2s_lml plus its gradient grad (HOST float64) in the order of gp2s_params: (r,
 * a_1..a_P, sigma_n^2), n_bumps + 2 values, for the stationary kernel; (r or r_1..r_d,
 * a_1..a_P, [c_1..c_P], sigma_n^2) otherwise. dLML/dtheta = 1/2 a^T dK a -
 * 1/2 tr(K^{-1} dK), the trace estimated as (1/S) sum_s q_s^T dK L^-T z_s with the
 * probe solutions q_s.
 * dK/dtheta is recomputed from the points for every stored entry; no per-parameter
 * matrix is formed. Requires a handle from gp2s_assemble and n_probes >= 1. */
gp2s_status gp2s_lml_grad(gp2s_ctx ctx, gp2s_matrix m, const double* y, const gp2s_solve_opts* opts,
                          double* a, gp2s_report* report, double* grad);

/* ---- posterior at test points ------------------------------------------------------
 * Posterior mean and variance of the latent function f at n_test test points x*
 * (Sec. 3, Eq. posterior, zero prior mean):
 *   mean_t = k(X, x*_t)^T a,   a = K^{-1} y as returned by gp2s_solve / gp2s_lml,
 *   var_t  = g(x*_t)^2 - k(X, x*_t)^T K^{-1} k(X, x*_t),
 * with k the noise-free kernel of the handle (k(x*, x*) = g(x*)^2; the noise belongs to
 * the observations, so a test point equal to a training point gets none). The
 * cross-covariance uses the training pattern (||x* - x_j|| < r, both points inside
 * some bump) and the handle's storage precision. The variance solves K v_t =
 * k(X, x*_t) with preconditioned CG (opts->precond), 64 test points per block, to the relative residual
 * opts->tol within opts->max_iter iterations (opts->n_probes is not used).
 *   x_test: DEVICE [n_test * dim] float64, row-major; a: DEVICE [n] float64, user order;
 *   mean: DEVICE [n_test] float64 (test order); var: DEVICE [n_test] float64, or NULL to
 *   skip the variance; report: HOST, may be NULL.
 * Requires a handle from gp2s_assemble. Non-finite test coordinates give
 * GP2S_E_NONFINITE; a variance block that misses the tolerance gives GP2S_E_NOCONV
 * with every output written. */
typedef struct {
  int64_t nnz_cross;    /* stored entries of k(X, x*) over all test points */
  int32_t var_blocks;   /* block solves run for the variance */
  int32_t var_iters;    /* most CG iterations of any block */
} gp2s_predict_report;
gp2s_status gp2s_predict(gp2s_ctx ctx, gp2s_matrix m, int64_t n_test, const double* x_test, const double* a,
                         const gp2s_solve_opts* opts, double* mean, double* var, gp2s_predict_report* report);

/* ---- batched instances -------------------------------------------------------------
 * Many independent instances (each its own points, dimension, targets and
 * hyperparameters; Sec. 3 per instance) evaluated together: one block-diagonal system
 * assembled in shared launches, solved by batched preconditioned CG (diagonal or
 * block-Jacobi per opts.precond, blocks inside each instance) whose iterations run as
 * replays of one captured hipGraph chunk, with per-instance step lengths, convergence
 * and Lanczos coefficients. A plan fixes the points, dimensions, bump centres and
 * widths, the precision and the solver options; runs may change r, the bump weights
 * and the noise variance.
 *
 * gp2s_batch_plan: n (HOST [n_inst]) point counts; x (HOST array of n_inst DEVICE
 * pointers, each [n[i] * dim_i] float64 row-major); params (HOST [n_inst]); opts
 * (n_probes must be a power of two in [1, 64]). Planning binds the points (they are
 * copied), picks the bin refinement and the lanes per row of both products by timing
 * candidates (the plan's autotuner), assembles once and reserves the CSR capacity
 * (1.25 x the planned entries). Returns GP2S_E_NONFINITE for non-finite points. */
typedef struct gp2s_batch_s* gp2s_batch;
gp2s_status gp2s_batch_plan(gp2s_ctx ctx, int32_t n_inst, const int64_t* n, const double* const* x,
                            const gp2s_params* params, gp2s_precision precision, const gp2s_solve_opts* opts,
                            gp2s_batch* out);
/* Total points, stored entries, reserved capacity and the tuned choices
 * tuned[3] = {bin refinement m, lanes per row of the single-RHS product, lanes per row
 * of the probe-block product: L > 1 for one lane per column in segments of L lanes, 1
 * for 16-byte column slices per lane, -G for G lanes splitting each row's stored
 * entries} (HOST outputs, each may be NULL). */
gp2s_status gp2s_batch_info(gp2s_batch b, int64_t* n_total, int64_t* nnz, int64_t* capacity, int32_t* tuned);
/* LML (and gradient) of every instance. y: HOST array of n_inst DEVICE pointers [n[i]];
 * params: HOST [n_inst] new hyperparameters, or NULL to keep the planned ones (dimension,
 * bump count, centres and width must match the plan, else GP2S_E_INVALID); lml: HOST
 * [n_inst]; grad: HOST array of n_inst HOST pointers to [n_bumps_i + 2] (r, a_1..a_P,
 * sigma^2), or NULL to skip the gradient; reports: HOST [n_inst] or NULL. If the new
 * radius needs more stored entries than reserved: GP2S_E_CAPACITY (plan again). */
gp2s_status gp2s_batch_run(gp2s_batch b, const double* const* y, const gp2s_params* params, double* lml,
                           double* const* grad, gp2s_report* reports);
gp2s_status gp2s_batch_free(gp2s_batch b);

#ifdef __cplusplus
}
#endif
#endif /* GP2S_H */
