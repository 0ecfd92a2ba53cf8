/*
 * gpmi.h -- C ABI of the MI355X (gfx950) low-precision Gaussian-process solver.
 *
 * Method: Maddox, Potapczynski & Wilson, "Low-Precision Arithmetic for Fast
 * Gaussian Processes", UAI 2022.  The library computes, without ever storing
 * the kernel matrix, the product (a^2 K(X1,X2) + s^2 I) V (Sec. 5.1, Eq. mvm)
 * and solves (a^2 K + s^2 I) U = B by conjugate gradients, either the standard
 * preconditioned form (App. A, Alg. 2) or the enhanced-stability form (Sec.
 * 5.2, Alg. 1: log-scale step sizes via logsumexp, re-orthogonalisation),
 * optionally preconditioned by a rank-k pivoted Cholesky factor through the
 * Woodbury identity (Sec. 5.2, Eq. woodbury).
 *
 * Conventions shared by every entry point:
 *  - Every call returns a gp_status; nothing throws across the ABI.  On any
 *    error the message is available from gp_last_error() (per host thread).
 *    On GP_ERR_ARG no output has been touched.
 *  - Matrices are row-major, float32, and DEVICE pointers unless a comment
 *    says "host".  The caller owns all memory it passes; the library owns the
 *    opaque handles it returns and its own workspaces.
 *  - Streams are HIP streams passed as void* (NULL = the default stream).
 *    Launches are asynchronous on that stream unless a comment says the call
 *    synchronises.
 *  - Library workspaces are cached per device and stream: calls issued on
 *    the same stream are safe; concurrent calls on one stream from several
 *    host threads race.
 */
#ifndef GPMI_H
#define GPMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gp_status;
#define GP_OK 0
#define GP_PENDING 1
#define GP_ERR_ARG (-1)
#define GP_ERR_NOMEM (-2)
#define GP_ERR_HIP (-3)
#define GP_ERR_NOT_PD (-4)
#define GP_ERR_BREAKDOWN (-5)
#define GP_ERR_TOO_LARGE (-6)
#define GP_ERR_UNKNOWN_TICKET (-7)
#define GP_ERR_CANCELLED (-8)
#define GP_ERR_STOPPED (-9)

/* A column's convergence is refused when its float64 true residual exceeds
 * GP_TRUE_RES_SLACK * max(tol, GP_TRUE_RES_FLOOR): the recursive residual
 * tracks the product's own operator, which in binary16 sits a little away
 * from K~ (the slack), and finite-precision CG's recursive residual keeps
 * falling after the true residual has reached the attainable accuracy (the
 * floor).  A solve that diverged is far beyond both.                      */
#define GP_TRUE_RES_SLACK 2.0
#define GP_TRUE_RES_FLOOR 1e-3

/* Covariance function (App. C; Matern-5/2 and -3/2 in the textbook
 * half-integer form, r^2 = sum_m ((x_m - x'_m)/l_m)^2):
 *   RBF        exp(-r^2/2)
 *   MATERN52   (1 + sqrt5 r + 5 r^2/3) exp(-sqrt5 r)
 *   MATERN12   exp(-r)
 *   MATERN32   (1 + sqrt3 r) exp(-sqrt3 r)                               */
#define GP_KERNEL_RBF 0
#define GP_KERNEL_MATERN52 1
#define GP_KERNEL_MATERN12 2
#define GP_KERNEL_MATERN32 3

/* Arithmetic of the kernel-matrix product (Sec. 5.1).
 *   GP_PREC_FP32: float32 inputs, kernel entries and accumulation.
 *   GP_PREC_FP16: inputs divided by the lengthscale are rounded to binary16,
 *                 the kernel tile entries and the scaled right-hand sides are
 *                 binary16 matrix-core operands, every product and sum is
 *                 accumulated in float32 ("block summation in single
 *                 precision"), and the output is float32.                     */
#define GP_PREC_FP32 0
#define GP_PREC_FP16 1
/*   GP_PREC_BF16: as GP_PREC_FP16 with bfloat16 (Sec. 2.1: float32's 8-bit
 *                 exponent, an 8-bit significand) in place of binary16: the
 *                 inputs divided by the lengthscale, the kernel tile entries
 *                 and the scaled right-hand sides are bfloat16 matrix-core
 *                 operands, accumulation is float32.  Kernel values keep
 *                 float32's range (no underflow to zero at 2^-25).           */
#define GP_PREC_BF16 2

/* Hyperparameters (Sec. 2.2 and Eq. mvm): kernel kind, lengthscale(s),
 * outputscale a^2 and noise s^2.  lengthscale is a HOST array of 1 value
 * (isotropic, ard = 0) or d values (ARD, ard = 1).  Requirements: every
 * lengthscale finite and > 0, a^2 finite and > 0, s^2 finite and >= 0
 * (> 0 for solves and preconditioners).                                       */
typedef struct gp_kernel {
  int32_t kind;
  int32_t ard;
  const float* lengthscale;
  float outputscale;
  float noise;
} gp_kernel;

/* Message describing the last error on the calling host thread ("" if none). */
const char* gp_last_error(void);

/* Library version string, e.g. "gpmi 0.1.0 gfx950". */
const char* gp_version(void);

/* Release the device memory the library keeps between calls: the per-stream
 * workspaces (each device is synchronised first) and the blocks kept for the
 * next preconditioner handle of the same size.  Later calls allocate again.
 * No library call may run on any host thread meanwhile.  *bytes_freed (may be
 * NULL) receives the total.  The library also releases the cached blocks by
 * itself, and retries once, when an allocation of a new handle fails.      */
gp_status gp_release_cached_memory(uint64_t* bytes_freed);

/*
 * gp_kmvm -- out = a^2 K(X1, X2) V + [add_noise] s^2 V          (Eq. mvm)
 *
 *  X1   n1 x d  points of the output rows
 *  X2   n2 x d  points of the summed columns
 *  V    n2 x r  right-hand sides
 *  out  n1 x r  result; must not overlap V, X1 or X2
 *  add_noise    1 adds s^2 V; requires X1 == X2 and n1 == n2 (the same set)
 *  precision    GP_PREC_FP32, GP_PREC_FP16 or GP_PREC_BF16
 *  scale_mode   FP16 and BF16: 0 scales column c of V by the power of two that
 *               puts max|v_c| in [2^14, 2^15) before rounding it to binary16,
 *               1 uses the paper's n2^(-1/2) (Sec. 5.1); the scale is undone
 *               on the float32 accumulator, so both give the same product up
 *               to rounding.
 *  Limits: 1 <= d <= 64, r >= 1, n1, n2 >= 0 (n1 == 0 is a no-op, n2 == 0
 *  gives out = [add_noise] s^2 V).  Asynchronous on `stream`.
 *  FP16 with X1 == X2, n1 == n2 >= 16384, d <= 14 and r <= 16 runs the
 *  symmetric form (each unique pair's kernel value computed once); its
 *  partial sums take about n^2 r_pad 4 / 3072 bytes of device memory (r_pad =
 *  16), and when they cannot be allocated the one-sided form, whose
 *  workspace is O(n), runs instead.  gp_cg_solve chooses the same way.
 *  Errors: GP_ERR_ARG (shapes, hyperparameters, null pointers, aliasing),
 *  GP_ERR_NOMEM (workspace), GP_ERR_HIP (launch failure).
 *  FP16 inputs whose |x/l| or squared norm exceeds the binary16 range give
 *  non-finite outputs.
 */
gp_status gp_kmvm(const gp_kernel* k, const float* X1, int64_t n1, const float* X2,
                  int64_t n2, int32_t d, const float* V, int32_t r, float* out,
                  int32_t add_noise, int32_t precision, int32_t scale_mode, void* stream);

/*
 * gp_kmvm_noalloc -- gp_kmvm for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, limits, errors and result as gp_kmvm; it calls
 * no hipMalloc, hipFree or allocating library routine.  Its scratch (the
 * prepared operands, the scaled right-hand sides and the split partial sums)
 * lives in one fixed block of gp_kmvm_noalloc_scratch_bytes() (64 MiB) per
 * device, held from the first call on that device until the process ends.
 * When the column-split count gp_kmvm would use does not fit, fewer splits
 * are used (only the order of the float32 partial sums changes); a product
 * that does not fit with one split fails with GP_ERR_TOO_LARGE before
 * anything runs (binary16 at d <= 14, r <= 16 needs about 128 n1 + 96 n2
 * bytes: n1 = n2 up to about 299,000 points).
 * Every call on one device shares that device's block and leaves its last
 * contents there: calls that overlap in time on one device (two streams, or
 * two host threads) race and give wrong results; order them on one stream.
 */
gp_status gp_kmvm_noalloc(const gp_kernel* k, const float* X1, int64_t n1, const float* X2,
                          int64_t n2, int32_t d, const float* V, int32_t r, float* out,
                          int32_t add_noise, int32_t precision, int32_t scale_mode,
                          void* stream);

/* Size in bytes of gp_kmvm_noalloc's per-device scratch block. */
uint64_t gp_kmvm_noalloc_scratch_bytes(void);

/*
 * gp_kmvm_truncated -- the binary16 product of gp_kmvm (precision FP16,
 * power-of-two column scales) over the finite support of the binary16 kernel
 * (Sec. 4.1; App. C): a kernel value below 2^-25 rounds to zero in binary16,
 * so pairs of points beyond the kernel's radius contribute nothing.  Both
 * point sets are put in Z-order of their scaled coordinates; each 256-point
 * row block skips the 128-point column stages whose bounding boxes are farther
 * apart than the scaled radius R at which the kernel value is 2^-26 (RBF
 * 6.00, Matern-5/2 10.44, Matern-3/2 12.19, Matern-1/2 18.02; half the
 * rounding threshold, far beyond the float32 error of the distance argument).
 *  skip  1: skip those tiles; 0: visit every tile of the same ordering.  The
 *        two give bit-identical outputs (the dropped terms are exact zeros and
 *        the float32 sums keep their order); against gp_kmvm they differ only
 *        by the order of float32 sums.
 *  stats optional HOST struct: tiles of the ordered product, tiles visited,
 *        and R.
 * Arguments and limits as gp_kmvm (n1, n2 < 2^30; X must be finite).
 * Asynchronous on `stream` unless stats is given (then synchronised).
 */
typedef struct gp_trunc_stats {
  int64_t tiles_total;
  int64_t tiles_visited;
  double radius;
} gp_trunc_stats;

gp_status gp_kmvm_truncated(const gp_kernel* k, const float* X1, int64_t n1, const float* X2,
                            int64_t n2, int32_t d, const float* V, int32_t r, float* out,
                            int32_t add_noise, int32_t skip, gp_trunc_stats* stats,
                            void* stream);

/*
 * gp_kmvm_summation -- accuracy ablations of the product (Sec. 5.1, Fig. 4;
 * App. B, summation approaches): the binary16 product of gp_kmvm with every
 * product and every sum in binary16 as well.  Kernel values of the binary16
 * inputs x / l are rounded to binary16 (k_hat), right-hand sides to
 * v_hat = fp16(v s_c), each term is p_j = fp16(k_hat_j v_hat_j), and the terms
 * of one output entry are summed in column order j = 0 .. n2-1:
 *   GP_SUM_BLOCK_HALF    blocks of `block` consecutive columns (the last one
 *                        shorter), each summed sequentially in binary16; the
 *                        block sums added sequentially in binary16;
 *   GP_SUM_BLOCK_SINGLE  the same block sums added sequentially in float32,
 *                        the total rounded to binary16;
 *   GP_SUM_KAHAN_HALF    one compensated (Kahan) sum over all columns with
 *                        every operation in binary16 (`block` is ignored).
 * Every binary16 or float32 operation rounds once to nearest even (no fused
 * multiply-add), so given the kernel values the total T is defined bit for
 * bit.  out = a^2 T / s_c + [add_noise] s^2 v, in float32.
 *  scale_mode  as gp_kmvm; 1 (s_c = n2^-1/2, the paper's) keeps binary16
 *              sums in range, 0 (largest |v_hat| in [2^14, 2^15)) overflows
 *              to inf after a few terms.
 *  block       1 <= block <= 2^30 (any value for GP_SUM_KAHAN_HALF).
 * One thread per output row on the vector ALUs: an accuracy reference, not a
 * fast path.  Arguments and limits otherwise as gp_kmvm.  Asynchronous on
 * `stream`.  Errors: GP_ERR_ARG, GP_ERR_NOMEM, GP_ERR_HIP.
 */
#define GP_SUM_BLOCK_HALF 0
#define GP_SUM_BLOCK_SINGLE 1
#define GP_SUM_KAHAN_HALF 2

gp_status gp_kmvm_summation(const gp_kernel* k, const float* X1, int64_t n1, const float* X2,
                            int64_t n2, int32_t d, const float* V, int32_t r, float* out,
                            int32_t add_noise, int32_t scheme, int32_t block, int32_t scale_mode,
                            void* stream);

/* ------------------------------------------------------------------------
 * Pivoted-Cholesky preconditioner (Sec. 5.2, "Preconditioning"; Eq. woodbury)
 * ------------------------------------------------------------------------ */
typedef struct gp_precond gp_precond; /* opaque, library-owned */

/*
 * gp_pivchol_precond -- rank-`rank` pivoted Cholesky factor L of a^2 K(X, X)
 * (greedy largest residual diagonal, lowest index on ties; stops early when
 * the largest residual diagonal is <= 1e-12 a^2) and the Woodbury form
 *   P^{-1} w = s^-2 w - s^-4 L (I + s^-2 L^T L)^{-1} L^T w.
 * The factor, the k x k inner matrix and its Cholesky inverse are float64 on
 * the device; a float32 copy of L serves the apply.
 *  X     n x d device points; only read during this call.
 *  rank  0 <= rank <= min(n, 128); 0 gives P^{-1} = s^-2 I.
 *  out   receives the handle; release it with gp_precond_destroy.
 * Synchronises `stream` before returning.  Errors: GP_ERR_ARG (arguments,
 * noise must be > 0), GP_ERR_NOMEM, GP_ERR_HIP, GP_ERR_NOT_PD (inner matrix
 * not positive definite).  An early stop is not an error: see gp_precond_info.
 */
gp_status gp_pivchol_precond(const gp_kernel* k, const float* X, int64_t n, int32_t d,
                             int32_t rank, gp_precond** out, void* stream);

/* Z = P^{-1} Rm for an n x r block (1 <= r <= 64); Rm, Z device, must not
 * overlap.  Asynchronous on `stream`; calls that share one handle must be
 * ordered on one stream (the handle holds the apply scratch).                */
gp_status gp_precond_apply(const gp_precond* P, const float* Rm, int32_t r, float* Z,
                           void* stream);

/* rank actually built, its pivots (HOST array of at least rank_used entries,
 * may be NULL) and trace(a^2 K - L L^T) = sum of the residual diagonal.      */
gp_status gp_precond_info(const gp_precond* P, int32_t* rank_used, int64_t* pivots,
                          double* trace_residual);

/* Release the handle (synchronises the device first).  NULL is a no-op.  Its
 * device memory (one block of about 12 n rank bytes plus ~34 MB of apply
 * partials) is kept by the library for the next handle of the same n and
 * rank on the same device, up to 4 GiB in total per process; beyond that it
 * is freed.  gp_release_cached_memory frees what is kept.                   */
gp_status gp_precond_destroy(gp_precond* P);

/* ------------------------------------------------------------------------
 * Conjugate-gradient solve of (a^2 K + s^2 I) U = B
 * ------------------------------------------------------------------------ */
#define GP_CG_STANDARD 0 /* App. A, Alg. 2 (preconditioned)                    */
#define GP_CG_ENHANCED 1 /* Sec. 5.2, Alg. 1: logsumexp step sizes, re-orth.   */

typedef struct gp_cg_opts {
  double tol;             /* per-column relative residual ||r_c|| / ||b_c||      */
  int32_t max_iter;       /* >= 0                                              */
  int32_t min_iter;       /* no column stops before this many iterations       */
  int32_t algo;           /* GP_CG_STANDARD or GP_CG_ENHANCED                  */
  int32_t reorth;         /* enhanced only: re-orthogonalise residuals         */
  int32_t use_lse;        /* enhanced only: log-scale step sizes               */
  int32_t precision;      /* kernel-matrix product: GP_PREC_FP32 / FP16 / BF16  */
  int32_t scale_mode;     /* FP16 and BF16, as in gp_kmvm                       */
  int32_t x0_given;       /* 1: U holds the initial guess x_0; 0: x_0 = 0      */
  int32_t true_res_every; /* < 0 never; 0 at exit; > 0 also after every that   */
                          /* many iterations (a host poll is forced there):    */
                          /* ||b - K~ u|| with float64 sums                    */
  int32_t poll_every;     /* iterations between host convergence polls (0=10) */
  const gp_precond* P;    /* NULL = no preconditioner; built on the same X     */
} gp_cg_opts;

/* Fill `o` with the defaults: tol 1.0, max_iter 100, min_iter 10, enhanced
 * with re-orthogonalisation and logsumexp, FP16 product, power-of-two scale,
 * x_0 = 0, true residual at exit, poll every 10 iterations, no preconditioner. */
void gp_cg_default_opts(gp_cg_opts* o);

typedef struct gp_cg_stats {
  /* HOST arrays of r entries, each may be NULL */
  int32_t* iters;          /* iterations each column ran                        */
  float* rel_res;          /* recursive relative residual at exit               */
  double* true_rel_res;    /* float64-accumulated ||b - K~ u|| / ||b|| (or -1)  */
  int8_t* converged;       /* reached tol: the recursive residual after min_iter
                              and, when the float64 true residual is computed at
                              exit, ||b - K~u|| / ||b|| <= GP_TRUE_RES_SLACK *
                              max(tol, GP_TRUE_RES_FLOOR) as well, so a solve
                              whose binary16 operator drifted from K~ (divergence)
                              cannot report convergence; a zero right-hand side
                              counts                                             */
  int8_t* breakdown;       /* a logsumexp argument or d^T K d was not > 0       */
  float* history;          /* HOST (max_iter + 1) x r relative residuals, or NULL */
  double* true_history;    /* gp_cg_solve with true_res_every = T > 0: HOST
                              (max_iter / T) x r, or NULL; row j holds the float64
                              true relative residual after (j + 1) T iterations
                              were launched (-1 where the solve ended earlier).
                              Not written by the batched and served solves.    */
  /* scalars written by the solver */
  int32_t total_iters;     /* iterations launched                                */
  int32_t mvms;            /* kernel-matrix products (excluding true residuals)  */
} gp_cg_stats;

/*
 * gp_cg_solve -- solve (a^2 K(X, X) + s^2 I) U = B column by column with one
 * step size per column (mBCG, App. A).
 *  X  n x d, B n x r, U n x r device arrays; 1 <= r <= 64, n >= 1.
 *  U  output; holds x_0 on entry when o->x0_given.
 *  o  options (NULL = gp_cg_default_opts); o->P must have been built for the
 *     same X and kernel.
 *  st statistics (may be NULL).
 * Each column freezes once ||r_c|| / ||b_c|| <= tol after min_iter
 * iterations, or when it breaks down; the solve ends when every column is
 * frozen or after max_iter iterations.  Returns GP_OK even if some columns did
 * not converge (see st); GP_ERR_BREAKDOWN if every column broke down.
 * Synchronises `stream` before returning.
 */
gp_status gp_cg_solve(const gp_kernel* k, const float* X, int64_t n, int32_t d, const float* B,
                      int32_t r, float* U, const gp_cg_opts* o, gp_cg_stats* st, void* stream);

/*
 * gp_true_residual_rows -- rows of the true residual of a solve, the check
 * the solver makes at exit (float32 kernel entries, every product and sum in
 * float64):
 *   res[t][c] = B[i][c] - (a^2 sum_j k(x_i, x_j) U[j][c] + s^2 U[i][c]),
 *   i = rows[t],
 * so that a problem too large for a float64 reference solve can be checked
 * row by row against an independent float64 product on sampled rows.
 *  X     n x d device points; B, U n x r device arrays (1 <= r <= 64)
 *  rows  nrows DEVICE int64 indices in [0, n) (repeats allowed)
 *  res   nrows x r DEVICE float64 output, must not overlap the inputs
 * Errors: GP_ERR_ARG (shapes, hyperparameters, an index outside [0, n),
 * found on the device and reported before the product runs; the call then
 * synchronises `stream`), GP_ERR_NOMEM, GP_ERR_HIP.  Otherwise asynchronous
 * on `stream` after that check.
 */
gp_status gp_true_residual_rows(const gp_kernel* k, const float* X, int64_t n, int32_t d,
                                const float* B, const float* U, int32_t r, const int64_t* rows,
                                int64_t nrows, double* res, void* stream);

/* ------------------------------------------------------------------------
 * Batched solves: many independent problems in one launch per step
 * ------------------------------------------------------------------------ */
typedef struct gp_problem {
  gp_kernel k;           /* per-problem kernel and hyperparameters               */
  const float* X;        /* n x d device points                                   */
  int64_t n;             /* >= 1                                                  */
  int32_t d;             /* 1 <= d <= 30                                          */
  const float* B;        /* n x r device right-hand sides                         */
  int32_t r;             /* 1 <= r <= 64                                          */
  float* U;              /* n x r device solution (x0 on entry if o->x0_given)    */
  int32_t precond_rank;  /* rank of the pivoted-Cholesky preconditioner, 0 = none */
} gp_problem;

/*
 * gp_cg_solve_batched -- solve nprob independent systems
 * (a_p^2 K_p + s_p^2 I) U_p = B_p (mBCG per problem, App. A) in one launch per
 * step for the whole batch: the binary16 fused product runs one work group per
 * (problem, row block, column split) item, longest first; every reduction is
 * per problem and merged in a fixed order, so each result is independent of
 * the other problems in the batch.  The iterations between host polls are
 * replayed from one captured HIP graph.
 *  o      options shared by all problems (NULL = defaults); o->precision must
 *         be GP_PREC_FP16 and o->P must be NULL (per-problem preconditioners
 *         are built from precond_rank, exactly as gp_pivchol_precond does).
 *  stats  NULL or an array of nprob gp_cg_stats (host arrays sized r_p).
 * Limits: 1 <= nprob <= 4096.  Synchronises `stream` before returning.
 * Returns GP_ERR_BREAKDOWN only if every column of every problem broke down.
 */
gp_status gp_cg_solve_batched(int32_t nprob, const gp_problem* probs, const gp_cg_opts* o,
                              gp_cg_stats* stats, void* stream);

/* ------------------------------------------------------------------------
 * Serving loop: many solves of different sizes sharing one GPU
 * ------------------------------------------------------------------------
 * A server owns one device, one HIP stream, a device arena of
 * hbm_budget_bytes and a host scheduler thread.  Each admitted request
 * occupies one slot: a contiguous region of the arena holding its points,
 * right-hand sides, iterate, CG vectors, basis and preconditioner, where its
 * whole CG state stays until it retires.  Between scheduling rounds the
 * scheduler admits queued requests (first come first served, while a slot
 * and arena space are free), builds their operands and preconditioners
 * together, then advances EVERY resident request by iters_per_round
 * iterations of the enhanced solve (the per-iteration launches of
 * gp_cg_solve_batched over the resident set), and retires requests whose
 * columns have all converged, broken down or reached max_iter: their true
 * residual is computed, the solution is copied to U_out and the slot's
 * region returns to the arena.  Each request computes exactly what
 * gp_cg_solve_batched computes for it alone (same reductions in the same
 * order), whatever else is resident.                                      */
typedef struct gp_serve_config {
  uint64_t hbm_budget_bytes;  /* arena size; a request larger is refused        */
  int32_t max_slots;          /* resident requests at most, 1..1024             */
  int32_t device;             /* HIP device ordinal                            */
  int32_t iters_per_round;    /* iterations between scheduling rounds (>= 1)   */
  int32_t min_iter;           /* as gp_cg_opts.min_iter                          */
  int32_t algo;               /* GP_CG_ENHANCED or GP_CG_STANDARD               */
  int32_t reorth;             /* enhanced only                                  */
  int32_t use_lse;            /* enhanced only                                  */
  int32_t scale_mode;         /* as gp_cg_opts.scale_mode                        */
} gp_serve_config;

/* Defaults: budget 8 GiB, 64 slots, device 0, 5 iterations per round,
 * min_iter 10, enhanced with re-orthogonalisation and logsumexp, scale 0. */
void gp_serve_default_config(gp_serve_config* c);

typedef struct gp_server gp_server;

/* One solve (a^2 K + s^2 I) U = B.  X, B and U_out are HOST arrays that the
 * caller keeps alive and unchanged until gp_serve_poll / gp_serve_wait
 * report something other than GP_PENDING; the server copies X and B to the
 * device when it admits the request and writes U_out (and stats, if not
 * NULL) before it reports completion.                                      */
typedef struct gp_request {
  gp_kernel k;
  const float* X;        /* n x d host points                                */
  int64_t n;             /* >= 1                                             */
  int32_t d;             /* 1..30                                            */
  const float* B;        /* n x r host right-hand sides                      */
  int32_t r;             /* 1..64                                            */
  float* U_out;          /* n x r host solution                              */
  double tol;            /* relative residual tolerance per column (>= 0)   */
  int32_t max_iter;      /* >= 0                                             */
  int32_t precond_rank;  /* 0..min(n, 128)                                   */
  gp_cg_stats* stats;    /* NULL or host arrays sized r                      */
} gp_request;

typedef struct gp_result {
  gp_status status;      /* GP_OK, GP_ERR_BREAKDOWN (every column broke down),
                            GP_ERR_NOT_PD, GP_ERR_CANCELLED, GP_ERR_HIP ...   */
  int32_t iters;         /* iterations run                                   */
  int32_t converged;     /* columns that met tol                             */
  int32_t breakdown;     /* columns that broke down                          */
  double max_rel_res;    /* largest recurrence relative residual             */
  double max_true_rel_res; /* largest float64 ||b - K~u|| / ||b||           */
  double t_submit;       /* seconds since the server was created            */
  double t_admit;
  double t_finish;
  uint64_t footprint_bytes; /* arena bytes the request occupied              */
  char message[128];     /* error text when status is an error               */
} gp_result;

typedef struct gp_serve_stats {
  int32_t queued;
  int32_t resident;
  int64_t submitted;
  int64_t completed;
  int64_t rounds;
  int64_t iterations;     /* sum over rounds of iterations x resident slots  */
  uint64_t bytes_in_use;
  uint64_t peak_bytes;
  double busy_seconds;    /* wall time the scheduler spent with work resident */
  double uptime_seconds;
} gp_serve_stats;

/* Create a server (allocates the arena on c->device, starts the scheduler).
 * Errors: GP_ERR_ARG, GP_ERR_NOMEM, GP_ERR_HIP.                            */
gp_status gp_serve_create(const gp_serve_config* c, gp_server** out);

/* Queue a request; thread-safe.  *ticket identifies it in poll / wait /
 * cancel.  Errors (nothing queued): GP_ERR_ARG, GP_ERR_TOO_LARGE (footprint
 * above the arena), GP_ERR_STOPPED (server failed or being destroyed).     */
gp_status gp_serve_submit(gp_server* s, const gp_request* q, uint64_t* ticket);

/* GP_PENDING while queued or resident; otherwise the request's final status,
 * *res filled, and the ticket is released (a later poll returns
 * GP_ERR_UNKNOWN_TICKET).  Thread-safe; never blocks on the GPU.          */
gp_status gp_serve_poll(gp_server* s, uint64_t ticket, gp_result* res);

/* As poll, but waits up to timeout_ms (< 0: no limit) for completion.      */
gp_status gp_serve_wait(gp_server* s, uint64_t ticket, int64_t timeout_ms, gp_result* res);

/* Cancel a queued or resident request: it completes with GP_ERR_CANCELLED
 * (at the next round boundary if resident) and U_out is not written.
 * GP_ERR_UNKNOWN_TICKET if the ticket is not pending.                     */
gp_status gp_serve_cancel(gp_server* s, uint64_t ticket);

gp_status gp_serve_stats_read(gp_server* s, gp_serve_stats* out);

/* Cancel everything pending, stop the scheduler, free the arena.          */
gp_status gp_serve_destroy(gp_server* s);

/* ------------------------------------------------------------------------
 * Predictive means with a cached solve (Sec. 4.1, the predictive-mean cache
 * v = K~^{-1} y and mu = K(x*, X) v) and their serving
 * ------------------------------------------------------------------------ */
typedef struct gp_model gp_model; /* opaque, library-owned, bound to a device */

typedef struct gp_model_info {
  int64_t n;
  int32_t d;
  int32_t iters;          /* iterations of the cache solve                    */
  int32_t converged;      /* the cache solve met its tolerance                */
  float rel_res;          /* its recursive relative residual                  */
  double true_rel_res;    /* its float64 ||y - K~ v|| / ||y|| (-1 if not run) */
} gp_model_info;

/* Options of the cache solve: gp_cg_default_opts with tol 1e-2, at most 1000
 * iterations and the float64 true residual at exit.                         */
void gp_model_default_opts(gp_cg_opts* o);

/*
 * gp_model_create -- copy X (n x d, device) and solve (a^2 K + s^2 I) v = y
 * (y: n device values) once with gp_cg_solve (o: NULL = gp_model_default_opts;
 * o->P must be NULL, a rank-precond_rank pivoted-Cholesky preconditioner is
 * built when precond_rank > 0).  The model keeps X and v on the current device.
 * Synchronises `stream`.  Errors: as gp_cg_solve and gp_pivchol_precond.
 */
gp_status gp_model_create(const gp_kernel* k, const float* X, int64_t n, int32_t d, const float* y,
                          const gp_cg_opts* o, int32_t precond_rank, void* stream,
                          gp_model** out);

/*
 * gp_model_predict -- mu[i] = a^2 sum_j k(x*_i, x_j) v_j for ns test points Xs
 * (ns x d, device; mu: ns device values), with the binary16 product
 * (precision FP16), the bfloat16 one (BF16) or the float32 one (FP32);
 * truncate = 1 (FP16 only) uses
 * gp_kmvm_truncated, whose result is the same binary16 product.  Asynchronous
 * on `stream`.  Errors: GP_ERR_ARG, GP_ERR_NOMEM, GP_ERR_HIP.
 */
gp_status gp_model_predict(const gp_model* m, const float* Xs, int64_t ns, float* mu,
                           int32_t precision, int32_t truncate, void* stream);

gp_status gp_model_info_read(const gp_model* m, gp_model_info* out);
/* Copy the cached v (n device values) into v_out; asynchronous on `stream`. */
gp_status gp_model_weights(const gp_model* m, float* v_out, void* stream);
/* Device the model lives on (-1 for NULL). */
int32_t gp_model_device(const gp_model* m);
/* Release the model (synchronises the device first).  NULL is a no-op.       */
gp_status gp_model_destroy(gp_model* m);

/*
 * Prediction requests to a server: the second request type of the serving
 * loop.  A prediction needs no slot or arena space; the server's prediction
 * thread runs the queued predictions in arrival order on its own stream
 * (host copy in, binary16 product against the model's cache, copy out),
 * concurrently with the solve rounds.  Its gp_result carries status, the
 * timestamps and iters = 0; busy_seconds in gp_serve_stats counts solve
 * rounds only.  The model must live on the server's device
 * and stay alive until the request completes; Xs and mu_out are HOST arrays
 * that must stay valid until then.
 */
typedef struct gp_predict_request {
  const gp_model* model;
  const float* Xs;        /* ns x d HOST test points                          */
  int64_t ns;             /* >= 1                                             */
  float* mu_out;          /* ns HOST predictive means                         */
  int32_t truncate;       /* 1: over the finite binary16 support             */
} gp_predict_request;

gp_status gp_serve_submit_predict(gp_server* s, const gp_predict_request* q, uint64_t* ticket);

/* ------------------------------------------------------------------------
 * Autotuner of the binary16 product's launch shape
 * ------------------------------------------------------------------------
 * Decisions (all change only the order of float32 partial sums, never what is
 * computed): column splits of the single-problem product per row-count
 * bucket (bucket b covers padded row counts from 4096 * 2^b), the per-problem
 * split rule of batched products (splits = clamp(stages / div, 1, 8), one
 * stage = 128 columns) and their launch form (one work group per work item,
 * or one persistent launch pulling items from an atomic counter).  Until
 * gp_autotune runs, built-in rules apply.  GPMI_TUNE_CACHE (environment) may
 * name a file: the table is loaded from it at first use and written by
 * gp_autotune.                                                             */
#define GP_TUNE_BUCKETS 8
typedef struct gp_tune_info {
  int32_t tuned;                            /* 1 after gp_autotune          */
  int32_t f16_splits[GP_TUNE_BUCKETS];      /* 0: built-in rule             */
  int64_t f16_bucket_rows[GP_TUNE_BUCKETS];
  double f16_gain[GP_TUNE_BUCKETS];         /* built-in time / tuned time   */
  int32_t batched_split_div;
  int32_t batched_persistent;
  double batched_gain;
} gp_tune_info;

/* Measure on the current device with synthetic operands (buckets 0..max_bucket
 * of the single-problem product, RBF, d = 8, 16 right-hand sides; a batch of
 * 48 problems with N from 500 to 20000, 8 iterations) and install the fastest
 * choices for this process.  Synchronises `stream`.  *out may be NULL.     */
gp_status gp_autotune(int32_t max_bucket, void* stream, gp_tune_info* out);
gp_status gp_tune_get(gp_tune_info* out);
/* Back to the built-in rules (the cache file is not read again). */
gp_status gp_tune_reset(void);
/* Install decisions made elsewhere (e.g. a previous gp_autotune): the split,
 * split-rule and launch-form fields of *in (f16_splits entries 0 = built-in
 * rule, otherwise 1..64; batched_split_div 1..1024).  GP_ERR_ARG on values
 * out of range.                                                            */
gp_status gp_tune_set(const gp_tune_info* in);

/* ------------------------------------------------------------------------
 * Hyperparameter training (Sec. 2.2 Eq. loss / gradient; Sec. 5.3 Eq. cg,
 * approx_loss, approx; App. C priors and optimiser)
 * ------------------------------------------------------------------------
 * Parameters theta are ordered (l_1..l_L, a^2, s^2), L = d with ARD, else 1.
 * At most GP_TRAIN_MAX_PARAMS entries (d <= 32 for training).              */
#define GP_TRAIN_MAX_DIM 32
#define GP_TRAIN_MAX_PARAMS (GP_TRAIN_MAX_DIM + 2)

/*
 * gp_mll_grad -- the gradient estimate of Eq. (approx) from one solve of
 * Eq. (cg):  dL/dtheta ~ 1/(2M) sum_j u_j^T dK~ z_j - 1/2 u_0^T dK~ u_0.
 *  X     n x d device points (1 <= d <= 32)
 *  B     n x r device right-hand sides [y, z_1..z_M] (r = M + 1, 2 <= r <= 64)
 *  U     n x r device solutions K~^{-1} B (e.g. from gp_cg_solve)
 *  row_begin, row_end   keep only the terms whose left index i lies in
 *        [row_begin, row_end) (0 and n for the whole gradient; a partition of
 *        the rows adds up to it, which is how the sum shards)
 *  grad  HOST array of L + 3 doubles: dL/dl_1..dL/dl_L, dL/da^2, dL/ds^2 and,
 *        last, 1/2 y^T u_0 over the row range (the data-fit half of Eq. loss).
 * The kernel's entries are float32 (no binary16 rounding); every sum is
 * combined in float64 in a fixed order, so results are deterministic.
 * Synchronises `stream`.  Errors: GP_ERR_ARG, GP_ERR_NOMEM, GP_ERR_HIP.
 */
gp_status gp_mll_grad(const gp_kernel* k, const float* X, int64_t n, int32_t d, const float* B,
                      const float* U, int32_t r, int64_t row_begin, int64_t row_end,
                      double* grad, void* stream);

/*
 * gp_rademacher -- probe vectors: out[i * ld + c] = +1 or -1 for i < rows,
 * c < cols, from value k = first + i * cols + c of the SplitMix64 stream
 * seeded with `seed` (Steele, Lea & Flood 2014): z = mix(seed + (k + 1) *
 * 0x9E3779B97F4A7C15), +1 when the top bit of z is 0.  Device `out`, ld >= cols.
 * Asynchronous on `stream`.
 */
gp_status gp_rademacher(uint64_t seed, uint64_t first, int64_t rows, int32_t cols, float* out,
                        int64_t ld, void* stream);

typedef struct gp_trainer gp_trainer; /* opaque */

typedef struct gp_train_config {
  int32_t kind;          /* GP_KERNEL_*                                         */
  int32_t ard;           /* 1: one lengthscale per input dimension              */
  int32_t probes;        /* M Rademacher probes per step, 1..63                 */
  int32_t precond_rank;  /* pivoted-Cholesky rank rebuilt every step, 0..128    */
  int32_t use_priors;    /* 1: Gamma(3, 6) on each l, Gamma(2, 0.15) on a^2,
                            Gamma(1.1, 0.05) on s^2 (rate parametrisation)     */
  int32_t pad_;
  double lr;             /* Adam step size                                      */
  double beta1, beta2, eps;
  uint64_t seed;         /* probe stream                                        */
  gp_cg_opts cg;         /* solve options; cg.P and cg.x0_given are ignored    */
} gp_train_config;

/* Defaults: RBF with ARD, 15 probes, rank 100, priors on, Adam 0.1 / 0.9 /
 * 0.999 / 1e-8, seed 0, CG tolerance 1.0 with at most 50 and at least 10
 * iterations, binary16 product, no true residual.                           */
void gp_train_default_config(gp_train_config* c);

/*
 * gp_trainer_create -- a trainer owning copies of X (n x d) and y (n) (device
 * arrays, read during this call only), the [y, probes] and solution blocks,
 * and the optimiser state on the device.  theta0 (HOST, L + 2 values) gives
 * the starting hyperparameters; NULL starts at l = a^2 = log 2 (raw value 0)
 * and s^2 = 2.  The positive parameters are optimised through raw values:
 * l = softplus(raw), a^2 = softplus(raw), s^2 = 1e-4 + softplus(raw).
 * The objective is (L(theta) - sum of log priors) / n.  All later calls run
 * on `stream`.  Errors: GP_ERR_ARG, GP_ERR_NOMEM, GP_ERR_HIP.
 */
gp_status gp_trainer_create(const gp_train_config* c, const float* X, const float* y, int64_t n,
                            int32_t d, const double* theta0, void* stream, gp_trainer** out);

typedef struct gp_train_step_info {
  int32_t step;                         /* 1 for the first step               */
  int32_t cg_iters;                     /* iterations of this step's solve    */
  int32_t cg_converged;                 /* columns that met cg.tol            */
  int32_t precond_rank;                 /* rank built                         */
  double max_rel_res;                   /* largest recursive relative residual */
  double theta[GP_TRAIN_MAX_PARAMS];    /* hyperparameters the step used      */
  double grad[GP_TRAIN_MAX_PARAMS];     /* dL/dtheta estimate (Eq. approx)    */
  double raw_grad[GP_TRAIN_MAX_PARAMS]; /* gradient of the objective in raw values */
  double theta_next[GP_TRAIN_MAX_PARAMS]; /* after the Adam update            */
  double data_fit;                      /* 1/2 y^T u_0                        */
  double seconds_precond, seconds_solve, seconds_grad;  /* wall time per phase */
} gp_train_step_info;

/* One training step: draw the probes of this step (counter
 * first = (step - 1) * n * M of gp_rademacher), build the preconditioner,
 * solve K~ U = [y, Z] with mBCG, estimate the gradient (gp_mll_grad), update
 * the raw values with Adam on the device.  Synchronises the stream.
 * Errors: as gp_pivchol_precond and gp_cg_solve; the state is unchanged
 * when the step fails.                                                      */
gp_status gp_trainer_step(gp_trainer* t, gp_train_step_info* info);

/* Optimiser state, for inspection, checkpoints and resumption. */
typedef struct gp_train_state {
  int32_t nparams;                      /* L + 2                              */
  int32_t step;                         /* steps taken                        */
  double raw[GP_TRAIN_MAX_PARAMS];
  double m[GP_TRAIN_MAX_PARAMS];        /* Adam first moment                  */
  double v[GP_TRAIN_MAX_PARAMS];        /* Adam second moment                 */
  double theta[GP_TRAIN_MAX_PARAMS];    /* constrained values of raw (read only) */
} gp_train_state;
gp_status gp_trainer_get_state(gp_trainer* t, gp_train_state* out);
/* Install raw, m, v and step (theta is recomputed); nparams must match.     */
gp_status gp_trainer_set_state(gp_trainer* t, const gp_train_state* in);
/* Copy the last step's n x (M + 1) blocks [y, Z] and U = K~^{-1}[y, Z] into
 * device arrays B_out and U_out (each may be NULL); GP_ERR_ARG before the
 * first step.  Synchronises the trainer's stream.                           */
gp_status gp_trainer_blocks(gp_trainer* t, float* B_out, float* U_out);
gp_status gp_trainer_destroy(gp_trainer* t);

/* ------------------------------------------------------------------------
 * Launch timing of the fused kernel-matrix product (measurement support)
 * ------------------------------------------------------------------------ */
/* When on, every launch of the fused product kernel (from gp_kmvm and
 * gp_cg_solve) is bracketed by HIP events on the stream it runs on.          */
gp_status gp_profile_enable(int32_t on);

/* Copy up to max_records launch records (HOST arrays, each may be NULL):
 * duration in ms, logical entries n1*n2, kernel kind; *count receives the
 * number recorded.  Waits for the recorded events.  A launch enqueued after a
 * solve's columns all froze exits at once and shows a near-zero duration.   */
gp_status gp_profile_read(int64_t max_records, float* ms, double* entries, int32_t* kinds,
                          int64_t* count);

/* Drop all records.                                                         */
gp_status gp_profile_reset(void);

/* Issue-rate and bandwidth probes of the current device (the peaks the
 * benchmark's roofline fractions are stated against).  Each runs one loop of
 * a single instruction kind (independent dependency chains, 8 work groups of
 * 256 threads per compute unit; the copy: `iters` passes over 1 GiB) once to
 * warm up and once timed with HIP events on `stream`, and writes *rate:
 *   GP_PROBE_EXP, GP_PROBE_SQRT, GP_PROBE_FMA   lane operations per second of
 *       v_exp_f32, v_sqrt_f32, v_fma_f32 (packed FP32 is disabled in the build)
 *   GP_PROBE_MFMA_F16_32, GP_PROBE_MFMA_F16_16, GP_PROBE_MFMA_F64   FLOP/s of
 *       v_mfma_f32_16x16x32_f16, v_mfma_f32_16x16x16_f16, v_mfma_f64_16x16x4_f64
 *   GP_PROBE_COPY   bytes read plus written per second by a device copy
 *   GP_PROBE_MIX_FMA, GP_PROBE_MIX_EXP   MFMA FLOP/s of a loop that issues,
 *       per iteration, four independent v_mfma_f32_16x16x32_f16 next to an
 *       independent vector stream (16 v_fma_f32 or 8 v_exp_f32 per lane):
 *       compared with the single-kind rates it shows how far the two overlap
 * Adding GP_PROBE_TWO_WAVES to a loop probe's kind runs it with 2 work groups
 * per compute unit (2 waves per SIMD) instead of 8.
 * 1 <= iters <= 2^24.  Allocates and frees its own small buffers (2 GiB for
 * the copy) and synchronises `stream`.  Errors: GP_ERR_ARG (unknown kind,
 * GP_PROBE_TWO_WAVES with the copy, iters out of range), GP_ERR_NOMEM,
 * GP_ERR_HIP.                                                              */
#define GP_PROBE_EXP 0
#define GP_PROBE_SQRT 1
#define GP_PROBE_FMA 2
#define GP_PROBE_MFMA_F16_32 3
#define GP_PROBE_MFMA_F16_16 4
#define GP_PROBE_MFMA_F64 5
#define GP_PROBE_COPY 6
#define GP_PROBE_MIX_FMA 7
#define GP_PROBE_MIX_EXP 8
#define GP_PROBE_TWO_WAVES 256
gp_status gp_probe_rate(int32_t which, int64_t iters, void* stream, double* rate);

#ifdef __cplusplus
}
#endif

#endif /* GPMI_H */
