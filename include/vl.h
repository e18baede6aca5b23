/*
 * vl.h -- C ABI of the MI355X (gfx950) library for iterative Vecchia-Laplace
 * inference in latent Gaussian process models.
 *
 * The operations follow Kuendig & Sigrist, "Iterative Methods for
 * Vecchia-Laplace Approximations for Latent Gaussian Process Models"
 * (arXiv 2310.12000):
 *   - Vecchia factor B, D of the prior precision B^T D^{-1} B   (Sec. 2.1)
 *   - Newton mode finding with preconditioned CG                (Sec. 2.2,
 *     eq. newton; Sec. 3, eqs. pcls1 / pcls2; appendix CG algorithm)
 *   - SLQ negative log-marginal likelihood and STE gradient     (eq. VLA_loss,
 *     eqs. logdetsplit / logdetsplit2 / def_SLQ / grad_STE; App. A.3, A.4)
 *   - VADU, LRAC, LVA and diagonal (P_1) preconditioners        (Sec. 3.1.1,
 *     Sec. 3.1.2, Sec. 3.1.4)
 *   - predictive means and simulated variances                  (Sec. 2.2.1,
 *     eq. latentpostpredictive; Sec. 3.3.1, Alg. simAlgo)
 *
 * Conventions (all entry points):
 *   - Arrays marked "device" are device pointers on the GPU the model was
 *     built on, addressed in the caller's point order (row i = i-th location
 *     of the ordering).  Arrays marked "host" are ordinary host memory.
 *   - Floating point is IEEE FP64, matrices row-major (n x t means element
 *     (i, c) at i * t + c).
 *   - The caller owns every input and output buffer; the library never frees
 *     them and never keeps a pointer to them after the call returns, except
 *     for the stream passed to vl_build_vecchia.
 *   - The model handle owns its device state (coordinates, neighbour sets,
 *     B, B^T, D, derivatives, mode, W, workspaces) until vl_free.
 *   - Work is enqueued on the model's HIP stream.  Calls that return host
 *     scalars (nll, gradient, statistics) synchronise that stream; other
 *     calls return once their work is enqueued, unless stated otherwise.
 *   - One model must not be used from two host threads at once.  Distinct
 *     models may be used concurrently (each with its own stream).
 *   - Every call returns a vl_status and never aborts the process.  On an
 *     error the outputs are unspecified unless stated otherwise;
 *     vl_last_error() gives a message.
 */
#ifndef VL_H
#define VL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vl_model vl_model;

typedef enum {
  VL_OK = 0,
  VL_ERR_INVALID_ARG = -1,    /* bad size, null pointer, unknown enum       */
  VL_ERR_NOT_SPD = -2,        /* a neighbour covariance is not positive
                                 definite (e.g. duplicate locations)        */
  VL_ERR_NO_CONVERGENCE = -3, /* a CG or Newton loop hit its cap; outputs
                                 are written and flagged in vl_stats        */
  VL_ERR_OOM = -4,            /* device allocation failed                   */
  VL_ERR_NONFINITE = -5,      /* NaN/Inf in inputs or intermediate results  */
  VL_ERR_HIP = -6,            /* a HIP runtime call failed                  */
  VL_ERR_STATE = -7,          /* call order violated (e.g. no mode yet)     */
  VL_ERR_TIMEOUT = -8         /* a device-side wait exceeded its bound      */
} vl_status;

typedef enum { VL_COV_EXPONENTIAL = 0, VL_COV_MATERN32 = 1 } vl_cov;

typedef enum {
  VL_LIK_BERNOULLI_LOGIT = 0, /* y in {0,1}, mu = logit P(y = 1)            */
  VL_LIK_POISSON_LOG = 1,     /* y in {0,1,2,...}, mu = log E[y]            */
  VL_LIK_GAUSSIAN = 2,        /* y real, aux[0] = noise variance tau^2      */
  VL_LIK_GAMMA = 3            /* y > 0, mu = log E[y], aux[0] = shape a > 0 */
} vl_lik;

typedef enum {
  VL_PREC_VADU = 0, /* B^T (W + D^{-1}) B (Sec. 3.1.1)                          */
  VL_PREC_LRAC = 1, /* L_k L_k^T + W^{-1} (Sec. 3.1.2)                          */
  VL_PREC_LVA = 2,  /* B^T D^{-1} B (Sec. 3.1.1); mode and likelihood only        */
  VL_PREC_DIAG = 3  /* P_1 = diag(W + B^T D^{-1} B) (Sec. 3.1.4); mode and
                       likelihood only                                          */
} vl_precond;
typedef enum { VL_FP64 = 0, VL_MIXED = 1 } vl_precision;

/* Predictive-variance method of vl_predict (Sec. 3.3): simulation (Alg.
 * simAlgo, s = num_pred_samples) or rank-k preconditioned Lanczos with
 * complete reorthogonalization (Sec. 3.3.2, k = lanczos_rank) with P_L1 =
 * B^T (W + D^{-1}) B or P_L2 = diag(sigma^2 + 1/W) on Sigma~ + W^{-1} (the
 * original covariance's diagonal sigma^2 stands in for diag Sigma~). */
typedef enum {
  VL_PRED_SIMULATION = 0,
  VL_PRED_LANCZOS_L1 = 1,
  VL_PRED_LANCZOS_L2 = 2
} vl_pred_method;

/* Options.  vl_default_opts fills the paper's defaults (Sec. 4.1): t = 50
 * probes, LRAC rank k = 50, CG tolerance 1e-2 for likelihoods and 1e-3 for
 * predictive variances, s = 2000 simulation samples. */
typedef struct {
  int max_newton;          /* Newton iteration cap (default 100)               */
  double newton_tol;       /* stop when |Psi_new - Psi_old| <= tol |Psi_old|   */
  int max_cg;              /* CG iteration cap per solve (default 1000)        */
  double cg_tol;           /* absolute tolerance on ||r||_2, likelihood solves */
  double pred_cg_tol;      /* absolute tolerance on ||r||_2, variance solves   */
  int num_probes;          /* t, Rademacher probes for SLQ / STE               */
  int num_pred_samples;    /* s, simulation samples for predictive variances   */
  uint64_t seed;           /* probe seed (counter-based SplitMix64)            */
  int precond;             /* vl_precond                                       */
  int lrac_rank;           /* k of the LRAC preconditioner                     */
  int precision;           /* vl_precision; VL_MIXED runs the preconditioner
                              solves of the block solves (SLQ, prediction) with
                              FP32 n x t blocks and FP64 sums inside the FP64
                              PCG (FP32 B values above 64 columns); Newton
                              stays FP64                                       */
  int pred_tile;           /* columns per predictive-variance CG block
                              (0 = all s at once)                              */
  const int* replay_cg_iters; /* host, nullable: fixed CG iteration counts that
                              replace the tolerance test (replay of another
                              run's counts, e.g. a reference implementation's):
                              vl_find_mode: entry k for the solve of Newton
                              iteration k; vl_neg_log_marglik: entries 0..t-1
                              for the probe columns, entry t for the implicit
                              gradient term's solve; vl_predict: entry c for
                              sample column c.  Entries past replay_len, and
                              negative entries, keep the tolerance test; the
                              max_cg cap always applies                     */
  int replay_len;          /* number of entries of replay_cg_iters            */
  int pred_method;         /* vl_pred_method (default simulation)             */
  int lanczos_rank;        /* k of the Lanczos variances, 1..min(n, 4096)
                              (default 100); FP64 in every precision form     */
} vl_opts;

/* Per-call statistics (host struct, filled by the call that receives it). */
typedef struct {
  int newton_iters;        /* Newton iterations of the last vl_find_mode       */
  int cg_iters_total;      /* CG iterations summed over solves (per column for
                              block solves: the maximum over columns)          */
  int cg_iters_max;        /* largest iteration count of one column            */
  int hit_cap;             /* 1 if a loop stopped at its cap                   */
  double t_ms;             /* wall time of the call                            */
  double t_build_us;       /* wall time of the model's latest factor build
                              (vl_build_vecchia or vl_set_theta)               */
  double t_mode_us;        /* ... of its latest vl_find_mode                   */
  double t_slq_us;         /* ... of its latest vl_neg_log_marglik             */
  double t_pred_us;        /* ... of its latest vl_predict (0 = none yet)      */
  double err_vs_fp64_est;  /* VL_MIXED block solves: relative 2-norm deviation
                              of the FP32 preconditioner application from the
                              FP64 one on the call's first right-hand side
                              (the CG iterates and stopping test are FP64, so
                              this is the perturbation the FP32 solves add to
                              the Lanczos coefficients); 0 for FP64 calls     */
} vl_stats;

/* ---------------------------------------------------------------------- */
/* Device memory of the library.  Every device buffer a model, batch or
 * server owns (its state and the temporaries of a call) is obtained from
 * the allocator installed here; by default the library uses the
 * stream-ordered hipMallocAsync / hipFreeAsync.
 *   alloc(bytes, stream, ctx)  returns a device pointer (NULL = out of
 *                              memory: the call fails with VL_ERR_OOM);
 *                              `stream` is the hipStream_t of the call
 *                              (the model's stream) on which the memory
 *                              will be used
 *   release(ptr, stream, ctx)  frees a pointer alloc returned; work on
 *                              `stream` that used it may still be pending,
 *                              so the allocator must order its reuse after
 *                              that stream's work (a caching allocator that
 *                              reuses a block only on its own stream does)
 * Both NULL restores the default; exactly one NULL is VL_ERR_INVALID_ARG.
 * A pointer is always released through the allocator that produced it,
 * also when another one was installed in between.  The functions may be
 * called from any host thread the library runs on (serving workers
 * included) and must be thread-safe.  Installing is thread-safe; buffers
 * already allocated are unaffected. */
typedef void* (*vl_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*vl_free_fn)(void* ptr, void* stream, void* ctx);
vl_status vl_set_allocator(vl_alloc_fn alloc, vl_free_fn release, void* ctx);

void vl_default_opts(vl_opts* o);
const char* vl_status_string(vl_status s);
/* Message of the most recent failing call on this host thread. */
const char* vl_last_error(void);

/* Build the Vecchia approximation of the prior (Sec. 2.1).
 *   coords     device, n x 2 locations in the ordering of the approximation
 *              (the row order IS the ordering; the paper's random ordering
 *              is the caller's order of i.i.d. locations, Sec. 4.1)
 *   n          number of locations, 1 <= n <= 262144 (VL_ERR_INVALID above:
 *              a build at n = 2,000,000 ended in a GPU memory fault whose
 *              cause is not found; the largest size run on the GPU is
 *              n = 200,000, and the limit sits below every size at which
 *              the build's launch shapes or transfer sizes change from
 *              the verified ones)
 *   m          neighbours per point, 0 <= m <= 31; N(i) = the min(i, m)
 *              nearest among locations 0..i-1 (ties: smaller index first)
 *   cov        vl_cov; theta_host = {sigma2 > 0, range rho > 0} (host)
 *   hip_stream hipStream_t to enqueue on (NULL = default stream)
 *   want_deriv nonzero: also keep dB/dtheta, dD/dtheta (App. derivatives of
 *              the Vecchia-approximated precision) for vl_neg_log_marglik's
 *              gradient
 *   out        receives the handle
 * Runs neighbour search, the batched neighbour Cholesky (A_i, D_i), and the
 * transpose B^T.  Synchronises the stream.  VL_ERR_NOT_SPD if some D_i <= 0
 * or a neighbour covariance fails its Cholesky.
 * Device memory per model beyond the arrays above: the inverse of B's
 * leading min(n, 4096) rows in two orientations (268 MB at n >= 4096), the
 * grouped B / B^T of the 32..64-column products (about 1.1 KB per location)
 * and the level schedules.  Two environment variables, read at build time,
 * tune the triangular solves: VL_HEAD_ROWS (rows solved in LDS per column,
 * default 12288) and VL_DENSE_ROWS (leading rows solved with the dense
 * inverse, default 4096, 0 to disable); neither changes results beyond
 * rounding. */
vl_status vl_build_vecchia(const double* coords, int64_t n, int m, int cov,
                           const double* theta_host, void* hip_stream,
                           int want_deriv, vl_model** out);

/* Recompute A_i, D_i (and derivatives if built with them) at a new theta,
 * reusing neighbour sets and B^T structure.  Invalidates the mode. */
vl_status vl_set_theta(vl_model* h, const double* theta_host);

/* Newton mode finding (eq. newton) from b = 0, each step halved (at most 30
 * times) while Psi(b) = log p(y|F+b) - b^T Sigma~^{-1} b / 2 falls below
 * Psi_old - 1e-12 |Psi_old| (a decrease beyond rounding);
 * stops when |Psi_new - Psi_old| <= o->newton_tol |Psi_old| or when no halving
 * increases Psi (b is kept).  With o->precond = VL_PREC_VADU, VL_PREC_LVA or
 * VL_PREC_DIAG each step solves (W + Sigma~^{-1}) b' = W b + g by CG
 * preconditioned with P_VADU, P_LVA or P_1 (eq. pcls1); with VL_PREC_LRAC it
 * solves (Sigma~ + W^{-1}) (W b') =
 * Sigma~ (W b + g) (eq. pcls2) preconditioned with P_LRAC = L_k L_k^T + W^{-1}
 * (Sec. 3.1.2), L_k the rank-o->lrac_rank pivoted Cholesky factor of Sigma,
 * built once per theta.
 *   y        device, n responses
 *   F        device, n offsets F(X) (NULL = 0)
 *   lik      vl_lik; aux_host: likelihood auxiliary parameters (host;
 *            Gaussian: {tau2}; Gamma: {shape}; may be NULL otherwise)
 *   mode_out device, n (NULL = keep it only inside the model)
 * Keeps y, F, b*, W(b*) in the model for the calls below.  Synchronises. */
vl_status vl_find_mode(vl_model* h, const double* y, const double* F, int lik,
                       const double* aux_host, const vl_opts* o,
                       double* mode_out, vl_stats* st);

/* SLQ negative log-marginal likelihood at the stored mode (eq. VLA_loss).
 *   nll_host        host, 1 double
 *   grad_theta_host host, 2 doubles d/d(sigma2, rho) (NULL = skip; needs
 *                   want_deriv at build and the VADU or the LRAC
 *                   preconditioner: the STE formulas of App. A.4.1 / A.4.2,
 *                   LRAC with the derivative of the pivoted Cholesky factor
 *                   at fixed pivots, k <= 128)
 * VADU: eq. (logdetsplit) with probes z = B^T (W + D^{-1})^{1/2} eps and
 * log det P = sum log(W + D^{-1}); LVA: z = B^T D^{-1/2} eps, log det P =
 * -sum log D; P_1: z = P_1^{1/2} eps, log det P = sum log (P_1)_ii; LRAC:
 * eq. (logdetsplit2) with z = L_k eps_k + W^{-1/2} eps_n, weight r0^T z0.
 * The mixed form leaves P_1 (no triangular solves) in FP64.
 * Synchronises. */
vl_status vl_neg_log_marglik(vl_model* h, const vl_opts* o, double* nll_host,
                             double* grad_theta_host, vl_stats* st);

/* Estimation of theta = (sigma2, rho) (Sec. 4.1): minimises the negative
 * log-marginal likelihood over log theta by L-BFGS (two-loop recursion,
 * history 10, backtracking Armijo line search) with a sample average
 * approximation: every evaluation uses the probes of o->seed, so the
 * objective is deterministic.  Each evaluation runs vl_set_theta,
 * vl_find_mode from b = 0 and vl_neg_log_marglik with the gradient (VADU or LRAC;
 * the model must have been built with want_deriv).
 *   theta_inout host, 2: start, then the estimate
 *   max_iter    L-BFGS iterations at most; grad_tol: stop when every
 *               component of the gradient in log theta is at most this
 *   nll_host, iters_host, evals_host (host, nullable): the objective at the
 *               estimate, the iterations and the likelihood evaluations used
 * Leaves the model at the estimate (mode and likelihood state of the last
 * evaluation).  VL_ERR_NO_CONVERGENCE when max_iter was reached (theta_inout
 * holds the last iterate).  Synchronises. */
vl_status vl_estimate(vl_model* h, const double* y, const double* F, int lik,
                      const double* aux_host, const vl_opts* o, double* theta_inout,
                      int max_iter, double grad_tol, double* nll_host, int* iters_host,
                      int* evals_host);

/* Joint estimation (Sec. 5: shape, covariance parameters and beta; Sec.
 * 4.1's L-BFGS with a sample average approximation, as vl_estimate) of
 * theta, the likelihood's auxiliary parameter xi (VL_LIK_GAUSSIAN: tau^2,
 * VL_LIK_GAMMA: shape; none for the others) and beta of F = X beta.  The
 * search runs on (log sigma2, log rho, [log xi], beta) with the gradient
 * from vl_neg_log_marglik, vl_grad_aux and vl_grad_beta.
 *   X            device, n x p row-major (NULL when p = 0: F = 0)
 *   params_inout host, 2 + r + p with r = 1 for a likelihood with xi, else
 *                0: {sigma2, rho, [xi], beta_0 .. beta_{p-1}}, start, then
 *                the estimate
 *   other arguments as for vl_estimate.
 * Leaves the model at the estimate.  VL_ERR_NO_CONVERGENCE when max_iter was
 * reached (params_inout holds the last iterate).  Synchronises. */
vl_status vl_estimate_glm(vl_model* h, const double* y, const double* X, int p, int lik,
                          const vl_opts* o, double* params_inout, int max_iter,
                          double grad_tol, double* nll_host, int* iters_host,
                          int* evals_host);

/* Gradient of the negative log-marginal likelihood in the offset F at the
 * stored mode (App. "Gradients of Vecchia-Laplace approximations"):
 *   dL/dF_i = -d log p(y_i|mu_i)/d mu_i + (1/2) d log det(Sigma~ W + I)/d mu_i
 *             + (dL/d b_mode)^T (d b_mode/dF_i),
 *   d b_mode/dF_i = -(W + Sigma~^{-1})^{-1} W e_i  (b_mode = the mode b*),
 * with d log det / d mu estimated by the VADU stochastic trace estimator and
 * its control variate (the same probes and solves as the theta-gradient).
 * Available after vl_neg_log_marglik with grad_theta_host != NULL (the same
 * call computes it, for one extra kernel); VL_ERR_STATE otherwise.
 *   grad_F device, n.  Synchronises. */
vl_status vl_grad_offset(vl_model* h, double* grad_F);

/* With F = X beta (Sec. 2, fixed effects): grad_beta_host (host, p) =
 * X^T dL/dF from the same call.  X device, n x p row-major.  Synchronises. */
vl_status vl_grad_beta(vl_model* h, const double* X, int p, double* grad_beta_host);

/* Gradient of the same call in the likelihood's auxiliary parameter xi
 * (App. "Gradients of Vecchia-Laplace approximations": the explicit term,
 * the STE of the log-determinant's xi-derivative with the VADU control
 * variate, and the mode's response A^{-1} d^2 log p / d xi d mu), for
 * VL_LIK_GAUSSIAN (xi = tau^2) and VL_LIK_GAMMA (xi = shape a).
 *   grad_xi_host host, 1.
 * VL_ERR_INVALID_ARG for a likelihood without xi; VL_ERR_STATE before a
 * gradient call or after a later vl_set_theta / vl_find_mode. */
vl_status vl_grad_aux(vl_model* h, double* grad_xi_host);

/* Predictive latent mean and simulated variance (eq. latentpostpredictive,
 * Alg. simAlgo) at n_p new locations conditioned on the m nearest training
 * locations.
 *   coords_p device, n_p x 2
 *   Fp       device, n_p offsets (NULL = 0)
 *   mean_out device, n_p
 *   var_out  device, n_p (NULL = means only)
 * Requires a mode.  Synchronises. */
vl_status vl_predict(vl_model* h, const double* coords_p, int64_t n_p,
                     const double* Fp, const vl_opts* o, double* mean_out,
                     double* var_out, vl_stats* st);

/* Copy internal state out, for inspection and tests.  `which`:
 *   0 neighbours   int32  n x m (-1 padded)
 *   1 B values     double n x m (entries -A_i; 0 in padded slots)
 *   2 D            double n
 *   3 mode b*      double n
 *   4 W(b*)        double n
 *   5 dB/dsigma2   double n x m     6 dB/drho  double n x m
 *   7 dD/dsigma2   double n         8 dD/drho  double n
 *   9 CG iteration counts of the last block solve, int32 (count = columns)
 *  10 CG iteration counts of the Newton solves of the last vl_find_mode,
 *     int32 (count = Newton iterations)
 *  11 SLQ quadratures e1^T log(T~_i) e1 of the last vl_neg_log_marglik,
 *     double t
 *  12 r0^T z0 weights of the last vl_neg_log_marglik, double t
 *  13 prediction neighbours of the last vl_predict, int32 n_p x m
 *  14 prediction factor entries -A_p (the off-diagonal of B_po), double
 *     n_p x m;  15 D_p, double n_p
 *  16 LRAC pivoted Cholesky factor L_k, double n x k (row-major)
 *  17 LRAC pivots, int32 k
 *  18 Cholesky factor of I + L^T W L with the W of the last LRAC call,
 *     double K x K lower (row-major), K = k rounded up to 16: rows and
 *     columns past k belong to the identity
 *  19 step halvings of each Newton iteration of the last vl_find_mode, int32
 * dst is a device pointer; `bytes` must equal the size of the array.
 * Synchronises. */
vl_status vl_export(vl_model* h, int which, void* dst, size_t bytes);

/* Size in elements of an exportable array (see vl_export), or -1. */
int64_t vl_export_count(vl_model* h, int which);

/* Sparse products with the Vecchia factor over a block of t columns
 * (device, row-major n x t):  Y = B X (transpose = 0) or Y = B^T X
 * (transpose = 1).  X and Y must not overlap.  Asynchronous.  For
 * 32 <= t <= 64 rows are computed in groups of 4 neighbouring locations with
 * dense weights, so a non-finite entry of X makes every row of its group
 * non-finite. */
vl_status vl_spmm(vl_model* h, int transpose, const double* X, double* Y, int t);

/* Triangular solves with the Vecchia factor over t columns (device,
 * row-major n x t):  B Y = X (transpose = 0) or B^T Y = X (transpose = 1).
 * X and Y must not overlap.  Asynchronous. */
vl_status vl_trsm(vl_model* h, int transpose, const double* X, double* Y, int t);

/* vl_trsm for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results as vl_trsm, for 1 <= t <= 64 columns, with every
 * scratch buffer of the solve (work-stream counters and abort flag of the
 * sync-free rows, partial products and folded right-hand sides of the
 * dense leading block) taken from one fixed 40 MiB device array per GPU,
 * which each GPU the library runs on holds until the process ends.  It
 * calls no allocation routine.  The caller passes inputs and outputs as
 * for vl_trsm.  t > 64, or a model whose dense leading block would need
 * more than the array (a VL_DENSE_ROWS above 4096 at large t), is
 * VL_ERR_INVALID_ARG.  Every call on a GPU shares that GPU's array: calls
 * that overlap on one GPU (different streams or host threads) race.  Each
 * call resets what must start at zero, so no call depends on an earlier
 * one.  Synchronises the model's stream. */
vl_status vl_trsm_noalloc(vl_model* h, int transpose, const double* X, double* Y, int t);

/* Measurement support: while enabled, every launch of the sparse kernel
 * classes below is bracketed by HIP events on the model's stream, and the
 * algorithmic bytes of the launch (8-byte values and 4-byte indices of the
 * nonzeros it touches, each operand column block read once, the result
 * written once, per-row vectors) are accumulated.  `kind`:
 *   0  Y = B X (B in ELL)                 1  Y = B^T X (B^T in CSR)
 *   2  sync-free rows of B Y = X          3  sync-free rows of B^T Y = X
 *   4  leading rows of B Y = X            5  leading rows of B^T Y = X
 *      (4-5: the dense products with the inverse of B's leading block, or
 *      with each problem's inverse in a batch)
 *   6  level-scheduled B Y = X            7  level-scheduled B^T Y = X
 *   8  level-scheduled B^T Y = X, levels of long rows (entries split over
 *      4 waves per row)
 *   9  level-scheduled B^T Y = X: the fold of the head rows' tail entries
 *      (one launch between the tail levels and the head levels)
 *  10  the leading rows of the level-scheduled solves, from the dense
 *      inverse of B's leading block (one record per solve)
 *      (6-10: blocks wider than 64 columns; 6-8 one launch, and one
 *      record, per level)
 * `enable` is a bit mask of the kinds to record (bit k = kind k; -1 = all,
 * 0 = off).  vl_timing_enable resets the records (and synchronises); vl_timing_read
 * synchronises and returns the summed kernel time (ms), the number of
 * launches and the summed algorithmic bytes of the records so far. */
vl_status vl_timing_enable(vl_model* h, int enable);
vl_status vl_timing_read(vl_model* h, int kind, double* total_ms, int64_t* launches,
                         double* bytes);

/* ---------------------------------------------------------------------- */
/* Batching form: many independent problems of different sizes fitted
 * together.  The problems are packed into one block-diagonal system (each
 * problem's neighbour sets stay inside its own points), so that every sparse
 * kernel, CG vector kernel and reduction launch serves all problems; the CG
 * scalars and the Newton iteration are kept per problem, and each problem's
 * reductions add its rows in the order of a solo run (vl_build_vecchia +
 * vl_find_mode + vl_neg_log_marglik on that problem alone gives the same
 * result up to the rounding of the B^T solve).  The solve path of the packed
 * system (sync-free rows, or one launch per level) is chosen per
 * block-width class by timing both on the packed system (autotuner). */
typedef struct vl_batch vl_batch;

typedef struct {
  const double* coords;    /* device, n x 2, in the problem's ordering        */
  int64_t n;               /* points, >= 1                                     */
  int m;                   /* neighbours, 0..31                                */
  int cov;                 /* vl_cov                                           */
  double theta[2];         /* sigma2 > 0, range rho > 0                        */
  const double* y;         /* device, n responses                              */
  const double* F;         /* device, n offsets (NULL = 0)                     */
  uint64_t seed;           /* probe seed of this problem (vl_opts.seed of a
                              solo run)                                        */
} vl_problem;

/* Build the packed model: per problem neighbour search and factor (Sec. 2.1),
 * then B^T and the solve schedules of the packed system.  At most 32 problems
 * and 65536 rows in total (VL_ERR_INVALID_ARG above): a 256-problem batch of
 * 3.2e6 rows faulted the GPU and the cause is not yet found.  All problems share
 * the likelihood `lik` (aux_host as for vl_find_mode).  The problem arrays are
 * copied; the caller keeps ownership.  Synchronises. */
vl_status vl_batch_create(const vl_problem* problems, int nprob, int lik,
                          const double* aux_host, void* hip_stream, vl_batch** out);

/* Newton mode finding (eq. newton, VADU, pcls1) and the SLQ negative
 * log-marginal likelihood (eqs. VLA_loss, logdetsplit, def_SLQ) of every
 * problem, with o->num_probes probes each (the problems' own seeds; o->seed
 * is not used).  FP64 and VADU only.  nll_host: host, nprob doubles.
 * Synchronises. */
vl_status vl_batch_fit(vl_batch* b, const vl_opts* o, double* nll_host);

/* The mode of problem p after vl_batch_fit into mode_out (device, n_p). */
vl_status vl_batch_mode(vl_batch* b, int p, double* mode_out);

/* Statistics of problem p of the last fit: newton_iters, cg_iters_max (the
 * SLQ probes' largest CG count), cg_iters_total (step halvings taken). */
vl_status vl_batch_stats(vl_batch* b, int p, vl_stats* st);

/* Solve path the autotuner picked for a width class (0: one column, 1: 2..64,
 * 2: more), 0 = sync-free rows, 1 = one launch per level, 2 = each
 * problem's factor inverted whole and applied as a dense product (offered
 * when every problem has at most 4096 locations and the inverses take at
 * most 8 GB); -1 if that class was not used yet. */
int vl_batch_tuned_path(vl_batch* b, int width_class);

void vl_batch_free(vl_batch* b);

/* ---------------------------------------------------------------------- */
/* Serving form: a continuous-batching loop of fit + predict requests.
 * Requests are queued in arrival order and admitted when one of `slots`
 * worker slots is free and the request's HBM estimate (vl_request_bytes)
 * fits into the budget next to the running requests; a finishing request
 * frees its slot and budget at once, so waiting requests join while others
 * still run.  Each slot runs its request on its own HIP stream and model
 * (vl_build_vecchia, vl_find_mode, vl_neg_log_marglik, vl_predict with the
 * server's options and the request's seed); requests overlap on the device,
 * and a request's results do not depend on the others. */
typedef struct vl_server vl_server;

typedef struct {
  const double* coords;    /* device, n x 2                                    */
  int64_t n;
  int m;
  int cov;                 /* vl_cov                                           */
  double theta[2];
  const double* y;         /* device, n                                        */
  const double* F;         /* device, n (NULL = 0)                             */
  int lik;                 /* vl_lik                                           */
  double aux;              /* Gaussian noise variance (other likelihoods: 0)  */
  uint64_t seed;           /* probe seed                                       */
  const double* coords_p;  /* device, n_p x 2 (n_p = 0: no prediction)        */
  int64_t n_p;
  const double* Fp;        /* device, n_p (NULL = 0)                           */
  double* mean_out;        /* device, n_p                                      */
  double* var_out;         /* device, n_p (NULL = means only)                  */
} vl_request;

/* Start `slots` (1..64) worker threads on the current device. */
vl_status vl_server_create(int slots, double hbm_budget_bytes, const vl_opts* o,
                           vl_server** out);
/* Queue a request (non-blocking, thread-safe); the caller keeps its buffers
 * alive and untouched until vl_server_wait returns for its ticket. */
vl_status vl_server_submit(vl_server* s, const vl_request* r, int64_t* ticket);
/* Block until the request finished; nll_out (host) gets its negative
 * log-marginal likelihood, st its statistics (t_ms = submit-to-done latency),
 * queue_ms the time it waited for admission.  Returns the request's status:
 * VL_ERR_NO_CONVERGENCE (with st->hit_cap = 1) when a Newton or CG loop of
 * the request stopped at its cap (its outputs are written). */
vl_status vl_server_wait(vl_server* s, int64_t ticket, double* nll_out, vl_stats* st,
                         double* queue_ms);
/* Largest admitted HBM estimate and largest number of requests running at once. */
vl_status vl_server_info(vl_server* s, double* peak_bytes, int* peak_running);
/* The HBM estimate admission uses for a request (bytes). */
double vl_request_bytes(const vl_request* r, const vl_opts* o);
/* Drop waiting requests (they complete with VL_ERR_STATE, so a thread
 * blocked in vl_server_wait for one of them returns), finish running ones,
 * stop the workers, and return once no thread is inside vl_server_wait. */
void vl_server_free(vl_server* s);

/* Release the handle and all its device memory. */
void vl_free(vl_model* h);

#ifdef __cplusplus
}
#endif
#endif /* VL_H */
