/*
 * laker.h -- C ABI of the MI355X (gfx950) LAKER solve path.
 *
 * LAKER (Tao & Tan, "Accelerating Regularized Attention Kernel Regression for
 * Spectrum Cartography") solves the regularised attention-kernel regression
 *     (lambda I + G) alpha = y,   G_ij = exp(s <e_i, e_j>)          (eq. sc-final, eq. sc-exp-kernel)
 * by preconditioned conjugate gradients (Alg. 1) with the preconditioner
 * P = Sigma_star^{-1/2} fitted by shrinkage-regularised CCCP maximum likelihood
 * on normalised random directions u_k = (lambda I + G) z_k       (Sec. IV-B..D),
 * and reconstructs the field r_hat(x) = sum_i G(x, x_i) alpha_i  (eq. sc-radio-map-reconstruction).
 * The paper's kernel has s = 1; s = 1/sqrt(d) is the same kernel on embeddings
 * scaled by s^{1/2}.
 *
 * Conventions for every entry point:
 *  - Pointers documented as "device" point to HIP device memory owned by the
 *    caller; the library never allocates or frees device memory.  Scratch space
 *    is passed in as a caller-owned workspace whose size comes from the
 *    matching *_workspace_bytes query; workspaces and preconditioner buffers
 *    start on a 256-byte boundary (as hipMalloc returns them), since the
 *    library carves them into 256-byte-aligned pieces that its kernels read
 *    with 16-byte vector loads.  Pointers documented as "host" are ordinary
 *    host memory.
 *  - Matrices are row-major and densely packed: E is n x d (row i = e_i), the
 *    random directions Z are n x n_r (column k = z_k).
 *  - y, alpha and r_hat are float64 at the boundary in every precision mode.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).  The
 *    solver and fitter read convergence flags back, so they return only after
 *    their work on `stream` has completed; stats structs are filled on return.
 *  - Errors are returned, never thrown; arguments are validated before any
 *    launch and an invalid call leaves outputs untouched (LAKER_EINVAL /
 *    LAKER_ENOMEM).  A HIP runtime failure returns LAKER_EHIP; numerical
 *    breakdown (p^T A p <= 0, a non-positive pivot, NaN) returns
 *    LAKER_EBREAKDOWN; hitting max_iter returns LAKER_ENOCONV with alpha holding
 *    the last iterate.
 *  - Reductions use a fixed order: repeated calls on the same inputs give
 *    bitwise-identical results.
 */
#ifndef LAKER_H
#define LAKER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LAKER_OK = 0,
  LAKER_EINVAL = -1,      /* invalid argument (sizes, null pointers, lambda <= 0, ...) */
  LAKER_ENOMEM = -2,      /* workspace or preconditioner buffer too small             */
  LAKER_EHIP = -3,        /* HIP runtime error                                         */
  LAKER_EBREAKDOWN = -4,  /* p^T A p <= 0, non-positive pivot, or a NaN/Inf             */
  LAKER_ENOCONV = -5,     /* max_iter reached before the tolerance                      */
  LAKER_ESTALL = -6       /* the residual fell by less than 2x over the last
                             laker_pcg_opts.stall_window iterations; alpha holds
                             the last iterate                                       */
} laker_status;

/* Arithmetic of the kernel products.
 *  LAKER_F64:   float64 scores, exp and accumulation; float64 PCG vectors.
 *  LAKER_F32:   float32 scores (MFMA), exp2 in float32, float32 PCG vectors.
 *  LAKER_BF16:  bfloat16 embeddings on MFMA with float32 accumulation, exp2 in
 *               float32, float32 PCG vectors.
 *  LAKER_F32 and LAKER_BF16 solves can run inside float64 iterative refinement
 *  (laker_pcg_opts.refine), which keeps the outer residual y - A alpha, the
 *  update of alpha and the stopping test in float64. */
typedef enum { LAKER_F64 = 0, LAKER_F32 = 1, LAKER_BF16 = 2 } laker_precision;

typedef enum {
  LAKER_PRECOND_NONE = 0,    /* P = I (plain CG)                                         */
  LAKER_PRECOND_JACOBI = 1,  /* P = diag(lambda I + G)^{-1} (Sec. V-A baseline)          */
  LAKER_PRECOND_CCCP = 2,    /* P = Sigma_star^{-1/2} from laker_fit_precond (eq. preconditioner-Sigmma) */
  LAKER_PRECOND_LEARNED = 3  /* P = S_theta^{-1} from laker_learned_precond              */
} laker_precond_kind;

/* The regression problem (Alg. 1 inputs).  Embedding construction is the
 * caller's: the paper leaves the position-to-embedding map unspecified. */
typedef struct {
  int64_t n;          /* number of measurement sites, >= 1                     */
  int32_t d;          /* embedding dimension, 1 <= d <= 128                    */
  int32_t reserved;
  const double* E;    /* device, n x d row-major embeddings e_i                */
  double lambda;      /* regularisation weight, > 0                            */
  double scale;       /* s in G_ij = exp(s <e_i,e_j>), > 0 (paper: 1)          */
} laker_problem;

/* Options of the preconditioner fit (Alg. 1, "Attention Kernel Regression Learning"). */
typedef struct {
  int32_t n_r;        /* number of random directions N_r, 1 <= n_r <= min(n, 1024) */
  int32_t max_iter;   /* CCCP iteration cap (> 0)                                   */
  double gamma;       /* nuclear-norm weight gamma >= 0 (eq. prob:kernel-mle)       */
  double rho;         /* shrinkage rho in [0, 1] (eq. kernel_shrinkage_cccp_Sigma)   */
  double eps;         /* safeguard eps > 0 (eq. kernel_shrinkage_cccp_F)             */
  double tol;         /* stop when ||Sigma_{t+1}-Sigma_t||_F/||Sigma_t||_F <= tol   */
  int32_t precision;  /* laker_precision of the products u_k = (lambda I + G) z_k    */
  int32_t reserved;
} laker_cccp_opts;

/* A fitted preconditioner: a header the host keeps plus a caller-owned device
 * buffer of laker_precond_bytes(n, n_r) bytes that the fit writes. */
typedef struct {
  int32_t kind;       /* laker_precond_kind                                    */
  int32_t n_r;        /* rank of the low-rank part (CCCP: N_r; learned: 64)    */
  int64_t n;
  void* data;         /* device buffer                                          */
  size_t bytes;       /* its size in bytes                                     */
} laker_precond;

typedef struct {
  double tol;         /* stop when ||r|| / ||y|| <= tol (recursive r, Alg. 1)  */
  int32_t max_iter;   /* PCG iteration cap (total over refinement steps)       */
  int32_t precision;  /* laker_precision of the inner products A p             */
  int32_t refine;     /* 1: float64 iterative refinement around an F32/BF16 PCG;
                         2: flexible CG in float64 whose preconditioner is that
                         inner PCG (robust when lambda is far below the
                         rounding of the reduced-precision product)             */
  int32_t ir_max;     /* outer step cap (refine 1: <= 64)                       */
  double inner_tol;   /* inner PCG tolerance per refinement step, relative to the
                         step's residual; raised to 0.5 tol / (current outer
                         residual) when that is larger                          */
  int32_t warm_start; /* 1: alpha holds the starting iterate alpha^0            */
  int32_t check_every;/* host polls the convergence flag every this many steps  */
  int32_t graph;      /* 1: each chunk of check_every iterations is captured once
                         into a HIP graph and replayed (same results)          */
  int32_t profile;    /* 1: time every kernel product of the loop with HIP events
                         on `stream` (eager launches; fills stats->kmv_ms)      */
  int32_t inner_max_iter; /* refinement: cap on the iterations of one inner PCG
                         (0: only max_iter)                                    */
  int32_t materialized; /* 1: G is formed once per call and stored in the
                         workspace (see laker_kmat_bytes); the float64 products
                         (outer residuals, float64 PCG) and, with precision
                         F32, the float32 products then stream it instead of
                         recomputing it.  Applies where the symmetric product
                         schedule does (laker_kmat_bytes > 0); bfloat16
                         products are always recomputed (a rounded stored G
                         need not be positive definite).  In
                         laker_pcg_solve_batched: the float64 outer residuals
                         of the maps it applies to; workspace
                         laker_batch_workspace_bytes + the sum over those maps
                         of (256 + laker_kmat_bytes(n_b, d, F64)) bytes        */
  int32_t stall_window; /* > 0: stop with LAKER_ESTALL when the residual (the
                         recursive one of PCG, the float64 outer one with
                         refinement) fell by less than a factor 2 over the last
                         stall_window PCG iterations; checked where the host
                         reads the residual (every check_every iterations, every
                         outer step).  0: no stall test                         */
  int32_t outer_history;/* refine 2: directions the flexible outer CG keeps and
                         makes each new direction A-conjugate to (1..8; 0: 1) */
  int32_t escalate;     /* refine 2: 1 makes the inner products finer (bfloat16 ->
                         float32 -> float64) when the outer residual has not
                         halved over 40 outer steps (for tolerances near the
                         float64 floor); counted in stats->escalations          */
  int32_t lanczos;      /* 1 (refine 0 only): record PCG's step sizes and
                         conjugation coefficients and estimate the extreme
                         eigenvalues of P A from the Lanczos tridiagonal they
                         define (stats->eig_min, eig_max, cond_est), over the
                         first 8192 iterations                                  */
} laker_pcg_opts;

typedef struct {
  int32_t iters;        /* PCG iterations (products with A in the loop)         */
  int32_t ir_steps;     /* refinement steps taken (0 without refinement)         */
  int32_t cccp_iters;   /* CCCP iterations (fit only)                            */
  int32_t status;       /* laker_status of the call                              */
  double relres;        /* final recursive relative residual                     */
  double relres_true;   /* ||y - (lambda I + G) alpha|| / ||y|| in float64        */
  double ir_relres[64]; /* float64 true residual after each refinement step      */
  double kmv_ms;        /* profile: mean duration of the loop's kernel products of
                           iterations that ran                                   */
  int32_t kmv_count;    /* profile: number of those products                      */
  int32_t kmv_launches; /* profile: product launches, including the ones enqueued
                           after convergence, which return at entry              */
  double kmv_launch_ms; /* profile: mean duration over all kmv_launches          */
  int32_t escalations;  /* refinement: times the inner product arithmetic was made
                           finer (bfloat16 -> float32 -> float64) after two
                           refinement steps without progress (an inner PCG that
                           breaks down in reduced precision ends with the
                           correction it has; only a float64 breakdown is an
                           error)                                               */
  int32_t fell_back;    /* laker_learned_solve: 0 the learned preconditioner
                           solved the system; 1 its solve stalled, 2 it broke
                           down (its build or its solve), and the solve went on
                           from the last iterate with a CCCP fit                 */
  int32_t learned_iters;/* laker_learned_solve: PCG iterations with the learned
                           preconditioner (all of them when fell_back is 0)      */
  int32_t lanczos_steps;/* opts->lanczos: PCG iterations in the estimate         */
  int32_t reserved;
  double eig_min;       /* opts->lanczos: smallest and largest eigenvalue of the  */
  double eig_max;       /*   Lanczos tridiagonal of the PCG coefficients (Ritz   */
  double cond_est;      /*   values of P A) and their ratio, kappa(P A)           */
} laker_stats;

/* ---- sizes ---------------------------------------------------------------- */

/* Bytes of the device buffer of a preconditioner of rank n_r on n sites. */
size_t laker_precond_bytes(int64_t n, int32_t n_r);
/* Workspace bytes of laker_fit_precond. */
size_t laker_fit_workspace_bytes(int64_t n, int32_t d, int32_t n_r);
/* Workspace bytes of laker_pcg_solve / laker_kernel_matvec / laker_predict
 * (m query points; pass m = 0 for the solver). */
size_t laker_solve_workspace_bytes(int64_t n, int32_t d, int64_t m);
/* Bytes of a stored G = exp(s E E^T) for opts->materialized (the tiles of the
 * symmetric product schedule on or right of the block diagonal: about
 * n^2 / 2 entries) in precision F64 or F32; 0 when the size is below the
 * symmetric schedule's threshold (then nothing is stored).  With
 * materialized set, laker_pcg_solve needs laker_solve_workspace_bytes(n, d, 0)
 * + laker_kmat_bytes(n, d, F64) (+ laker_kmat_bytes(n, d, F32) with
 * precision F32) bytes of workspace. */
size_t laker_kmat_bytes(int64_t n, int32_t d, int32_t precision);

/* ---- entry points ---------------------------------------------------------- */

/* w = (lambda I + G) p, the product the whole method is built on (Alg. 1 step
 * size and residual update; Sec. IV-D remark: G is never formed).
 * p, w: device float64 vectors of length n.  precision: laker_precision. */
laker_status laker_kernel_matvec(const laker_problem* prob, const double* p, double* w,
                                 int32_t precision, void* workspace, size_t workspace_bytes,
                                 void* stream);

/* w = (lambda I + G) p as laker_kernel_matvec computes it (the same kernels,
 * bitwise the same result), for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It takes no workspace and allocates nothing: its scratch (the
 * prepared embedding copy and the product's partial sums) is a file-scope
 * device array of 64 MiB, one per GPU, held until the process ends.  Problems
 * whose scratch exceeds it return LAKER_ENOMEM before any launch (it holds
 * every precision at n <= 32768 with d <= 64).  All calls on one GPU share
 * that GPU's array, so calls that overlap on one GPU (on different streams or
 * host threads) race; calls ordered on one stream do not.  p, w: device
 * float64 vectors of length n. */
laker_status laker_kernel_matvec_noalloc(const laker_problem* prob, const double* p, double* w, int32_t precision,
                                         void* stream);

/* theta = P r: the preconditioner step of every PCG iteration (Alg. 1; for
 * CCCP P = Sigma_star^{-1/2}, eq. preconditioner-Sigmma), computed once with
 * the same kernels the solver runs in its loop.  For a low-rank precond
 * (CCCP or learned) theta = c r + Bt (B^T r), with c the scalar b^{-1/2}
 * (CCCP) or the diagonal D^{-1} (learned); Jacobi: theta_i = r_i / A_ii;
 * kind LAKER_PRECOND_NONE: theta = r.  precision selects the factors the
 * solver would read (LAKER_F64: float64 B, Bt; otherwise the float32 copies
 * of a CCCP fit; the learned factors are float64 in every precision).
 * r, theta: device float64 vectors of length precond->n (not aliased).
 * workspace: laker_precond_apply_workspace_bytes(n, n_r) bytes (unused for
 * LAKER_PRECOND_NONE). */
size_t laker_precond_apply_workspace_bytes(int64_t n, int32_t n_r);
laker_status laker_precond_apply(const laker_precond* precond, const double* r, double* theta, int32_t precision,
                                 void* workspace, size_t workspace_bytes, void* stream);

/* Fit P = Sigma_star^{-1/2} (Alg. 1, preconditioner learning):
 * u_k = (lambda I + G) z_k, u_bar_k = u_k/||u_k|| (eq. random_directions);
 * shrinkage-CCCP Sigma_{t+1} = n Sigma_tilde / tr(Sigma_tilde) with
 * Sigma_tilde = (1-rho) F_gamma(Sigma_t) + rho I from Sigma_0 = I
 * (eqs. kernel_shrinkage_cccp_F/Sigma/normalization), carried exactly in
 * low-rank form Sigma = b I + a U_bar diag(w) U_bar^T; then P = Sigma^{-1/2}.
 * Z: device, n x n_r row-major float64 standard normal draws (column k = z_k);
 * the draws are inputs so that results are reproducible.
 * out: kind/n/n_r are set by the call; out->data must hold
 * laker_precond_bytes(n, n_r) bytes.  stats->cccp_iters is filled. */
laker_status laker_fit_precond(const laker_problem* prob, const double* Z, const laker_cccp_opts* opts,
                               laker_precond* out, void* workspace, size_t workspace_bytes,
                               laker_stats* stats, void* stream);

/* ---- measurements that arrive over time -----------------------------------
 *
 * The paper leaves online spectrum cartography, where measurements arrive
 * sequentially, to future work (Sec. VI).  When sites are appended to a map,
 * the fit of Alg. 1 is extended instead of redone: the random directions keep
 * their previous entries and gain new ones (z_k of the enlarged problem), so
 * only the products with the new rows are formed,
 *     U[old] += G[old, new] Z[new],   U[new] = G[new, :] Z + lambda Z[new],
 * and the CCCP iteration starts from the previous fit's (a, b, w) instead of
 * Sigma_0 = I.  The same solution as a fresh fit (the fixed point depends on
 * the directions only); a PCG warm-started from [alpha_prev; 0]
 * (laker_pcg_opts.warm_start) then finishes the enlarged solve. */

/* Bytes of the state buffer for up to n_cap sites and n_r directions. */
size_t laker_online_state_bytes(int64_t n_cap, int32_t n_r);

/* Fit P = Sigma_star^{-1/2} for the n sites of prob, the first n_prev of which
 * were fitted by the previous call on the same state (n_prev = 0: a full fit
 * that starts the state).  Rows of E and Z keep their order: E rows
 * [0, n_prev) and Z rows [0, n_prev) (n x n_r row-major, device) must equal
 * the previous call's.  state: device, caller-owned, laker_online_state_bytes
 * (n_cap, n_r) bytes with n_cap >= n; it holds the float64 directions and the
 * CCCP weights between calls.  opts->precision must be LAKER_F64.  out,
 * workspace (laker_fit_workspace_bytes(n, d, n_r)) and stats as for
 * laker_fit_precond. */
laker_status laker_fit_precond_online(const laker_problem* prob, int64_t n_prev, const double* Z,
                                      const laker_cccp_opts* opts, void* state, size_t state_bytes,
                                      laker_precond* out, void* workspace, size_t workspace_bytes,
                                      laker_stats* stats, void* stream);

/* Jacobi preconditioner P_J = diag(lambda I + G)^{-1} (Sec. V-A numerical-layer
 * baseline); out->data must hold laker_precond_bytes(n, 0) bytes. */
laker_status laker_jacobi_precond(const laker_problem* prob, laker_precond* out, void* stream);

/* Solve (lambda I + G) alpha = y by PCG (Alg. 1, Sec. IV-E).
 * precond: NULL or kind LAKER_PRECOND_NONE for plain CG.
 * y: device float64 (n); alpha: device float64 (n), read as alpha^0 when
 * opts->warm_start, written with the solution.  stats is filled on return. */
laker_status laker_pcg_solve(const laker_problem* prob, const laker_precond* precond, const double* y,
                             double* alpha, const laker_pcg_opts* opts, void* workspace,
                             size_t workspace_bytes, laker_stats* stats, void* stream);

/* r_hat_j = sum_i exp(s <eq_j, e_i>) alpha_i for m query embeddings
 * (eq. sc-radio-map-reconstruction).  Eq: device, m x d row-major float64;
 * alpha: device (n); rhat: device (m). */
laker_status laker_predict(const laker_problem* prob, const double* alpha, int64_t m, const double* Eq,
                           double* rhat, int32_t precision, void* workspace, size_t workspace_bytes,
                           void* stream);

/* ---- learned rank-64-plus-diagonal preconditioner --------------------------
 *
 * Replaces the CCCP fit of Alg. 1 by a per-point network trained on CCCP fits.
 * Network: x_i = [e_i, log lambda, log(n)/10, mean_j e_j, mean_j e_j^2]
 * (3 d + 2 inputs) -> 256 -> 256 -> 65 with SiLU activations, bfloat16 MFMA
 * products with float32 accumulation and float32 master weights.  Outputs
 * o_i = (v_i in R^64, log delta_i) define S = diag(delta) + V V^T, a surrogate
 * of Sigma_star^{1/2} (Sec. IV; SPD for any weights), and P = S^{-1} by the
 * Woodbury identity.  Training minimises ||Z - S^{-1} U||_F^2 / (n m) over
 * Gaussian probes Z with U = Sigma_star^{1/2} Z from laker_precond_sigma_half.
 *
 * Model buffer (device, caller-owned, laker_mlp_layout.bytes): three blocks of
 * block_bytes -- weights theta, Adam first moments, Adam second moments -- each
 * holding `count` floats with W1 (in x 256), b1, W2 (256 x 256), b2,
 * W3 (256 x 65), b3 at the element offsets off[0..5] (weights fan_in x fan_out,
 * row-major).  Callers write the initial weights and zero the moments. */
typedef struct {
  int32_t d;          /* embedding dimension                                   */
  int32_t in_dim;     /* 3 d + 2                                               */
  int64_t count;      /* floats in one block                                   */
  int64_t off[6];     /* element offsets of W1 b1 W2 b2 W3 b3                   */
  size_t block_bytes; /* bytes of one block (256-byte multiple)                 */
  size_t bytes;       /* bytes of the model buffer                              */
} laker_mlp_layout;

typedef struct {
  double lr, beta1, beta2, eps; /* Adam hyper-parameters                        */
  int32_t step;       /* Adam step t >= 1 (bias correction)                     */
  int32_t update;     /* 1: apply the Adam step; 0: gradient only               */
} laker_train_opts;

/* Layout of the model buffer for embeddings of dimension d (1..128). */
laker_status laker_mlp_layout_query(int32_t d, laker_mlp_layout* out);
/* Workspace bytes of the learned entry points for n points and m probes
 * (m = 0 for inference). */
size_t laker_learned_workspace_bytes(int64_t n, int32_t d, int32_t m);

/* Network outputs o (n x 65 float32, device) for the problem's embeddings. */
laker_status laker_learned_forward(const laker_problem* prob, const void* model, float* out, void* workspace,
                                   size_t workspace_bytes, void* stream);

/* One training step on one problem: loss ||Z - S^{-1} U||_F^2 / (n m) and its
 * gradient; with opts->update the Adam step is applied to the model buffer.
 * Z, U: device float64, n x m row-major.  grad_out: optional device float
 * buffer of `count` floats (the gradient block); loss_out: optional host
 * double (the call then synchronises `stream`). */
laker_status laker_learned_train_step(const laker_problem* prob, void* model, int32_t m, const double* Z,
                                      const double* U, const laker_train_opts* opts, float* grad_out,
                                      double* loss_out, void* workspace, size_t workspace_bytes, void* stream);

/* P = S^{-1} of the trained network into out->data (laker_precond_bytes(n, 64)
 * bytes): kind LAKER_PRECOND_LEARNED, n_r = 64, P = D^{-1} + Bt B^T with
 * B = D^{-1} V, Bt = -B (I + V^T D^{-1} V)^{-1}. */
laker_status laker_learned_precond(const laker_problem* prob, const void* model, laker_precond* out,
                                   void* workspace, size_t workspace_bytes, void* stream);

/* Workspace bytes of laker_learned_solve (precision and materialized as in
 * the laker_pcg_opts it will get). */
size_t laker_learned_solve_workspace_bytes(int64_t n, int32_t d, int32_t n_r, int32_t precision,
                                           int32_t materialized);

/* Solve (lambda I + G) alpha = y with the learned preconditioner, falling back
 * to the paper's CCCP preconditioner (Alg. 1) when that solve does not get
 * there: the network builds P = S^{-1} (laker_learned_precond) and
 * laker_pcg_solve runs with `opts` (opts->stall_window > 0 turns on the stall
 * test).  If the learned build breaks down, or its solve stalls (LAKER_ESTALL),
 * breaks down or reaches opts->max_iter, CCCP is fitted with the directions Z
 * and options `cccp` (laker_fit_precond) into the same buffer and the solve
 * continues from the last iterate with the same opts (a fresh max_iter, no
 * stall test).  precond: caller-owned buffer of laker_precond_bytes(n,
 * max(64, cccp->n_r)) bytes; on return it holds the preconditioner used last
 * (kind LAKER_PRECOND_LEARNED or LAKER_PRECOND_CCCP).  stats: iters counts
 * both solves; fell_back (0, 1 stall or cap, 2 breakdown) and learned_iters
 * say what happened; cccp_iters is the fit's.  opts->warm_start and
 * opts->lanczos must be 0.  Returns the status of the last solve. */
laker_status laker_learned_solve(const laker_problem* prob, const void* model, const double* Z,
                                 const laker_cccp_opts* cccp, const double* y, double* alpha,
                                 const laker_pcg_opts* opts, laker_precond* precond, void* workspace,
                                 size_t workspace_bytes, laker_stats* stats, void* stream);

/* Workspace bytes of laker_precond_sigma_half. */
size_t laker_sigma_half_workspace_bytes(int64_t n, int32_t n_r, int32_t m);

/* U = Sigma_star^{1/2} Z for a CCCP preconditioner P = Sigma_star^{-1/2}
 * (eq. preconditioner-Sigmma), computed as Sigma_star (P Z) with
 * Sigma_star = b I + B B^T.  Z, U: device float64 n x m row-major. */
laker_status laker_precond_sigma_half(const laker_precond* precond, int32_t m, const double* Z, double* U,
                                      void* workspace, size_t workspace_bytes, void* stream);

/* ---- several right-hand sides on one map ----------------------------------
 *
 * Bands or snapshots measured at the same sites share E, G and the
 * preconditioner: k <= 8 right-hand sides y_1 .. y_k are solved together.
 * Each column runs the PCG iteration of laker_pcg_solve (Alg. 1) with its own
 * scalars, stopping test and retirement; the kernel product of an iteration
 * is one launch for all columns, whose score tiles and exponentials are formed
 * once and multiplied by the k directions.  Matrices of k columns are stored
 * column after column: column q of Y at Y + q n. */

/* Workspace bytes of laker_kernel_matvec_multi and laker_pcg_solve_multi. */
size_t laker_multi_workspace_bytes(int64_t n, int32_t d, int32_t k);

/* W = (lambda I + G) P for k <= 8 columns (P, W: device, n x k, column-major as
 * above); precision as for laker_kernel_matvec. */
laker_status laker_kernel_matvec_multi(const laker_problem* prob, int32_t k, const double* P, double* W,
                                       int32_t precision, void* workspace, size_t workspace_bytes, void* stream);

/* Solve (lambda I + G) alpha_q = y_q for q < k (Y, Alpha: device, n x k,
 * column-major).  opts: tol, max_iter (per column), precision, check_every
 * as for laker_pcg_solve; refine, warm_start, graph, stall_window and lanczos
 * must be 0.  precond: NULL or one preconditioner for all columns.  stats:
 * host array of k entries (iters, relres, relres_true, status per column).
 * Returns LAKER_OK when every column converged, else the worst status. */
laker_status laker_pcg_solve_multi(const laker_problem* prob, const laker_precond* precond, int32_t k,
                                   const double* Y, double* Alpha, const laker_pcg_opts* opts, void* workspace,
                                   size_t workspace_bytes, laker_stats* stats, void* stream);

/* ---- batched solve --------------------------------------------------------
 *
 * Many independent maps of uneven size (bands, snapshots) solved together: each
 * pass of a PCG iteration is one launch for the whole batch (the kernel products
 * as one grid of (map, row block, column range) tiles), each map keeps its own
 * scalars and retires at its own tolerance (Alg. 1 per map), with the same
 * float64 refinement as laker_pcg_solve when opts->refine is set. */
typedef struct {
  int32_t cols_per_split; /* -1: autotuned per size class (maps with the same
                             floor(log2 n); the product of the class's largest
                             map timed per candidate length, cached per class);
                             0: the single-map plan of each map (bitwise the same
                             iterates as laker_pcg_solve); > 0: this many columns */
  int32_t xcd_order;      /* 1: tiles ordered so that each XCD walks its own
                             contiguous stretch of the tile list                */
  int32_t cols_used;      /* out: the length used for the largest map
                             (0: its single-map plan)                          */
  int32_t reserved;
} laker_batch_opts;

/* Workspace bytes of laker_pcg_solve_batched for maps of n[0..count) sites and
 * embedding dimension d. */
size_t laker_batch_workspace_bytes(int32_t count, const int64_t* n, int32_t d);

/* Solve (lambda_b I + G_b) alpha_b = y_b for b < count.  probs: count problems
 * with the same d; preconds: NULL (plain CG) or count preconditioners of one
 * kind; y, alpha: host arrays of count device float64 pointers.  opts as for
 * laker_pcg_solve (warm_start must be 0; profile is ignored); stats: host array
 * of count entries; refine 0 or 1.  Returns LAKER_OK when every map converged,
 * else the worst status (each map's status is in its stats entry). */
laker_status laker_pcg_solve_batched(int32_t count, const laker_problem* probs, const laker_precond* preconds,
                                     const double* const* y, double* const* alpha, const laker_pcg_opts* opts,
                                     laker_batch_opts* bopts, void* workspace, size_t workspace_bytes,
                                     laker_stats* stats, void* stream);

/* Human-readable name of a status code (static string). */
const char* laker_status_str(int32_t status);

#ifdef __cplusplus
}
#endif
#endif /* LAKER_H */
