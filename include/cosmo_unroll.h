/*
 * cosmo_unroll.h -- C ABI of the batched, unrolled COSMO hot path on MI355X.
 *
 * Problem (eq:conic-standard):  minimize 1/2 x'Px + q'x  s.t.  Ax + s = b, s in K,
 * K a product of zero, nonnegative, second-order (SOC) and PSD cones.
 *
 * One forward step k (Sec. "Conic Operator Splitting Method", indirect mode
 * eq:cosmo_linear_system_reduced; per-block penalty rectification of App. E,
 * "Hyperparameter policy"):
 *   rho_hat = rectify(rho^k)                       (mean over each SOC/PSD block)
 *   x~  solves (P + sigma I + A' D(rho_hat) A) x~ = sigma x - q + A'(y + rho_hat o (b - s))
 *        by Jacobi-preconditioned CG (Table 2, "Linear solve"), matrix-free
 *   s~  = b - A x~
 *   x+  = alpha x~ + (1 - alpha) x,   s^ = alpha s~ + (1 - alpha) s
 *   s+  = Pi_K(s^ + y / rho_hat)                  (PSD: eigendecompose, clip; eq:psd-proj)
 *   y+  = y + rho_hat o (s^ - s+)
 * The backward pass is the matrix-free implicit rule of Sec. "Matrix-Free
 * Implicit Differentiation" (adjoint CG with the same operator, eq:grad_rho)
 * and the Daleckii-Krein rule for the PSD projection (eq:psd-cotangent-dk,
 * eq:lowner).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Super-batch (App. C, "super-batches"): B independent instances are stacked;
 *   instance i owns columns [n_off[i], n_off[i+1]) and rows [m_off[i], m_off[i+1]).
 *   A and P are block diagonal by instance.
 * - Real arrays hold `dtype` elements (float or double).  Index arrays are
 *   int64 row pointers and int32 column indices.
 * - PSD blocks use the svec encoding: a p x p symmetric block occupies
 *   p(p+1)/2 consecutive rows, column-major over the upper triangle (column j
 *   holds rows i = 0..j), off-diagonal entries scaled by sqrt(2).
 * - "device" pointers are HIP device memory owned by the caller; "host"
 *   pointers are read during the call only (unless stated otherwise).
 * - `stream` is a hipStream_t (NULL = default stream).  Unroll, loss and
 *   projection launches are asynchronous on it.  After cosmo_plan_create the
 *   unroll and loss calls allocate nothing; every O(n + m) buffer (workspace,
 *   tape) is caller-owned, sized by cosmo_workspace_size.
 * - Errors: host-checkable misuse returns COSMO_EINVAL before anything is
 *   launched; a HIP runtime failure returns COSMO_EHIP.  Numerical conditions
 *   detected on the device (CG not converged, eigen-sweeps exhausted,
 *   non-finite values) never abort a call: they are counted in cosmo_stats.
 *   cosmo_last_error() returns a message for the last failure on this thread.
 * - A plan is not safe for concurrent calls; distinct plans are independent.
 */
#ifndef COSMO_UNROLL_H
#define COSMO_UNROLL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  COSMO_OK = 0,
  COSMO_EINVAL = -1,        /* invalid argument or descriptor */
  COSMO_ENOMEM = -2,        /* a plan-owned allocation failed */
  COSMO_EHIP = -3,          /* HIP runtime error (launch, copy, device) */
  COSMO_EUNSUPPORTED = -4   /* valid request outside the implemented envelope */
} cosmo_status;

/* The last enumerator of each enum taken from callers widens its range to
 * every int32 value, so a caller's out-of-range value is a valid (rejected)
 * enum value on the library side, not undefined behaviour. */
typedef enum { COSMO_F32 = 0, COSMO_F64 = 1, COSMO_DTYPE_MAX_ENUM = 0x7fffffff } cosmo_dtype;

typedef enum {
  COSMO_CONE_ZERO = 0,      /* s = 0            (equality rows)          */
  COSMO_CONE_NONNEG = 1,    /* s >= 0                                     */
  COSMO_CONE_SOC = 2,       /* (t, w): ||w||_2 <= t, size = rows (>= 1)   */
  COSMO_CONE_PSD = 3,       /* svec(S), S psd, size = matrix order p      */
  COSMO_CONE_MAX_ENUM = 0x7fffffff
} cosmo_cone_kind;

/* Largest PSD order handled: the one-sided Jacobi eigensolver keeps one
 * p x p block in the 160 KiB LDS of a workgroup. */
#define COSMO_MAX_PSD_ORDER_F32 200
#define COSMO_MAX_PSD_ORDER_F64 140

typedef struct cosmo_plan cosmo_plan;

/* A dense sub-block of A (Sec. "Matrix-Free Implicit Differentiation": the
 * method only ever applies A and A' to vectors, at O(n + nnz(A)) cost, so a
 * dense block is read as a dense block instead of as CSR with an index per
 * entry).  The matrix the library uses is
 *     A = (the CSR arrays of cosmo_problem)
 *         + sum over dense blocks and their placements of scale[p] * G
 *           placed at rows row0[p] .. row0[p] + rows - 1 and columns
 *           col0 .. col0 + cols - 1,
 * so the CSR arrays hold only the entries outside the dense blocks.  One G
 * may be placed at several row offsets with different scales (e.g. [G; -G]):
 * every operator application then reads G once.
 * Constraints (COSMO_EINVAL otherwise, before any device access): all rows
 * and columns of a block lie inside one instance; no row of A lies in two
 * placements (of any blocks); no column lies in two blocks; 1 <= cols <=
 * COSMO_DENSE_MAX_COLS; ld >= cols and ld a multiple of 16 / (bytes per
 * stored value); val 16-byte aligned; val_f32 the same for every block of a
 * plan.  While dense blocks are present the CG runs in form 0
 * (cosmo_plan_set_pcg_form with form > 0 returns COSMO_EUNSUPPORTED).
 *
 * Storage type: with val_f32 = 1 a float64 plan reads the values of G as
 * float32 and does all its arithmetic in float64; G then is, by definition,
 * those float32 values.  A product with G is bound by reading G (one value
 * per multiply-add), so problems whose data are float32 numbers (e.g. data
 * generated in float64 and rounded to float32) run float64 iterations at the
 * float32 cost of their dense blocks.  In a float32 plan val_f32 may be 0 or
 * 1 (both mean float32). */
#define COSMO_DENSE_MAX_PLACEMENTS 4
#define COSMO_DENSE_MAX_COLS 1024
typedef struct {
  const void *val;             /* (d) rows x ld, row-major, dtype or float32 (val_f32); valid and unchanged
                                  until cosmo_plan_destroy                              */
  int32_t rows;                /* >= 1                                                  */
  int32_t cols;                /* 1 .. COSMO_DENSE_MAX_COLS                             */
  int64_t ld;                  /* elements between consecutive rows of val              */
  int64_t col0;                /* first column of the block in the stacked A           */
  int32_t n_place;             /* placements, 1 .. COSMO_DENSE_MAX_PLACEMENTS           */
  int32_t val_f32;             /* 1: val holds float32 values (see above); 0: dtype    */
  int64_t row0[COSMO_DENSE_MAX_PLACEMENTS];   /* first row of each placement            */
  double scale[COSMO_DENSE_MAX_PLACEMENTS];   /* finite multiplier of each placement    */
} cosmo_dense_block;

/* Problem data of a super-batch.  Arrays marked (d) are device pointers that
 * must stay valid and unchanged until cosmo_plan_destroy; (h) are host arrays
 * read during cosmo_plan_create only. */
typedef struct {
  int32_t B;                   /* number of instances, >= 1                           */
  const int64_t *n_off;        /* (h) [B+1], n_off[0] = 0, non-decreasing, n_tot = n_off[B] */
  const int64_t *m_off;        /* (h) [B+1], m_off[0] = 0, strictly increasing         */
  const int64_t *A_rowptr;     /* (d) [m_tot+1] CSR of A (m_tot x n_tot)               */
  const int32_t *A_col;        /* (d) [nnz(A)], columns inside the row's instance;
                                  16-byte aligned (rows are read in 16-byte pieces)     */
  const void *A_val;           /* (d) [nnz(A)] dtype, 16-byte aligned                   */
  int64_t A_nnz;
  const int64_t *P_rowptr;     /* (d) [n_tot+1] CSR of P, symmetric, full storage;
                                  may be NULL when P_nnz == 0                            */
  const int32_t *P_col;        /* (d) [nnz(P)]                                          */
  const void *P_val;           /* (d) [nnz(P)] dtype                                    */
  int64_t P_nnz;
  const void *q;               /* (d) [n_tot] dtype                                     */
  const void *b;               /* (d) [m_tot] dtype                                     */
  int32_t n_cones;             /* cone blocks, laid out contiguously in list order,
                                  covering rows 0..m_tot, none straddling instances     */
  const int32_t *cone_kind;    /* (h) [n_cones] cosmo_cone_kind                         */
  const int32_t *cone_size;    /* (h) [n_cones] rows (zero/nonneg/soc) or order p (psd) */
  int32_t n_dense;             /* dense sub-blocks of A (0: A is the CSR arrays alone)  */
  const cosmo_dense_block *dense;   /* (h) [n_dense] descriptors; the blocks' values
                                       are device arrays (see cosmo_dense_block)        */
} cosmo_problem;

typedef struct {
  cosmo_dtype dtype;           /* arithmetic and storage type of all real arrays        */
  int32_t K;                   /* unrolled steps, >= 1                                  */
  double sigma;                /* > 0; the paper fixes 1e-6                             */
  double cg_tol;               /* PCG stops when ||xi - M x~||_2 <= cg_tol ||xi||_2      */
  int32_t cg_max_iter;         /* >= 1                                                   */
  int32_t eig_max_sweeps;      /* Jacobi sweep cap, >= 1                                 */
  double eig_tol;              /* Jacobi column-orthogonality threshold; 0 = dtype default */
  int32_t eig_refine;          /* 1: refine the float32 eigenpairs of every PSD block
                                  once (Ogita-Aishima step with float64-accumulated
                                  residual products) and form the projection by
                                  Rayleigh-Ritz on the positive subspace; 0: use
                                  the Jacobi eigenpairs as they are.  Must be 0 or 1;
                                  ignored for COSMO_F64, whose sweeps run in float64. */
  int32_t eig_warm_start;      /* 1: start every step's Jacobi sweeps from the same
                                  block's eigenvectors of the previous step (same
                                  decomposition, fewer sweeps); 0: start from S.        */
} cosmo_options;

/* Per-instance device counters, updated with atomics (max / or); the caller
 * zeroes them before a call if it wants per-call values (the sums wrap past
 * 2^31). */
typedef struct {
  int32_t cg_iters_max;        /* largest PCG iteration count of any solve             */
  int32_t cg_not_converged;    /* solves that ended with the true residual above tol
                                  (iteration cap, or the working precision's floor)     */
  int32_t eig_sweeps_max;      /* largest Jacobi sweep count of any PSD block          */
  int32_t eig_not_converged;   /* PSD eigensolves that hit eig_max_sweeps              */
  int32_t nonfinite;           /* 1 if a non-finite value reached the iterate          */
  int32_t eig_sweeps_total;    /* Jacobi sweeps summed over the PSD block solves       */
  int32_t eig_solves;          /* PSD block eigensolves (eig_sweeps_total / eig_solves
                                  is the mean sweep count)                              */
  int32_t cg_iters_total;      /* PCG iterations summed over the solves                */
  int32_t cg_passes_total;     /* float64 true-residual passes summed over the solves
                                  (each is one more operator application)               */
  int32_t eig_refine_steps_total; /* float32 eigenpair refinement steps summed over the
                                  PSD block solves (1 to 3 per solve)                   */
} cosmo_stats;

const char *cosmo_status_string(cosmo_status s);
const char *cosmo_last_error(void);
int32_t cosmo_abi_version(void);

/* Validate the problem, copy its structure to the host, build the transposed
 * CSR of A, cone tables and work lists, and upload them (plan-owned device
 * memory, freed by cosmo_plan_destroy).  Synchronous.  *plan is NULL on error. */
cosmo_status cosmo_plan_create(cosmo_plan **plan, const cosmo_problem *prob, const cosmo_options *opt);
cosmo_status cosmo_plan_destroy(cosmo_plan *plan);

/* Bytes of caller-owned device memory: forward workspace, tape (K steps of
 * checkpoints: iterates z^0..z^K, x~ and s~ of every step, eigenvalues and
 * eigenvectors of every PSD block -- O(n + m + sum p^2) per step), backward
 * workspace.  Any pointer may be NULL. */
cosmo_status cosmo_workspace_size(const cosmo_plan *plan, size_t *fwd_ws_bytes, size_t *tape_bytes,
                                  size_t *bwd_ws_bytes);

/* Byte offsets, inside the tape, of iterate k (0 <= k <= K) and of x~, s~ of
 * step k (0 <= k < K; pass NULL for those when k == K). */
cosmo_status cosmo_tape_offsets(const cosmo_plan *plan, int32_t k, size_t *x_off, size_t *s_off,
                                size_t *y_off, size_t *xt_off, size_t *st_off);

/* K forward steps.
 *   rho   (d) [K][m_tot] > 0, per row; rectified per SOC/PSD block inside.
 *   alpha (d) [K][B] in (0, 2), one relaxation per instance and step.
 *   x0 (d) [n_tot], s0, y0 (d) [m_tot]; NULL = zeros (App. D default start).
 *   xK, sK, yK (d) outputs (may be NULL).
 *   tape  (d) [tape_bytes] or NULL for a forward-only run (then the backward
 *         pass is unavailable and only the final iterate is kept).
 *   ws    (d) [fwd_ws_bytes].   stats (d) [B] cosmo_stats or NULL. */
cosmo_status cosmo_unroll_forward(cosmo_plan *plan, const void *rho, const void *alpha, const void *x0,
                                  const void *s0, const void *y0, void *xK, void *sK, void *yK, void *tape,
                                  void *ws, void *stats, void *stream);

/* Reverse pass over the K steps recorded in `tape` by cosmo_unroll_forward
 * with the same rho / alpha.  Incoming cotangents gxK, gsK, gyK (d) of the
 * final iterate (NULL = 0).  Outputs (d), each may be NULL:
 *   grho [K][m_tot] w.r.t. the raw per-row rho (rectification included),
 *   galpha [K][B], gx0 [n_tot], gs0, gy0 [m_tot].
 *   ws (d) [bwd_ws_bytes].  Deterministic: no floating-point atomics. */
cosmo_status cosmo_unroll_backward(cosmo_plan *plan, const void *rho, const void *alpha, const void *tape,
                                   const void *gxK, const void *gsK, const void *gyK, void *grho,
                                   void *galpha, void *gx0, void *gs0, void *gy0, void *ws, void *stats,
                                   void *stream);

/* ---- Learned hyperparameter policy inside the unroll ---------------------
 * App. E "Policy Parameterization" (widths, bounds and initial values from
 * Table 2) and the log-residual loss of Sec. "Experiments".  At iterate z^k
 * a per-row network over xi_rho,i = (l_rho,i, s_i, y_i, rbar_p,i,
 * log(|rbar_d|_inf + 1e-12), s_i - s~_i, s_i - s^{k-1}_i) and a per-instance
 * network over xi_alpha = (l_alpha, log(|rbar_p|_inf + 1e-12),
 * log(|rbar_d|_inf + 1e-12), log(|s - s~|_inf + 1e-12), log(|s - s^{k-1}|_inf
 * + 1e-12)) move the logits, l^{k+1} = l^k + MLP(xi^k), and
 *   rho^k = exp(log 1e-3 + (log 1e3 - log 1e-3) sigmoid(l_rho^{k+1})),
 *   alpha^k = 2 sigmoid(l_alpha^{k+1})
 * drive the step z^k -> z^{k+1} (rho^k rectified per SOC/PSD block).  Here
 * r_p = A x + s - b, r_d = P x + q - A'y (the sign of cosmo_residual_loss),
 * rbar = r / N with N_p = max(|Ax|, |s|, |b|)_inf, N_d = max(|Px|, |q|,
 * |A'y|)_inf (rbar = 0 when N = 0); the two ADMM residuals are 0 at k = 0.
 * Loss per instance: L = sum_{k=1..K} log(|r_d^k|^2 / D_d + |r_p^k|^2 / D_p),
 * with D = the squared norms at z^0 held constant (1 when zero).
 *
 * theta (d) [COSMO_POLICY_PARAMS] of the plan's dtype, shared by the batch:
 *   penalty network: W1 [7][32] (input-major), b1 [32], W2 [32][32]
 *   (input-major), b2 [32], w3 [32], b3 [1]; then the relaxation network the
 *   same with W1 [5][32]; then l_rho^0 [4] for zero, nonnegative, SOC and PSD
 *   rows, and l_alpha^0 [1].  Hidden layers are ReLU.
 * Reverse mode: ties in an infinity norm or a normaliser's max share the
 * cotangent evenly; |.| has derivative 0 at 0.  Calls run eagerly (they are
 * not recorded into graphs) and, like the other calls, use no floating-point
 * atomics: results are deterministic. */
#define COSMO_POLICY_PARAMS 2631

/* Bytes of the policy's own device memory: ptape (the logits of every step
 * and the loss denominators; written by the forward, read by the backward)
 * and pws (scratch, used by both).  Either pointer may be NULL. */
cosmo_status cosmo_policy_sizes(const cosmo_plan *plan, size_t *ptape_bytes, size_t *pws_bytes);

/* K steps with the policy choosing (rho^k, alpha^k).
 *   theta (d) as above.  x0, s0, y0 (d, nullable: zeros).
 *   rho (d) [K][m_tot], alpha (d) [K][B]: outputs, the penalties and
 *   relaxations chosen (pass them to cosmo_policy_backward).
 *   xK, sK, yK (d, nullable) outputs.  loss (d) [B] output.
 *   tape (d) [tape_bytes] (NULL: forward only), ptape (d) [ptape_bytes],
 *   ws (d) [fwd_ws_bytes], pws (d) [pws_bytes], stats (d, nullable). */
cosmo_status cosmo_policy_forward(cosmo_plan *plan, const void *theta, const void *x0, const void *s0,
                                  const void *y0, void *rho, void *alpha, void *xK, void *sK, void *yK, void *loss,
                                  void *tape, void *ptape, void *ws, void *pws, void *stats, void *stream);

/* Gradient of the summed loss over the batch.  theta, rho, alpha, tape,
 * ptape as written by cosmo_policy_forward.  Outputs (d): gtheta
 * [COSMO_POLICY_PARAMS] (required), grho [K][m_tot] and galpha [K][B]
 * (required: the cotangents of the chosen penalties and relaxations),
 * gx0, gs0, gy0 (nullable).  ws (d) [bwd_ws_bytes], pws (d) [pws_bytes]. */
cosmo_status cosmo_policy_backward(cosmo_plan *plan, const void *theta, const void *rho, const void *alpha,
                                   const void *tape, const void *ptape, void *gtheta, void *grho, void *galpha,
                                   void *gx0, void *gs0, void *gy0, void *ws, void *pws, void *stats,
                                   void *stream);

/* ---- Vanilla COSMO run to tolerance ---------------------------------------
 * The baseline of Sec. "Experiments" (App. D: zero start, fixed alpha; the
 * residual-balancing penalty the paper cites from OSQP: one scalar per
 * instance, times eq_scale on zero-cone rows).  Each instance runs until
 *   |r_p|_inf <= eps_abs + eps_rel N_p  and  |r_d|_inf <= eps_abs + eps_rel N_d
 * (r_p = A x + s - b, r_d = P x + q - A'y, N_p = max(|Ax|, |s|, |b|)_inf,
 * N_d = max(|Px|, |q|, |A'y|)_inf), checked every K steps (the plan's K;
 * K = 1 counts steps exactly).  With `adapt`, every `interval` steps (a
 * multiple of K) the penalty of each instance not yet converged becomes
 * clip(rho sqrt((|r_p|/N_p) / (|r_d|/N_d)), rho_min, rho_max) when that
 * moves it by more than a factor tol_factor.  The batch runs until every
 * instance has passed the test or max_iter steps are done; an instance that
 * passed keeps iterating with the others (its count is the first check it
 * passed). */
typedef struct {
  double rho0;        /* initial penalty scalar (> 0) */
  double eq_scale;    /* multiplier on zero-cone rows (> 0) */
  double alpha;       /* relaxation, in (0, 2) */
  double eps_abs, eps_rel;   /* >= 0, not both 0 */
  double tol_factor;  /* >= 1 */
  double rho_min, rho_max;   /* 0 < rho_min <= rho0 <= rho_max */
  int32_t max_iter;   /* >= 1 */
  int32_t interval;   /* >= 1, a multiple of K */
  int32_t adapt;      /* 0 or 1 */
  int32_t pad;
} cosmo_solve_options;

/* Bytes of the solver's own device scratch (penalties and relaxations of a
 * chunk, residual vectors and per-instance norms, a copy of the iterate). */
cosmo_status cosmo_solve_size(const cosmo_plan *plan, size_t *sws_bytes);

/* x (d) [n_tot], s, y (d) [m_tot]: the start (in) and, per instance, the
 * iterate at its own count (out; the last one where max_iter came first).
 * iters (h) [B]: steps to tolerance, -1 where max_iter was reached first.
 * rho_out (h, nullable) [B]: the final penalty scalars.  ws (d)
 * [fwd_ws_bytes], sws (d) [sws_bytes], stats (d, nullable).  Returns when the
 * solve is done: the host reads the B residual norms after every K steps. */
cosmo_status cosmo_solve(cosmo_plan *plan, const cosmo_solve_options *opt, void *x, void *s, void *y,
                         int32_t *iters, double *rho_out, void *ws, void *sws, void *stats, void *stream);

/* Final-residual loss per instance, L_i = ||A x + s - b||^2 + ||P x + q - A'y||^2
 * (the dual residual sign follows the fixed point of the iteration above,
 * at which P x + q - A'y = 0), and its gradient when gx, gs, gy are non-NULL:
 *   gx = 2A'r_p + 2P r_d,  gs = 2 r_p,  gy = -2 A r_d.
 * loss (d) [B].  ws (d) [fwd_ws_bytes] of the same plan. */
cosmo_status cosmo_residual_loss(cosmo_plan *plan, const void *x, const void *s, const void *y, void *loss,
                                 void *gx, void *gs, void *gy, void *ws, void *stream);

/* Standalone projections (the same kernels as the unroll).  Block layouts are
 * host arrays; they are copied into the caller's workspace `ws` with a
 * blocking copy before the asynchronous launch.  `offset` is the first row of
 * each block inside `in` / `out`.  Block rows must not overlap. */

/* Bytes of device workspace for psd_proj / psd_proj_vjp / socp_proj(_vjp):
 * block descriptors plus 3 p^2 float64 of eigensolver scratch per PSD block. */
size_t cosmo_proj_workspace_size(int32_t nblk, const int32_t *order_or_dim);

/* eq:psd-proj per block: out = svec(U max(L, 0) U') of S = smat(in).
 * eigvals (d, nullable) [sum p], in no particular order inside a block;
 * eigvecs (d, nullable) [sum p^2], block b column-major p x p at offset
 * sum_{b'<b} p_{b'}^2, column i paired with eigvals i.  `refine` as in
 * cosmo_options.eig_refine. */
cosmo_status psd_proj(int32_t nblk, const int32_t *order, const int64_t *offset, cosmo_dtype dtype,
                      const void *in, void *out, void *eigvals, void *eigvecs, int32_t max_sweeps,
                      double eig_tol, int32_t refine, void *ws, void *stream);

/* psd_proj for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same operation, arguments and results as psd_proj, without `ws`.  The
 * scratch is the library's own device array of COSMO_PSD_STATIC_SCRATCH_BYTES
 * (one per device, held until the process ends); blocks whose
 * cosmo_proj_workspace_size exceeds it return COSMO_EUNSUPPORTED before any
 * launch.  The call allocates nothing.  Every call on a device shares that
 * device's array: calls that overlap on one device (several host threads or
 * streams) race and must be serialised by the caller. */
#define COSMO_PSD_STATIC_SCRATCH_BYTES (64u << 20)
cosmo_status psd_proj_static_scratch(int32_t nblk, const int32_t *order, const int64_t *offset, cosmo_dtype dtype,
                                     const void *in, void *out, void *eigvals, void *eigvecs, int32_t max_sweeps,
                                     double eig_tol, int32_t refine, void *stream);

/* eq:psd-cotangent-dk per block, reusing the decomposition of psd_proj:
 * gin = svec(U (L o (U' smat(gout) U)) U'), L the Loewner matrix of max(., 0)
 * (eq:lowner; f'(0) taken as 0). */
cosmo_status psd_proj_vjp(int32_t nblk, const int32_t *order, const int64_t *offset, cosmo_dtype dtype,
                          const void *eigvals, const void *eigvecs, const void *gout, void *gin, void *ws,
                          void *stream);

/* Comparison backward rules of the PSD projection (Sec. "Differentiating
 * Through the PSD Projection", paragraph "Alternative Approaches", and the
 * appendix on the PSD backward experiments).  Same arguments, layout and
 * errors as psd_proj_vjp, plus:
 *   rule COSMO_PSD_RULE_DK (0): eq:psd-cotangent-dk, identical to psd_proj_vjp;
 *   rule COSMO_PSD_RULE_NAIVE (1): eq:psd-cotangent with the cotangents that
 *     reverse mode gives U and L for U max(L, 0) U', F_ij = 1/(l_j - l_i)
 *     formed as written: on tied eigenvalues the result is inf or NaN, on
 *     close ones it loses accuracy (this is the rule's behaviour, not an
 *     error: no status reports it);
 *   rule COSMO_PSD_RULE_TIKHONOV (2): rule 1 for the projection of S + eps I,
 *     from the decomposition of S (same U, eigenvalues l + eps).
 * eps (finite) is read by rule 2 only.  Unknown rule: COSMO_EINVAL. */
#define COSMO_PSD_RULE_DK 0
#define COSMO_PSD_RULE_NAIVE 1
#define COSMO_PSD_RULE_TIKHONOV 2
cosmo_status psd_proj_vjp_rule(int32_t nblk, const int32_t *order, const int64_t *offset, cosmo_dtype dtype,
                               int32_t rule, double eps, const void *eigvals, const void *eigvecs, const void *gout,
                               void *gin, void *ws, void *stream);

/* Newton-Schulz comparison rule (eq:newton-schulz): the projection
 * Pi(S) = (S + sign(S) S) / 2 with sign(S) approximated by `iters` steps of
 * S_{k+1} = S_k (3 I - S_k^2) / 2 from S_0 = S / ||S||_F, and the reverse pass
 * through those unrolled products.  Blocks as for psd_proj (svec rows at
 * `offset`, order p <= COSMO_NS_MAX_ORDER, 0 <= iters <= COSMO_NS_MAX_ITERS);
 * out = svec of the symmetric part of Pi, gin = the input cotangent for the
 * output cotangent gout.
 * `tape` (device, caller-owned, psd_ns_tape_size bytes for the same blocks,
 * dtype and iters, 8-byte aligned) holds block descriptors, the norms and
 * (2 iters + 8) p^2 elements per block: every iterate and its square, kept by
 * psd_proj_ns for psd_proj_ns_vjp, which must follow with the same blocks,
 * dtype and iters on the same stream.  psd_proj_ns copies the descriptors in
 * and waits for that copy; both are otherwise stream-asynchronous.
 * psd_ns_tape_size returns 0 for invalid arguments. */
#define COSMO_NS_MAX_ORDER 1024
#define COSMO_NS_MAX_ITERS 200
size_t psd_ns_tape_size(int32_t nblk, const int32_t *order, cosmo_dtype dtype, int32_t iters);
cosmo_status psd_proj_ns(int32_t nblk, const int32_t *order, const int64_t *offset, cosmo_dtype dtype,
                         int32_t iters, const void *in, void *out, void *tape, void *stream);
cosmo_status psd_proj_ns_vjp(int32_t nblk, const int32_t *order, const int64_t *offset, cosmo_dtype dtype,
                             int32_t iters, const void *gout, void *gin, void *tape, void *stream);

/* Projection onto SOC blocks (t, w) of `dim` rows (closed form), and its VJP
 * (J is symmetric: identity inside the cone, zero inside its polar, else
 * 1/2 [[1, u'], [u, (1 + t/|w|) I - (t/|w|) u u']] with u = w/|w|). */
cosmo_status socp_proj(int32_t ncones, const int32_t *dim, const int64_t *offset, cosmo_dtype dtype,
                       const void *in, void *out, void *ws, void *stream);
cosmo_status socp_proj_vjp(int32_t ncones, const int32_t *dim, const int64_t *offset, cosmo_dtype dtype,
                           const void *in, const void *gout, void *gin, void *ws, void *stream);

/* Schedules of the CG solves (Table 2; Sec. "Matrix-Free Implicit
 * Differentiation"): form 0 = one workgroup per instance iterating to its own
 * tolerance (the default); form f = 1..4 = one cooperative launch over the
 * whole device with at most f workgroups per compute unit, the operator
 * passes of all instances spread over every workgroup and grid barriers
 * between phases (falls back to form 0 where cooperative launch is not
 * available).  Both forms compute the same iteration with the same stopping
 * rule; their sums are taken in different orders, each deterministic.
 * set_pcg_form: form outside 0..4 is COSMO_EINVAL; a cooperative form while
 * graph mode is on, or on a plan with dense blocks, is COSMO_EUNSUPPORTED.
 * With dense blocks, form 0 reads each block once per operator application:
 * the row products G v, the penalty weights and the transposed products
 * G'(D (A v)) are fused per row of G inside the instance's workgroup. */
cosmo_status cosmo_plan_set_pcg_form(cosmo_plan *plan, int32_t form);
cosmo_status cosmo_plan_get_pcg_form(const cosmo_plan *plan, int32_t *form);

/* Graph mode (enable = 0 or 1, default 0).  When on, cosmo_unroll_forward and
 * cosmo_unroll_backward record their whole launch sequence (all K steps, the
 * order-class streams included) into a HIP graph on the first call with a
 * given set of pointer arguments, and on every call replay it on `stream`
 * with one graph launch: one host call per unroll instead of several
 * launches per step.  The data behind the pointers may change between calls
 * (new rho, alpha, initial iterates); a call with any other pointer set
 * records anew (and frees the previous recording), so callers that replay
 * keep their buffers.  Recording happens on a stream the plan owns, so the
 * caller's stream may be the default stream.  While profiling is enabled the
 * calls launch eagerly.  Results are bitwise the same as eager launches.
 * Enabling it with a cooperative CG form selected is COSMO_EUNSUPPORTED
 * (cooperative launches are not recorded).  Set-up calls. */
cosmo_status cosmo_plan_set_graph(cosmo_plan *plan, int32_t enable);
cosmo_status cosmo_plan_get_graph(const cosmo_plan *plan, int32_t *enabled);

/* Autotuner: runs the forward unroll (no tape) under each schedule -- CG
 * forms 0, 2, 4 launched eagerly, and form 0 replayed from a graph -- on the
 * given rho, alpha and forward workspace, times the second of two runs with
 * events on `stream`, and keeps the fastest (CG form and graph mode) in the
 * plan.  Then, on plans with PSD blocks, it picks the PSD launch shapes (see
 * cosmo_plan_set_psd_schedule): each order class's eigensolve is timed alone
 * over forward runs under the class defaults and under the alternatives, and
 * the DK VJP on the last step's eigenpairs under both thread counts; each
 * keeps the faster (an error in that phase leaves the PSD shapes the plan
 * had).  A setup call, not for the hot path: it allocates scratch buffers
 * and waits for the stream, and it discards the plan's profiling records
 * (cosmo_plan_profile_read counts from zero afterwards).  ms (host, nullable) [4] receives the CG
 * timings in that order (-1 for schedules not run: problems whose reduced
 * matrix is diagonal have no CG, and only the eager and graph runs of form
 * 0 are timed for them); cosmo_plan_psd_tune_ms returns the PSD timings. */
cosmo_status cosmo_plan_autotune(cosmo_plan *plan, const void *rho, const void *alpha, void *ws, void *stream,
                                 double *ms);

/* Launch shapes of the PSD kernels (eq:psd-proj and eq:psd-cotangent-dk; a
 * schedule choice, not part of the method).  eig_threads (host) [4]: threads
 * per workgroup of the eigensolve for the order classes p <= 32, <= 64,
 * <= 128 and larger; each is the class default {64, 256, 512, 1024} or twice
 * it for the three smaller classes {128, 512, 1024} (the largest class has
 * no alternative).  vjp_threads: 1024 (16 waves, default) or 512 (8 waves)
 * per workgroup of the DK VJP.  Other values are COSMO_EINVAL.  The VJP
 * gives bitwise the same result in both shapes; the eigensolve's workgroup
 * sums are taken in a different order (results agree to rounding).  Setting
 * drops graph recordings.  Set-up calls. */
cosmo_status cosmo_plan_set_psd_schedule(cosmo_plan *plan, const int32_t *eig_threads, int32_t vjp_threads);
cosmo_status cosmo_plan_get_psd_schedule(const cosmo_plan *plan, int32_t *eig_threads, int32_t *vjp_threads);
/* Timings (ms) of the last cosmo_plan_autotune's PSD phase.  ms (host) [10]:
 * ms[c] for c = 0..3 is order class c's eigensolve over one forward under
 * the defaults, ms[4] one DK VJP pass under 1024 threads; ms[5 + c] and
 * ms[9] the same under the alternatives; -1 where nothing was timed (absent
 * classes, plans without PSD blocks, before the first autotune). */
cosmo_status cosmo_plan_psd_tune_ms(const cosmo_plan *plan, double *ms);

/* A plan's whole launch schedule (the choices cosmo_plan_autotune makes). */
typedef struct {
  int32_t pcg_form;            /* CG form, 0..4 (cosmo_plan_set_pcg_form)              */
  int32_t graph;               /* graph mode, 0 or 1 (cosmo_plan_set_graph)             */
  int32_t eig_threads[4];      /* eigensolve threads per order class                    */
  int32_t vjp_threads;         /* DK VJP threads, 1024 or 512                            */
} cosmo_schedule;

/* get: the plan's current schedule.  set: applies all of it or nothing (each
 * field is checked as by the single setters; on an error the plan keeps its
 * CG form and graph mode and the error names the field).  Set-up calls. */
cosmo_status cosmo_plan_get_schedule(const cosmo_plan *plan, cosmo_schedule *sched);
cosmo_status cosmo_plan_set_schedule(cosmo_plan *plan, const cosmo_schedule *sched);

/* Problem signature of a plan, the key of the schedule cache: the device's
 * target name (e.g. gfx950) and compute-unit count, dtype, K, B, n_tot,
 * m_tot, and a 64-bit FNV-1a hash of the options, the per-instance offsets,
 * the nonzero counts of A and P, the cone structure (SOC count, PSD order
 * classes with their sizes and largest orders) and the dense blocks' shapes.
 * The values of the problem data are not part of it.  buf (host) receives a
 * NUL-terminated string of printable characters; len < its length + 1 is
 * COSMO_EINVAL (256 bytes always suffice). */
cosmo_status cosmo_plan_signature(const cosmo_plan *plan, char *buf, int64_t len);

/* Schedule cache: a text file of JSON objects, one per line,
 *   {"key": "<signature>", "pcg_form": f, "graph": g,
 *    "eig_threads": [a, b, c, d], "vjp_threads": v}
 * load: *found = 1 and *sched set from the last line with that key, else
 * *found = 0 (a missing file is a miss).  Lines this library did not write
 * are skipped.  store: rewrites the file (through `path`.tmp, then rename)
 * with every other key's lines kept and this key's line replaced or added;
 * an unwritable path is COSMO_EINVAL.  Keys are 1..255 printable characters
 * without quotes or backslashes (COSMO_EINVAL otherwise).  Host-only calls;
 * concurrent stores to one file from several processes may lose entries. */
cosmo_status cosmo_schedule_cache_load(const char *path, const char *key, cosmo_schedule *sched, int32_t *found);
cosmo_status cosmo_schedule_cache_store(const char *path, const char *key, const cosmo_schedule *sched);

/* Autotuner with the cache: looks up the plan's signature in the file at
 * `path`; on a hit (*hit = 1) applies that schedule without timing anything;
 * otherwise (*hit = 0) runs cosmo_plan_autotune on rho, alpha and ws and
 * stores the chosen schedule under the signature.  An entry the plan
 * rejects is treated as a miss and replaced. */
cosmo_status cosmo_plan_autotune_cached(cosmo_plan *plan, const void *rho, const void *alpha, void *ws, void *stream,
                                        const char *path, int32_t *hit);

/* Per-step taps for the PSD-backward comparison study (Fig. 3 of the paper:
 * each backward rule applied to the matrix the solver actually projects and
 * to the cotangent the reverse pass actually delivers).  tap (d): [K][2][m_tot]
 * of the plan's dtype, or NULL to stop.  While set, cosmo_unroll_backward
 * stores for each unrolled step k, at tap + 2 k m_tot, the projection input
 * v^k = s^ + y / rho_hat, and at tap + (2 k + 1) m_tot the cotangent of the
 * projection's output s+ (net of the dual update's share), both on every row.  The tap is caller-owned and must stay valid while
 * set; a recorded backward is recorded again when it changes. */
cosmo_status cosmo_plan_set_tap(cosmo_plan *plan, void *tap);

/* Measurement support (not needed on the hot path).  With profiling on, the
 * library records a pair of HIP events on the call's stream around every
 * launch of a kernel family: 0 = PSD eigensolve + reconstruction (all order
 * classes, fork to join), 1 = DK VJP, 2 = PCG solves, 3 = row/column SpMV
 * passes, and 4 + c = the eigensolve kernel of PSD order class c alone
 * (c = 0: p <= 32, 1: p <= 64, 2: p <= 128, 3: p <= 200), timed on the
 * stream it runs on.  profile_read waits for the recorded events and returns
 * the number of launches and their summed duration since profiling was
 * (re)enabled; kind outside 0..7 is COSMO_EINVAL. */
cosmo_status cosmo_plan_set_profiling(cosmo_plan *plan, int32_t enable);
cosmo_status cosmo_plan_profile_read(cosmo_plan *plan, int32_t kind, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* COSMO_UNROLL_H */
