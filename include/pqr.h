/*
 * pqr.h -- C ABI of libpqr: weighted-l1 penalized quantile regression (PQR)
 * solved by FS-QRPPA, the feature-splitting proximal point algorithm
 * (Algorithm 1 of "Scalable Ultra-High-Dimensional Quantile Regression with
 * Genomic Applications", arXiv 2601.02826), on one AMD MI355X (gfx950).
 *
 * The problem (eq. vanilla_QR with the weighted-l1 penalty):
 *
 *     min_beta  (1/n) sum_i rho_tau(y_i - x_i^T beta) + sum_{j>=1} lambda_j |beta_j|,
 *     rho_tau(u) = (tau - 1{u < 0}) u,   x_i = (1, x_i1, ..., x_ip),
 *
 * with lambda_j = lambda * w_j and an unpenalized intercept (lambda_0 = 0).
 * When the design is standardized the solver works on x~_ij = (x_ij - m_j)/s_j
 * (population sd) and reports coefficients on both scales.
 *
 * Conventions for every entry point:
 *  - Every call returns a pqr_status; nothing aborts or throws across the ABI.
 *    On failure pqr_last_error(ctx) holds a message.
 *  - "device pointer" means memory from hipMalloc (or a PyTorch HIP tensor);
 *    "host pointer" means ordinary process memory.
 *  - All device work runs on the stream given in pqr_options.stream (NULL =
 *    the default stream).  Calls on one context must not overlap.
 */
#ifndef PQR_H
#define PQR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PQR_OK = 0,
  PQR_ERR_INVALID_ARG = 1,   /* bad size, tau outside (0,1), negative or non-finite input */
  PQR_ERR_OOM = 2,           /* device allocation failed */
  PQR_ERR_DEVICE = 3,        /* a HIP call failed */
  PQR_ERR_NOT_CONVERGED = 4, /* max_iter reached; outputs hold the best certified iterates */
  PQR_ERR_DIVERGED = 5,      /* the H-norm monitor tripped twice after eta was doubled */
  PQR_ERR_UNSUPPORTED = 6    /* combination of formats or options not provided */
} pqr_status;

/* Storage formats of the design matrix X (values, not the intercept). */
typedef enum {
  PQR_X_F64 = 0,     /* IEEE double                                           */
  PQR_X_F32 = 1,     /* IEEE float                                            */
  PQR_X_BF16 = 2,    /* bfloat16; exact for the dosages 0, 1, 2               */
  PQR_X_FP8E4M3 = 3, /* OCP FP8 E4M3; exact for the dosages 0, 1, 2           */
  PQR_X_I8 = 4,      /* unsigned byte codes (dosages 0..2, any 0..255 value)  */
  PQR_X_2BIT = 5     /* 2-bit codes 0..3, four rows per byte                  */
} pqr_xfmt;

/* Iterate precision: the arithmetic of the FS-QRPPA state (beta, z, theta). */
typedef enum { PQR_ITER_F32 = 0, PQR_ITER_F64 = 1 } pqr_iter_prec;

/* Design matrix handed to pqr_create.
 *  data   : device pointer, column-major, element (i, j) at data[j*ld + i],
 *           i < n, j < p; src_fmt is PQR_X_F64, PQR_X_F32 or PQR_X_I8.
 *           Caller-owned; pqr_create copies it into the context's own padded
 *           store (format store_fmt), after which it may be freed.
 *  store_fmt : internal storage; integer-valued sources may use any format,
 *           floating sources PQR_X_F64 / PQR_X_F32 (converting a float source
 *           to BF16 is allowed and is then lossy).
 *  standardize : 1 = solve on standardized columns (zero-variance columns are
 *           excluded: their coefficient is 0), 0 = use X as given.          */
typedef struct {
  int64_t n, p, ld;
  int src_fmt;
  const void* data;
  int store_fmt;
  int standardize;
} pqr_design;

/* Solver options.  Zero/negative values select the documented defaults. */
typedef struct {
  double mu;            /* augmentation parameter (eq. fsppa_update); default
                           mu = mu_scale * sqrt(G+1) / (n * sd(y)), recomputed per y */
  double mu_scale;      /* default 0.1                                         */
  int G;                /* number of column blocks (decomposition of X); default 48,
                           capped at ceil(p/16); block boundaries are multiples of 16 */
  double eta_margin;    /* eta_g = (1 + margin) * mu * Lambda_g; default 0.01; a value in
                           (-1, 0) violates eta_g > mu Lambda_max on purpose (to exercise
                           the monitor that doubles eta and reports PQR_ERR_DIVERGED) */
  int lanczos_steps;    /* steps of the Lanczos estimate of Lambda_g; default 40 */
  int iter_prec;        /* pqr_iter_prec; default PQR_ITER_F32                 */
  double tol_gap;       /* stop when the FP64 relative duality gap <= tol_gap; default 1e-6 */
  int cert_every;       /* iterations between FP64 certificates; default 50     */
  int64_t max_iter;     /* default 1e6                                         */
  void* stream;         /* hipStream_t; NULL = default stream                  */
  int profile;          /* 1 = time every sweep launch with HIP events on `stream` */
  int intercept_block;  /* 1 (default) = the intercept is a block of its own (p_1 = 1,
                           Lambda = n) and the G feature blocks follow; 0 = the
                           intercept is the first column of the first feature block.
                           Set through pqr_default_options; 0 is honoured as given. */
  int rows_per_lane;    /* 0 = automatic (16 when n >= 8192 or for 2-bit, else 4); 4 or 16
                           forces the row geometry (the batched solver needs 16) */
  int launch_mode;      /* 0 (default) = pqr_solve replays each chunk of cert_every
                           iterations as one captured HIP graph (captured on a private
                           stream of the context, launched on `stream`; re-captured when
                           the step parameters change); 1 = every kernel launched from
                           the host.  Both run the same kernels in the same order.
                           With opt.profile the kernels are always launched directly. */
  int tile_override;    /* 0 (default) = batched solves choose their launch variants by
                           timing them (pqr_batch_tiles); 1 + PQR_TILE_VARIANTS b + a
                           forces back-product variant b (0..3) and union-product
                           variant a (0..2), for tests */
} pqr_options;

typedef struct pqr_ctx pqr_ctx;

/* Solution and report.  Output arrays are host pointers supplied by the
 * caller (any may be NULL to skip it):
 *   beta      p+1 doubles, coefficients on the original scale (intercept first)
 *   beta_std  p+1 doubles, coefficients on the solver's (standardized) scale
 *   z, theta  n doubles each: the auxiliary and dual variables of Algorithm 1
 * The gap is certified from the best bounds seen at any certificate: beta,
 * beta_std and z come from the evaluated iterate with the smallest P(beta), theta
 * from the evaluated iterate whose feasible dual point had the largest dual value,
 * so pqr_kkt(beta_std, theta) reproduces primal, dual and rel_gap.  (A warm start
 * from such a result begins from these two iterates; PQR_START_DEVICE continues
 * from the last iterate instead.) */
typedef struct {
  double* beta;
  double* beta_std;
  double* z;
  double* theta;
  int64_t iters;        /* FS-QRPPA iterations run                              */
  int64_t x_passes;     /* full reads of X (iterations + certificates + setup of this call) */
  int64_t certs;        /* duality-gap certificates evaluated                   */
  int64_t nnz;          /* nonzero coefficients (intercept excluded)            */
  double primal;        /* P(beta) in FP64                                      */
  double dual;          /* dual objective of the feasible point built from theta */
  double rel_gap;       /* (primal - dual) / primal                            */
  double lambda_max;    /* smallest lambda with the null fit optimal (same tau, weights) */
  double mu;            /* the mu used                                          */
  double seconds;       /* wall time of the call                                */
  double sweep_ms;      /* with opt.profile: summed duration of the sweep kernels
                           (pqr_solve_batch: of the batched back-product kernel)  */
  int64_t sweep_launches;
} pqr_result;

typedef enum {
  PQR_START_ZERO = 0,   /* beta = 0, z = y, theta = 0                           */
  PQR_START_HOST = 1,   /* from warm->beta_std, warm->z, warm->theta (host); z and
                           theta may be NULL (derived from beta, see pqr_solve)  */
  PQR_START_DEVICE = 2  /* continue from the state the previous solve left on the device
                           (warm starts along a lambda path; same y, tau and mu) */
} pqr_start;

/* Sets every field of *opt to its default. */
void pqr_default_options(pqr_options* opt);

/* Encodes X into the context's store, computes the column statistics (one
 * pass, integer sums for integer formats), partitions the columns into G
 * blocks and estimates Lambda_g = Lambda_max(X~_g^T X~_g) for every block by
 * Lanczos (text after eq. fsppa_update: power method or Lanczos).
 * On success *out owns its device memory until pqr_destroy. */
pqr_status pqr_create(pqr_ctx** out, const pqr_design* X, const pqr_options* opt);

/* Solves PQR for one (tau, lambda) by Algorithm 1.
 *  y        host, n doubles (copied)
 *  weights  host, p+1 doubles w_j >= 0 (w_0 ignored), or NULL for unit weights
 *  start    pqr_start; for PQR_START_HOST, warm must point to arrays of the
 *           sizes above (beta_std, z, theta).  warm->z may be NULL: then
 *           z = y - X~beta - beta0 (the residual of beta, so r = 0); warm->theta
 *           may be NULL: then theta_i = (tau - 1{z_i < 0}) / n, centred so
 *           that sum(theta) = 0 (a subgradient of the check loss at z)
 *  out      results; see pqr_result.  On PQR_ERR_NOT_CONVERGED out still holds
 *           the best certified iterates and their gap. */
pqr_status pqr_solve(pqr_ctx* ctx, const double* y, double tau, double lambda,
                     const double* weights, int start, const pqr_result* warm,
                     pqr_result* out);

/* FP64 optimality report for a given point (Prop. 1 and the dual of the
 * Lagrangian, eq. main_lagrangian).  beta_std: host p+1 doubles on the
 * solver's scale; theta: host n doubles.  Pure: no state changes.
 * rep[0] = primal P(beta), rep[1] = dual objective of the projected theta,
 * rep[2] = relative gap, rep[3] = max_j |x~_j^T theta'| / lambda_j over
 * penalized columns (<= 1 means dual feasible before scaling).  Columns with
 * weight 0 are unpenalized: theta' is first projected onto {sum theta = 0,
 * x~_j^T theta = 0 on them} and scaled back into the box (at most 4096 such
 * columns; the equalities hold to rounding, like sum theta = 0 for the
 * intercept). */
pqr_status pqr_kkt(pqr_ctx* ctx, const double* y, double tau, double lambda,
                   const double* weights, const double* beta_std, const double* theta,
                   double rep[4]);

/* lambda_max for (y, tau, weights) and, optionally, the per-column score
 * S_j = x~_j^T psi / n (host, p doubles) where psi is the null-fit dual
 * (psi_i = tau above the tau-quantile of y, tau-1 below, balanced on ties). */
pqr_status pqr_lambda_max(pqr_ctx* ctx, const double* y, double tau, const double* weights,
                          double* lambda_max, double* score);

/* Blocks in use.  *G receives the total number of blocks B (the G of
 * eq. fsppa_update, intercept block included when it is separate).  bounds
 * (host, B+1 ints) are feature-column boundaries: block b holds the feature
 * columns [bounds[b], bounds[b+1]); block 0 also holds the intercept (with
 * intercept_block = 1 it holds only the intercept: bounds[0] = bounds[1] = 0).
 * Lambda (host, B doubles) are the estimates of Lambda_max(X~_b^T X~_b). */
pqr_status pqr_blocks(pqr_ctx* ctx, int* G, int* bounds, double* Lambda);

/* One or more iterations from a given state with every parameter explicit,
 * for step-level checks.  beta_std (p+1), z (n), theta (n) are host doubles,
 * read and overwritten; eta is host, G doubles.  Runs exactly `iters`
 * iterations of Algorithm 1 with no stopping test. */
pqr_status pqr_iterate(pqr_ctx* ctx, const double* y, double tau, double lambda,
                       const double* weights, double mu, const double* eta, int64_t iters,
                       double* beta_std, double* z, double* theta);

/* Folded-concave penalties by L-step local linear approximation (Algorithm 2):
 * stage 0 is pqr_solve at unit weights from `start` (PQR_START_ZERO, or
 * PQR_START_DEVICE to continue from the state the previous solve on ctx left, e.g.
 * the last stage at the previous lambda of a path: the warm start of the paper's
 * path runs; same y and tau); stage l = 1..L solves
 * the weighted problem with lambda_j = lambda w_j, w_j = max(p'_lambda(|b_j|) /
 * lambda, wfloor), b the previous stage's coefficients on the standardized scale
 * and p' the SCAD derivative (eq. scad, penalty 0, a > 2) or the MCP derivative
 * (eq. mcp, penalty 1, a > 1), warm-started on the device from the previous stage
 * (PQR_START_DEVICE).  Zero weights (SCAD beyond a lambda, MCP beyond a lambda)
 * make columns unpenalized; the certificate then projects its dual point onto
 * x~_j^T theta = 0 for them (see pqr_kkt), so wfloor = 0 runs Algorithm 2 exactly;
 * a positive floor changes a stage's objective by at most wfloor lambda sum_j |b_j|
 * over the floored columns.
 *  weights_out  NULL or host, p+1 doubles: the last stage's weights (w_0 = 0)
 *  stage_iters  NULL or host, L+1 iteration counts
 *  out          the last stage's result (as pqr_solve); with opt.profile, sweep_ms
 *               and sweep_launches are summed over all stages
 * Stops at the first stage that does not return PQR_OK and returns its status. */
pqr_status pqr_solve_lla(pqr_ctx* ctx, const double* y, double tau, double lambda,
                         int penalty, double a, int L, double wfloor, int start,
                         double* weights_out, int64_t* stage_iters, pqr_result* out);

/* K problems that share X, y and the weights, with their own (tau_k, lambda_k),
 * solved together (Algorithm 1 for every k, iterated in lockstep).  The back-
 * products X~^T Theta of all k run on the int8 matrix cores over digit slices of
 * theta (exact integer arithmetic); every k is stopped by its own duality-gap
 * certificate (Prop. 1) on an exactly representable dual point: the projected theta'
 * truncated toward zero to multiples of unit_k = c 2^-27 (c the power of two
 * >= max(tau_k, 1 - tau_k)/n), its integer sum moved onto the largest or smallest
 * entry so that it sums to zero exactly, the dual ratios x~_j^T theta_q exact in
 * integers from one int8 matrix-core pass for all due k (pqr_kkt's FP64 pass for a k
 * whose sum cannot be moved inside the box).  Needs an int8 store with codes 0..127,
 * rows_per_lane 16, FP32 iterates, positive weights and, for the integer sums to
 * stay exact in int32 with 32-bit buffer offsets, n_pad * max(max_code, 1) * 65 <
 * 2^31, 512 n_pad < 2^31 and p_pad <= 16 * 64 * floor((2^31 - 1) / (64 max(max_code,
 * 1)) / 64) (the union product's 16 splits; about 4.2 million columns at max_code
 * 127), n_pad = n rounded up to a multiple of 1024 (PQR_ERR_UNSUPPORTED otherwise);
 * 1 <= K <= 128.
 *  y, weights  as in pqr_solve;  taus, lambdas  host, K doubles each
 *  outs        host array of K pqr_result (output arrays optional, as in pqr_solve);
 *              beta and z are the final iterate (a certified right-hand side stops
 *              iterating), theta the iterate whose dual point gave the best dual value,
 *              so primal, dual and rel_gap are reproduced from the exported beta, theta
 * Returns PQR_ERR_NOT_CONVERGED (outputs filled) if max_iter ends the solve first.
 * The single right-hand-side device state is discarded (PQR_START_DEVICE needs a
 * new pqr_solve afterwards). */
pqr_status pqr_solve_batch(pqr_ctx* ctx, const double* y, int K, const double* taus,
                           const double* lambdas, const double* weights, pqr_result* outs);

/* The launch variants the autotuner chose for batched solves of width K on this
 * context, and the mean time (ms) it measured for each candidate: the four of the
 * back-product (bgemm_ms, host, PQR_TILE_VARIANTS doubles, unused entries 0; timed on
 * the first batched solve of that width before its iterations) and the three of the
 * union product (baxpy_ms, same size; timed at the end of the first chunk of
 * cert_every iterations whose union of nonzero columns holds at least 1024 columns,
 * on that live union; baxpy_variant -1 if none has).  Variant 0 of each is the
 * default configuration; every variant computes identical results.  union_cols
 * receives the number of union columns the union product was timed on (0 if it was
 * not).  Any output pointer may be NULL.  PQR_ERR_INVALID_ARG if no batched solve of
 * that width has run on ctx. */
#define PQR_TILE_VARIANTS 8
pqr_status pqr_batch_tiles(pqr_ctx* ctx, int K, int* bgemm_variant, int* baxpy_variant,
                           double* bgemm_ms, double* baxpy_ms, int64_t* union_cols);

/* Many independent problems (X_i, y_i, tau_i, lambda_i), one per context, solved
 * together from zero starts: every still-running problem takes one FS-QRPPA
 * iteration (Algorithm 1, eq. fsppa_update) per round of five grouped kernel
 * launches on ctxs[0]'s stream, each grid covering the blocks of all problems;
 * each problem stops on its own FP64 duality-gap certificate (its own
 * cert_every, tol_gap, max_iter) and leaves the group.
 *  nprob        >= 1 distinct contexts; all need the same store format,
 *               rows_per_lane and iterate precision (PQR_ERR_UNSUPPORTED otherwise)
 *  ys           host, nprob pointers to n_i doubles
 *  taus, lambdas host, nprob doubles each
 *  weights      NULL, or host, nprob pointers (each NULL or p_i+1 doubles)
 *  outs         NULL or host array of nprob pqr_result, filled as by pqr_solve;
 *               with ctxs[0]'s profile option, sweep_ms is the summed duration of
 *               the grouped sweep launches (all problems), the same in every out
 *  statuses     NULL or host array of nprob statuses, one per problem
 * Returns PQR_OK if every problem converged, else the first problem's failure
 * (its message on that context).  Contexts must not be used concurrently. */
pqr_status pqr_solve_grouped(int nprob, pqr_ctx* const* ctxs, const double* const* ys,
                             const double* taus, const double* lambdas,
                             const double* const* weights, pqr_result* outs,
                             pqr_status* statuses);

/* pqr_kkt plus every column's dual value: v (host, p doubles) receives
 * x~_j^T theta' for the projected theta' of the certificate. */
pqr_status pqr_kkt_columns(pqr_ctx* ctx, const double* y, double tau, double lambda,
                           const double* weights, const double* beta_std, const double* theta,
                           double rep[4], double* v);

/* A context over the columns cols[0..ncols) (host, 0-based, in increasing order)
 * of parent: the design store and the column statistics are copied from the
 * parent on the device (the standardization is the parent's), blocks and step
 * sizes are set up for the subset.  opt NULL = the parent's options.  Independent
 * of the parent afterwards. */
pqr_status pqr_create_subset(pqr_ctx** out, pqr_ctx* parent, const int64_t* cols,
                             int64_t ncols, const pqr_options* opt);

/* Interleaved column order (the Discussion's block-permutation direction: a
 * column order that lowers Lambda_max(X_g^T X_g) of every block allows smaller
 * eta_g, i.e. longer beta steps in eq. beta_update).  cols (host, p int64)
 * receives the feature columns 0..p-1 ordered by (j mod G, j).  A context made
 * with pqr_create_subset(parent, cols, p, opt) and opt->G = G then has block b
 * (a contiguous run of its columns) holding residue class b up to the 16-column
 * alignment of the block bounds, so columns j and j + 1 of the parent sit in
 * different blocks; where correlation decays with column distance (an AR(1)
 * design, linkage along a chromosome) the blocks' Gram matrices lose their
 * off-diagonal mass.  The subset context's per-column arrays (weights, beta,
 * scores) follow the new order: element 1 + q is parent column cols[q].
 * Host only (no device work).  Errors: p < 1, G < 1, G > p or cols NULL. */
pqr_status pqr_interleaved_order(int64_t p, int G, int64_t* cols);

/* ---- learned warm start: the per-feature scoring network ------------------
 * Network 4 -> 64 -> 64 -> 2 with SiLU activations; 4610 FP32 parameters in the
 * order W1[64][4], b1[64], W2[64][64], b2[64], W3[2][64], b3[2], used as BF16
 * (round to nearest even) in every pass, FP32 activations and accumulations.
 * Features of column j (pqr_features): sqrt(n) S_j / sqrt(tau (1 - tau)) with
 * S_j the null-fit score of pqr_lambda_max, m_j / 2, tau, log(lambda/lambda_max).
 * Outputs: o0 = proposed beta~_j / sd(y), o1 = logit of beta~_j != 0.
 * All buffers below are device pointers; stream is a hipStream_t (NULL = default). */
int64_t pqr_mlp_param_count(void);
/* feats: device, p x 4 floats (row j = column j); also returns lambda_max */
pqr_status pqr_features(pqr_ctx* ctx, const double* y, double tau, double lambda,
                        const double* weights, float* feats, double* lambda_max);
pqr_status pqr_mlp_forward(const float* params, const float* feats, int64_t B, float* out,
                           void* stream);
/* Loss (mean over the B rows of w_reg (o0 - t)^2 + w_pos a softplus(-o1)
 * + (1 - a) softplus(o1)) and its gradient; workspace of pqr_mlp_workspace_bytes(B). */
int64_t pqr_mlp_workspace_bytes(int64_t B);
pqr_status pqr_mlp_grad(const float* params, const float* feats, const float* target,
                        const float* active, int64_t B, double w_reg, double w_pos,
                        void* workspace, float* grad, float* loss, void* stream);
/* pqr_mlp_grad without a workspace and without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight training
 * loops, harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * pqr_mlp_grad; the partial gradients live in a library-owned device array of
 * PQR_MLP_NOALLOC_MAX_ROWS / 128 * 4 * (4610 + 1) floats (4.7 MB, one per GPU,
 * held until the process ends), looked up on the current device.  Calls that
 * overlap on one GPU share that array and race; sequential calls need no
 * clearing (every partial used is written first).  Errors: NULL pointers or
 * B < 1: PQR_ERR_INVALID_ARG; B > PQR_MLP_NOALLOC_MAX_ROWS: PQR_ERR_UNSUPPORTED. */
#define PQR_MLP_NOALLOC_MAX_ROWS 8192
pqr_status pqr_mlp_grad_noalloc(const float* params, const float* feats, const float* target,
                                const float* active, int64_t B, double w_reg, double w_pos,
                                float* grad, float* loss, void* stream);
/* One Adam step (step >= 1 counts from 1) on the 4610 parameters. */
pqr_status pqr_mlp_adam(float* params, const float* grad, float* m, float* v, int step,
                        double lr, double beta1, double beta2, double eps, void* stream);

typedef struct {
  int rounds;               /* reduced solves run                                   */
  int fallback;             /* 1 if the plain zero-start solve produced the answer */
  int64_t active_initial;   /* columns proposed by the network                      */
  int64_t active_final;     /* columns of the last reduced problem                  */
  int64_t reduced_iters;    /* iterations spent in reduced solves                   */
  double seconds_proposal, seconds_reduced, seconds_check;   /* cumulative          */
  /* with ctx's profile option: the reduced solves' sweep kernels, their summed
     duration, launches and algorithmic bytes (n |A| b + 4n + 20|A| per launch)   */
  double reduced_sweep_ms, reduced_sweep_bytes;
  int64_t reduced_sweep_launches;
} pqr_learned_report;

/* Learned warm start: the network (params, device) proposes coefficients and an
 * active set A = {j : o1_j > threshold} plus the 32 columns with the largest o1.
 * FS-QRPPA solves the problem restricted to A from that proposal (beta_j =
 * o0_j sd(y) on A, beta_0 = the tau-quantile of y, z = y - X~beta - beta_0 and
 * theta_i = (tau - 1{z_i < 0}) / n centred, as PQR_START_HOST with only beta);
 * the FP64 certificate on the full design then judges the result.  The first
 * round stops at 10 tol_gap when more rounds are allowed (enough to expose
 * violators), later rounds at tol_gap.  If the full gap exceeds tol_gap, the
 * columns outside A whose |x~_j^T theta'| exceeds lambda_j (1 + 1e-6) join A and
 * the next round starts from the previous solution; with no violator the next
 * round is solved 4x tighter (at most max_rounds reduced solves).  If no round
 * passes, the plain FS-QRPPA solve from a zero start on the full design gives the
 * answer (rep->fallback = 1).  The reported rel_gap is always the full design's
 * certificate. */
pqr_status pqr_solve_learned(pqr_ctx* ctx, const double* y, double tau, double lambda,
                             const double* weights, const float* params, double threshold,
                             int max_rounds, pqr_result* out, pqr_learned_report* rep);

/* Screened warm start (the Discussion's screening direction, Sec. 8, made exact by
 * the certificate; a non-learned counterpart of pqr_solve_learned): the sequential
 * strong rule on the null-fit scores S_j of pqr_lambda_max proposes the active set
 * A = {j : |S_j| >= (2 lambda - lambda_prev) w_j} (budget = 0; lambda_prev <= 0 means
 * lambda_max), or the `budget` columns with the largest |S_j| / w_j (budget > 0);
 * zero weights always join A, and an empty A starts from the 32 best scores.
 * FS-QRPPA then solves the problem restricted to A from beta = 0, beta_0 = the
 * tau-quantile of y, and the same rounds as pqr_solve_learned follow: the FP64
 * certificate on the full design decides, columns outside A with |x~_j^T theta'| >
 * lambda_j (1 + 1e-6) join A, and after max_rounds the plain zero-start solve
 * answers.  The reported rel_gap is always the full design's certificate; rep is
 * filled as for pqr_solve_learned.  Errors: max_rounds < 1, budget < 0 or a negative
 * or non-finite lambda_prev: PQR_ERR_INVALID_ARG. */
pqr_status pqr_solve_screened(pqr_ctx* ctx, const double* y, double tau, double lambda,
                              const double* weights, double lambda_prev, int64_t budget,
                              int max_rounds, pqr_result* out, pqr_learned_report* rep);

void pqr_destroy(pqr_ctx* ctx);
const char* pqr_last_error(const pqr_ctx* ctx);
const char* pqr_status_string(pqr_status s);

#ifdef __cplusplus
}
#endif
#endif /* PQR_H */
