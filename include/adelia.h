/*
 * adelia.h: C ABI of the MI355X (gfx950) library for the INLA objective over
 * block-tridiagonal-arrowhead (BTA) precision matrices and its exact reverse-mode gradient.
 *
 * Paper: "ADELIA: Automatic Differentiation for Efficient Laplace Inference Approximations"
 * (arXiv 2605.06392).  Section/equation numbers below refer to that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Precision: FP64 everywhere.  Matrices are column-major.
 * - BTA shape (Sec. II-B): n diagonal blocks of size b x b, sub-diagonal blocks
 *   B_i = [Q]_{i+1,i} (i = 0..n-2), arrow blocks C_i = [Q]_{T,i} of size a x b and the
 *   arrowhead tip T (a x a).  N = n*b + a.  Vectors of length N are time-major with the
 *   tip last.
 * - Device pointers unless stated otherwise.  The caller owns every buffer; no entry point
 *   keeps a pointer after it returns (except an inla_model, which owns its own copies).
 * - Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).  Every call
 *   only enqueues work on that stream and returns without synchronising, allocating or
 *   printing, so calls may be captured into a hipGraph.  Exceptions: adelia_create,
 *   inla_model_create/destroy (set-up time).  Bound on captures: an INLA call whose estimated
 *   number of kernel launches exceeds 60,000 (e.g. an FD Hessian of many passes) returns
 *   ADELIA_E_UNSUPPORTED, before enqueueing anything, when its stream is capturing: a capture
 *   of about 96,000 launches ended the process on the host, one of 44,000 ran normally, and the
 *   cause is not established.  Called eagerly, such calls run normally.
 * - Return codes: 0 = enqueued.  -k = argument k (1-based) is invalid.  ADELIA_E_* below.
 *   Numerical failure is reported asynchronously through a device int `info`: 0 = success,
 *   j > 0 = the leading minor of global order j is not positive definite (LAPACK POTRF
 *   convention); outputs are then undefined.  Nothing aborts and no exception crosses the ABI.
 * - Workspaces are caller-allocated device memory of at least the queried size, 256-byte
 *   aligned.  Workspace contents are scratch unless stated otherwise.
 * - Threading: a context is read-only after creation.  A workspace (and a model's saved
 *   factors inside it) must be used by one stream at a time.
 */
#ifndef ADELIA_H
#define ADELIA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ADELIA_OK 0
#define ADELIA_E_SHAPE (-100)       /* inconsistent or unsupported sizes                   */
#define ADELIA_E_WORKSPACE (-101)   /* workspace too small or misaligned                     */
#define ADELIA_E_HIP (-102)         /* a HIP runtime call failed                             */
#define ADELIA_E_UNSUPPORTED (-103) /* a valid request this build does not implement         */
#define ADELIA_E_STATE (-104)       /* e.g. inla_grad with REUSE but no saved forward pass   */

typedef struct adelia_ctx_s* adelia_ctx;
typedef struct inla_model_s* inla_model;
typedef struct inla_batch_s* inla_batch;

/* Largest block size b (also k * ns of an INLA model).  The matrix cores read every operand of
 * the sweeps (up to a b x (b + 65) block) through 32-bit buffer descriptors, so a block of 2 GiB
 * or more could not be addressed; larger shapes are rejected with ADELIA_E_SHAPE (workspace
 * queries return 0) rather than computed wrongly. */
#define ADELIA_MAX_BLOCK 16320

typedef struct {
  int32_t n; /* number of diagonal blocks, >= 1        */
  int32_t b; /* block size, 1..ADELIA_MAX_BLOCK         */
  int32_t a; /* arrowhead width, 0..64                  */
} adelia_bta_shape;

/* Context bound to one HIP device (made current by the call).  Returns 0 or ADELIA_E_HIP. */
int adelia_create(adelia_ctx* ctx, int device);
int adelia_destroy(adelia_ctx ctx);
/* Static English text for a return code. */
const char* adelia_strerror(int code);
/* Library version string. */
const char* adelia_version(void);

/* ---------------------------------------------------------------------------------------
 * Batched FP64 GEMM on matrix cores (v_mfma_f64_16x16x4): for z in [0, batch):
 *   C_z = alpha * op(A_z) * op(B_z) + beta * C_z,  op(X) = X or X^T (trans* = 0 or 1),
 * with A_z = A + z*strideA etc.  C is M x N (ld ldc); op(A) is M x K; op(B) is K x N.
 * `uplo` = 0 writes all of C, 1 writes only the lower triangle (r >= c) of C.
 * A helper entry point used by the factorisations; exported for testing and for callers
 * that want the same tile kernel.  beta == 0 never reads C.  Errors: -k for argument k;
 * ADELIA_E_SHAPE when uplo == 1 and M != N, or when one operand (of one batch entry) spans
 * 2 GiB or more (the tile kernel addresses each operand through a 32-bit buffer range).
 * --------------------------------------------------------------------------------------- */
int adelia_dgemm(adelia_ctx ctx, int transA, int transB, int M, int N, int K, double alpha,
                 const double* A, int lda, long long strideA, const double* B, int ldb,
                 long long strideB, double beta, double* C, int ldc, long long strideC,
                 int batch, int uplo, void* stream);

/* ---------------------------------------------------------------------------------------
 * BTA factorisation (Sec. III-A-1, Alg. 1): the fused block Cholesky with the lower
 * triangular solve.  For i = 1..n:
 *   L_Di = chol(D_i - L_B{i-1} L_B{i-1}^T),  L_Bi = B_i L_Di^-T,
 *   L_Ci = (C_i - L_C{i-1} L_B{i-1}^T) L_Di^-T,  z_i = L_Di^-1 (r_i - L_B{i-1} z_{i-1}),
 * then L_T = chol(T - sum_i L_Ci L_Ci^T) and z_T = L_T^-1 (r_T - sum_i L_Ci z_i).
 * In/out (device, column-major):
 *   D    n blocks b x b (block i at D + i*b*b, ld b).  Lower triangle read; on exit holds L_Di
 *        (lower; the upper triangle of each block is overwritten with zeros).
 *   B    n-1 blocks b x b (ld b): in B_i = [Q]_{i+1,i}, out L_Bi.  May be NULL iff n == 1.
 *   C    n blocks a x b (ld a): in C_i, out L_Ci.  May be NULL iff a == 0.
 *   T    a x a (ld a): lower triangle in, out L_T (upper zeroed).  May be NULL iff a == 0.
 *   Dinv n blocks b x b (ld b): out G_i = L_Di^-1 (lower, upper zeroed).  Required: it is the
 *        form in which bta_solve and bta_selinv consume the diagonal factors.
 *   rhs  NULL, or length N: in r, out z = L^-1 r (forward solve fused into the sweep).
 *   logdet  device scalar out: log|Q| = 2 sum log diag(L).
 *   info    device int32 out (see conventions).
 * Workspace: adelia_bta_workspace_bytes(shape, ADELIA_WS_FACTOR).
 * --------------------------------------------------------------------------------------- */
#define ADELIA_WS_FACTOR 1
#define ADELIA_WS_SOLVE 2
#define ADELIA_WS_SELINV 4
size_t adelia_bta_workspace_bytes(adelia_bta_shape shape, int which);

int bta_factor(adelia_ctx ctx, adelia_bta_shape shape, double* D, double* B, double* C,
               double* T, double* Dinv, double* rhs, double* logdet, int32_t* info, void* ws,
               size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * bta_factor without a workspace argument, for callers that cannot allocate device memory
 * (code under hipGraph capture, serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, in/out contract, numbering of argument errors and results as bta_factor, minus
 * `ws` and `ws_bytes`: the call allocates nothing and works in a static device array of
 * ADELIA_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on until the
 * process ends (its address is taken by adelia_create, with the context's device current).
 * Shapes whose factor workspace, adelia_bta_workspace_bytes(shape, ADELIA_WS_FACTOR), exceeds
 * that size return ADELIA_E_WORKSPACE before anything is enqueued (adelia_last_error says
 * how much the shape needs); ADELIA_E_HIP if the array's address could not be obtained.
 * Every call on a device shares that device's array: calls that overlap in time on one device
 * (other streams, other contexts or threads) race and give undefined results; calls in order
 * on one stream are safe.  The array keeps the last call's contents; everything a call reads
 * from it is written by that call first.
 * --------------------------------------------------------------------------------------- */
#define ADELIA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int bta_factor_noalloc(adelia_ctx ctx, adelia_bta_shape shape, double* D, double* B, double* C,
                       double* T, double* Dinv, double* rhs, double* logdet, int32_t* info,
                       void* stream);

/* ---------------------------------------------------------------------------------------
 * Uneven batch (Sec. III-A-1, Alg. 1, applied to many independent matrices at once; the
 * batched evaluation of many instances is the setting of Sec. IV): factorises `count`
 * independent BTA matrices whose (n, b, a) differ, with the same in/out contract per matrix
 * as bta_factor.  Matrices with equal b share every launch of their block sweep (one launch
 * per step covers all of them; a matrix with fewer blocks drops out of the launches past its
 * last block, a smaller arrow is padded with identity rows).  Groups with different b run one
 * after the other on `stream`.
 *   shapes               host array [count]: the (n, b, a) of each matrix.
 *   D, B, C, T, Dinv     host arrays [count] of device pointers, laid out as for bta_factor
 *                        (B[i] may be NULL iff n_i == 1, C[i] and T[i] iff a_i == 0).
 *   rhs                  NULL (no solve), or a host array [count] of device pointers, all
 *                        non-NULL: length N_i, in r_i, out z_i = L_i^-1 r_i.
 *   logdet, info         device arrays [count].
 * Workspace: adelia_bta_batched_workspace_bytes(count, shapes, rhs != NULL).  Matrices are
 * copied into the workspace and back, so they must not overlap each other.
 * Errors: ADELIA_E_SHAPE for an invalid shape (nothing is launched); argument errors as for
 * bta_factor, numbered for the first offending matrix.
 * --------------------------------------------------------------------------------------- */
size_t adelia_bta_batched_workspace_bytes(int count, const adelia_bta_shape* shapes, int with_rhs);
int bta_factor_batched(adelia_ctx ctx, int count, const adelia_bta_shape* shapes,
                       double* const* D, double* const* B, double* const* C, double* const* T,
                       double* const* Dinv, double* const* rhs, double* logdet, int32_t* info,
                       void* ws, size_t ws_bytes, void* stream);

/* log|Q| from a factor produced by bta_factor (Sec. II-A: log|Q| = 2 sum log diag L):
 * reads the diagonals of the n blocks LD (ld b) and of LT (a x a, ld a; NULL iff a == 0).
 * out: device scalar. */
int bta_logdet(adelia_ctx ctx, adelia_bta_shape shape, const double* LD, const double* LT,
               double* out, void* ws, size_t ws_bytes, void* stream);

/* Solve Q x = rhs with the factor (Sec. III-A-2, Eqs. 3-5 for the upper sweep).
 * Dinv, LB, LC, LT as produced by bta_factor.  x: length N; in rhs (or z = L^-1 rhs when
 * flags & ADELIA_Z_INPUT), out Q^-1 rhs. */
#define ADELIA_Z_INPUT 1
int bta_solve(adelia_ctx ctx, adelia_bta_shape shape, const double* Dinv, const double* LB,
              const double* LC, const double* LT, double* x, int flags, void* ws,
              size_t ws_bytes, void* stream);

/* Selected inversion (Sec. III-A, Phase A): the blocks of Q^-1 on the BTA pattern,
 *   ZD_i = [Q^-1]_{i,i} (b x b, full symmetric), ZB_i = [Q^-1]_{i+1,i} (b x b),
 *   ZC_i = [Q^-1]_{T,i} (a x b, ld a), ZT = [Q^-1]_{T,T} (a x a),
 * swept from block n to 1 from the factor (Dinv, LB, LC, LT).  ZB may be NULL iff n == 1;
 * ZC, ZT may be NULL iff a == 0. */
int bta_selinv(adelia_ctx ctx, adelia_bta_shape shape, const double* Dinv, const double* LB,
               const double* LC, const double* LT, double* ZD, double* ZB, double* ZC,
               double* ZT, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * INLA model (Sec. II-A, II-B; Sec. III-B for k coregionalised fields).
 * The model is given by HOST arrays; inla_model_create validates every index, builds the
 * per-column observation lists and the union pattern of the spatial base matrices (integer
 * work), and copies everything to device memory it owns until inla_model_destroy.
 * A model also owns a second stream (default priority): the forward sweep of a gradient
 * (inla_grad, inla_grad_terms, inla_objective with ADELIA_SAVE_FACTORS) forms the block
 * inverses L_Di^-1 there while the sweep continues on the caller's stream; events order the
 * two, so the call behaves as one stream-ordered operation on the caller's stream (and can be
 * captured into a graph).  Calls on one model must come from one host thread at a time.
 * --------------------------------------------------------------------------------------- */
#define ADELIA_PARAM_UNIVARIATE 1 /* theta = [log scale, range, temporal, log tau], k == 1 */
#define ADELIA_PARAM_COREG 2      /* theta = [range(k), temporal(k), prec(k),
                                       lambda(k(k-1)/2) row-major strictly lower, log tau(k)] */
typedef struct {
  int32_t param;   /* ADELIA_PARAM_*                                                     */
  int32_t k;       /* fields, 1..4                                                        */
  int32_t ns;      /* spatial nodes per field; b = k*ns <= ADELIA_MAX_BLOCK                */
  int32_t nt;      /* time steps (n)                                                       */
  int32_t a;       /* fixed effects (arrowhead width), 0..64                               */
  int32_t n_obs;   /* observations                                                         */
  /* spatial base matrices c0, g1, g2 (ns x ns, symmetric) in CSR */
  const int32_t* c0_ptr; const int32_t* c0_idx; const double* c0_val;
  const int32_t* g1_ptr; const int32_t* g1_idx; const double* g1_val;
  const int32_t* g2_ptr; const int32_t* g2_idx; const double* g2_val;
  /* temporal matrices M0, M1, M2 (nt x nt, symmetric tridiagonal): diagonal (nt) and
   * sub-diagonal (nt-1) */
  const double* m0_diag; const double* m0_off;
  const double* m1_diag; const double* m1_off;
  const double* m2_diag; const double* m2_off;
  /* observations, sorted by (time, field): each touches 4 nodes of one field at one time
   * step with bilinear weights, plus the a covariates */
  const int32_t* obs_t; const int32_t* obs_field; const int32_t* obs_node; /* n_obs x 4 */
  const double* obs_w;  /* n_obs x 4 */
  const double* X;      /* n_obs x a, row-major */
  const double* y;      /* n_obs */
  double sigma_prior;   /* theta_k ~ N(0, sigma^2) */
  double tip_prec;      /* prior precision of the fixed effects */
} inla_model_desc;

/* Returns 0, ADELIA_E_SHAPE (with a message available from adelia_last_error), or a
 * negative argument index. */
int inla_model_create(adelia_ctx ctx, const inla_model_desc* desc, inla_model* out);
int inla_model_destroy(inla_model model);
/* Number of hyperparameters d of the model. */
int inla_model_dim(inla_model model);
/* Thread-local text of the last validation failure (set-up calls only). */
const char* adelia_last_error(void);

/* Workspace for evaluating `batch` theta points (mode = ADELIA_MODE_OBJECTIVE), or for the
 * gradients of `batch` points (mode = ADELIA_MODE_GRAD): the forward factors of Qc and Qp are
 * kept in it between inla_objective(SAVE) and inla_grad(REUSE).  A gradient workspace keeps
 * every block's factor, W and G^T G: about (4n + 6) b^2 doubles per matrix and point. */
#define ADELIA_MODE_OBJECTIVE 0
#define ADELIA_MODE_GRAD 1
/* A carry-only gradient workspace (see ADELIA_CARRY_ONLY): about n b^2 + 10 b^2 doubles per
 * matrix and point instead of (4n + 6) b^2. */
#define ADELIA_MODE_GRAD_CARRY 2
/* Workspaces of one objective or gradient by the two-sided split (ADELIA_SPLIT, batch 1): the
 * two halves' chains (about half the blocks each) and the one-block reduced system. */
#define ADELIA_MODE_OBJECTIVE_SPLIT 3
#define ADELIA_MODE_GRAD_SPLIT 4
size_t inla_workspace_bytes(inla_model model, int batch, int mode);

/* f(theta) of Eq. 1 for `batch` points theta (device, batch x d, row-major):
 *   f = 1/2 log|Qp| - 1/2 log|Qc| - 1/2 x*^T Qp x* + log l(y|x*,theta) + log p(theta),
 * Gaussian likelihood with precision tau_m = exp(theta_tau_m) per field, theta_k ~ N(0,s^2),
 * Qp = blkdiag(Q_x(theta), tip_prec I).  f: device, batch.  info: device int32, batch.
 * flags & ADELIA_SAVE_FACTORS (batch == 1, GRAD workspace): keep the factors for inla_grad. */
#define ADELIA_SAVE_FACTORS 1
/* flags & ADELIA_SPLIT (inla_objective with batch 1, inla_grad; workspace mode
 * ADELIA_MODE_OBJECTIVE_SPLIT / ADELIA_MODE_GRAD_SPLIT; not with SAVE, REUSE or CARRY_ONLY):
 * the two-phase decomposition of Sec. III-C with P = 2 partitions on one GPU.  The blocks are
 * split at the separator block s = (n - 1) / 2: blocks 0..s-1 are eliminated from the top and
 * blocks n-1..s+1 from the bottom (the sub-diagonal blocks of the model are symmetric, so the
 * reversed half is again a BTA chain), both halves' chains in the same launches, so the
 * sequence of block steps is about half as long; their Schur complements meet in the separator
 * block and the tip, which form the reduced system (one block and the arrowhead), factored
 * next.  The gradient runs the reduced system's selected inversion first and then both halves'
 * reverse passes from it.  Same results as without the flag up to rounding; `info` numbers a
 * failing column within its own half.  ADELIA_E_UNSUPPORTED for models with fewer than three
 * time steps. */
#define ADELIA_SPLIT 4
int inla_objective(inla_model model, const double* theta, int32_t batch, double* f,
                   int32_t* info, void* ws, size_t ws_bytes, int flags, void* stream);

/* f and its exact gradient (Sec. III-A-3, Eq. 5: Phases A, B, C plus the likelihood and
 * prior terms; Eqs. 10-11 for the coregional parameters).  theta, grad: device, d.
 * flags & ADELIA_REUSE_FACTORS: skip the forward pass and use the factors saved by the
 * preceding inla_objective(SAVE_FACTORS) on the same workspace and theta.  The reverse pass
 * consumes them (it overwrites G^T G with Z_D): a second REUSE call, or a REUSE call after any
 * other call on that workspace, returns ADELIA_E_STATE.  (A captured graph that replays a
 * REUSE call must replay the SAVE call before it.) */
#define ADELIA_REUSE_FACTORS 1
/* flags & ADELIA_CARRY_ONLY (workspace of mode ADELIA_MODE_GRAD_CARRY; not with REUSE): the
 * memory mode of Sec. III-A-1/2.  The forward keeps only each block's Schur-updated diagonal
 * block D_i - S_{i-1} (the carry, b x b) and its arrow rows [L_C | z]; the backward rebuilds
 * L_D and L_B block by block (one more block Cholesky per block), with G, W and G^T G in rings
 * of two blocks.  The result equals the stored-factor gradient up to rounding. */
#define ADELIA_CARRY_ONLY 2
int inla_grad(inla_model model, const double* theta, double* f, double* grad, int32_t* info,
              void* ws, size_t ws_bytes, int flags, void* stream);

/* f and the exact gradient at `batch` points (theta: device, batch x d, row-major; f, info:
 * batch; grad: batch x d, row-major) in one pass: every launch of the forward sweeps and of
 * the reverse pass covers the 2 * batch chains (Qc and Qp of each point) at once.  Workspace:
 * inla_workspace_bytes(model, batch, GRAD) or larger.  The saved factors are not reusable
 * with REUSE afterwards unless batch == 1.  Errors: -k for argument k, ADELIA_E_WORKSPACE,
 * ADELIA_E_HIP. */
int inla_grad_batched(inla_model model, const double* theta, int32_t batch, double* f,
                      double* grad, int32_t* info, void* ws, size_t ws_bytes, void* stream);

/* inla_grad with its decomposition, for diagnostics and identities: terms (device,
 * 5 + 6d doubles) = [f, log|Qp|, log|Qc|, |z|^2 (z = L_c^-1 r), tr([Qc^-1]_{T,T}),
 * PhaseA(d), PhaseB(d), PhaseC(d), dlog l/dtheta(d), dlog p/dtheta(d), grad(d)], where
 * PhaseA = -1/2 tr(Qc^-1 dQc), PhaseB = -1/2 x*^T dQp x*, PhaseC = 1/2 tr(Qp^-1 dQp)
 * (Sec. III-A-3, Eq. 5).  Same workspace and flags as inla_grad. */
int inla_grad_terms(inla_model model, const double* theta, double* terms, int32_t* info,
                    void* ws, size_t ws_bytes, int flags, void* stream);

/* Central finite-difference gradient (Sec. II-D, Eq. 2) on the GPU: the 2d+1 points
 * theta, theta +- h e_j are evaluated as batched objectives (in sub-batches of at most
 * `max_batch` points, sized by the caller's workspace = inla_workspace_bytes(model,
 * max_batch, OBJECTIVE)); grad_j = (f(theta+h e_j) - f(theta-h e_j)) / 2h, f = f(theta).
 * info: device int32, 2d+1 entries. */
int inla_fd_grad(inla_model model, const double* theta, double h, int32_t max_batch,
                 double* f, double* grad, int32_t* info, void* ws, size_t ws_bytes,
                 void* stream);

/* Posterior Hessian from exact gradients (Sec. III-D, Eq. 12): the exact gradients at the 2d+1
 * points theta, theta +- h e_j (in that order: +e_j at 1+2j, -e_j at 2+2j) are computed as in
 * inla_grad_batched, at most `max_batch` points per pass, and column j of H is
 * (grad f(theta + h e_j) - grad f(theta - h e_j)) / 2h, as the equation defines it (not
 * symmetrised).  The paper's step is h = 5e-3.  H: device, d x d, column-major.  f, grad:
 * device, f and its gradient at theta.  info: device int32, 2d+1 entries (one per gradient).
 * Workspace: inla_workspace_bytes(model, max_batch, GRAD) or larger.  Errors: -k for argument
 * k (h must be positive), ADELIA_E_WORKSPACE, ADELIA_E_HIP. */
int inla_hessian(inla_model model, const double* theta, double h, int32_t max_batch, double* f,
                 double* grad, double* H, int32_t* info, void* ws, size_t ws_bytes,
                 void* stream);

/* The finite-difference Hessian that Eq. 12 replaces (Sec. II-D): second-order central
 * differences over 2d^2+1 objective evaluations, batched in sub-batches of at most `max_batch`
 * points (workspace = inla_workspace_bytes(model, max_batch, OBJECTIVE)):
 *   H_jj = (f(theta + h e_j) - 2 f(theta) + f(theta - h e_j)) / h^2,
 *   H_jk = (f(+e_j+e_k) - f(+e_j-e_k) - f(-e_j+e_k) + f(-e_j-e_k)) / 4h^2  (steps of size h).
 * H: device, d x d, column-major (symmetric).  f: device, f(theta).  info: device int32,
 * 2d^2+1 entries: the centre, theta +- h e_j at 1+2j and 2+2j, then four points per pair
 * j < k in the order above.  Errors as inla_fd_grad. */
int inla_fd_hessian(inla_model model, const double* theta, double h, int32_t max_batch,
                    double* f, double* H, int32_t* info, void* ws, size_t ws_bytes,
                    void* stream);


/* ---------------------------------------------------------------------------------------
 * Uneven batch of INLA instances (Sec. III-A over many independent models at once; the
 * batched evaluation of Sec. IV): `count` models of different sizes -- time steps, spatial
 * size, fixed effects, observations -- evaluated together, each at its own theta.  Models with
 * the same block size b = k * ns form a group whose Qc and Qp chains share every launch of the
 * sweeps; inside a group the fixed effects are padded to the group's largest a with zero
 * covariate columns (f and the gradient are unchanged: the padded effects are decoupled and
 * keep their prior precision in Qp and Qc alike) and an instance with fewer time steps drops
 * out of the launches past its last block.  Groups run one after another on the stream.
 *   inla_batch_create: set-up call (allocates the per-member descriptors and padded covariate
 *     copies, and the batch's own side streams).  All models must live on the context's device
 *     and share the parameterisation, k and d; models of one block size must have the same
 *     spatial size.  The batch references the models, which must outlive it.  Returns 0,
 *     -k for argument k, ADELIA_E_SHAPE (message in adelia_last_error) or ADELIA_E_HIP.
 *   inla_batch_workspace_bytes: mode ADELIA_MODE_OBJECTIVE or ADELIA_MODE_GRAD (0 if invalid).
 *   inla_batch_objective: f of Eq. 1 for instance i at theta[i*d .. i*d+d) (device, row-major,
 *     count x d); f: device, count; info: device int32, count (as inla_objective).
 *   inla_batch_grad: f and the exact gradient (as inla_grad) of every instance; grad: device,
 *     count x d row-major.
 * Both evaluate calls enqueue only (capturable into a hipGraph) and return -k for argument k,
 * ADELIA_E_WORKSPACE or ADELIA_E_HIP.
 * --------------------------------------------------------------------------------------- */
int inla_batch_create(adelia_ctx ctx, int count, const inla_model* models, inla_batch* out);
int inla_batch_destroy(inla_batch batch);
/* Number of block-size groups of the batch (0 for NULL). */
int inla_batch_groups(inla_batch batch);
size_t inla_batch_workspace_bytes(inla_batch batch, int mode);
int inla_batch_objective(inla_batch batch, const double* theta, double* f, int32_t* info,
                         void* ws, size_t ws_bytes, void* stream);
int inla_batch_grad(inla_batch batch, const double* theta, double* f, double* grad,
                    int32_t* info, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * GEMM tile shapes and the autotuner (the tile choice per block size of the batched
 * evaluation).  Every dense product of the sweeps runs on 64 x 64 or 32 x 32 output tiles per
 * 256-thread workgroup; which one is kept in a process-wide table keyed by (block size b,
 * role), read when a launch is enqueued (a captured graph keeps the choices of its capture).
 * Roles (the profiler's GEMM groups): 1 trailing update, 2 block inversion, 4 Schur update,
 * 5 selected inversion V = L_C G, 6 Z_B, 7 Z_D.  Role 3, the panel rows of the split schedule, is
 * formed in place and always takes 64 x 64 tiles (each tile must hold all columns of its rows).
 * Entries not set take 64.  A context created while $ADELIA_TUNE_CACHE names a readable JSON file
 * ({"tiles": [{"b": 128, "role": "schur_update", "tile": 32}, ...]}) loads it; the autotuners
 * write the table back to that file.
 *   adelia_tune_set: -1 bad b, -2 bad role, -3 tile not 32 or 64.  adelia_tune_get: the tile
 *   (0 for invalid arguments).  adelia_tune_save / _load: 0 / entries read; ADELIA_E_UNSUPPORTED
 *   if the file cannot be written or read, ADELIA_E_SHAPE for a malformed file (nothing loaded).
 *   inla_autotune: for the model's block size, each role in turn tries both tiles with the
 *   others as chosen so far, timing `reps` runs of a batched objective (mode
 *   ADELIA_MODE_OBJECTIVE) or gradient (ADELIA_MODE_GRAD) evaluation at the `batch` <= 2d + 1
 *   points theta (device, batch x d), and keeps a tile only for a gain of more than 2%.
 *   Workspace: inla_workspace_bytes(model, batch, mode).  *changed (host): roles whose choice
 *   changed.  Synchronises the stream (set-up time; ADELIA_E_UNSUPPORTED while capturing).
 *   inla_batch_autotune: the same for every block-size group of an uneven batch, timing that
 *   group's part of inla_batch_objective / inla_batch_grad at theta (device, count x d).
 * --------------------------------------------------------------------------------------- */
int adelia_tune_set(int b, int role, int tile);
int adelia_tune_get(int b, int role);
int adelia_tune_clear(void);
int adelia_tune_save(const char* path);
int adelia_tune_load(const char* path);
int inla_autotune(inla_model model, const double* theta, int32_t batch, int mode, int reps,
                  void* ws, size_t ws_bytes, void* stream, int32_t* changed);
int inla_batch_autotune(inla_batch batch, const double* theta, int mode, int reps, void* ws,
                        size_t ws_bytes, void* stream, int32_t* changed);

/* ---------------------------------------------------------------------------------------
 * Opt-in kernel timing for measurement runs.  Between adelia_profile_start and
 * adelia_profile_stop every launch of the library's main kernels is bracketed by two HIP events
 * recorded on the launch's own stream (this inserts small gaps between launches, so time
 * whole calls without it).  stop() synchronises the device and returns, per kernel, the number
 * of launches, the summed event time, and the algorithmic flops and HBM bytes of those launches
 * (the work the method needs, not the padded tile work).  Not hipGraph-capture safe.
 * --------------------------------------------------------------------------------------- */
typedef struct {
  char name[32];
  int64_t launches;
  double ms;
  double flops;
  double bytes;
} adelia_kernel_stats;
int adelia_profile_start(adelia_ctx ctx, int max_launches);
int adelia_profile_stop(adelia_ctx ctx, adelia_kernel_stats* out, int max_entries, int* n_entries);

#ifdef __cplusplus
}
#endif
#endif /* ADELIA_H */
