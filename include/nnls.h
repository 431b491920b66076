/*
 * nnls.h -- C ABI of the MI355X (gfx950) anti-lopsided NNLS library (libnnls.so).
 *
 * The method (Nguyen & Ho, "Anti-lopsided Algorithm for Large-scale Non-negative Least
 * Squares", arXiv 1502.01645):
 *   Problem (1)   minimise 1/2 ||A x - b||^2 subject to x >= 0, A in R^{d x n}.
 *   Problem (2)   the same as f(x) = 1/2 x^T H x + h^T x with H = A^T A, h = -A^T b.
 *   Algorithm 1   rescale to Problem (5): Q_ij = H_ij / sqrt(H_ii H_jj), q_i = h_i / sqrt(H_ii),
 *                 solve for y, return x = y / sqrt(diag H) (rescaling (4)); H_ii = 0 keeps x_i = y_i.
 *   Algorithm 2   from y = 0 with gradient q: passive set P = {y_i > 0 or grad_i < 0}, masked
 *                 gradient gbar, exact step alpha = ||gbar||^2 / gbar^T Q gbar, projected update
 *                 y <- [y - alpha gbar]_+, incremental gradient grad += Q (y_new - y).
 *
 * Conventions shared by every entry point:
 *   - Array arguments are DEVICE pointers owned by the caller; the library keeps no pointer after
 *     a call returns (a batched plan keeps the pointers it was created with).
 *   - Matrices are row-major.  A is [d, n] with leading dimension lda >= n; B is [d, k] with
 *     ldb >= k; Q is [n, n]; q, Y0 and X are [n, k] (leading dimension k).
 *   - Every call is asynchronous and ordered on `stream` (a hipStream_t; NULL = the null stream).
 *     No call synchronises the device or allocates device memory: scratch space comes from the
 *     caller's workspace `ws` of `ws_bytes` bytes, sized by nnls_workspace_bytes().  The
 *     exceptions are set-up and file calls, each saying so: the batched plan's create and
 *     destroy, nnls_autotune, and the checkpoint calls nnls_mlp_save / nnls_mlp_load.
 *   - Arguments are validated on the host before any HIP call.  The return value is a
 *     nnls_error code; NNLS_OK means the work was enqueued.  Per-column outcomes of a solve are
 *     written on the device as nnls_col_status values.
 *   - Calls that share a workspace must not overlap; distinct workspaces make calls independent.
 */
#ifndef NNLS_H
#define NNLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Host-side return codes. */
enum nnls_error {
    NNLS_OK = 0,
    NNLS_E_ARG = -1,         /* a size, pointer, leading dimension or mode is invalid */
    NNLS_E_WORKSPACE = -2,   /* ws_bytes is smaller than nnls_workspace_bytes() */
    NNLS_E_HIP = -3,         /* a HIP runtime call failed (see nnls_last_hip_error) */
    NNLS_E_UNSUPPORTED = -4, /* valid arguments this build does not handle (e.g. n too large) */
    NNLS_E_IO = -5           /* a file could not be read or written, or is not a valid
                                checkpoint of this network (nnls_autotune's cache,
                                nnls_mlp_save / nnls_mlp_load) */
};

/* Per-column outcome of a solve, written to the device array `status`. */
enum nnls_col_status {
    NNLS_CONVERGED = 0,  /* relative KKT residual <= tol, or empty passive set */
    NNLS_MAXITER = 1,    /* max_iter updates done without meeting tol */
    NNLS_BREAKDOWN = 2,  /* line-search denominator gbar^T Q gbar not positive and finite; or
                            the workgroups of a whole-GPU solver stopped waiting for one another
                            (then iters = -1 and kkt = NaN) */
    NNLS_NONFINITE = 3,  /* NaN or Inf in the inputs or the iterate */
    NNLS_FELL_BACK = 4   /* warm start rejected (it raised the objective); solved from y = 0 */
};

/* Arithmetic of the Gram product H = A^T A, h = -A^T B. */
enum nnls_gram_mode {
    NNLS_GRAM_FP64 = 0,   /* FP64 inputs, FP64 products (for dtype NNLS_F64) */
    NNLS_GRAM_FP32 = 1,   /* FP32 inputs, plain FP32 fused multiply-adds (accuracy cross-check) */
    NNLS_GRAM_BF16X3 = 2  /* FP32 inputs split as hi + lo bfloat16; hi*hi + hi*lo + lo*hi on the
                             matrix cores with FP32 accumulation */
};

/* Element type of A, B, Q, q, Y0 and X. */
enum nnls_dtype { NNLS_F32 = 0, NNLS_F64 = 1 };

/* Operations for nnls_workspace_bytes. */
enum nnls_op {
    NNLS_OP_PREPARE = 0,
    NNLS_OP_SOLVE = 1,
    NNLS_OP_REFINE = 2,
    NNLS_OP_SCALES = 3,
    NNLS_OP_GRAM = 4
};

/* Bytes of device workspace that operation `op` needs for the given shape, mode and dtype
 * (0 if it needs none).  Host function; for NNLS_OP_SOLVE it reads the compute-unit count of the
 * current device (the whole-GPU solver keeps one partial vector per workgroup). */
size_t nnls_workspace_bytes(int op, int64_t d, int64_t n, int64_t k, int mode, int dtype);

/*
 * nnls_prepare -- Algorithm 1 up to the call of the solver: the Gram product of Problem (2)
 * and the rescaling to Problem (5).
 *
 *   d, n, k   rows of A, unknowns, right-hand sides (d >= 1, n >= 1, k >= 0)
 *   A         [d, n] (lda >= n), element type `dtype`
 *   B         [d, k] (ldb >= k); may be NULL when k == 0
 *   mode      nnls_gram_mode; NNLS_F64 requires NNLS_GRAM_FP64, NNLS_F32 requires FP32/BF16X3
 *   Q         out [n, n]: Q_ij = H_ij / (s_i s_j), Q_ii = 1 where H_ii > 0 (the Remark of
 *             Section 3), row and column i zero where H_ii = 0
 *   q         out [n, k]: q_ic = -(A^T B)_ic / s_i
 *   s         out [n] FP64: s_i = ||A_i||_2 computed in FP64 from the stored entries of A,
 *             or 1 where the column is zero
 * Element type of Q and q is `dtype`.
 */
int nnls_prepare(int64_t d, int64_t n, int64_t k, const void* A, int64_t lda, const void* B,
                 int64_t ldb, int mode, int dtype, void* Q, void* q, double* s, void* ws,
                 size_t ws_bytes, void* stream);

/*
 * nnls_prepare with NNLS_GRAM_BF16X3 (FP32 data) in its two launches, for a caller that times
 * or orders them separately; the workspace (nnls_workspace_bytes(NNLS_OP_PREPARE, ...,
 * NNLS_GRAM_BF16X3, NNLS_F32)) carries the split operands from the first call to the second,
 * so the same workspace must be passed to both and not be used in between.
 *   nnls_prepare_split    [A | B] split once into BF16 hi and lo planes (stored by column, in
 *                         ws), and s [n] FP64 = ||A_i||_2 (1 for a zero column) from the same
 *                         read of A.  Arguments as for nnls_prepare.
 *   nnls_prepare_product  Q [n, n] and q [n, k] from the planes in ws and s: the matrix-core
 *                         Gram of Problem (2) with the rescale of Problem (5) in its epilogue.
 * Errors as for nnls_prepare.
 */
int nnls_prepare_split(int64_t d, int64_t n, int64_t k, const float* A, int64_t lda,
                       const float* B, int64_t ldb, double* s, void* ws, size_t ws_bytes,
                       void* stream);
int nnls_prepare_product(int64_t d, int64_t n, int64_t k, const double* s, float* Q, float* q,
                         void* ws, size_t ws_bytes, void* stream);

/*
 * nnls_prepare is also these two calls in sequence, in any mode; they are exported so a caller
 * can time or reuse them separately.
 *
 * nnls_column_scales -- the scale vector of the rescaling (4): s_i = ||A_i||_2 in FP64, 1 where
 * the column is zero.  A [d, n] (lda >= n) of element type `dtype`; s out [n] FP64.
 * Workspace: nnls_workspace_bytes(NNLS_OP_SCALES, ...).
 *
 * nnls_gram_rescaled -- the Gram product of Problem (2) with the rescale of Problem (5) applied
 * in the epilogue, given s from nnls_column_scales: Q, q as for nnls_prepare.
 * Workspace: nnls_workspace_bytes(NNLS_OP_GRAM, ...).
 */
int nnls_column_scales(int64_t d, int64_t n, const void* A, int64_t lda, int dtype, double* s,
                       void* ws, size_t ws_bytes, void* stream);

/*
 * nnls_gram -- the Gram product of Problem (2) without the rescale: H = A^T A [n, n] (exactly
 * symmetric, its diagonal as computed) and h = -A^T B [n, k] (h may be NULL when k = 0).  Solving
 * (H, h) with nnls_solve and s = NULL runs Algorithm 2 on the unscaled problem, the method
 * without the anti-lopsided transformation (the contrast of Figure 1 against Figure 2).
 * Arguments, modes, layouts and errors as for nnls_gram_rescaled; workspace
 * nnls_workspace_bytes(NNLS_OP_GRAM, ...).
 */
int nnls_gram(int64_t d, int64_t n, int64_t k, const void* A, int64_t lda, const void* B,
              int64_t ldb, int mode, int dtype, void* H, void* h, void* ws, size_t ws_bytes,
              void* stream);
int nnls_gram_rescaled(int64_t d, int64_t n, int64_t k, const void* A, int64_t lda,
                       const void* B, int64_t ldb, int mode, int dtype, const double* s, void* Q,
                       void* q, void* ws, size_t ws_bytes, void* stream);

/*
 * nnls_solve -- Algorithm 2 on every column of q (they share Q), then x = y / s (rescaling (4)).
 *
 *   n, k      unknowns and right-hand sides (k >= 1)
 *   Q, q      the rescaled problem (as written by nnls_prepare, or any symmetric Q)
 *   s         [n] FP64 scales for the unscale step, or NULL to return y itself
 *   tol       stop when r(y) = ||min(y, Qy + q)||_2 / ||q||_2 <= tol (||q|| = 0: unnormalised);
 *             the test runs on a freshly recomputed gradient before a column is accepted
 *   max_iter  cap on updates per column; 0 means 5 n
 *   Y0        [n, k] start in the rescaled variables, or NULL for y = 0 (negative entries are
 *             clipped to 0)
 *   X         out [n, k]: x = y / s (the many-right-hand-side solver also keeps the start
 *             gradients of a warm start there until each column is done; X may be Y0 itself)
 *   iters     out [k] int32 updates done; kkt out [k] FP64 r(y) of the returned iterate in the
 *             arithmetic of the solve; status out [k] int32 nnls_col_status
 *   rows_read out [k] int64, may be NULL: rows of Q the solve's products read in total (passive
 *             rows of the line-search products, clipped rows of the gradient corrections, rows
 *             of exact gradient recomputations); 4 n bytes each for FP32 Q.  This is the
 *             S(n)-weighted work of the complexity lemma of Section 4.
 *   trace     out [k, trace_len, 2] FP32, may be NULL (then trace_len is ignored; otherwise
 *             trace_len >= 1): per column c and update count t < trace_len,
 *             trace[c][t][0] = r(y_t) and trace[c][t][1] = ||gbar_t||^2 of the iterate y_t after
 *             t updates, as the solve evaluated them (the convergence record that Figures 3 and
 *             4 of Section 5 plot against time).  Where the solve recomputed the gradient
 *             exactly at y_t, the entry holds the recomputed values.  Entries for t > iters[c]
 *             are not written.
 * The workspace size depends on the solver chosen for the shape; NNLS_OP_SOLVE sizes it for
 * the current device.  The environment variable NNLS_SOLVER=wg|regq|persistent|mrhs forces
 * the one-workgroup-per-column solver, the whole-GPU single-right-hand-side solver with Q held
 * in registers (n <= 5120) or streamed from memory, or the matrix-core many-right-hand-side
 * solver, where valid.  The many-right-hand-side solver forms its products in FP32 on the
 * matrix cores (for n <= 256 with Q held in registers).  NNLS_MRHS_PRODUCT=split16 opts into a
 * faster form for n <= 256: Q held as FP16 hi and lo parts (rows scaled by powers of two), each
 * update's two products formed as three FP16 matrix-core products with FP32 accumulation, every
 * term within 3 2^-22 of the FP32 product; the exact gradient behind every accepted stop is
 * still formed from the FP32 Q.  Every wait of the whole-GPU solvers is bounded (2^24 polls; the
 * environment variable NNLS_SPIN_LIMIT=m, 0 <= m <= 2^24, lowers it to test the give-up path):
 * a workgroup that gives up sets an abort word that ends the waits of all the others, and the
 * solve reports BREAKDOWN with iters = -1.
 */
int nnls_solve(int64_t n, int64_t k, int dtype, const void* Q, const void* q, const double* s,
               double tol, int32_t max_iter, const void* Y0, void* X, int32_t* iters,
               double* kkt, int32_t* status, int64_t* rows_read, float* trace,
               int32_t trace_len, void* ws, size_t ws_bytes, void* stream);

/*
 * nnls_solve_noalloc -- nnls_solve for callers that cannot allocate device memory or pass a
 * workspace: code under graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, solvers, results and errors as nnls_solve, without ws / ws_bytes: the solver
 * state lives in a fixed device array of NNLS_NOALLOC_SCRATCH_BYTES inside the library, one
 * per GPU, held from the first call on that GPU until the process ends.  The call allocates
 * nothing (no hipMalloc, no allocating library routine); the caller still owns Q, q, s, Y0 and
 * the outputs.
 *   - Returns NNLS_E_WORKSPACE when the solve would need more than NNLS_NOALLOC_SCRATCH_BYTES
 *     (nnls_workspace_bytes(NNLS_OP_SOLVE, ...) tells; the per-column solver needs 12 n k bytes
 *     for FP32, so that path is limited to n k <= 699050).
 *   - Every call on one GPU shares that GPU's array and the solvers reset what they read before
 *     they read it, so consecutive calls are independent; calls that overlap in time on one GPU
 *     (different streams, or host threads) race on the array and must not be issued.
 */
#define NNLS_NOALLOC_SCRATCH_BYTES (8u << 20)
int nnls_solve_noalloc(int64_t n, int64_t k, int dtype, const void* Q, const void* q,
                       const double* s, double tol, int32_t max_iter, const void* Y0, void* X,
                       int32_t* iters, double* kkt, int32_t* status, int64_t* rows_read,
                       float* trace, int32_t trace_len, void* stream);

/*
 * nnls_refine -- FP64 check and one refinement step against the ORIGINAL data (A, B).
 * For every column: r = A x - b and grad = A^T r in FP64; in the rescaled variables one masked
 * exact-line-search projected step of Algorithm 2 (the step length from ||A (gbar ./ s)||^2 in
 * FP64); the step is kept only if it lowers the KKT residual (below) without raising
 * 1/2 ||A x - b||^2.  Writes back X (FP32 or FP64 as `dtype`) and, for the returned x:
 *   kkt64 out [k]  relative KKT residual ||min(s .* x, grad ./ s)|| / ||A^T b ./ s|| in FP64,
 *                  with s the FP64 column norms of A (the rescaled-space residual of y = s .* x)
 *   obj64 out [k]  F = 1/2 ||A x - b||^2 of Problem (1) in FP64, summed from the residuals
 *                  A x - b (never from the Gram form 1/2 x^T H x + h^T x + 1/2 ||b||^2, which
 *                  cancels near a noiseless fit).  May be NULL: then F is not formed.  For
 *                  k > 4 forming it costs one more FP64 product A X (2 d n k flops); for
 *                  k <= 4 the residuals are formed anyway.
 * A, B, X have element type `dtype`.  Workspace: nnls_workspace_bytes(NNLS_OP_REFINE, ...);
 * errors NNLS_E_ARG (sizes < 1, null pointers other than obj64, lda < n, ldb < k),
 * NNLS_E_WORKSPACE.
 */
int nnls_refine(int64_t d, int64_t n, int64_t k, const void* A, int64_t lda, const void* B,
                int64_t ldb, int dtype, void* X, double* kkt64, double* obj64, void* ws,
                size_t ws_bytes, void* stream);

/*
 * Uneven batch: many independent problems (each Problem (1) with its own A_i [d_i, n_i] and a
 * single right-hand side b_i), solved by Algorithm 1 each, as one captured hipGraph: a batched
 * Gram with the rescale of Problem (5) (every tile of every problem an independent work item:
 * first the diagonal tiles, which give the scales, then the others), then per solver class a
 * resident grid that takes its problems from an atomic queue in longest-first order and runs
 * Algorithm 2 on each.  FP32 data, BF16x3 Gram, n_i <= 1024.
 *
 * Problems fall in size classes by n (n <= 64, 128, 256, 512, 1024); each class has a Gram tile
 * size (64 or 128) and a solver workgroup size (256, 512 or 1024 threads), the defaults (128,
 * 256) or the ones nnls_autotune measured fastest on this device.
 *
 * Pools are caller-owned device arrays; descriptor offsets are element offsets into them:
 *   A_pool  FP32, problem i's A_i row-major [d_i, n_i] at offA
 *   B_pool  FP32, b_i [d_i] at offB
 *   Q_pool  FP32 out, Q_i [n_i, n_i] at offQ
 *   q_pool  FP32 out, q_i [n_i] at offq;  s_pool FP64 out, s_i [n_i] at offq
 *           (s_i = sqrt of the computed Gram diagonal, 1 where it is 0)
 *   X_pool  FP32 out, x_i [n_i] at offX
 *   iters, kkt, status, rows_read (may be NULL): per problem, as for nnls_solve
 * The plan keeps these pointers; each launch recomputes every output.
 */
typedef struct {
    int64_t d, n, offA, offB, offQ, offq, offX;
} nnls_problem_desc;
typedef struct nnls_plan nnls_plan;

/* Device workspace bytes a plan over these problems needs (descriptors, Gram work items, queue
 * orders and counters, three FP32 vectors per unknown); 0 for invalid arguments.  Host
 * function. */
size_t nnls_batched_workspace_bytes(const nnls_problem_desc* host_desc, int64_t count);

/* Validates the descriptors, copies them, the Gram work items and the longest-first orders into
 * `ws` (blocking host-to-device copies, done once here), captures the graph on capture_stream (a
 * created stream, not the null stream) and instantiates it.  The workspace must stay allocated
 * and unused by other calls while the plan lives.  tol and max_iter as for nnls_solve (max_iter
 * 0: 5 n_i per problem).  tune_cache: path of a cache written by nnls_autotune, or NULL; its
 * entries for this device's architecture set the per-class parameters (a missing or unreadable
 * file leaves the defaults). */
int nnls_batched_plan_create(const nnls_problem_desc* host_desc, int64_t count, double tol,
                             int32_t max_iter, const char* tune_cache, const float* A_pool,
                             const float* B_pool, float* Q_pool, float* q_pool, double* s_pool,
                             float* X_pool, int32_t* iters, double* kkt, int32_t* status,
                             int64_t* rows_read, void* ws, size_t ws_bytes, void* capture_stream,
                             nnls_plan** out);

/* One launch of the plan's graph on `stream` (asynchronous). */
int nnls_batched_plan_launch(nnls_plan* plan, void* stream);

/* Releases the plan's graph (not the pools or the workspace). */
void nnls_batched_plan_destroy(nnls_plan* plan);

/* Operations nnls_autotune can tune. */
enum nnls_tune_op {
    NNLS_TUNE_BATCHED = 1  /* the uneven batch: Gram tile size and solver workgroup size */
};

/*
 * nnls_autotune -- measures, on this device, the per-size-class parameters of operation `op`
 * for problems of the given shapes and records the fastest in the JSON cache file cache_path
 * (created or updated; entries are keyed by architecture, operation, size class and dtype, and
 * an entry measured now replaces the old one with its key; the file is written to a temporary
 * name and renamed, and reads and writes of cache files in one process are serialised).
 *   shapes  host array of `count` pairs (d_i, n_i), 1 <= n_i <= 1024, d_i <= 16384: the
 *           problems the tuned plans will see (each class is measured on up to 1024 of them).
 * For NNLS_TUNE_BATCHED each class present is timed with HIP events on synthetic problems of
 * its shapes (A U[0, 1], x 60 % zeros else U[0, 1], b = A x with 1 % noise, drawn on the device
 * from SplitMix64): the batched Gram at tile sizes 64 and 128, then the batched solver at 256,
 * 512 and 1024 threads per workgroup (tolerance 5e-6, at most 20000 updates), best of 3 runs
 * after a warm-up each.  Unlike the other calls this one is a setup step: it allocates and
 * frees its own device memory and synchronises `stream`.  Errors: NNLS_E_ARG (bad pointers,
 * shapes or op), NNLS_E_IO (the cache could not be written), NNLS_E_UNSUPPORTED (n_i > 1024 or
 * d_i > 16384), NNLS_E_HIP.
 */
int nnls_autotune(const char* cache_path, int op, const int64_t* shapes, int64_t count,
                  void* stream);

/* ---- Learned warm start --------------------------------------------------------------------
 * Algorithm 2 may start from any y0 >= 0 (the worked example of Section 3 starts from a nonzero
 * point).  This addition, which the paper does not have, predicts y0 for the fixed-size case
 * n = 256 with a 256 -> 1024 -> 1024 -> 256 network (GELU hidden layers, exact x * Phi(x)) that
 * reads u = q / ||q|| (one column of q) and returns one head z per column:
 *     direction of y0:  v = ReLU(z)  (Problem (5) is positively homogeneous in q, so the
 *                       direction of y* depends on q / ||q|| only)
 *     logit of "y*_i > 0" = z_i.
 * Training minimises, averaged over the batch,
 *     1/2 ||ReLU(z) - t||^2 + lambda * BCE(z, 1[t > 0]),   t = y* / ||y*||,
 * with Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on FP32 master weights; the
 * products run on a BF16 copy with FP32 accumulation.
 *
 * The input is standardised first, in FP32: x = (u - shift) * scale per feature, then rounded to
 * BF16 (for a fixed A the informative part of u is a small fraction of its size).
 *
 * Parameters live in one device blob of nnls_mlp_blob_bytes() bytes, owned by the caller:
 *     float master[P] | float adam_m[P] | float adam_v[P] | bf16 copy[P] |
 *     float shift[256] | float scale[256],              P = nnls_mlp_param_count()
 * with master laid out as W1 [256, 1024] | b1 [1024] | W2 [1024, 1024] | b2 [1024] |
 * W3 [1024, 256] | b3 [256] (row-major, input index first: h = x W1 + b1).  The caller writes the
 * master weights and shift/scale (or fits them with nnls_mlp_fit_input) and calls
 * nnls_mlp_reset_state() to clear the Adam moments and make the BF16 copy;
 * nnls_mlp_train_step() keeps the copy in step with the master.
 *
 * batch must be a positive multiple of 64 (at most 2^24).  u, target and z are FP32 [batch, 256]
 * row-major.  Workspaces are sized by nnls_mlp_workspace_bytes(batch, train) with train = 0 for
 * the forward pass and 1 for gradients and training steps. */
int64_t nnls_mlp_param_count(void);
size_t nnls_mlp_blob_bytes(void);
size_t nnls_mlp_workspace_bytes(int64_t batch, int train);

/* Sets shift = per-feature mean and scale = 1 / per-feature standard deviation (population; 1
 * where it is 0) of the `count` rows of U [count, 256] FP32 (device), accumulated in FP64.
 * Workspace: nnls_mlp_fit_input_workspace_bytes() bytes. */
size_t nnls_mlp_fit_input_workspace_bytes(void);
int nnls_mlp_fit_input(int64_t count, void* blob, const float* U, void* ws, size_t ws_bytes,
                       void* stream);

/* Clears the Adam moments and rounds the master weights to the BF16 copy (shift and scale are
 * left as they are). */
int nnls_mlp_reset_state(void* blob, void* stream);

/* z = network(u) for `batch` rows. */
int nnls_mlp_forward(int64_t batch, const void* blob, const float* u, float* z, void* ws,
                     size_t ws_bytes, void* stream);

/* Loss (FP32 scalar, device) and the gradient of every parameter (FP32 [P], the master layout)
 * for one batch, without changing the blob.  grad_out and loss_out may each be NULL. */
int nnls_mlp_gradients(int64_t batch, const void* blob, const float* u, const float* target,
                       float lambda, float* grad_out, float* loss_out, void* ws, size_t ws_bytes,
                       void* stream);

/* One Adam step with learning rate lr; step counts from 1 (bias correction).  loss_out (device,
 * may be NULL) receives the batch loss before the step. */
int nnls_mlp_train_step(int64_t batch, void* blob, const float* u, const float* target, float lr,
                        int64_t step, float lambda, float* loss_out, void* ws, size_t ws_bytes,
                        void* stream);

/* Checkpoints of the network blob, so that training can stop and resume exactly.
 * nnls_mlp_save copies the whole blob (master weights, both Adam moments, the BF16 copy and the
 * input standardisation) to the host on `stream`, waits for the copy, and writes
 *     64-byte header | blob (nnls_mlp_blob_bytes() bytes, the device layout above)
 * to `path` (through `path`.tmp and a rename, so a reader never sees a partial file).  The
 * header is little-endian: magic "NNLSCKP1", u32 version 1, u32 widths 256, 1024, 256,
 * i64 parameter count, u64 blob bytes, i64 `step` (the number of Adam steps taken, which
 * the next nnls_mlp_train_step continues from as step + 1), u64 FNV-1a hash of the blob, u64 0.
 * nnls_mlp_load reads and checks the whole file (header fields, size, hash) before it touches
 * the device, then copies the blob into `blob` on `stream`, waits for the copy, and stores the
 * step in *step (may be NULL).  Both synchronise `stream` and allocate host memory only.
 * Errors: NNLS_E_ARG (null blob or path), NNLS_E_IO (the file cannot be opened, read or
 * written, or it is not a checkpoint of this network: wrong magic, version, widths or size, or
 * a hash mismatch), NNLS_E_HIP.  The caller keeps `blob` alive and unused by other work on
 * other streams during the call. */
int nnls_mlp_save(const void* blob, int64_t step, const char* path, void* stream);
int nnls_mlp_load(void* blob, int64_t* step, const char* path, void* stream);

/* Network inputs and training targets from a rescaled problem with n = 256: for each column c
 * of q [256, k], U[c, :] = q[:, c] / ||q_c|| and, if Y [256, k] (a solution of Problem (5), e.g.
 * from nnls_solve with s = NULL) is given, T[c, :] = Y[:, c] / ||Y_c||.  U and T are FP32
 * [k, 256]; T may be NULL when Y is.  A zero column is divided by 1. */
int nnls_mlp_inputs(int64_t n, int64_t k, const float* q, const float* Y, float* U, float* T,
                    void* stream);

/* Warm start for k (1 <= k <= 2^24) right-hand sides of a rescaled problem with n = 256 (other
 * n return NNLS_E_UNSUPPORTED).  Q [256, 256] (symmetric) and q [256, k] FP32 as produced by
 * nnls_prepare.  Per column, with v = ReLU(z) from the network, a = v^T Q v and b = q^T v:
 *     y0 = c* v,  c* = -b / a  (the exact minimiser of f along v),  f(y0) = -b^2 / (2a) < f(0),
 * written to Y0 [256, k] FP32 for nnls_solve.  Where b >= 0 or a <= 0 (v = 0, or no descent
 * along v) or anything is not finite, that column of Y0 is 0, the cold start, and
 * fell_back[k] (int32, device) is 1 there, else 0.
 * Workspace: nnls_warm_start_workspace_bytes(n, k). */
size_t nnls_warm_start_workspace_bytes(int64_t n, int64_t k);
int nnls_warm_start(int64_t n, int64_t k, const float* Q, const float* q, const void* blob,
                    float* Y0, int32_t* fell_back, void* ws, size_t ws_bytes, void* stream);

/* nnls_transpose -- dst[j, i] = src[i, j] for FP32 src [rows, cols] (row-major, leading
 * dimension ld_src >= cols) into dst [cols, rows] (ld_dst >= rows); device pointers, caller-owned,
 * not overlapping.  The data movement of the alternating NNLS update of a nonnegative matrix
 * factorisation V ~ W H (the use the Introduction motivates): the W half solves NNLS with the
 * matrix H^T and right-hand sides V^T.  NNLS_E_ARG for bad sizes or pointers,
 * NNLS_E_UNSUPPORTED for more than 65535 x 64 rows. */
int nnls_transpose(int64_t rows, int64_t cols, const float* src, int64_t ld_src, float* dst,
                   int64_t ld_dst, void* stream);

/* nnls_rescale_start -- Y0 = s .* X (row i of the FP32 [n, k] X times s[i], FP64 product rounded
 * to FP32): a start given in the original variables x, such as the previous factor in an
 * alternating NNLS loop, mapped to the rescaled variables y = D^(1/2) x of rescaling (4) in which
 * nnls_solve takes its start (the worked example of Section 3 starts the same way).  s as
 * written by nnls_prepare; device pointers; NNLS_E_ARG for bad sizes or pointers. */
int nnls_rescale_start(int64_t n, int64_t k, const double* s, const float* X, float* Y0,
                       void* stream);

/* Which solver nnls_solve uses for this shape on the current device: "regq" (one right-hand
 * side, Q held in the register file of the whole GPU), "persistent" (one right-hand side, Q
 * streamed from memory), "mrhs" (many right-hand sides on the matrix cores) or "wg" (one
 * workgroup per column); "" if the shape is not supported.  Host function; the string is
 * static. */
const char* nnls_solver_name(int64_t n, int64_t k, int dtype);

/* Text of the last HIP error seen by this thread (empty if none). */
const char* nnls_last_hip_error(void);

/* Library version string. */
const char* nnls_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NNLS_H */
