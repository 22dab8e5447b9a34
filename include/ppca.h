/*
 * ppca.h -- C ABI of the primed-PCA (pPCA) hot path for AMD Instinct MI355X
 * (gfx950).
 *
 * Primed PCA ("Speeding up PCA with priming", Alg. 1): a cheap approximate
 * PCA method (the priming) produces K = k + l directions V (Sec. 3.3), the
 * data is projected on span(V) and an exact PCA of the projected data
 * returns the first k principal components.  This library implements the
 * data-parallel passes of that method on the GPU:
 *
 *   ppca_center_quantize   centre the data and store it as f32 / bf16 / fp8
 *   ppca_prime_power       block power (subspace) iteration with CholeskyQR2
 *   ppca_prime_oja         minibatch Oja / Sanger rule
 *   ppca_prime_eigengame   minibatch EigenGame utility ascent
 *   ppca_project_gram      Y = X V', G = Y^T Y, B = V'^T V'   (Alg. 1 steps 2-3)
 *   ppca_rayleigh_ritz     full PCA of the projected data      (Alg. 1 step 4)
 *   ppca_prime_power_grouped / ppca_rayleigh_ritz_grouped
 *                          the same for hundreds of small bf16 problems at once
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument is a device pointer (HIP global memory) that
 * the caller owns; the library never allocates or frees memory and keeps no
 * state between calls.  Scratch space is the caller-provided workspace
 * `ws` of `ws_bytes` bytes (256-byte aligned); its required size is returned
 * by ppca_workspace_bytes().  Workspace contents are undefined between calls.
 *
 * Streams.  `stream` is a hipStream_t (NULL = the legacy default stream).
 * Every call validates its arguments on the host, enqueues its kernels on
 * `stream`, waits for the stream to drain and returns a status: device-side
 * failures (non-positive Cholesky pivot, non-finite values, eigensolver sweep
 * cap) are reported through a status word kept in the workspace.  Calls on
 * different streams with different workspaces may run concurrently; two
 * calls that share a workspace must not overlap.
 *
 * Layouts.  X is row-major n x d with row stride `ld` elements (ld >= d).
 * The base pointer must be 16-byte aligned and ld * element_size must be a
 * multiple of 16 bytes.  V, Z and E are row-major d x K float32 (V[j*K+c]).
 * Gram matrices G and B are row-major K x K float64.
 *
 * Signs and order.  Eigenvalues are returned in descending order; each
 * returned eigenvector column is flipped so that its largest-magnitude
 * entry is positive (ties: lowest row index).  Eigenvectors of repeated
 * eigenvalues are any orthonormal basis of their eigenspace.
 *
 * Errors.  No entry point throws or aborts; outputs are unspecified when the
 * status is not PPCA_OK.
 */
#ifndef PPCA_H
#define PPCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PPCA_OK                  0
#define PPCA_ERR_ARG            (-1)  /* invalid size, pointer, count or parameter */
#define PPCA_ERR_DTYPE          (-2)  /* unknown dtype, or col_scale given/missing wrongly */
#define PPCA_ERR_NOT_SPD        (-3)  /* a Cholesky pivot <= K*eps*a_jj: V (or Z) is rank deficient */
#define PPCA_ERR_NONFINITE      (-4)  /* NaN/Inf met in a Gram matrix or in Z */
#define PPCA_ERR_NO_CONVERGENCE (-5)  /* Jacobi eigensolver reached its sweep cap */
#define PPCA_ERR_WORKSPACE      (-6)  /* ws is NULL, misaligned or smaller than required */
#define PPCA_ERR_HIP            (-7)  /* a HIP runtime call failed */
#define PPCA_ERR_ALIGN          (-8)  /* X base or row stride violates the 16-byte rule */
#define PPCA_ERR_PLACEMENT      (-9)  /* single-read pass: a cluster's workgroups were not on one XCD */
#define PPCA_ERR_TIMEOUT       (-10)  /* single-read pass: a bounded wait between workgroups expired */

/* ---- storage types of X ------------------------------------------------- */
#define PPCA_F32       0   /* float32 */
#define PPCA_BF16      1   /* bfloat16 (bits of the upper half of a float32) */
#define PPCA_FP8_E4M3  2   /* OCP fp8 e4m3 "fn" (bias 7, max 448, no inf) with per-column
                              float32 scales: the value of x_ij is code_ij * col_scale[j] */

/* ---- workspace query operations ------------------------------------------ */
#define PPCA_OP_CENTER      0
#define PPCA_OP_POWER       1
#define PPCA_OP_OJA         2
#define PPCA_OP_EIGENGAME   3
#define PPCA_OP_PROJECT     4
#define PPCA_OP_RR          5
#define PPCA_OP_STREAM      6
#define PPCA_OP_POWER_SEQ   7   /* ppca_prime_power_seq */

/* Largest K = k + l supported by the kernels. */
#define PPCA_MAX_K 128

/* A centred data matrix as the GPU path sees it. */
typedef struct {
  const void*  x;          /* device, row-major n x d, row stride ld (elements) */
  int64_t      n;          /* rows (data points), n >= 1 */
  int64_t      d;          /* columns (dimension), d >= 1 */
  int64_t      ld;         /* row stride in elements, ld >= d */
  int32_t      dtype;      /* PPCA_F32, PPCA_BF16 or PPCA_FP8_E4M3 */
  const float* col_scale;  /* device [d]; required for PPCA_FP8_E4M3, NULL otherwise */
} ppca_matrix;

/* Minibatch schedule and optimiser of the SGD-style primings (Sec. 2.2,
 * Sec. 2.3 and the training setup of Sec. 5: SGD, optionally with
 * (Nesterov) momentum).  Step t (counted from start_step) uses the rows
 * (t*batch + i) mod n, i < batch, and the rate eta_t = eta0 / (1 + t/t0)
 * (t0 <= 0: constant eta0).  With momentum mu > 0 the buffer follows
 * buf <- mu*buf + g and the step is g + mu*buf (Nesterov) or buf. */
typedef struct {
  int32_t  batch;           /* b, 1 <= b <= n */
  int64_t  steps;           /* number of minibatch steps T >= 0 */
  double   eta0;            /* > 0 and finite */
  double   t0;              /* decay constant of the rate; <= 0 for a constant rate */
  double   momentum;        /* mu in [0, 1) */
  int32_t  nesterov;        /* 0 or 1 */
  int64_t  start_step;      /* global index of the first step (resume), >= 0 */
  float*   mom_buf;         /* device d x K float32 in/out (zero to start); required iff mu > 0 */
  int32_t  snapshot_every;  /* m > 0: copy V after every m-th step into snapshots */
  float*   snapshots;       /* device [floor(steps/m)][d*K] or NULL */
  int32_t  orthonormalise_start; /* 1: V <- CholQR2(V) before the first step */
} ppca_sgd_params;

/* Centre a float32 matrix and store it in the requested type (the paper
 * assumes a centred dataset, Sec. 1).  mu_j = (sum_r x_rj) / n with the sum
 * taken in double-double arithmetic and rounded once (order independent);
 * c_rj = float32(double(x_rj) - mu_j).  PPCA_F32 stores c; PPCA_BF16 stores
 * the nearest bf16 of c (ties to even); PPCA_FP8_E4M3 stores the nearest
 * e4m3 of float32(c_rj / s_j) (ties to even, saturating at +-448) with
 * s_j = float32(max_r |c_rj| / 448) (1 for an all-zero column) written to
 * col_scale.  x: device float32 [n][ldx]; out: device [n][ldo] of out_dtype;
 * mean: device double [d] (may be NULL); col_scale: device float [d],
 * required iff out_dtype is fp8.  x and out must not overlap unless both
 * are float32 with ldx == ldo (in-place centring). */
int ppca_center_quantize(const float* x, int64_t n, int64_t d, int64_t ldx,
                         int32_t out_dtype, void* out, int64_t ldo,
                         float* col_scale, double* mean,
                         void* ws, size_t ws_bytes, void* stream);

/* Block power priming (Sec. 2.1, block form of the cited simultaneous
 * iteration): V_0 = CholQR2(V); for t = 1..iters: one pass over X gives
 * Y = X V'_{t-1}, Z = X^T Y (float32 accumulation) and G_{t-1} = Y^T Y
 * (float64 across row panels); V_t = CholQR2(Z) in float64.
 * V: device d x K float32, in = starting directions (full rank), out = V_iters
 * (orthonormal columns).  K = k + l with 1 <= k, 0 <= l, K <= min(d, n, 128).
 * gram_hist / b_hist (optional, device [iters][K*K] float64): G_{t-1} and
 * B_{t-1} = V'^T V' of the operand V' that multiplied X in pass t, so that
 * the Ritz values of every iterate can be evaluated afterwards. */
int ppca_prime_power(const ppca_matrix* X, int32_t k, int32_t l, int32_t iters,
                     float* V, double* gram_hist, double* b_hist,
                     void* ws, size_t ws_bytes, void* stream);

/* Block power priming with the termination rule of Sec. 2.1 (the power
 * method stops when |x_i - x_{i+1}| < eps), read for a block as: stop after
 * the first iteration t at which every new direction lies within eps of the
 * previous iterate's span, max_j |v_j^t - V_{t-1} V_{t-1}^T v_j^t|_2 < eps
 * (for one unit vector: the sine of the angle it turned, |x_i - x_{i+1}| to
 * first order; the columns of a block keep turning inside its span long
 * after the span has settled, so their individual changes are not used).
 * Otherwise as
 * ppca_prime_power with at most max_iters iterations.  iters_done: host int
 * (the number of iterations run); changes: host double [max_iters] or NULL
 * (the span change of each iteration run).  The host reads the change after every
 * iteration (one synchronisation per pass).  Workspace: PPCA_OP_POWER. */
int ppca_prime_power_eps(const ppca_matrix* X, int32_t k, int32_t l, int32_t max_iters,
                         double eps, float* V, int32_t* iters_done, double* changes,
                         void* ws, size_t ws_bytes, void* stream);

/* The power method of Sec. 2.1 for K = k + l directions found one after the
 * other: direction i starts from column i of V, orthogonalised against the
 * directions before it and normalised, and iterates
 * u <- P X^T X u / |P X^T X u| with P = I - V_<i V_<i^T (the orthogonalisation
 * after every step that keeps it in the complement of the directions found),
 * until |u_t - u_{t+1}| < eps or max_steps steps.  Each step is one streaming
 * pass with K = 1 plus a one-workgroup update in float64; the host reads the
 * state every 8 steps (steps past convergence change nothing).
 * V: device d x K float32 in/out (orthonormal columns out); steps: host int
 * [K], the steps each direction took.  Workspace: PPCA_OP_POWER_SEQ. */
int ppca_prime_power_seq(const ppca_matrix* X, int32_t k, int32_t l, double eps,
                         int32_t max_steps, float* V, int32_t* steps,
                         void* ws, size_t ws_bytes, void* stream);

/* Minibatch Sanger / generalised Oja priming (Sec. 2.2): for each step the
 * minibatch mean of dw_m = y_m (x - sum_{l<=m} y_l w_l), in matrix form
 * g = (Z_b - V triu(G_b)) / b with Z_b = X_b^T X_b V', G_b = V'^T X_b^T X_b V';
 * then V <- V + eta_t * step.  V: device d x K float32 in/out. */
int ppca_prime_oja(const ppca_matrix* X, int32_t k, int32_t l,
                   const ppca_sgd_params* p, float* V,
                   void* ws, size_t ws_bytes, void* stream);

/* Minibatch EigenGame priming (Sec. 2.3, eqs. (1)-(3)) with
 * M = X_b^T X_b / b: grad_j = dU_j/dv_j = (2/b)(Z_j - sum_{i<j} G_ij/G_ii Z_i),
 * projected on the tangent space of the sphere (grad_j - (v_j.grad_j) v_j),
 * stepped (with optional momentum) and every v_j renormalised to unit norm.
 * All players update together from the same minibatch. */
int ppca_prime_eigengame(const ppca_matrix* X, int32_t k, int32_t l,
                         const ppca_sgd_params* p, float* V,
                         void* ws, size_t ws_bytes, void* stream);

/* One streaming pass over the rows r0, r0+1, ..., r0+nrows-1 (mod n) of X:
 * the product every priming step is built from (power step of Sec. 2.1,
 * minibatch steps of Sec. 2.2 and 2.3): Y = X V' (never stored in full),
 * Z = X^T Y (d x K float32, float32 accumulation within a row split, float64
 * across splits) and G = Y^T Y (K x K float64).  V' is the operand described
 * at ppca_project_gram; Z and G are unnormalised sums over the rows.
 * G may be NULL: then only Z is computed, by the same kernels as a block
 * power step.  0 <= r0 < n, 1 <= nrows.  Workspace: PPCA_OP_STREAM with
 * batch = nrows. */
int ppca_stream_pass(const ppca_matrix* X, int32_t K, const float* V, int64_t r0,
                     int64_t nrows, float* Z, double* G,
                     void* ws, size_t ws_bytes, void* stream);

/* Projection of the data on span(V) and its Gram matrix (Alg. 1 steps 2-3;
 * Sec. 4.2: the variance of the projected data along v in S is v^T X^T X v).
 * One pass over X: Y = X V' is never stored; G = Y^T Y (float64 across row
 * panels), B = V_eff^T V_eff in float64, where V' is the operand that
 * multiplied X (V itself for f32 data; bf16(V) for bf16 data;
 * bf16(s_j V_jc) for fp8 data) and V_eff = V' (f32, bf16) or diag(1/s) V'
 * (fp8), so that G = V_eff^T Xhat^T Xhat V_eff for the stored data Xhat.
 * G, B: device K x K float64.  V: device d x K float32. */
int ppca_project_gram(const ppca_matrix* X, int32_t K, const float* V,
                      double* G, double* B, void* ws, size_t ws_bytes, void* stream);

/* The projection of ppca_project_gram over the rows r0, r0+1, ...,
 * r0+nrows-1 (mod n) only: the cheaper final pass of the large-scale runs of
 * Sec. 5.2, which project a tenth of the rows.  G is the unnormalised Gram of
 * those rows; pass a matrix descriptor with n = nrows to ppca_rayleigh_ritz so
 * that H = R^-T G R^-1 / nrows.  0 <= r0 < n, 1 <= nrows <= n.  Workspace:
 * PPCA_OP_PROJECT with batch = nrows. */
int ppca_project_gram_rows(const ppca_matrix* X, int32_t K, const float* V, int64_t r0,
                           int64_t nrows, double* G, double* B,
                           void* ws, size_t ws_bytes, void* stream);

/* Rayleigh-Ritz: exact PCA of the projected data (Alg. 1 step 4).
 * R = chol(B); H = R^-T G R^-1 / n; H = W Theta W^T (parallel Jacobi,
 * float64); E = V_eff R^-1 W[:, :k].  X supplies n, d, dtype and col_scale
 * (its data is not read), so that V_eff is rebuilt exactly as
 * ppca_project_gram built it.  evals: device double [k] (descending);
 * E: device d x k float32 (may be NULL to get the eigenvalues only). */
int ppca_rayleigh_ritz(const ppca_matrix* X, int32_t K, int32_t k,
                       const double* G, const double* B, const float* V,
                       float* E, double* evals,
                       void* ws, size_t ws_bytes, void* stream);

/* Rayleigh-Ritz that allocates nothing, for callers that cannot allocate
 * device memory or pass a workspace: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, results
 * and errors as ppca_rayleigh_ritz without ws / ws_bytes: its scratch is a
 * fixed device array of PPCA_NOALLOC_SCRATCH_BYTES inside the library (one
 * copy per GPU, held until the process ends).  The Rayleigh-Ritz workspace
 * does not grow with n or d (the rotation reads V directly; its sign rule
 * keeps at most 1024 x K column maxima): at most about 2.7 MiB, at
 * K = PPCA_MAX_K, so every valid call fits; a call whose workspace
 * (ppca_workspace_bytes(PPCA_OP_RR, X, K, 0)) exceeded the array would return
 * PPCA_ERR_WORKSPACE without running.  `stream` must belong to the current
 * device (else PPCA_ERR_ARG).  All calls on one GPU share the array: calls
 * that overlap on one GPU (different streams or threads) race and must be
 * serialised by the caller.  No hipMalloc, hipFree or allocating library
 * routine is called. */
#define PPCA_NOALLOC_SCRATCH_BYTES (4u << 20)
int ppca_rayleigh_ritz_noalloc(const ppca_matrix* X, int32_t K, int32_t k,
                               const double* G, const double* B, const float* V,
                               float* E, double* evals, void* stream);

/* ---- grouped problems ----------------------------------------------------
 * Many independent PCA problems of uneven n, d and K solved together: every
 * power pass of all problems is one persistent launch (the problems' rows are
 * cut into work items of a few MiB, sorted by size and dealt round-robin to
 * the workgroups), and CholeskyQR2 and Rayleigh-Ritz run one workgroup per
 * problem.  Each problem follows the single-problem path step for step
 * (ppca_prime_power, then ppca_project_gram, then ppca_rayleigh_ritz) for
 * bf16 data: V' = bf16(V), Y' = bf16(X V'), Z = X^T Y', G = Y'^T Y'.
 * Limits per problem: dtype PPCA_BF16, 1 <= d <= PPCA_GROUP_MAX_D,
 * ld <= PPCA_GROUP_MAX_LD, 1 <= k, 0 <= l, K = k + l <= min(PPCA_GROUP_MAX_K,
 * n, d). */
#define PPCA_GROUP_MAX_D 768
#define PPCA_GROUP_MAX_K 64
#define PPCA_GROUP_MAX_LD (1 << 24)
#define PPCA_GROUP_GRAPH 1   /* flag: replay the power iteration as a captured HIP graph */

typedef struct {
  ppca_matrix X;   /* bf16 data, allocated as n x ld */
  int32_t k, l;    /* K = k + l directions, k wanted components */
  float*  V;       /* device d x K f32: starting directions in, primed V out */
  double* G;       /* device K x K f64: Gram of the projection on the primed V */
  double* B;       /* device K x K f64: V_eff^T V_eff of that projection's operand */
  float*  E;       /* device d x k f32 (Rayleigh-Ritz output; may be NULL) */
  double* evals;   /* device k f64 (Rayleigh-Ritz output) */
} ppca_problem;

/* Block power priming of every problem (Sec. 2.1, as ppca_prime_power), then
 * the projection pass on the primed directions (Alg. 1 steps 2-3, as
 * ppca_project_gram): V_0 = CholQR2(V); iters times { one pass over X gives
 * Z = X^T Y', V <- CholQR2(Z) }; then G = Y'^T Y' and B for the final V.
 * probs: host array of nprob >= 1 problems (V, G, B required; E, evals not
 * used).  flags: 0 or PPCA_GROUP_GRAPH (the iteration is captured once on
 * `stream` and replayed; `stream` must not be the legacy NULL stream).
 * Workspace: ppca_grouped_workspace_bytes(probs, nprob).  The status is the
 * first failure of any problem. */
int ppca_prime_power_grouped(const ppca_problem* probs, int32_t nprob, int32_t iters,
                             int32_t flags, void* ws, size_t ws_bytes, void* stream);

/* Rayleigh-Ritz of every problem (Alg. 1 step 4, as ppca_rayleigh_ritz) from
 * its G, B and V: evals (descending) and, when E is not NULL, the Ritz
 * vectors E = V_eff R^-1 W[:, :k] with the sign rule of the header. */
int ppca_rayleigh_ritz_grouped(const ppca_problem* probs, int32_t nprob,
                               void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes of the grouped calls for these problems (0 if invalid),
 * at the current work-item size (ppca_set_group_item_bytes). */
size_t ppca_grouped_workspace_bytes(const ppca_problem* probs, int32_t nprob);

/* The same at work-item size item_bytes (0 if invalid or out of range). */
size_t ppca_grouped_workspace_bytes_for(const ppca_problem* probs, int32_t nprob,
                                        int64_t item_bytes);

/* Work split of the grouped calls: the rows of every problem are cut into
 * work items of about `bytes` bytes of X (whole 16-row tiles), dealt largest
 * first to one persistent workgroup per CU.  Smaller items balance the end of
 * a pass better, larger ones write fewer partial sums.  0 restores the default
 * (3 MiB); otherwise 64 KiB <= bytes <= 1 GiB, else PPCA_ERR_ARG.  Process-
 * wide; affects the plans (and workspace sizes) of later calls; results differ
 * between item sizes only in the order of float32 partial sums. */
int ppca_set_group_item_bytes(int64_t bytes);

/* Autotuner of that work split: for each of the ncand candidate item sizes
 * (cand == NULL or ncand == 0: 1, 2, 3, 4, 6 and 8 MiB) forms the bf16
 * operand of every problem's V as it stands, runs the fused power pass once
 * untimed and once timed with HIP events on `stream`, and returns the fastest
 * candidate in *best_bytes (each time in times_ms[i] when times_ms is not
 * NULL).  Nothing the caller owns is written (V is not orthonormalised; the
 * sums stay in the workspace).  The setting is not changed: pass *best_bytes
 * to ppca_set_group_item_bytes.  Workspace: the largest of
 * ppca_grouped_workspace_bytes_for over the candidates (the smallest
 * candidate needs the most). */
int ppca_tune_group_items(const ppca_problem* probs, int32_t nprob, const int64_t* cand,
                          int32_t ncand, void* ws, size_t ws_bytes, void* stream,
                          int64_t* best_bytes, double* times_ms);

/* Bytes of workspace needed by operation `op` (PPCA_OP_*) for data X with
 * K directions and minibatch `batch` (rows of the pass for PPCA_OP_STREAM;
 * for PPCA_OP_PROJECT 0 = all n rows, else the rows of the window of
 * ppca_project_gram_rows; ignored by the other non-minibatch operations).
 * Returns 0 for invalid arguments. */
size_t ppca_workspace_bytes(int32_t op, const ppca_matrix* X, int32_t K, int32_t batch);

/* Static description of a status code. */
const char* ppca_strerror(int status);

/* Optional per-kernel timing of the streaming kernels.  When enabled, the
 * library records a pair of HIP events on the caller's stream around every
 * launch of each streaming kernel and accumulates their elapsed times.
 * kernel: 0 = X V' pass (ppca_xv), 1 = X^T Y / Gram pass (ppca_xty),
 * 2 = fused grouped pass (power and projection passes of the grouped calls,
 * eager mode only), 3 = single-read power pass (ppca_set_fused_pass),
 * 4 = projection pass (ppca_project_gram, ppca_project_gram_rows),
 * 5 = streaming-read probe (ppca_read_probe).
 * ppca_kernel_stats returns the number of launches and the total ms since
 * the last reset.  Not thread safe; meant for benchmarks. */
void ppca_set_kernel_timing(int32_t enable);
int  ppca_kernel_stats(int32_t kernel, int64_t* launches, double* total_ms);

/* Streaming-read probe, a measurement aid (not a step of the method): reads
 * every byte of the stored X (rows [0, n), ld * element-size bytes each)
 * exactly once and does no arithmetic on it, so that the streaming kernels'
 * rates can be set against what this GPU reads in their access pattern.
 * mode 0: plain 16-byte vector loads striding over the matrix;
 * mode 1: the LDS-DMA pipeline of the power pass (three 32 KB LDS stages,
 *         two in flight) walking tiles of 32768 / seg_bytes rows seg_bytes of
 *         every row per step; seg_bytes = 128, 256 or 512.
 * sink: device uint32 array of at least sink_len entries, written with the
 * XOR of the 32-bit words each workgroup read (so the reads are kept; the
 * XOR over the whole array is the XOR of all words read).  sink_len must be
 * at least 1024 (mode 0) or 256 (mode 1), else PPCA_ERR_ARG; bad mode or
 * seg_bytes: PPCA_ERR_ARG; X as in the other calls (PPCA_ERR_ALIGN, _DTYPE).
 * Synchronises the stream; timed as kernel 5 when kernel timing is on. */
int ppca_read_probe(const ppca_matrix* X, int32_t mode, int32_t seg_bytes, uint32_t* sink,
                    int64_t sink_len, void* stream);

/* Tuning knob of the streaming passes: rows per chunk (0 = whole pass in
 * one launch pair).  Chunks bound the size of the Y staging buffer and keep
 * a chunk of X resident in the last-level cache between the two kernels. */
void ppca_set_chunk_rows(int64_t rows);

/* Single-read power pass (Sec. 2.1 power step): for bf16 data with K padded
 * to a multiple of 32 (K <= 128) and d <= 8192, the Z-only passes of
 * ppca_prime_power and ppca_stream_pass (G == NULL) compute Z = X^T bf16(X V')
 * in one read of X: clusters of workgroups on one XCD split the columns of X,
 * exchange their float32 partials of Y through the XCD's L2 and keep their
 * column slice of Z on chip (kernel timing slot 3).  enable = 0 (the
 * default) runs these passes as two kernels (Y = X V', then Z = X^T Y) like
 * every other pass: at 2,000,000 x 2048, K = 128 on an MI355X the single-read
 * pass measured 5.4 ms against 3.35 ms for the two kernels (its 32-row tiles
 * are bound by L2 round trips of the exchange and by the MFMA latency of two
 * accumulators, not by HBM).  The setting is process-wide and enters the workspace
 * plans of later calls (the single-read pass needs its own exchange buffers:
 * query ppca_workspace_bytes after changing it).  Results of the two forms
 * differ only in the order of the float32 sums that form Y before its bf16
 * rounding. */
void ppca_set_fused_pass(int32_t enable);

#ifdef __cplusplus
}
#endif
#endif /* PPCA_H */
