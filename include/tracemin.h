/*
 * tracemin.h -- C ABI of the MI355X (gfx950) trace-minimization eigensolver.
 *
 * Computes the m lowest eigenpairs of a real, symmetric, sparse N x N matrix
 * H: the sum E_G of the m lowest eigenvalues (Eq. 2 of Tsuchida & Choe,
 * "Iterative diagonalization of symmetric matrices in mixed precision") and an
 * orthonormal basis C of their subspace, by minimizing E(C) = tr(C^T H C)
 * subject to C^T C = I (Sec. 2.1, Eq. 4-7) with nonlinear conjugate gradients
 * (Fig. 1).  Every step of the iteration runs in hand-written HIP kernels on
 * the device.
 *
 * Conventions used by every entry point
 *   - Blocks of m vectors (C, X = HC, G, P, ...) are N x ld row-major arrays:
 *     element (r, j) lives at index r * ld + j.  ld = tm_leading_dim(m) (m
 *     rounded up to a multiple of 32); columns m .. ld-1 must hold zeros and
 *     are kept at zero.
 *   - m x m matrices are dense row-major with leading dimension m.
 *   - Pointers documented as "device" must point to device memory on the
 *     context's device; "host" pointers to host memory.  The library never
 *     frees memory it did not allocate.  All device work is enqueued on the
 *     context's stream; an entry point returns once its work is enqueued,
 *     except where "synchronous" is stated.
 *   - Every entry point returns a tm_status.  On failure the detail text is
 *     available from tm_last_error() (thread-local).  No C++ exception crosses
 *     this boundary.
 *   - One context per host thread at a time; a context is not thread-safe.
 */
#ifndef TRACEMIN_H
#define TRACEMIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
typedef enum tm_status {
    TM_OK = 0,
    TM_EINVAL = -1,   /* invalid argument (sizes, pointers, malformed CSR)     */
    TM_ENOMEM = -2,   /* device allocation failed                             */
    TM_ENOTSPD = -3,  /* C^T C not positive definite in the Cholesky step     */
    TM_ENOCONV = -4,  /* max_iter reached; result filled, converged = 0       */
    TM_ENAN = -5,     /* NaN or Inf in the energy or gradient norm            */
    TM_EDEVICE = -6,  /* HIP runtime error (text in tm_last_error)            */
    TM_ENOTSUP = -7,  /* option combination not supported                    */
    TM_EAGAIN = -8    /* a served request is still queued or running          */
} tm_status;

/* TM_BF16X3: FP32 blocks multiplied on BF16 matrix cores with each operand
 * split into two BF16 terms (hi + lo, three products, FP32 accumulation);
 * accepted by tm_gram only. */
typedef enum tm_dtype { TM_F64 = 0, TM_F32 = 1, TM_BF16X3 = 2 } tm_dtype;

/* Precision policies (Sec. 2.2).  Every policy keeps the m x m Cholesky,
 * triangular inverse and Rayleigh-Ritz eigensolve in FP64, and reports E_G and
 * residuals from an FP64 evaluation at the end.
 *   TM_FULL_DP  every operation in FP64 (the paper's "full DP").
 *   TM_FULL_SP  every N-sized operation in FP32 (the paper's "full SP").
 *   TM_MP2      the paper's MP2: SpMM, X' = X - C H_D and S = C^T C in FP64;
 *               H' = C^T X' and C H' on FP32 matrix cores; G and P stored
 *               in FP32; C_out = C L_D + C L' with the second term in FP32.
 *   TM_MIXED    FULL_SP until the residual reaches switch_tol (or the FP32
 *               energy stalls), then MP2 with subspace rotations every k_rot
 *               iterations until tol -- the switch the paper recommends in
 *               Sec. 3 and Sec. 5.
 *   TM_MIXED_BF16  TM_MIXED with the bulk phase's H' = C^T X' on BF16 matrix
 *               cores (two-term BF16 operands, FP32 accumulation); the MP2
 *               refinement restores FP64 accuracy.
 *   TM_FULL_BF16   the bulk phase of TM_MIXED_BF16 alone (no refinement):
 *               its accuracy floor, for error reports.
 *   TM_MP1      the paper's MP1: everything as TM_FULL_DP except (i) G and P
 *               stored in FP32 (G formed in FP64, then rounded) and (ii)
 *               C_out = C L_D + C L' with the second term on FP32 matrix
 *               cores (Eq. 11-13); H' = C^T X' and C H' stay FP64.
 *   TM_MP2_MP1  TM_MP2 until rho <= switch_tol (or its energy stalls), then
 *               TM_MP1 to tol, with the CG state carried across the switch
 *               (G and P are FP32 in both): the switch Sec. 3 and Sec. 5
 *               recommend in place of rotations. */
typedef enum tm_precision {
    TM_FULL_DP = 0,
    TM_FULL_SP = 1,
    TM_MP2 = 2,
    TM_MIXED = 3,
    TM_MIXED_BF16 = 4,
    TM_FULL_BF16 = 5,
    TM_MP1 = 6,
    TM_MP2_MP1 = 7
} tm_precision;

/* ---------------------------------------------------------------- objects */
typedef struct tm_ctx tm_ctx;
typedef struct tm_mat tm_mat;

/* Device allocator hook.  alloc returns device memory of at least `bytes`
 * bytes (256-byte aligned) or NULL; free releases it.  Both are called on
 * the thread that calls into the library. */
typedef struct tm_allocator {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} tm_allocator;

/* Matrix-free H = kinetic_scale * (-Lap_h) + diag(V) on a regular grid with
 * spacing 1.  order 2: 1-D stencil (-1, 2, -1); order 4: (1, -16, 30, -16, 1)/12.
 * dims[0] is the fastest axis; grid point (x, y, z) is row (z*ny + y)*nx + x.
 * With ndim = 2, periodic = 0, kinetic_scale = 1 and V = NULL this is the
 * paper's 2-D Dirichlet Laplacian H_N (Eq. 14-15). */
typedef struct tm_stencil {
    int32_t ndim;          /* 2 or 3                                         */
    int32_t dims[3];       /* grid extents (dims[2] ignored when ndim = 2)   */
    int32_t order;         /* 2 (7-point in 3-D) or 4 (13-point in 3-D)      */
    int32_t periodic;      /* 1 periodic, 0 Dirichlet (zero outside)         */
    double kinetic_scale;  /* 0.5 for -1/2 Lap; 1.0 for the paper's H_N       */
    const double *V;       /* host, N values added to the diagonal, or NULL  */
} tm_stencil;

/* Progress report of a running solve: called on the solving thread each
 * time the host polls the device (every k_check iterations) with the
 * iterations done, the current energy E_i, rho_i and the phase (0 first,
 * 1 second).  Must not call back into the library. */
typedef void (*tm_progress_fn)(int32_t iterations, double E, double rho, int32_t phase,
                               void *user);

typedef struct tm_opts {
    int32_t precision;     /* tm_precision                                   */
    int32_t max_iter;      /* total CG iterations over all phases            */
    int32_t k_rot;         /* subspace rotation every k_rot iterations (0 = off) */
    int32_t k_check;       /* host polls the device convergence flag every k_check iterations */
    int32_t precondition;  /* 1: diagonal M of Eq. 18, M_ii = 1/(H_ii - sigma);
                              2: polynomial M = p(H - sigma I) of cheb_degree
                              Chebyshev-iteration steps for (H - sigma I) z = G
                              on the Gershgorin interval, sigma = lo -
                              cheb_shift (hi - lo), applied in the precision of
                              G (FP32 in every policy but TM_FULL_DP) */
    int32_t history;       /* 1: record E_i and rho_i per iteration         */
    int32_t transport;     /* 1 (default): a subspace rotation C <- C U also maps
                              P <- P U and G_prev <- G_prev U and CG continues;
                              0: CG restarts after each rotation */
    int32_t graphs;        /* 1: replay batches of k_check iterations without a
                              rotation from captured HIP graphs (same kernels) */
    double switch_tol;     /* TM_MIXED: leave FP32 when rho <= switch_tol (<= 0: automatic) */
    double rise_tol;       /* restart CG when E rises by more than rise_tol*|E| */
    double stall_tol;      /* TM_MIXED*: also leave the bulk phase when E drops by less
                              than stall_tol*|E| over 25 iterations (<= 0: 1e-7) */
    uint64_t seed;         /* tm_solve with C0 = NULL: the start block is
                              tm_random_block(seed) (standard normal entries) */
    int32_t cheb_degree;   /* precondition = 2: steps (>= 1; 2 by default)   */
    int32_t reserved;      /* 0 */
    double cheb_shift;     /* precondition = 2: sigma below the Gershgorin
                              interval, as a fraction of its width (0.02)   */
    tm_progress_fn progress;  /* NULL: no reports                            */
    void *progress_user;
} tm_opts;

typedef struct tm_result {
    double E_G;            /* sum of the m Ritz values after the final FP64 Rayleigh-Ritz */
    double rho;            /* ||X - C A||_F at the last iteration            */
    double max_residual;   /* max_j ||H c_j - lambda_j c_j||_2, FP64        */
    double frob_residual;  /* sqrt(sum_j ||H c_j - lambda_j c_j||^2), FP64  */
    double orth_err;       /* max |C^T C - I|, FP64                          */
    double seconds;        /* wall time of the solve (synchronous)           */
    double seconds_phase[3];  /* wall time of [0] the first phase (the FP32/BF16
                              bulk of TM_MIXED*, the MP2 part of TM_MP2_MP1,
                              all iterations of a one-phase policy), [1] the
                              second phase, [2] the start (upload, first
                              orthonormalization) plus the final FP64
                              Rayleigh-Ritz and residuals                    */
    int32_t iterations;    /* CG iterations taken (all phases)               */
    int32_t iters_sp;      /* iterations of the first phase (= iterations for a
                              one-phase policy)                              */
    int32_t converged;     /* 1 if rho <= tol was reached                    */
    int32_t restarts;      /* CG restarts (gamma = 0), including i = 0       */
    int32_t rotations;     /* subspace rotations performed                   */
    int32_t iters_phase2;  /* iterations of the second phase (0 if none)    */
} tm_result;

/* ------------------------------------------------------------- lifecycle */

/* Leading dimension used for an m-column block: m rounded up to 32. */
int32_t tm_leading_dim(int32_t m);

/* Create a context on HIP device `device`.  alloc may be NULL (hipMalloc /
 * hipFree are used).  stream is a hipStream_t or NULL for the null stream;
 * the caller keeps ownership of it. */
tm_status tm_create(int32_t device, const tm_allocator *alloc, void *stream,
                    tm_ctx **out);
void tm_destroy(tm_ctx *ctx);
const char *tm_status_string(int32_t status);
const char *tm_last_error(void);

/* Flags of tm_set_matrix_csr. */
#define TM_CHECK_SYMMETRY 1u   /* verify H = H^T entry by entry (duplicates summed);
                                  TM_EINVAL if not                              */
#define TM_DEVICE_PTRS 2u      /* rowptr, col and val are device pointers       */

/* H from CSR arrays (Sec. 2.1: real, symmetric, sparse with O(N) nonzeros).
 * rowptr (n+1, int64), col (nnz, int32) and val (nnz, FP64) are copied by the
 * library (host arrays unless flags has TM_DEVICE_PTRS); the caller may free
 * them afterwards.  Columns must lie in [0, n), rowptr must be non-decreasing
 * with rowptr[0] = 0 and values finite (TM_EINVAL otherwise).  Symmetry is
 * checked when flags has TM_CHECK_SYMMETRY, else it is the caller's
 * responsibility.  Unknown flag bits are TM_EINVAL. */
tm_status tm_set_matrix_csr(tm_ctx *ctx, int64_t n, const int64_t *rowptr,
                            const int32_t *col, const double *val, uint32_t flags,
                            tm_mat **out);
tm_status tm_set_matrix_stencil(tm_ctx *ctx, const tm_stencil *s,
                                tm_mat **out);
void tm_free_matrix(tm_mat *mat);
int64_t tm_matrix_rows(const tm_mat *mat);

/* ------------------------------------------------------------------ solve */

void tm_opts_default(tm_opts *opts);

/* Fill the device block out (n x ld FP64, ld = tm_leading_dim(m)) with
 * standard normal entries in columns 0..m-1 and zeros in the padding: the
 * random start block of Sec. 3 ("random numbers, then orthonormalization").
 * Entry (r, j) is a pure function of (seed, r * m + j): Philox4x32-10
 * (Salmon et al., SC'11) with key (seed low, seed high) on the counter
 * (k, 0, 0, 0), k = (r * m + j) / 2, gives four 32-bit words; words 0-1 and
 * 2-3 form two 53-bit uniforms u1 in (0, 1], u2 in [0, 1) and the Box-Muller
 * pair sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2) gives entries 2k and 2k + 1. */
tm_status tm_random_block(tm_ctx *ctx, int64_t n, int32_t m, uint64_t seed, double *out);

/* Trace minimization (Fig. 1) from the start block C0 (device, N x ld FP64,
 * need not be orthonormal; it is orthonormalized first by Fig. 4; NULL: the
 * block tm_random_block makes from opts->seed) until
 * rho = ||X - C A||_F <= tol, where X = HC and A = C^T X.  Synchronous.
 * m may be up to 2048 (TM_ENOTSUP above).
 *   C_out     device N x ld FP64 or NULL: the Ritz vectors, ascending.
 *   eig_out   device m FP64 or NULL: the Ritz values lambda_1..lambda_m.
 *   history   host array of 2*history_len doubles or NULL: (E_i, rho_i)
 *             for i < min(iterations, history_len) (opts->history = 1).
 * Returns TM_ENOCONV (with *res filled) if max_iter was reached. */
tm_status tm_solve(tm_ctx *ctx, const tm_mat *H, int32_t m, double tol,
                   const tm_opts *opts, const double *C0, double *C_out,
                   double *eig_out, tm_result *res, double *history,
                   int32_t history_len);

/* The generalized problem H x = lambda S x with S symmetric positive
 * definite (Sec. 2.1: the extension the trace minimization allows for
 * nonorthogonal basis functions): minimizes tr(C^T H C) subject to
 * C^T S C = I.  Each iteration is Algorithm-2 in the S metric (Z = S C,
 * X' = X - Z H_D, H' = C^T X', G = -2 (X' - Z H')), the Polak-Ribiere step,
 * the line step with S-norms p_j^T S p_j, and Fig. 4 in the S inner product
 * (C^T S C = R^T R, C <- C R^{-1}).  Arguments as tm_solve; S is a matrix of
 * the same context and size (CSR or stencil; a diagonal entry <= 0 is
 * TM_EINVAL, a Cholesky breakdown TM_ENOTSPD).  rho = ||X - Z A||_F; the
 * residuals are ||H c_j - lambda_j S c_j|| and orth_err is max |C^T S C - I|.
 * Runs in TM_FULL_DP (other precisions: TM_ENOTSUP). */
tm_status tm_solve_generalized(tm_ctx *ctx, const tm_mat *H, const tm_mat *S, int32_t m,
                               double tol, const tm_opts *opts, const double *C0,
                               double *C_out, double *eig_out, tm_result *res,
                               double *history, int32_t history_len);

/* ---------------------------------------------------------------- batches
 * Many small problems on one grid: the Hamiltonian of Sec. 3 is a kinetic
 * operator plus a potential on the diagonal, so problems on the same grid
 * differ only there.  A batch matrix holds k operators H_g = A + diag(d_g)
 * (g = 0..k-1) sharing one CSR A; a batched solve runs Fig. 1 for all of
 * them at once on one n x ld block where problem g owns columns
 * g * ldg .. g * ldg + m - 1 (the rest of its ldg columns are zero): each
 * sparse product reads A once for all problems and adds d_g in its
 * epilogue, the Gram, rotation and TRMM products run once on the whole
 * block with their m_b x m_b results (m_b = k * ldg) kept block-diagonal,
 * and every scalar of the CG step (Eq. 8's gamma, the step alpha, the
 * convergence and phase tests) is a problem's own. */

/* k operators H_g = A + diag(d_g): A as for tm_set_matrix_csr (host arrays
 * only; flags may hold TM_CHECK_SYMMETRY), d host k x n row-major (d_g at
 * d + g * n), copied.  1 <= k <= 256; TM_EINVAL for a non-finite d.  Such a
 * matrix is taken by tm_solve_batch and tm_spmm (in the batch layout) and
 * refused by the other calls. */
tm_status tm_set_matrix_batch(tm_ctx *ctx, int64_t n, const int64_t *rowptr,
                              const int32_t *col, const double *val, int32_t k,
                              const double *d, uint32_t flags, tm_mat **out);
/* The batch layout of k problems of m columns: *ldg columns per problem (m
 * rounded up to 16, then up to a multiple of 64 for k * ldg) and the block's
 * leading dimension *ld = tm_leading_dim(k * ldg). */
tm_status tm_batch_layout(int32_t k, int32_t m, int32_t *ldg, int32_t *ld);
/* Solve the k problems of the batch matrix H for m eigenpairs each until
 * every problem has rho_g <= tol.  C0: device n x ld FP64 in the batch
 * layout, or NULL: problem g starts from the block tm_random_block makes
 * with seed opts->seed + g.  C_out: device n x ld FP64 or NULL; eig_out:
 * device k * m FP64 or NULL (problem g's ascending values at g * m); res:
 * host array of k results (seconds and rotations are the batch's).  A
 * converged problem takes no further steps (alpha = 0) while others run; a
 * two-phase policy changes phase once every problem has ended its first
 * phase.  k * ldg <= 2048.  Precisions: all but the BF16 policies;
 * precondition 0, or 2 with cheb_degree = 2 (each problem on its own
 * Gershgorin interval); other options TM_ENOTSUP; history is not recorded;
 * opts->progress receives the furthest problem's iteration count, the sum
 * of the energies and the largest rho.  TM_ENOCONV (results filled) if some
 * problem did not converge. */
tm_status tm_solve_batch(tm_ctx *ctx, const tm_mat *H, int32_t m, double tol,
                         const tm_opts *opts, const double *C0, double *C_out,
                         double *eig_out, tm_result *res);

/* ---------------------------------------------------------------- serving
 * Continuous batching of independent solves on one GPU (for callers that
 * serve many eigenproblems of different N and m).  Requests queue in arrival
 * order and are admitted as soon as one of max_slots slots is idle and the
 * request's memory bound (tm_solve_footprint) fits the free part of
 * hbm_budget; admitted requests run concurrently, each on its own HIP stream
 * and host thread.  A request computes exactly what tm_solve computes for the
 * same inputs: the kernels, launch shapes and reduction orders do not depend
 * on what else is running.
 * With max_batch > 1, a slot that admits the head of the queue also takes
 * later queued requests that can share one tm_solve_batch with it: same n,
 * m, tol and options (no BF16 policy; no preconditioner or the degree-2
 * polynomial), the same sparsity pattern and off-diagonal values (one grid,
 * one kinetic operator), any diagonal -- up to max_batch requests,
 * max_batch_cols block columns (tm_batch_layout) and 2^25 block entries
 * (n times columns: sizes where one batched solve costs less than its
 * requests alone),
 * as far as the batch's memory bound fits.  A batched request is solved to the same tolerance but
 * in another rounding order than alone.  The server is internally
 * synchronized; all entry points may be called from any host thread. */
typedef struct tm_server tm_server;

typedef struct tm_server_opts {
    int32_t device;        /* HIP device                                        */
    int32_t max_slots;     /* solves in flight, 1..16                           */
    uint64_t hbm_budget;   /* device bytes reserved at creation for requests    */
    int32_t max_batch;     /* requests per batched solve, 0 or 1: no batching;
                              at most 256                                       */
    int32_t max_batch_cols;/* columns of a batched solve's block (k * ldg),
                              64..2048 (0: 512)                                 */
} tm_server_opts;

typedef struct tm_request {
    int64_t n;             /* rows of H                                         */
    const int64_t *rowptr; /* host CSR of H (as tm_set_matrix_csr); copied      */
    const int32_t *col;
    const double *val;
    int32_t m;             /* eigenpairs wanted, 1 <= m <= n                    */
    int32_t reserved;      /* must be 0 */
    double tol;            /* stop when ||X - C A||_F <= tol                    */
    const double *C0;      /* host n x m FP64 start block, row-major; copied    */
    const tm_opts *opts;   /* NULL: tm_opts_default with precision TM_MIXED     */
} tm_request;

typedef struct tm_server_stats {
    int64_t submitted, completed, failed, rejected, queued, running;
    double p50_latency_s;  /* submit -> result, nearest-rank percentiles over   */
    double p99_latency_s;  /* all finished requests                             */
    double max_latency_s;
    double mean_latency_s;
    double span_s;         /* first submit -> last completion                   */
    double solves_per_s;   /* finished requests / span_s                        */
    uint64_t hbm_budget;
    uint64_t hbm_peak;     /* largest sum of admitted memory bounds             */
    double p50_wait_s;     /* submit -> admission (queue wait), percentiles     */
    double p99_wait_s;
    double p50_service_s;  /* admission -> result (the solve on the GPU)        */
    double p99_service_s;
    int64_t solver_runs;   /* finished solver runs (a batched run counts once)  */
} tm_server_stats;

/* Device bytes tm_solve may allocate for an n x m problem with nnz stored
 * nonzeros under opts (NULL: defaults), plus the start block and the
 * eigenvalues: the admission bound used by the server. */
tm_status tm_solve_footprint(int64_t n, int64_t nnz, int32_t m, const tm_opts *opts,
                             uint64_t *bytes);
/* Reserves hbm_budget bytes on the device and starts max_slots worker
 * threads.  TM_EINVAL for bad options, TM_ENOMEM if the reservation fails. */
tm_status tm_server_create(const tm_server_opts *opts, tm_server **out);
/* Queues a request (inputs are copied; the caller may free them on return).
 * TM_ENOMEM if its memory bound exceeds the whole budget (counted as
 * rejected), TM_EINVAL for malformed input. */
tm_status tm_server_submit(tm_server *srv, const tm_request *req, uint64_t *id);
/* TM_EAGAIN while the request is queued or running.  Once finished: fills
 * *res and eig_out (host, m doubles; either may be NULL), returns the solve's
 * status (tm_last_error holds its text) and forgets the request. */
tm_status tm_server_poll(tm_server *srv, uint64_t id, tm_result *res, double *eig_out);
/* As tm_server_poll, blocking up to timeout_s seconds (< 0: no limit). */
tm_status tm_server_wait(tm_server *srv, uint64_t id, double timeout_s, tm_result *res,
                         double *eig_out);
tm_status tm_server_get_stats(tm_server *srv, tm_server_stats *out);
/* Drops queued requests, waits for running ones, releases everything. */
void tm_server_destroy(tm_server *srv);

/* ------------------------------------------------ steps of the iteration
 * The kernels of one iteration, exposed one by one so that each can be
 * checked on its own.  All pointers are device pointers; dtype selects FP64
 * or FP32 blocks; sizes: n = rows, m = columns, ld = tm_leading_dim(m). */

/* X = H C (Fig. 2, step (1)). */
tm_status tm_spmm(tm_ctx *ctx, const tm_mat *H, int32_t m, int32_t dtype,
                  const void *C, void *X);

/* out = A^T B, an m x m FP64 result (the Gram products H' = C^T X' of
 * Fig. 2 step (6) and S = C^T C of Fig. 4 step (1)).  When h is not NULL, B
 * is replaced by B - A diag(h) (Fig. 2 step (5), formed on the fly).  The
 * products run on matrix cores in the block's precision with FP64 sums
 * across row chunks. */
tm_status tm_gram(tm_ctx *ctx, int64_t n, int32_t m, int32_t dtype,
                  const void *A, const void *B, const double *h, double *out);

/* tm_gram without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, products and result as tm_gram, to rounding:
 * the padded h and the split-K partials live in a fixed 32 MiB device array
 * of the library (one per GPU, held until the process ends), so the row
 * splits are capped to fit it, which may change the summation order.  The
 * call only enqueues work on the context's stream (no synchronization, no
 * memset, no allocation); out is valid once the stream gets there.  Every
 * call on a GPU uses that GPU's one array: calls that overlap on one GPU
 * (several streams or host threads) race and must be serialized by the
 * caller.  TM_ENOMEM if even one row split does not fit (m about 2040 or
 * more). */
tm_status tm_gram_noalloc(tm_ctx *ctx, int64_t n, int32_t m, int32_t dtype,
                          const void *A, const void *B, const double *h, double *out);

/* out = A W with A an n x ld block and W an m x m FP64 matrix (the subspace
 * rotation C U of the Rayleigh-Ritz step, Eq. 9).  W is rounded to the
 * block's precision. */
tm_status tm_rotate(tm_ctx *ctx, int64_t n, int32_t m, int32_t dtype,
                    const void *A, const double *W, void *out);

/* Energy and gradient by Fig. 2, Algorithm-2, with FP64 blocks:
 * X = HC; h = diag(C^T X); E = sum h; X' = X - C diag(h); H' = C^T X' with
 * diag(H') := 0; G = -2 (X' - C H').  C must be orthonormal, as the method
 * keeps it: H' = C^T H C - diag(h) is then symmetric and is formed from its
 * upper 64- or 128-column block tiles, mirrored (it differs from the full
 * product by (C^T C - I) diag(h), which only moves G within span(C)).
 * Outputs: X (n x ld), G (n x ld), h (m), Hp (m x m), E (1 double); all
 * device.
 * precision TM_FULL_DP: all FP64.  TM_MP2: steps (6) and (7) on FP32
 * matrix cores (Sec. 2.2, MP2).  TM_MP1: FP64 products, G rounded to FP32
 * (Sec. 2.2, MP1 (i)).  G is returned in FP64 in every case. */
tm_status tm_energy_grad(tm_ctx *ctx, const tm_mat *H, int32_t m,
                         int32_t precision, const double *C, double *X,
                         double *G, double *h, double *Hp, double *E);

/* In-place Cholesky orthonormalization of an FP64 block (Fig. 4, read as
 * Cholesky-QR): S = C^T C = R^T R, C <- C R^{-1}.  precision TM_FULL_DP uses
 * an FP64 triangular product; TM_MP2 uses the MP1 (ii) split
 * C R^{-1} = C D + C R' with D = diag(R^{-1}) in FP64 and R' in FP32 (Eq. 11-13). */
tm_status tm_orthonormalize(tm_ctx *ctx, int64_t n, int32_t m,
                            int32_t precision, double *C);

/* R^{-1} of the Cholesky factor S = R^T R, R upper triangular (Fig. 4,
 * steps (2)-(3)), for an m x m FP64 S, 1 <= m <= 2048.  Rinv is m x m, upper triangular with
 * zeros below the diagonal.  Synchronous; TM_ENOTSPD if a pivot is not
 * positive. */
tm_status tm_cholesky_inverse(tm_ctx *ctx, int32_t m, const double *S,
                              double *Rinv);

/* Eigen-decomposition of a symmetric m x m FP64 A (1 <= m <= 2048) by
 * parallel block Jacobi (the diagonalization of H in Eq. 9): w ascending (m),
 * U (m x m, column j is the eigenvector of w[j]).  A is not modified.
 * TM_ENOCONV if the off-diagonal norm has not fallen below 1e-15 ||A||_F
 * within the sweep cap (no result is returned then). */
tm_status tm_sym_eig(tm_ctx *ctx, int32_t m, const double *A, double *U,
                     double *w);

/* ----------------------------------------------------------- measurement
 * Average device duration of one kernel of the iteration at H's size,
 * measured with HIP events on the context's stream around `reps` back-to-back
 * launches (after two warm-up launches), on library-allocated blocks filled
 * with a constant byte pattern.  Synchronous.  kernel selects:
 *   TM_K_SPMM       X = H C                               (dtype)
 *   TM_K_GRAM_SHIFT H' = C^T (X - C diag(h)) upper tiles, split-K part (dtype)
 *   TM_K_GRAM_SYM   S = C^T C upper tiles, split-K part     (dtype)
 *   TM_K_ROT_GRAD   G = -2 (X' - C H')                     (dtype)
 *   TM_K_TRMM       C D + C R'                             (dtype)
 *   TM_K_GRAM_MP2   H' upper tiles from FP64 blocks on FP32 matrix cores
 *                   (dtype ignored)
 *   TM_K_ROT_GRAD_MP2 G from FP64 C and X, FP32 H' and FP32 G (dtype ignored)
 *   TM_K_TRMM_MP2   FP64 C D + C R' with R' on FP32 matrix cores (dtype ignored)
 *   TM_K_CHOL       S = R^T R and R^{-1}, m x m FP64 (dtype ignored)
 *   TM_K_GRAM_BF16X3 H' from FP32 blocks on BF16 matrix cores, two-term
 *                   operands (dtype ignored) */
typedef enum tm_kernel_id {
    TM_K_SPMM = 0,
    TM_K_GRAM_SHIFT = 1,
    TM_K_GRAM_SYM = 2,
    TM_K_ROT_GRAD = 3,
    TM_K_TRMM = 4,
    TM_K_GRAM_MP2 = 5,
    TM_K_ROT_GRAD_MP2 = 6,
    TM_K_TRMM_MP2 = 7,
    TM_K_CHOL = 8,
    TM_K_GRAM_BF16X3 = 9
} tm_kernel_id;

tm_status tm_time_kernel(tm_ctx *ctx, const tm_mat *H, int32_t kernel, int32_t m,
                         int32_t dtype, int32_t reps, double *avg_ms);

#ifdef __cplusplus
}
#endif

#endif /* TRACEMIN_H */
