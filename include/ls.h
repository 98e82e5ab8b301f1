/*
 * ls.h -- C ABI of libls, an MI355X (gfx950) implementation of iterative sketching, the randomized
 * least-squares solver of E. N. Epperly, "Fast and forward stable randomized algorithms for linear
 * least-squares problems" (arXiv 2311.04362).
 *
 * Problem (eq. ls):  x = argmin_y ||b - A y||  for full-rank A (m x n), m >= n.
 * Method (Algorithm 2):  S <- d x m sparse-sign embedding;  B <- S A;  (Q, R) <- QR(B);
 *   x_0 <- R^{-1} Q^T (S b);  for i < q:  r_i = b - A x_i;  c_i = A^T r_i;
 *   d_i = R^{-1} (R^{-T} c_i);  x_{i+1} = x_i + d_i.
 *
 * Conventions shared by every entry point
 *  - Matrices are row-major: element (i, j) of a matrix with leading dimension ld is at [i*ld + j].
 *  - All array arguments are DEVICE pointers on the context's GPU, allocated and freed by the
 *    caller; they must be 8-byte aligned.  The library owns only its internal workspace (and
 *    the side stream of ls_create's note).
 *  - `stream` is a hipStream_t (NULL: the device's null stream).  Every call enqueues its work on
 *    that stream and returns without waiting, except ls_sync and ls_solve (which waits to report).
 *  - Argument errors are reported synchronously (LS_ERR_ARG) before anything is enqueued.
 *    Conditions the GPU detects (rank deficiency, NaN/Inf) are deferred: they are collected in a
 *    device status word and returned by the next ls_sync on that context.
 *  - Nothing aborts and no exception crosses the ABI.  ls_last_error gives a readable detail.
 *  - Results are deterministic: the same inputs, options and seed give bitwise-identical outputs
 *    (no floating-point atomics; every reduction has a fixed order).
 *  - A context is not thread-safe; use one per host thread.  Calls on one context that overlap
 *    on different streams share its workspace and must be ordered by the caller.
 */
#ifndef LS_H
#define LS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LS_OK = 0,
    LS_ERR_ARG = 1,          /* invalid argument (synchronous)                                   */
    LS_ERR_ALLOC = 2,        /* device allocation failed                                         */
    LS_ERR_DEVICE = 3,       /* HIP runtime error, or no usable device                           */
    LS_ERR_RANK = 4,         /* deferred: |R_kk| <= n u max_j |R_jj| (A taken as rank deficient) */
    LS_ERR_NONFINITE = 5,    /* deferred: NaN or Inf met in B, R or x                            */
    LS_ERR_DIVERGED = 6,     /* deferred: the stopping rule saw the residual grow without bound  */
    LS_ERR_UNSUPPORTED = 7,  /* a size beyond the library's compiled limits (see ls_limits)      */
    LS_ERR_TIMEOUT = 8       /* ls_server_wait: the request did not finish within the timeout    */
} ls_status;

typedef struct ls_ctx ls_ctx;

/* Compiled limits of the library (returned by ls_limits). */
#define LS_MAX_ZETA 32       /* nonzeros per column of S                                         */
#define LS_MAX_N 2048        /* columns of A                                                     */

/* Context: binds a GPU, its compiled kernels, a growable workspace and the status word.
 * device >= 0 selects a GPU.  device = -1 creates a host-only context that validates arguments
 * and then returns LS_ERR_DEVICE from every compute call (for testing argument checks without a
 * GPU).  Returns LS_ERR_DEVICE if the GPU cannot be used.  The first QR of a large sketch
 * (d*n >= 3e7, cooperative panels) also creates one non-blocking side stream and two events in
 * the context; that QR's trailing updates run partly on it, joined back into the caller's stream
 * by events before the call's later work, so ordering on the caller's stream is unchanged. */
ls_status ls_create(int device, ls_ctx **out);
void ls_destroy(ls_ctx *ctx);         /* frees the workspace, side stream, events; NULL is a no-op */
const char *ls_last_error(const ls_ctx *ctx);       /* detail of the last failure, never NULL  */
ls_status ls_limits(int32_t *max_zeta, int32_t *max_n);

/* Options (ls_set_option / ls_get_option).  Integer options take ival, real ones dval. */
enum {
    LS_OPT_ZETA = 1,        /* nonzeros per column of S used by ls_solve (default 8, Sec. 3.3)   */
    LS_OPT_SEED = 2,        /* seed of S used by ls_solve (default 0)                           */
    LS_OPT_UPDATE = 3,      /* 0: x += d (Alg. 2); 1: damping; 2: momentum (eq. damping_momentum) */
    LS_OPT_ALPHA = 4,       /* alpha of the damping/momentum update (dval; <= 0: from eps)      */
    LS_OPT_BETA = 5,        /* beta of the momentum update (dval; < 0: from eps)                */
    LS_OPT_PRECISION = 6,   /* 0: FP64 throughout; 1: mixed (see "Mixed precision" below)        */
    LS_OPT_PROFILE = 7,     /* 1: time every launch of the fused pass kernel with HIP events    */
    LS_OPT_QR_PANEL = 8,    /* 0: one cooperative launch per QR panel when the device allows it;
                               1: one launch per column (the fallback path)                     */
    LS_OPT_STOP = 9,        /* 1: ls_solve stops by the rule of Section 3.3, q being the maximum  */
    LS_OPT_GAMMA = 10,      /* gamma of that rule (dval, default 1)                              */
    LS_OPT_RHO = 11,        /* rho of that rule (dval, default 0.04)                             */
    LS_OPT_GATHER = 12      /* 0: the column-sliced sketch gather when the shape suits it (n >= 448,
                               65536 <= m < 2^26); 1: one wave per sketch row always.  Same bits. */
};
ls_status ls_set_option(ls_ctx *ctx, int key, int64_t ival, double dval);
ls_status ls_get_option(const ls_ctx *ctx, int key, int64_t *ival, double *dval);

/* ---- Sparse-sign embedding (eq. sparse_sign, Section 2.2) -------------------------------------
 * S = zeta^{-1/2} [s_1 ... s_m] (d x m); column s_j holds zeta distinct nonzeros +-1.  Positions and
 * signs come from the counter-based SplitMix64 stream `seed` (Steele, Lea & Flood 2014): column j
 * uses outputs j*2^16 + t, t = 0, 1, ...; a draw z proposes row (z >> 11) mod d, a repeated row is
 * rejected, an accepted draw gives sign -1 if bit 0 of z is set, else +1; a column that exhausted
 * its 2^16 draws is completed with the smallest free rows, sign +1.
 *
 * ls_sketch_embedding writes the nonzeros column by column, in acceptance order:
 *   rows[j*zeta + e] (int32, in [0, d)), signs[j*zeta + e] (int8, +-1), j < m, e < zeta.
 * Requires m >= 1, 1 <= zeta <= min(d, LS_MAX_ZETA), d < 2^31, m*zeta < 2^31. */
ls_status ls_sketch_embedding(ls_ctx *ctx, void *stream, int64_t m, int64_t d, int32_t zeta,
                              uint64_t seed, int32_t *rows, int8_t *signs);

/* The same S transposed into compressed rows: for sketch row k, entries rowptr[k] .. rowptr[k+1]-1
 * of `cols` hold the columns j with S[k, j] != 0 in ascending j; bit 31 of an entry is set when
 * S[k, j] < 0 and bits 0..30 hold j.  rowptr has d+1 entries, cols has m*zeta. */
ls_status ls_sketch_csr(ls_ctx *ctx, void *stream, int64_t m, int64_t d, int32_t zeta,
                        uint64_t seed, int32_t *rowptr, int32_t *cols);

/* ---- Sketch (Algorithm 2, "B <- S A"; S b for the sketch-and-solve start, eq. sketched_ls) ------
 * B (d x n, ldb >= n) = S A and Sb (d) = S b for A (m x n, lda >= n), b (m).  Row k of B is the sum
 * of +-A[j, :] over the columns j of sketch row k in ascending j, then multiplied once by
 * fl(1/sqrt(zeta)).  Gathered by rows of A; each sum has a single writer that adds its terms in
 * that order, so results are deterministic (and the same under LS_OPT_GATHER 0 and 1).  b and Sb
 * may both be NULL.
 * Requires n >= 1, m >= 1, d >= 1, lda >= n, ldb >= n and the embedding limits above. */
ls_status ls_sketch(ls_ctx *ctx, void *stream, int64_t m, int64_t n, const double *A, int64_t lda,
                    const double *b, int64_t d, int32_t zeta, uint64_t seed, double *B, int64_t ldb,
                    double *Sb);

/* ---- Householder QR of the sketch and the sketch-and-solve start (Alg. 2, third and fourth
 * lines; eq. it-sk-qr, eq. sketched_ls) --------------------------------------------------------
 * Factors [B | Sb] (d x (n+1)) by blocked Householder reflections (compact-WY trailing updates on
 * FP64 matrix cores).  Q is never formed: Q^T is applied to Sb as the last column.
 * Writes R (n x n upper triangular, ldr >= n; the strict lower triangle is set to zero) and
 * x0 = R^{-1} (Q^T Sb)[0:n] (n, nullable).  R[k,k] = -sign(alpha) * ||column||, sign(0) = +1.
 * B and Sb are read only (the factorization works on a copy in the workspace).
 * Deferred: LS_ERR_RANK if |R_kk| <= n u max|R_jj|; LS_ERR_NONFINITE on NaN/Inf in R or x0.
 * Requires 1 <= n <= LS_MAX_N, d >= n, ldb >= n. */
ls_status ls_qr_sketch(ls_ctx *ctx, void *stream, int64_t d, int64_t n, const double *B,
                       int64_t ldb, const double *Sb, double *R, int64_t ldr, double *x0);

/* ---- One evaluation of the refinement right-hand side (Alg. 2 loop, stable form of Sec. 3.2) ----
 * c = A^T (b - A x) with the residual formed first, in FP64, and never stored; rnorm2 (nullable,
 * one double) = ||b - A x||^2.  A is read once.  Requires 1 <= n <= LS_MAX_N, m >= 1, lda >= n. */
ls_status ls_gradient(ls_ctx *ctx, void *stream, int64_t m, int64_t n, const double *A, int64_t lda,
                      const double *b, const double *x, double *c, double *rnorm2);

/* ---- ls_gradient without allocation ---------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, kernels and bits as ls_gradient, but the
 * per-work-group partials of c and ||r||^2 live in a fixed 33 MiB scratch array that the library
 * holds on each GPU it runs on until the process ends (its address is looked up once per device by
 * ls_create), not in the context's workspace.  Nothing is allocated or freed (no hipMalloc, no
 * events: LS_OPT_PROFILE does not time this call).  Every call on one GPU, from any context and any
 * stream, uses that GPU's one array: calls that overlap on one GPU race and must be ordered by the
 * caller; a call's results are complete once its stream has reached them.  The array needs no
 * clearing (every partial is written before it is read).  LS_ERR_UNSUPPORTED if the partials
 * exceed the array (not reachable for n <= LS_MAX_N); other errors as ls_gradient. */
ls_status ls_gradient_noalloc(ls_ctx *ctx, void *stream, int64_t m, int64_t n, const double *A,
                              int64_t lda, const double *b, const double *x, double *c, double *rnorm2);

/* ---- The two triangular solves of Alg. 2: d = R^{-1} (R^{-T} c) by forward then back
 * substitution (never an explicit inverse).  R: n x n upper triangular, ldr >= n. */
ls_status ls_precond_solve(ls_ctx *ctx, void *stream, int64_t n, const double *R, int64_t ldr,
                           const double *c, double *d);

/* ---- q refinement steps (Alg. 2 loop; eq. it-sk-it-ref) ---------------------------------------
 * x (n, in: x_i, out: x_{i+q}) is updated q times by x <- x + R^{-1} R^{-T} A^T (b - A x).
 * rnorm2 (nullable, q doubles) receives ||b - A x_i||^2 for each step.  q = 0 leaves x unchanged.
 * With LS_OPT_UPDATE = 1 or 2 the update is x_{i+1} = x_i + alpha d_i + beta (x_i - x_{i-1})
 * (eq. damping_momentum) with x_{-1} = x_i on entry; eps = sqrt(n/d) needs d, so these options
 * take explicit LS_OPT_ALPHA / LS_OPT_BETA here.  Requires q >= 0 and the ls_gradient limits. */
ls_status ls_iterate(ls_ctx *ctx, void *stream, int64_t m, int64_t n, const double *A, int64_t lda,
                     const double *b, const double *R, int64_t ldr, double *x, int32_t q,
                     double *rnorm2);

/* ---- Whole solve (Algorithm 2) ------------------------------------------------------------------
 * x (n) = x_q for A (m x n, lda), b (m), embedding dimension d and q steps, with zeta and seed from
 * the options.  d <= 0 selects eq. (dimension): d = max(ceil((6 + 4 sqrt 2) n exp(W((6 - 4 sqrt 2)
 * (m / n^2) ln(1/u)))), 20 n) with u = 2^-53 and W the principal branch of Lambert's W.
 * With LS_OPT_STOP = 1, q is the maximum number of steps and the iteration ends at the first x_i
 * with ||r(x_i) - r(x_{i-1})|| <= u (gamma normest ||x_i|| + rho condest ||r(x_i)||) (Section 3.3);
 * normest is ceil(ln n) steps of the power method on R from g_i = 2 u_i - 1, u_i the 53 high bits
 * of SplitMix64 output i of the stream seed + 0x632BE59BD9B4E019 scaled to [0, 1); condest is
 * ||R||_1 times Hager's estimate of ||R^{-1}||_1.  The decision is taken on the device; a residual
 * that grows past 100 ||r(x_0)|| ends the iteration with LS_ERR_DIVERGED.
 * Enqueues sketch, QR and iterations, then waits on `stream` and returns the deferred status (as
 * ls_sync).  With LS_OPT_PRECISION = 1 it also waits once after the QR, to take the fallback
 * decision described under "Mixed precision".  Requires d >= n and the limits above. */
ls_status ls_solve(ls_ctx *ctx, void *stream, int64_t m, int64_t n, const double *A, int64_t lda,
                   const double *b, int64_t d, int32_t q, double *x);

/* After ls_solve: the embedding dimension used, the number of refinement steps made (those of the
 * FP64 solve after a fallback), normest and condest when they were computed (LS_OPT_STOP = 1 or
 * LS_OPT_PRECISION = 1; NaN otherwise; from the FP32 factor on the mixed path), and the precision
 * the result came from (LS_PRECISION_*).  Any pointer may be NULL. */
ls_status ls_solve_info(ls_ctx *ctx, int64_t *d_used, int32_t *steps, double *normest,
                        double *condest, int32_t *precision);

/* ---- Mixed precision (LS_OPT_PRECISION = 1) ------------------------------------------------------
 * The paper computes in FP64 only.  In this variant the sketch is stored in FP32 (each entry of the
 * FP64 sum rounded once), its Householder QR runs in FP32 (trailing updates on FP32 matrix cores),
 * and the two triangular solves of every step run in FP32 on c scaled by 2^-e, e the binary
 * exponent of max |c_i| (frexp convention), with d scaled back exactly in FP64; the A^T (b - A x)
 * pass and the update stay FP64, so the refinement still reaches FP64 accuracy when the FP32 factor
 * is a usable preconditioner.  ls_solve falls back to the FP64 solve, from the start, when
 *   condest(R) * 2^-24 > 0.05 (condest in FP32 arithmetic on the FP32 R), or the FP32 QR flags R
 *   as rank deficient or non-finite                                   -> LS_PRECISION_FELL_BACK_COND
 *   ||r_i||^2 grows three steps in a row, each time by more than a relative 2^-20, or is not
 *   finite                                                            -> LS_PRECISION_FELL_BACK_GROWTH
 * The pieces are exposed for testing: */
#define LS_PRECISION_FP64 0
#define LS_PRECISION_MIXED 1
#define LS_PRECISION_FELL_BACK_COND 2
#define LS_PRECISION_FELL_BACK_GROWTH 3

/* ls_sketch with FP32 outputs: B (d x n, ldb >= n) and Sb (d, nullable with b) are the FP64 sums of
 * ls_sketch rounded once to FP32.  B and Sb must be 4-byte aligned. */
ls_status ls_sketch_f32(ls_ctx *ctx, void *stream, int64_t m, int64_t n, const double *A, int64_t lda,
                        const double *b, int64_t d, int32_t zeta, uint64_t seed, float *B, int64_t ldb,
                        float *Sb);

/* ls_qr_sketch in FP32: R (n x n, FP32, ldr >= n, zero strict lower triangle) and x0 (FP64,
 * nullable) = the FP32 back substitution R^{-1} (Q^T Sb)[0:n], widened.  Deferred: LS_ERR_RANK if
 * |R_kk| <= n 2^-24 max|R_jj|; LS_ERR_NONFINITE.  B, Sb, R must be 4-byte aligned. */
ls_status ls_qr_sketch_f32(ls_ctx *ctx, void *stream, int64_t d, int64_t n, const float *B,
                           int64_t ldb, const float *Sb, float *R, int64_t ldr, double *x0);

/* d = R^{-1} (R^{-T} c) with an FP32 R (4-byte aligned, ldr >= n) by FP32 substitution on c scaled
 * by a power of two as above; c and d are FP64. */
ls_status ls_precond_solve_f32(ls_ctx *ctx, void *stream, int64_t n, const float *R, int64_t ldr,
                               const double *c, double *d);

/* ---- Served stream (many independent solves resident on one GPU) -------------------------------
 * A server solves submitted problems with ls_solve's algorithm (zeta = 8, fixed q, plain update; FP64,
 * or mixed precision after ls_server_set_precision) and returns, for each, the same bits ls_solve
 * returns for it alone with the same precision option.  Problems are admitted first
 * in, first out while the footprint stays within `budget_bytes` and at most `max_active` are
 * admitted.  The footprint counts, for every admitted problem, its resident bytes (A and b, 8mn + 8m,
 * plus its device block: R, R^T, pass partials, c) and the workspaces the eight setup lanes hold
 * (embedding, lists, sketch and QR work matrix of the largest problem each set up; an idle lane
 * gives its workspace back when the next problem would not fit otherwise); ls_server_footprint
 * reports both figures for a shape.  The sketch, QR and
 * start of each are computed on one of eight setup streams (eight problems at a time), then every
 * admitted problem takes one refinement step per round on a serve stream (one batched launch per
 * kernel for all of them: continuous batching -- problems join and leave between rounds).  A
 * scheduler thread owned by the server does all device work.  A, b and x are device pointers owned
 * by the caller: A and b must stay unchanged and x untouched until the request is finished; x then
 * holds x_q.  ls_server_submit and ls_server_wait may be called from any host thread.
 * 1 <= max_active <= 4096.  device = -1 creates a host-only server for argument checks (submit
 * returns LS_ERR_DEVICE). */
typedef struct ls_server ls_server;
ls_status ls_server_create(int device, int64_t budget_bytes, int32_t max_active, ls_server **out);
/* Finishes every submitted request, then frees the server. */
void ls_server_destroy(ls_server *server);
/* What admission charges for a problem of this shape: *resident (bytes held while it is admitted)
 * and *setup (the setup-lane workspace its sketch and QR need).  A problem is refused at submission
 * (LS_ERR_ALLOC) when resident + setup exceeds the budget. */
ls_status ls_server_footprint(ls_server *server, int64_t m, int64_t n, int64_t d, int64_t *resident,
                              int64_t *setup);
/* Queues one solve (arguments as ls_solve; d >= n) and returns its ticket.  LS_ERR_ALLOC if its
 * footprint alone exceeds the budget.  Never blocks on the device.  A finished request keeps only a
 * small host record (result and times) until the server is destroyed; its event and pinned status
 * word are reused by later requests. */
ls_status ls_server_submit(ls_server *server, int64_t m, int64_t n, const double *A, int64_t lda,
                           const double *b, int64_t d, int32_t q, uint64_t seed, double *x,
                           int64_t *ticket);
/* Waits until the request is finished (timeout_s < 0: no limit) and stores its status (LS_OK, or a
 * deferred error of that problem alone) in *result; LS_ERR_TIMEOUT if it is still running. */
ls_status ls_server_wait(ls_server *server, int64_t ticket, double timeout_s, ls_status *result);
/* Arithmetic of the requests submitted after this call: LS_PRECISION_FP64 (the default) or
 * LS_PRECISION_MIXED, the mixed-precision variant of ls_solve with LS_OPT_PRECISION = 1 (see "Mixed
 * precision" above): the FP64 sketch, an FP32 QR and FP32 R-solves, FP64 passes and updates.  Its setup waits on the host once, in the
 * scheduler thread, for the fallback decision; a request whose growth monitor fires in the rounds
 * is queued again and solved in FP64.  LS_ERR_ARG for any other value. */
ls_status ls_server_set_precision(ls_server *server, int32_t precision);
/* The precision a request's result comes from (LS_PRECISION_*); final once the request is finished. */
ls_status ls_server_request_precision(ls_server *server, int64_t ticket, int32_t *used);
/* times[0..3]: submission, admission, first round, completion (seconds since ls_server_create;
 * completion is when the scheduler saw the last round end). */
ls_status ls_server_request_info(ls_server *server, int64_t ticket, double *times);
/* stats[0..7]: submitted, finished, queued, admitted and unfinished, footprint now, peak footprint,
 * rounds launched, bytes of the footprint held by the setup lanes' workspaces. */
ls_status ls_server_stats(ls_server *server, int64_t *stats);
const char *ls_server_last_error(ls_server *server);

/* Waits for `stream`, then returns and clears the deferred device status of the context. */
ls_status ls_sync(ls_ctx *ctx, void *stream);

/* Kernel timing (LS_OPT_PROFILE = 1): every launch of the fused pass kernel (the A^T (b - A x)
 * pass of ls_gradient, ls_iterate and ls_solve) is bracketed by HIP events on the caller's stream.
 * ls_profile waits for the recorded events and returns the summed kernel time in milliseconds and
 * the number of launches since the last reset (reset != 0 clears the counters afterwards). */
ls_status ls_profile(ls_ctx *ctx, double *pass_ms, int64_t *pass_launches, int32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* LS_H */
