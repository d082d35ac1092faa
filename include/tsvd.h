/*
 * tsvd.h -- C ABI of the MI355X (gfx950) truncated-SVD library.
 *
 * The library computes the k leading singular triplets of a real matrix A by
 * the power method with deflation (Boureima et al., "Distributed
 * Out-of-Memory SVD on CPU/GPU Architectures": Algorithm 1, the driver;
 * Algorithm 2, the power method on the Gram matrix; Algorithm 3, the Gram as
 * a sum of block products; Equations 1-3 and Algorithm 4, the deflated
 * product applied to a vector without forming the residual).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All matrices are dense and addressed by plain pointers and leading
 *   dimensions.  A is ROW-major (element (i, j) at A[i * lda + j], lda >= n).
 *   U (m x k), V (n x k) and the iterate matrices X are COLUMN-major (column j
 *   contiguous at X + j * ldx, ldx >= rows): one singular vector per column.
 *   Gram matrices B are stored in full (both triangles), row-major, ldb >= d.
 * - Device pointers are HIP device allocations on the context's device
 *   (torch.cuda tensors qualify).  "host" pointers are ordinary host memory
 *   unless stated "pinned".
 * - The caller owns A, the CSR arrays and every output buffer.  The library
 *   only borrows them for the duration of the call.  The library owns the
 *   context, its workspaces and its internal streams.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Entry
 *   points that return a status derived from device results (convergence,
 *   rank deficiency) synchronise `stream` before returning; those documented
 *   as "asynchronous" do not.
 * - Nothing throws across the ABI.  On failure the status says what went
 *   wrong and tsvd_last_error(ctx) holds a message (per context).
 * - Calls on one context are not thread safe; use one context per host thread.
 *
 * Sign convention: the largest-magnitude entry of each v_j is positive (ties:
 * lowest index) and u_j follows from u_j = A v_j / sigma_j.
 */
#ifndef TSVD_H
#define TSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TSVD_OK = 0,
  TSVD_ERR_INVALID_ARG = 1,    /* bad shape, k, pointer, leading dimension or option */
  TSVD_ERR_OUT_OF_MEMORY = 2,  /* device allocation failed or would exceed opts.hbm_budget */
  TSVD_ERR_NOT_CONVERGED = 3,  /* eps > 0 and some triplet hit max_iter; all outputs are still filled */
  TSVD_ERR_NONFINITE = 4,      /* NaN/Inf met in the Gram, a product or a norm */
  TSVD_ERR_HIP = 5,            /* a HIP runtime call failed */
  TSVD_ERR_REJECTED = 6,       /* the server cannot admit the request even when idle */
  TSVD_ERR_UNSUPPORTED = 7,    /* valid request outside what the library implements */
  TSVD_ERR_INTERNAL = 8        /* an internal consistency check failed (e.g. a bounded device wait timed out) */
} tsvd_status;

typedef enum { TSVD_F32 = 0, TSVD_F64 = 1 } tsvd_dtype;

typedef enum { TSVD_LOC_DEVICE = 0, TSVD_LOC_PINNED_HOST = 1 } tsvd_loc;

/* How the Gram (Algorithm 2's B = X^T X or X X^T) is computed.
 * FP32:   FP32 operands, FP32 MFMA, FP32 accumulation.
 * BF16X3: each FP32 element a is split into hi = bf16(a), lo = bf16(a - hi);
 *         the Gram is hi^T hi + hi^T lo + lo^T hi on BF16 MFMA with FP32
 *         accumulation (lo^T lo is dropped).  Same HBM traffic as FP32.
 * FP64:   FP64 operands and accumulation (FP64 MFMA); requires FP64 A.
 * AUTO:   FP64 for FP64 A, BF16X3 for FP32 A.                               */
typedef enum { TSVD_GRAM_AUTO = 0, TSVD_GRAM_FP32 = 1, TSVD_GRAM_BF16X3 = 2, TSVD_GRAM_FP64 = 3 } tsvd_gram;

/* Which Gram: RIGHT = A^T A (n x n, iterate on v), LEFT = A A^T (m x m, iterate on u). */
typedef enum { TSVD_SIDE_RIGHT = 0, TSVD_SIDE_LEFT = 1 } tsvd_side;

typedef struct {
  int32_t k;               /* triplets wanted; -1 = min(m, n) (Algorithm 1) */
  double eps;              /* stopping test |v0 . v1| >= 1 - eps of Algorithm 2, evaluated in FP64;
                              eps <= 0 runs exactly max_iter iterations per triplet */
  int32_t max_iter;        /* iteration cap per triplet (the paper's loop has none); default 10000 */
  const int32_t* fixed_iters; /* optional HOST array of k counts: triplet l runs exactly fixed_iters[l]
                                 iterations (trajectory mode); overrides eps */
  const double* v0;        /* DEVICE, k x d row-major, d = length of the iterated vector (n for the
                              right branch, m for the left): row l is the N(0, I) start vector of
                              triplet l (Algorithm 2 draws one per call).  Required. */
  int32_t gram;            /* tsvd_gram */
  int64_t rows_per_block;  /* contraction rows (columns, for m < n) per Gram chunk (in HBM) or per
                              streamed batch (pinned host); 0 = library default */
  int64_t hbm_budget;      /* device bytes the call may allocate for workspace; 0 = no limit */
  int32_t branch;          /* 0: m >= n iterates on v (A^T A); 1: m > n as printed in Algorithm 1 */
  int32_t queue_depth;     /* device buffers in the host->device batch pipelines, 1..16 (default 2; the
                              pinned-A Gram pipeline takes at least 2): A's row (or column) batches, sparse tile
                              batches, and the factor batches below */
  int32_t method;          /* dense A only (tsvd_method): how Algorithm 2's product is applied */
  int32_t factor_loc;      /* implicit paths (sparse A, method IMPLICIT): where the iterated factor X lives
                              (V on the right branch, U on the left): TSVD_LOC_DEVICE (default), or
                              TSVD_LOC_PINNED_HOST: the caller's V (or U) output is pinned host memory, and
                              every projection against the found vectors streams X to the device in
                              factor_batches row batches through queue_depth device buffers (the paper's
                              out-of-memory handling of the heavy co-factor, Sec. V-C) */
  int32_t factor_batches;  /* n_b for factor_loc = PINNED_HOST: X's rows are cut into this many batches,
                              each rounded up to a multiple of 4096 rows (so fewer may result); 0 = 1 */
} tsvd_opts;

/* How a dense t-SVD applies Algorithm 2's operator.
 * GRAM:     form B = A^T A (or A A^T) once (Algorithm 3) and iterate on it; the
 *           power iteration runs on chip when the iterate fits the on-chip
 *           kernel, else as a host-driven loop of HBM-streamed B x products.
 * IMPLICIT: never form B: every iteration applies A^T (A x) (or A (A^T x)) as
 *           two mat-vecs over A (Equation 2 evaluated right to left); A in
 *           pinned host memory is then streamed once per iteration (row
 *           batches for m >= n, pitched column batches for m < n).
 * AUTO:     GRAM when its workspace (B, split-K partials, finish sums, plus the
 *           row-batch buffers for pinned A) fits hbm_budget and the device's
 *           free memory, else IMPLICIT.                                       */
typedef enum { TSVD_METHOD_AUTO = 0, TSVD_METHOD_GRAM = 1, TSVD_METHOD_IMPLICIT = 2 } tsvd_method;

typedef struct {
  int32_t k_done;          /* triplets computed before a zero product stopped the run */
  int32_t rank_deficient;  /* 1 if a zero product or sigma = 0 was met */
  int32_t converged;       /* 1 if every triplet met the stopping test (always 1 in fixed modes) */
  int32_t branch_right;    /* 1: v first on A^T A; 0: u first on A A^T */
  int32_t* iters;          /* optional HOST array of k: iterations taken per triplet (filled) */
  double* lambda;          /* optional HOST array of k: ||B_l x|| at the last iteration (filled) */
  double t_gram_ms;        /* device time of the Gram phase (HIP events) */
  double t_eig_ms;         /* device time of the power-iteration phase */
  double t_final_ms;       /* device time of the FP64 finishing pass (U = A V / sigma, signs) */
  double t_total_ms;       /* device time of the whole call */
  int64_t workspace_bytes; /* device workspace the call used */
  int64_t h2d_bytes;       /* bytes copied host -> device (pinned-host input) */
  double latency_ms;       /* server requests: submission -> completion, host clock; else 0 */
  double t_stream_copy_ms;    /* pinned-host A, Gram pass: time the copy stream spent copying batches
                                 (sum of per-batch HIP event intervals); else 0 */
  double t_stream_compute_ms; /* the same pass: time the compute stream spent in the batches' Grams */
  double t_stream_overlap_ms; /* time during which both ran at once (intersection of the two streams'
                                 per-batch event intervals) */
} tsvd_info;

typedef struct tsvd_ctx tsvd_ctx;

/* Create a context on HIP device `device`.  Queries the device (CU count,
 * LDS size) and creates the library's internal streams.  Returns
 * INVALID_ARG for a bad device, HIP on runtime failure. */
tsvd_status tsvd_ctx_create(int device, tsvd_ctx** out);

/* Destroy a context and free its workspaces.  NULL is ignored. */
void tsvd_ctx_destroy(tsvd_ctx* ctx);

/* Static string for a status code. */
const char* tsvd_status_string(tsvd_status s);

/* Message of the last failing call on `ctx` ("" if none).  Owned by ctx. */
const char* tsvd_last_error(const tsvd_ctx* ctx);

/* Gram-dimension classes of the batched Gram's per-class unit shapes (tsvd_tuning). */
#define TSVD_GRAM_CLASSES 8

/* Launch-shape tuning of a context (chosen by the library when 0).  The
 * autotuner (paper_2208_08410_amd.autotune) measures candidates per shape class
 * and sets these before a call. */
typedef struct {
  int32_t gram_tile;     /* BF16X3 Gram tile edge: 0 (library choice), 128 or 256 */
  int32_t gram_chunks;   /* contraction chunks (split-K) per Gram launch: 0 = library choice */
  int32_t power_blocks;  /* workgroups of the power-iteration launch: 0 = one per CU; for batches the cap
                            on every team and on the engine launch's grid */
  int32_t team_kib;      /* batched engine launch: KiB of a problem's Gram per team workgroup, which
                            sets the team size (ceil(4 d^2 / (team_kib * 1024)) workgroups);
                            0 = 256; range [8, 65536] */
  int32_t group_kchunk;  /* batched Gram: contraction rows per work unit; 0 = 2048; range [32, 2^20] */
  int32_t sparse_row_bits; /* sparse products: tiles of 2^bits rows, one per wave (0 = library choice,
                              about two workgroups of 8 chunks per CU, 32..1024 rows); range [0, 11];
                              applies to handles created after the call */
  int32_t sparse_col_bits; /* sparse products: column slices of 2^bits (0 = 2^18: 1 MiB of FP32 x);
                              row + column bits <= 32 */
  int32_t power_path;    /* Gram power iteration: 0 = the on-chip persistent kernel when the iterate fits
                            it, else the host-driven loop of HBM-streamed B x products; 1 = always that
                            loop (B is then left undeflated: deflation is a projection per iteration) */
  /* Batched Gram work-unit shape per Gram-dimension class c (TSVD_GRAM_CLASSES classes: c = 0 for
     d <= 128, c for 2^(6+c) < d <= 2^(7+c), the last for d > 8192).  A unit is one tile_edge x
     tile_edge triangle tile over a chunk of contraction rows.  The edge does not change any result
     bit (every Gram entry sums the same contraction steps in the same order); the chunk length sets
     the split-K order of the FP32 sums, per problem, so a problem still gives the same bits alone and
     in any mix. */
  int32_t group_tile[TSVD_GRAM_CLASSES];       /* tile edge of class c: 0 = library choice (128), 64 or 128 */
  int32_t group_kchunk_cls[TSVD_GRAM_CLASSES]; /* contraction rows per unit of class c: 0 = group_kchunk;
                                                  range [32, 2^20] */
} tsvd_tuning;

/* Set / read the context's tuning.  INVALID_ARG for out-of-range values. */
tsvd_status tsvd_ctx_set_tuning(tsvd_ctx* ctx, const tsvd_tuning* tuning);
tsvd_status tsvd_ctx_get_tuning(const tsvd_ctx* ctx, tsvd_tuning* tuning);

/* Fill opts with defaults: k = -1, eps = 1e-8, max_iter = 10000, gram = AUTO,
 * everything else 0/NULL, queue_depth = 2. */
void tsvd_opts_default(tsvd_opts* opts);

/* ---------------------------------------------------------------------------
 * Step entry points (each is one row of the method; tsvd_dense chains them)
 * ------------------------------------------------------------------------- */

/* Gram product, Algorithm 2's B = X^T X (side RIGHT) or X X^T (side LEFT),
 * formed as Algorithm 3's sum of block products over chunks of the
 * contraction dimension.  A: DEVICE, dtype, m x n row-major (lda).  B: DEVICE,
 * d x d (d = n for RIGHT, m for LEFT) row-major (ldb), FP32 for gram FP32 /
 * BF16X3, FP64 for gram FP64; both triangles are written.  accumulate != 0
 * adds to B (B += A^T A) instead of overwriting it.  rows_per_block: chunk of
 * the contraction dimension per work unit (0 = default).  Asynchronous. */
tsvd_status tsvd_gram_dense(tsvd_ctx* ctx, const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                            int32_t gram, int32_t side, int64_t rows_per_block, void* B, int64_t ldb,
                            int32_t accumulate, void* stream);

/* Power iteration with deflation on a symmetric d x d Gram (Algorithm 2, run
 * for l = 1..k as Algorithm 1 does).  B: DEVICE, row-major (ldb), dtype FP32
 * or FP64; it is OVERWRITTEN by the deflated Gram (I - v v^T) B (I - v v^T)
 * after each triplet.  opts->v0 (k x d start vectors), k, eps, max_iter,
 * fixed_iters apply.  X: DEVICE FP64 d x k column-major (ldx): the unit
 * iterate vectors, re-orthogonalised in FP64 against the earlier columns.
 * Synchronises `stream`; fills info (k_done, converged, iters, lambda). */
tsvd_status tsvd_power_gram(tsvd_ctx* ctx, void* B, int32_t dtype, int64_t d, int64_t ldb,
                            const tsvd_opts* opts, double* X, int64_t ldx, tsvd_info* info, void* stream);

/* Finishing pass of Algorithm 1 for all k triplets at once, in FP64:
 * W = A X (side RIGHT: X is n x k, W is m x k) or W = A^T X (side LEFT: X is
 * m x k, W is n x k); S[j] = ||W[:, j]||; W[:, j] /= S[j] (columns with
 * S[j] = 0 are left zero).  A: DEVICE dtype row-major (lda); X, W: DEVICE FP64
 * column-major; S: DEVICE FP64 k.  Asynchronous. */
tsvd_status tsvd_finish_dense(tsvd_ctx* ctx, const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                              int32_t side, const double* X, int64_t ldx, int32_t k, double* W, int64_t ldw,
                              double* S, void* stream);

/* The finishing pass of tsvd_finish_dense with no device allocation, for
 * callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments and results, bit for
 * bit (the same kernels run); the scratch that tsvd_finish_dense takes from the
 * context's workspace ((ceil(M / 128) + 2) x k doubles, M = m for RIGHT, n for
 * LEFT) lives instead in a fixed device array of 2^20 doubles (8 MiB) that each
 * device holds for the life of the process.  Larger requests return
 * UNSUPPORTED with a message.  Every call on one device shares that array:
 * calls that overlap on one device (other streams, other contexts, other host
 * threads) race and must be serialised by the caller.  Asynchronous. */
tsvd_status tsvd_finish_dense_noalloc(tsvd_ctx* ctx, const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                                      int32_t side, const double* X, int64_t ldx, int32_t k, double* W, int64_t ldw,
                                      double* S, void* stream);

/* ---------------------------------------------------------------------------
 * Whole t-SVD (Algorithm 1), dense A
 * ------------------------------------------------------------------------- */

/* A: dtype, m x n row-major (lda); loc DEVICE (in HBM) or PINNED_HOST (pinned
 * host memory, streamed to the device along the Gram's contraction through a
 * double-buffered copy pipeline: row batches for m >= n, pitched column
 * batches for m < n; FP32 only).  U: DEVICE FP64 m x k
 * column-major (ldu); S: DEVICE FP64 k; V: DEVICE FP64 n x k column-major
 * (ldv).  Triplets past info->k_done are zero.  Synchronises `stream`.
 * Returns OK, NOT_CONVERGED (outputs filled), NONFINITE, INVALID_ARG,
 * OUT_OF_MEMORY, UNSUPPORTED or HIP. */
tsvd_status tsvd_dense(tsvd_ctx* ctx, const void* A, int32_t dtype, int32_t loc, int64_t m, int64_t n,
                       int64_t lda, const tsvd_opts* opts, double* U, int64_t ldu, double* S, double* V,
                       int64_t ldv, tsvd_info* info, void* stream);

/* ---------------------------------------------------------------------------
 * Many dense problems in one pass (persistent batched kernel)
 * ------------------------------------------------------------------------- */

/* One problem of a batch: the arguments of tsvd_dense for a DEVICE FP32 A. */
typedef struct {
  const void* A;           /* DEVICE, m x n row-major (lda) */
  int32_t dtype;           /* TSVD_F32 (the only type the batched path takes) */
  int64_t m, n, lda;
  tsvd_opts opts;          /* k, eps, max_iter, fixed_iters, v0 (DEVICE), gram (AUTO, FP32 or BF16X3),
                              branch; rows_per_block, hbm_budget and queue_depth are not used */
  double* U;               /* DEVICE FP64 m x k column-major (ldu) */
  int64_t ldu;
  double* S;               /* DEVICE FP64 k */
  double* V;               /* DEVICE FP64 n x k column-major (ldv) */
  int64_t ldv;
} tsvd_problem;

/* Algorithm 1 for `count` independent problems of any mix of shapes.  One
 * persistent engine launch takes work items from one list in order: per
 * problem (queued longest first) its Gram units (problem x split-K chunk x
 * triangle tile, Algorithm 3's block products; tile edge and chunk rows per
 * Gram-dimension class from the context's tuning), the reduction of each tile's
 * chunk partials into the problem's B, and the seats of its power team (a
 * team runs Algorithm 2 with deflation on its problem, then its members take
 * further items), so later problems' Gram work runs beside earlier problems'
 * teams; then one grouped FP64 finishing product.  Each problem's result is
 * what tsvd_dense computes for it, up to the rounding of a different
 * reduction order.  hbm_budget bounds the workspace of the whole batch (0 =
 * no limit).  infos (optional, count entries) receive per-problem k_done,
 * converged, iters, lambda and the batch's phase times (t_gram_ms covers only
 * the clears before the engine launch, t_eig_ms the engine: Gram, reductions
 * and power iterations together); statuses
 * (optional HOST array of count) receive per-problem statuses.  Synchronises
 * `stream`.  Returns OK when every problem is OK, else the status of the first
 * failing problem (argument errors are found before any launch). */
tsvd_status tsvd_dense_batched(tsvd_ctx* ctx, int32_t count, const tsvd_problem* problems, int64_t hbm_budget,
                               tsvd_info* infos, int32_t* statuses, void* stream);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of dense requests
 * ------------------------------------------------------------------------- */

typedef struct tsvd_server tsvd_server;

typedef struct {
  int64_t hbm_budget;      /* device bytes the server allocates once and admits requests into (> 0).
                              1/16 of it (16 MiB..512 MiB, at most half) holds the running batch's
                              tables; the rest holds admitted requests' workspaces and staged A */
  int32_t max_slots;       /* requests admitted and not yet completed, at most; 0 = 256 */
  int32_t max_batch;       /* requests per batch launch, at most; 0 = max_slots */
  int32_t lanes;           /* batches that may run on the device at once, 1..8; 0 = 1.  A further batch
                              launches only into the CUs the running engine launches have released, with
                              the requests whose team fits them, so all launches always fit the chip
                              together */
} tsvd_server_config;

typedef struct {
  int64_t submitted, completed, failed, rejected;  /* completed = finished with OK */
  int64_t batches;         /* batch launches so far */
  double mean_batch;       /* requests per batch launch */
  double p50_ms, p99_ms, mean_ms, max_ms; /* submit -> completion latency of finished (not rejected)
                                             requests, nearest-rank percentiles */
  int64_t peak_bytes;      /* high-water mark of admitted request footprints */
  int64_t in_flight;       /* admitted or running now */
  int64_t waiting;         /* submitted, not yet admitted */
  int64_t lanes_busy_max;  /* most batches on the device at once so far */
  int64_t overlapped;      /* batch launches made while another batch was on the device */
} tsvd_server_stats;

/* Start a server on ctx's device: one device allocation of cfg->hbm_budget
 * bytes, a compute stream per lane, a host->device copy stream and a worker
 * thread.  The worker owns ctx until tsvd_server_destroy: make no other call
 * on ctx meanwhile.  Each worker cycle admits waiting requests in arrival
 * order while a slot is free and the budget covers the request's footprint
 * (its Gram, split-K partials and finish sums, plus its A when A is in pinned
 * host memory, which is then copied at once on the copy stream); whenever a
 * lane is idle it launches admitted requests on it as one batch (as
 * tsvd_dense_batched) into the CUs that no running engine launch holds (the
 * launches' workgroups report their exit through pinned host memory), taking
 * the requests whose team fits; when a lane's batch completes it frees that
 * batch's memory and completes its tickets.  So a request that arrives while
 * another batch runs starts as soon as that batch's teams have released
 * enough CUs, and its work overlaps the rest of the running batch.  A
 * request's result is the same whether it runs alone or in any mix (its
 * launch shapes depend on it alone). */
tsvd_status tsvd_server_create(tsvd_ctx* ctx, const tsvd_server_config* cfg, tsvd_server** out);

/* Queue one request; returns at once with a ticket.  The problem struct is
 * copied (with opts.fixed_iters); A (loc DEVICE or PINNED_HOST), opts.v0, U, S
 * and V are borrowed until the ticket completes.  Argument errors are returned
 * here (INVALID_ARG / UNSUPPORTED); a request whose footprint exceeds the
 * budget completes with REJECTED.  Thread safe. */
tsvd_status tsvd_server_submit(tsvd_server* srv, const tsvd_problem* problem, int32_t loc, uint64_t* ticket);

/* Non-blocking: *done = 1 once the ticket completed; then info (optional; its
 * iters / lambda arrays, if set, receive k entries) and *status (optional) are
 * filled and the ticket is released.  INVALID_ARG for an unknown ticket. */
tsvd_status tsvd_server_poll(tsvd_server* srv, uint64_t ticket, int32_t* done, tsvd_info* info, int32_t* status);

/* Block until the ticket completes; fill info and release the ticket.
 * Returns the request's status. */
tsvd_status tsvd_server_wait(tsvd_server* srv, uint64_t ticket, tsvd_info* info);

/* Counters and latency percentiles so far. */
tsvd_status tsvd_server_get_stats(tsvd_server* srv, tsvd_server_stats* stats);

/* Message of the server's last failure ("" if none). */
const char* tsvd_server_last_error(const tsvd_server* srv);

/* Finish every submitted request, stop the worker, free the device memory.
 * NULL is ignored. */
void tsvd_server_destroy(tsvd_server* srv);

/* ---------------------------------------------------------------------------
 * Sparse A (CSR): the implicit deflated product of Equation 2 / Algorithm 4
 * ------------------------------------------------------------------------- */

typedef struct tsvd_csr tsvd_csr;

/* Register an m x n CSR matrix held on the device: rowptr int64 [m+1],
 * col int32 [nnz] (0 <= col < n), val FP32 [nnz].  The arrays are BORROWED and
 * must outlive the handle.  The structure is validated on the device first
 * (monotone row pointers, rowptr[0] = 0, rowptr[m] = nnz, column range);
 * a violation returns INVALID_ARG before any product reads through it.  Then
 * the transpose is built once as a CSC copy owned by the handle (counting sort
 * by column, rows ascending inside each column), so that both A x and A^T y
 * are gather-only products.  Synchronises `stream`. */
tsvd_status tsvd_csr_create(tsvd_ctx* ctx, int64_t m, int64_t n, int64_t nnz, const int64_t* rowptr,
                            const int32_t* col, const float* val, tsvd_csr** out, void* stream);

/* Register an m x n CSR matrix held in PINNED HOST memory (rowptr int64
 * [m+1], col int32 [nnz], val FP32 [nnz]; hipHostMalloc / pinned torch
 * tensors), for matrices kept out of HBM: the paper's out-of-memory case of
 * degree 1 (Sec. III, Sec. V-C).  The arrays are read only during this call.
 * The sliced tiles of A and of A^T are built on the device batch by batch
 * (whole row chunks of at most batch_bytes of tiles per batch, 0 = 512 MiB;
 * A^T's batches are gathered by streaming the CSR once per batch of its
 * columns) and kept in pinned host memory owned by the handle (16 bytes per
 * nonzero).  Every product then streams its tiles to the device through
 * queue_depth device slots (0 = 2, at most 16) on the handle's copy stream,
 * while the previous slot's product runs; the handle holds those slots
 * (queue_depth x the largest batch x 8 bytes) and the tile pointers on the
 * device.  Products, tsvd_spmv and tsvd_sparse give bitwise the results of a
 * device handle of the same matrix (same tiles, same order).
 * tsvd_csr_get_csc is UNSUPPORTED on such a handle.  Structure errors return
 * INVALID_ARG as for tsvd_csr_create.  Synchronises `stream`. */
tsvd_status tsvd_csr_create_pinned(tsvd_ctx* ctx, int64_t m, int64_t n, int64_t nnz, const int64_t* rowptr,
                                   const int32_t* col, const float* val, int64_t batch_bytes, int32_t queue_depth,
                                   tsvd_csr** out, void* stream);

/* Where a handle's tiles live (*loc: TSVD_LOC_DEVICE or TSVD_LOC_PINNED_HOST),
 * how many row batches a product of A streams (0 for device handles), and
 * the device bytes the handle holds.  Any output may be NULL. */
tsvd_status tsvd_csr_info(const tsvd_csr* csr, int32_t* loc, int64_t* batches, int64_t* device_bytes);

/* Free the handle's CSC copy and tiles.  NULL is ignored. */
void tsvd_csr_destroy(tsvd_csr* csr);

/* Copy the CSC transpose into caller DEVICE buffers: colptr int64 [n+1],
 * rowidx int32 [nnz], val FP32 [nnz].  Asynchronous. */
tsvd_status tsvd_csr_get_csc(tsvd_ctx* ctx, const tsvd_csr* csr, int64_t* colptr, int32_t* rowidx, float* val,
                             void* stream);

/* Sparse product with FP64 accumulation: trans = 0: y = A x (x: n entries,
 * y: m entries); trans = 1: y = A^T x (x: m, y: n).  x DEVICE FP32 (x_dtype
 * TSVD_F32) or FP64 (TSVD_F64); y DEVICE FP64.  Asynchronous. */
tsvd_status tsvd_spmv(tsvd_ctx* ctx, const tsvd_csr* csr, int32_t trans, const void* x, int32_t x_dtype, double* y,
                      void* stream);

/* Whole t-SVD of a CSR matrix (Algorithm 1 with the implicit product of
 * Algorithm 4 in factored form).  Each power iteration computes
 * z = P A^T (A x) (right branch, m >= n) or z = P A (A^T x) (left branch):
 * FP32 values, FP64 accumulation, FP64 projection P = I - V V^T against the
 * triplets already found, with the start vector projected once.  Then
 * u = A v / ||A v|| (or the mirror) in FP64.  opts->v0 is k x d (d = n right,
 * m left).  U, S, V as in tsvd_dense.  Synchronises `stream` (one small
 * device-to-host read per iteration for the stopping test). */
tsvd_status tsvd_sparse(tsvd_ctx* ctx, const tsvd_csr* csr, const tsvd_opts* opts, double* U, int64_t ldu,
                        double* S, double* V, int64_t ldv, tsvd_info* info, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TSVD_H */
