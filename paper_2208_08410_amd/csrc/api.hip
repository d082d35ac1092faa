// C-ABI implementation: context, workspace, argument checks and the dense
// driver that chains Gram -> power iteration -> FP64 finishing pass
// (Algorithm 1 with Algorithm 2 on the Gram of Algorithm 3).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tsvd.h"
#include "common.h"

#include "ctx.h"
#include "internal.h"

namespace tsvd {

static thread_local std::string g_hip_msg;

int hip_fail(hipError_t e, const char* what, const char* file, int line) {
  char buf[512];
  snprintf(buf, sizeof buf, "HIP error '%s' (%d) in %s at %s:%d", hipGetErrorString(e), (int)e, what, file, line);
  g_hip_msg = buf;
  (void)hipGetLastError();  // clear the sticky error so later calls do not report it again
  return TSVD_ERR_HIP;
}

}  // namespace tsvd

using namespace tsvd;

namespace tsvd {


tsvd_status fail(tsvd_ctx* ctx, tsvd_status st, const char* fmt, ...) {
  if (ctx) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->last_error = buf;
  }
  return st;
}

tsvd_status from_internal(tsvd_ctx* ctx, int rc, const char* where) {
  if (rc == 0) return TSVD_OK;
  if (rc == TSVD_ERR_HIP) return fail(ctx, TSVD_ERR_HIP, "%s: %s", where, g_hip_msg.c_str());
  return fail(ctx, TSVD_ERR_INTERNAL, "%s: internal error %d", where, rc);
}

tsvd_status ensure_ws(tsvd_ctx* ctx, size_t bytes, int64_t budget) {
  if (budget > 0 && (int64_t)bytes > budget)
    return fail(ctx, TSVD_ERR_OUT_OF_MEMORY, "workspace of %zu bytes exceeds hbm_budget %lld", bytes,
                (long long)budget);
  if (ctx->ws_bytes >= bytes) return TSVD_OK;
  if (ctx->ws) {
    hipDeviceSynchronize();
    hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  hipError_t e = hipMalloc(&ctx->ws, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ctx->ws = nullptr;
    return fail(ctx, TSVD_ERR_OUT_OF_MEMORY, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  ctx->ws_bytes = bytes;
  return TSVD_OK;
}

int gram_mode(int32_t gram, int32_t dtype) {
  if (gram == TSVD_GRAM_AUTO) return dtype == TSVD_F64 ? MODE_FP64 : MODE_BF16X3;
  if (gram == TSVD_GRAM_FP32) return MODE_FP32;
  if (gram == TSVD_GRAM_BF16X3) return MODE_BF16X3;
  if (gram == TSVD_GRAM_FP64) return MODE_FP64;
  return -1;
}

tsvd_status check_mode(tsvd_ctx* ctx, int mode, int32_t dtype) {
  if (mode < 0) return fail(ctx, TSVD_ERR_INVALID_ARG, "unknown gram mode");
  if (dtype != TSVD_F32 && dtype != TSVD_F64) return fail(ctx, TSVD_ERR_INVALID_ARG, "unknown dtype %d", dtype);
  if (mode == MODE_FP64 && dtype != TSVD_F64)
    return fail(ctx, TSVD_ERR_UNSUPPORTED, "gram FP64 needs FP64 A");
  if (mode != MODE_FP64 && dtype != TSVD_F32)
    return fail(ctx, TSVD_ERR_UNSUPPORTED, "gram FP32/BF16X3 needs FP32 A");
  return TSVD_OK;
}

bool right_side(int64_t m, int64_t n, int32_t branch) { return branch == 1 ? (m > n) : (m >= n); }

}  // namespace tsvd

extern "C" {

const char* tsvd_status_string(tsvd_status s) {
  switch (s) {
    case TSVD_OK: return "ok";
    case TSVD_ERR_INVALID_ARG: return "invalid argument";
    case TSVD_ERR_OUT_OF_MEMORY: return "out of device memory";
    case TSVD_ERR_NOT_CONVERGED: return "not converged";
    case TSVD_ERR_NONFINITE: return "non-finite value";
    case TSVD_ERR_HIP: return "HIP runtime error";
    case TSVD_ERR_REJECTED: return "request rejected";
    case TSVD_ERR_UNSUPPORTED: return "unsupported";
    case TSVD_ERR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* tsvd_last_error(const tsvd_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

tsvd_status tsvd_ctx_set_tuning(tsvd_ctx* ctx, const tsvd_tuning* t) {
  if (!ctx) return TSVD_ERR_INVALID_ARG;
  if (!t) return fail(ctx, TSVD_ERR_INVALID_ARG, "null tuning");
  if (t->gram_tile != 0 && t->gram_tile != 128 && t->gram_tile != 256)
    return fail(ctx, TSVD_ERR_INVALID_ARG, "gram_tile must be 0, 128 or 256");
  if (t->gram_chunks < 0 || t->gram_chunks > 4096) return fail(ctx, TSVD_ERR_INVALID_ARG, "gram_chunks out of range");
  if (t->power_blocks < 0 || t->power_blocks > ctx->num_cu)
    return fail(ctx, TSVD_ERR_INVALID_ARG, "power_blocks must be in [0, %d]", ctx->num_cu);
  if (t->sparse_row_bits < 0 || t->sparse_row_bits > 13 || t->sparse_col_bits < 0 || t->sparse_col_bits > 31 ||
      t->sparse_row_bits + t->sparse_col_bits > 32)
    return fail(ctx, TSVD_ERR_INVALID_ARG, "sparse tile bits out of range (rows <= 13, rows + cols <= 32)");
  if (t->team_kib != 0 && (t->team_kib < 8 || t->team_kib > 65536))
    return fail(ctx, TSVD_ERR_INVALID_ARG, "team_kib must be 0 or in [8, 65536]");
  if (t->group_kchunk != 0 && (t->group_kchunk < 32 || t->group_kchunk > (1 << 20)))
    return fail(ctx, TSVD_ERR_INVALID_ARG, "group_kchunk must be 0 or in [32, 2^20]");
  ctx->tuning = *t;
  return TSVD_OK;
}

tsvd_status tsvd_ctx_get_tuning(const tsvd_ctx* ctx, tsvd_tuning* t) {
  if (!ctx || !t) return TSVD_ERR_INVALID_ARG;
  *t = ctx->tuning;
  return TSVD_OK;
}

void tsvd_opts_default(tsvd_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof *o);
  o->k = -1;
  o->eps = 1e-8;
  o->max_iter = 10000;
  o->gram = TSVD_GRAM_AUTO;
  o->queue_depth = 2;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free finishing pass: its scratch (column sums per row tile and
// the scale/sign factors) lives in one file-scope device array instead of the
// context's workspace.  Each device holds its own copy of the array; host
// code reaches it only through the address hipGetSymbolAddress returns for
// that device (kept in g_scratch_ptr), never through the array's name.
// ---------------------------------------------------------------------------
static constexpr int64_t kNoallocScratchDoubles = (int64_t)1 << 20;  // 8 MiB per device
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];
static constexpr int kMaxDevices = 64;
static double* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// called with `device` current (tsvd_ctx_create); once per device
static tsvd_status noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return TSVD_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return TSVD_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return TSVD_ERR_HIP;
  }
  g_scratch_ptr[device] = (double*)p;
  return TSVD_OK;
}

static double* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch_ptr[device];
}

extern "C" {

tsvd_status tsvd_ctx_create(int device, tsvd_ctx** out) {
  if (!out) return TSVD_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
    (void)hipGetLastError();
    return TSVD_ERR_HIP;
  }
  if (device < 0 || device >= count) return TSVD_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return TSVD_ERR_HIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return TSVD_ERR_HIP;
  tsvd_ctx* c = new tsvd_ctx();
  c->device = device;
  c->num_cu = prop.multiProcessorCount;
  c->max_lds = prop.maxSharedMemoryPerMultiProcessor < prop.sharedMemPerBlock ? prop.maxSharedMemoryPerMultiProcessor
                                                                             : prop.sharedMemPerBlock;
  for (int i = 0; i < 4; i++) {
    if (hipEventCreate(&c->ev[i]) != hipSuccess) {
      delete c;
      return TSVD_ERR_HIP;
    }
  }
  if (hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return TSVD_ERR_HIP;
  }
  if (device < kMaxDevices && noalloc_scratch_init(device) != TSVD_OK) {
    tsvd_ctx_destroy(c);
    return TSVD_ERR_HIP;
  }
  *out = c;
  return TSVD_OK;
}

void tsvd_ctx_destroy(tsvd_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  if (ctx->ws) {
    hipDeviceSynchronize();
    hipFree(ctx->ws);
  }
  for (int i = 0; i < 4; i++)
    if (ctx->ev[i]) hipEventDestroy(ctx->ev[i]);
  if (ctx->copy_stream) hipStreamDestroy(ctx->copy_stream);
  delete ctx;
}

tsvd_status tsvd_gram_dense(tsvd_ctx* ctx, const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                            int32_t gram, int32_t side, int64_t rows_per_block, void* B, int64_t ldb,
                            int32_t accumulate, void* stream) {
  if (!ctx) return TSVD_ERR_INVALID_ARG;
  if (!A || !B) return fail(ctx, TSVD_ERR_INVALID_ARG, "null pointer");
  if (m < 1 || n < 1 || lda < n) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad shape m=%lld n=%lld lda=%lld",
                                              (long long)m, (long long)n, (long long)lda);
  if (side != TSVD_SIDE_RIGHT && side != TSVD_SIDE_LEFT) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad side");
  const int64_t d = side == TSVD_SIDE_RIGHT ? n : m;
  const int64_t K = side == TSVD_SIDE_RIGHT ? m : n;
  if (ldb < d) return fail(ctx, TSVD_ERR_INVALID_ARG, "ldb < d");
  if (rows_per_block < 0) return fail(ctx, TSVD_ERR_INVALID_ARG, "rows_per_block < 0");
  const int mode = gram_mode(gram, dtype);
  tsvd_status st = check_mode(ctx, mode, dtype);
  if (st) return st;
  hipSetDevice(ctx->device);
  SyrkPlan sp;
  syrk_plan(mode, d, K, rows_per_block, ctx->num_cu, &sp, ctx->tuning.gram_tile, ctx->tuning.gram_chunks);
  st = ensure_ws(ctx, align256(sp.partial_bytes), 0);
  if (st) return st;
  int rc = syrk_launch(mode, side, A, m, n, lda, sp, ctx->ws, B, ldb, accumulate, (hipStream_t)stream);
  return from_internal(ctx, rc, "tsvd_gram_dense");
}

// shared power-phase driver (workspace carved from `bump`)
static tsvd_status run_power(tsvd_ctx* ctx, Bump& bump, void* B, int is_f64, int64_t d, int64_t ldb, int k,
                             const tsvd_opts* o, double* X, int64_t ldx, const PowerPlan& pp, int* d_status,
                             int* d_iters, double* d_lambda, int* d_fixed, hipStream_t stream) {
  PowerArgs a;
  memset(&a, 0, sizeof a);
  a.B = B;
  a.ldb = ldb;
  a.d = (int)d;
  a.k = k;
  a.eps = o->eps;
  a.max_iter = o->max_iter > 0 ? o->max_iter : 10000;
  a.fixed_iters = o->fixed_iters ? d_fixed : nullptr;
  a.v0 = o->v0;
  a.X = X;
  a.ldx = ldx;
  a.lambda = d_lambda;
  a.iters = d_iters;
  a.status = d_status;
  const size_t words = pp.xex_words + pp.pex_words + pp.vex_words + pp.wex_words;
  uint64_t* ex = (uint64_t*)bump.take(words * 8);
  a.xex = ex;
  a.pex = a.xex + pp.xex_words;
  a.vex = a.pex + pp.pex_words;
  a.wex = a.vex + pp.vex_words;
  a.kscr = (double*)bump.take((size_t)pp.G * 2 * (k + 2) * 8);
  a.vec_ok = (((uintptr_t)B & 15) == 0) && (ldb % (is_f64 ? 2 : 4) == 0);
  a.spin_limit = (int64_t)1 << 21;
  if (o->fixed_iters) {
    if (hipMemcpyAsync(d_fixed, o->fixed_iters, (size_t)k * 4, hipMemcpyHostToDevice, stream) != hipSuccess)
      return fail(ctx, TSVD_ERR_HIP, "copy fixed_iters");
  }
  if (int rc = zero_bytes_launch(d_status, 16, stream)) return from_internal(ctx, rc, "clear status");
  int rc = power_launch(is_f64, pp, a, stream);
  if (rc == -2) return fail(ctx, TSVD_ERR_UNSUPPORTED, "power kernel does not fit on a CU");
  return from_internal(ctx, rc, "power iteration");
}

static size_t power_ws_bytes(const PowerPlan& pp, int k) {
  const size_t words = pp.xex_words + pp.pex_words + pp.vex_words + pp.wex_words;
  return align256(words * 8) + align256((size_t)pp.G * 2 * (k + 2) * 8) + 4 * 256 + align256((size_t)k * 4) +
         align256((size_t)k * 8) + align256((size_t)k * 4) + 1024;
}

tsvd_status tsvd_power_gram(tsvd_ctx* ctx, void* B, int32_t dtype, int64_t d, int64_t ldb, const tsvd_opts* o,
                            double* X, int64_t ldx, tsvd_info* info, void* stream_) {
  if (!ctx) return TSVD_ERR_INVALID_ARG;
  if (!B || !o || !X || !o->v0) return fail(ctx, TSVD_ERR_INVALID_ARG, "null pointer");
  if (d < 1 || ldb < d || ldx < d) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad shape");
  if (dtype != TSVD_F32 && dtype != TSVD_F64) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad dtype");
  int k = o->k == -1 ? (int)d : o->k;
  if (k < 1 || k > d) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad k=%d for d=%lld", o->k, (long long)d);
  if (o->fixed_iters)
    for (int l = 0; l < k; l++)
      if (o->fixed_iters[l] < 1) return fail(ctx, TSVD_ERR_INVALID_ARG, "fixed_iters[%d] < 1", l);
  hipSetDevice(ctx->device);
  hipStream_t stream = (hipStream_t)stream_;
  const int is_f64 = dtype == TSVD_F64;
  PowerPlan pp;
  if (power_plan(is_f64 ? 8 : 4, (int)d, k, ctx->num_cu, ctx->max_lds, ctx->tuning.power_blocks, &pp))
    return fail(ctx, TSVD_ERR_UNSUPPORTED, "d=%lld too large for the LDS-resident iterate", (long long)d);
  tsvd_status st = ensure_ws(ctx, power_ws_bytes(pp, k), o->hbm_budget);
  if (st) return st;
  Bump bump(ctx->ws, ctx->ws_bytes);
  int* d_status = (int*)bump.take(256);
  int* d_iters = (int*)bump.take((size_t)k * 4);
  double* d_lambda = (double*)bump.take((size_t)k * 8);
  int* d_fixed = (int*)bump.take((size_t)k * 4);
  if (int rc = zero_cols_launch(X, ldx, d, k, stream)) return from_internal(ctx, rc, "clear X");
  st = run_power(ctx, bump, B, is_f64, d, ldb, k, o, X, ldx, pp, d_status, d_iters, d_lambda, d_fixed, stream);
  if (st) return st;
  int hs[4];
  std::vector<int> hit(k);
  std::vector<double> hl(k);
  if (hipMemcpyAsync(hs, d_status, 16, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipMemcpyAsync(hit.data(), d_iters, (size_t)k * 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipMemcpyAsync(hl.data(), d_lambda, (size_t)k * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return fail(ctx, TSVD_ERR_HIP, "power status readback: %s", hipGetErrorString(hipGetLastError()));
  if (info) {
    info->k_done = hs[0];
    info->converged = hs[1];
    info->rank_deficient = hs[3];
    info->branch_right = 1;
    info->latency_ms = 0;
    if (info->iters) memcpy(info->iters, hit.data(), (size_t)k * 4);
    if (info->lambda) memcpy(info->lambda, hl.data(), (size_t)k * 8);
  }
  if (hs[2] == 1) return fail(ctx, TSVD_ERR_INTERNAL, "power iteration: a bounded wait timed out");
  if (hs[2] == 2) return fail(ctx, TSVD_ERR_NONFINITE, "non-finite value in the power iteration");
  if (hs[2] == 3) return fail(ctx, TSVD_ERR_INVALID_ARG, "a start vector is zero");
  if (!hs[1] && !o->fixed_iters && o->eps > 0)
    return fail(ctx, TSVD_ERR_NOT_CONVERGED, "some triplet reached max_iter");
  return TSVD_OK;
}

tsvd_status tsvd_finish_dense(tsvd_ctx* ctx, const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                              int32_t side, const double* X, int64_t ldx, int32_t k, double* W, int64_t ldw,
                              double* S, void* stream) {
  if (!ctx) return TSVD_ERR_INVALID_ARG;
  if (!A || !X || !W || !S) return fail(ctx, TSVD_ERR_INVALID_ARG, "null pointer");
  if (m < 1 || n < 1 || lda < n) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad shape");
  if (dtype != TSVD_F32 && dtype != TSVD_F64) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad dtype");
  const int64_t K = side == TSVD_SIDE_RIGHT ? n : m, M = side == TSVD_SIDE_RIGHT ? m : n;
  if (k < 1 || k > (m < n ? m : n) || ldx < K || ldw < M) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad k/ld");
  hipSetDevice(ctx->device);
  const size_t need = align256((size_t)finish_workspace_doubles(m, n, side, k) * 8);
  tsvd_status st = ensure_ws(ctx, need, 0);
  if (st) return st;
  int rc = finish_launch(dtype == TSVD_F64, side, A, m, n, lda, X, ldx, k, W, ldw, S, (double*)ctx->ws,
                         (hipStream_t)stream);
  if (rc) return from_internal(ctx, rc, "finish");
  rc = finish_scale_sign_launch(W, ldw, M, S, nullptr, 0, 0, nullptr, 0, 0, k, 0,
                                (double*)ctx->ws + finish_tiles(m, n, side) * k, (hipStream_t)stream);
  return from_internal(ctx, rc, "finish scale");
}

tsvd_status tsvd_finish_dense_noalloc(tsvd_ctx* ctx, const void* A, int32_t dtype, int64_t m, int64_t n, int64_t lda,
                                      int32_t side, const double* X, int64_t ldx, int32_t k, double* W, int64_t ldw,
                                      double* S, void* stream) {
  if (!ctx) return TSVD_ERR_INVALID_ARG;
  if (!A || !X || !W || !S) return fail(ctx, TSVD_ERR_INVALID_ARG, "null pointer");
  if (m < 1 || n < 1 || lda < n) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad shape");
  if (dtype != TSVD_F32 && dtype != TSVD_F64) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad dtype");
  if (side != TSVD_SIDE_RIGHT && side != TSVD_SIDE_LEFT) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad side");
  const int64_t K = side == TSVD_SIDE_RIGHT ? n : m, M = side == TSVD_SIDE_RIGHT ? m : n;
  if (k < 1 || k > (m < n ? m : n) || ldx < K || ldw < M) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad k/ld");
  const int64_t need = finish_workspace_doubles(m, n, side, k);
  if (need > kNoallocScratchDoubles)
    return fail(ctx, TSVD_ERR_UNSUPPORTED,
                "allocation-free finish needs %lld doubles of scratch ((ceil(%lld / 128) + 2) x k); its device array "
                "holds %lld",
                (long long)need, (long long)M, (long long)kNoallocScratchDoubles);
  double* ws = noalloc_scratch(ctx->device);
  if (!ws) return fail(ctx, TSVD_ERR_HIP, "allocation-free scratch has no address on device %d", ctx->device);
  hipSetDevice(ctx->device);
  int rc = finish_launch(dtype == TSVD_F64, side, A, m, n, lda, X, ldx, k, W, ldw, S, ws, (hipStream_t)stream);
  if (rc) return from_internal(ctx, rc, "finish (allocation-free)");
  rc = finish_scale_sign_launch(W, ldw, M, S, nullptr, 0, 0, nullptr, 0, 0, k, 0, ws + finish_tiles(m, n, side) * k,
                                (hipStream_t)stream);
  return from_internal(ctx, rc, "finish scale (allocation-free)");
}

// Dense t-SVD of an FP32 A held in pinned host memory (Algorithm 3's
// out-of-memory batching).  Rows are streamed in batches through
// `queue_depth` device buffers: the copy stream fills buffer b % Q while the
// compute stream runs the Gram (pass 1) or the FP64 finishing product (pass 2)
// on the previous batch; events order reuse.  The power iteration runs on the
// device-resident Gram between the passes, overlapped with the first copies of
// pass 2.
static tsvd_status dense_pinned(tsvd_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda, const tsvd_opts* o,
                                int k, int mode, double* U, int64_t ldu, double* S, double* V, int64_t ldv,
                                tsvd_info* info, hipStream_t s) {
  if (!right_side(m, n, o->branch))
    return fail(ctx, TSVD_ERR_UNSUPPORTED, "pinned-host input needs the A^T A branch (m >= n)");
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, A) != hipSuccess || attr.type != hipMemoryTypeHost) {
    (void)hipGetLastError();
    return fail(ctx, TSVD_ERR_INVALID_ARG, "A is not pinned host memory (allocate it with hipHostMalloc / pin_memory)");
  }
  const int Q = o->queue_depth >= 2 ? o->queue_depth : 2;
  if (Q > 16) return fail(ctx, TSVD_ERR_INVALID_ARG, "queue_depth > 16");
  const int64_t d = n;
  const int64_t ldb = (d + 3) & ~3;
  const bool explicit_rows = o->rows_per_block > 0;
  // batch rows: rows_per_block rounded up to a multiple of 128 (the finishing
  // pass's row tile), or 4 GiB worth of rows rounded down to one
  int64_t R = explicit_rows ? ((o->rows_per_block + 127) / 128) * 128 : (((int64_t)4 << 30) / (n * 4)) / 128 * 128;
  if (R < 128) R = 128;
  if (R > m) R = m;
  const int64_t nbatch = (m + R - 1) / R;
  // Gram plan per batch (one chunk per batch when the batch size is given, so
  // the result is bitwise that of the in-HBM path with the same rows_per_block)
  SyrkPlan sp_full, sp_last;
  const int64_t last_rows = m - (nbatch - 1) * R;
  syrk_plan(mode, d, R, explicit_rows ? R : 0, ctx->num_cu, &sp_full, ctx->tuning.gram_tile, ctx->tuning.gram_chunks);
  syrk_plan(mode, d, last_rows, explicit_rows ? last_rows : 0, ctx->num_cu, &sp_last, ctx->tuning.gram_tile,
            ctx->tuning.gram_chunks);
  const size_t part_bytes = sp_full.partial_bytes > sp_last.partial_bytes ? sp_full.partial_bytes : sp_last.partial_bytes;
  PowerPlan pp;
  if (power_plan(4, (int)d, k, ctx->num_cu, ctx->max_lds, ctx->tuning.power_blocks, &pp))
    return fail(ctx, TSVD_ERR_UNSUPPORTED, "n=%lld too large for the LDS-resident iterate", (long long)d);
  const int64_t tiles_total = (m + 127) / 128 + nbatch;  // finish row tiles, one partial tile per batch at most
  const size_t buf_bytes = align256((size_t)R * n * 4);
  const size_t b_bytes = align256((size_t)d * ldb * 4);
  const size_t ssq_bytes = align256((size_t)(tiles_total + 2) * k * 8);
  const size_t need = (size_t)Q * buf_bytes + b_bytes + align256(part_bytes) + power_ws_bytes(pp, k) + ssq_bytes + 4096;
  tsvd_status st = ensure_ws(ctx, need, o->hbm_budget);
  if (st) return st;
  Bump bump(ctx->ws, ctx->ws_bytes);
  float* buf[16];
  for (int q = 0; q < Q; q++) buf[q] = (float*)bump.take(buf_bytes);
  void* B = bump.take(b_bytes);
  void* partial = bump.take(part_bytes);
  double* ssq = (double*)bump.take(ssq_bytes);
  int* d_status = (int*)bump.take(256);
  int* d_iters = (int*)bump.take((size_t)k * 4);
  double* d_lambda = (double*)bump.take((size_t)k * 8);
  int* d_fixed = (int*)bump.take((size_t)k * 4);

  hipEvent_t copied[16], consumed[16];
  int made = 0;
  auto cleanup = [&]() {
    for (int i = 0; i < made; i++) { hipEventDestroy(copied[i]); hipEventDestroy(consumed[i]); }
  };
  for (; made < Q; made++) {
    if (hipEventCreateWithFlags(&copied[made], hipEventDisableTiming) != hipSuccess) { cleanup(); return fail(ctx, TSVD_ERR_HIP, "event"); }
    if (hipEventCreateWithFlags(&consumed[made], hipEventDisableTiming) != hipSuccess) {
      hipEventDestroy(copied[made]);
      cleanup();
      return fail(ctx, TSVD_ERR_HIP, "event");
    }
  }
  hipStream_t cs = ctx->copy_stream;
  int rc = 0;
  auto copy_batch = [&](int64_t b, int slot, bool wait_slot) -> int {
    const int64_t r0 = b * R;
    const int64_t rows = (b == nbatch - 1) ? last_rows : R;
    if (wait_slot && hipStreamWaitEvent(cs, consumed[slot], 0) != hipSuccess) return TSVD_ERR_HIP;
    if (hipMemcpy2DAsync(buf[slot], (size_t)n * 4, A + r0 * lda, (size_t)lda * 4, (size_t)n * 4, (size_t)rows,
                         hipMemcpyHostToDevice, cs) != hipSuccess)
      return TSVD_ERR_HIP;
    if (hipEventRecord(copied[slot], cs) != hipSuccess) return TSVD_ERR_HIP;
    return 0;
  };

  hipEventRecord(ctx->ev[0], s);
  if (hipStreamWaitEvent(cs, ctx->ev[0], 0) != hipSuccess) { cleanup(); return fail(ctx, TSVD_ERR_HIP, "wait"); }
  if (zero_cols_launch(U, ldu, m, k, s) || zero_cols_launch(V, ldv, n, k, s) || zero_cols_launch(S, k, k, 1, s)) {
    cleanup();
    return fail(ctx, TSVD_ERR_HIP, "clear outputs");
  }
  // ---- pass 1: B = sum_b A_b^T A_b
  for (int64_t b = 0; b < nbatch && !rc; b++) {
    const int slot = (int)(b % Q);
    if ((rc = copy_batch(b, slot, b >= Q))) break;
    if (hipStreamWaitEvent(s, copied[slot], 0) != hipSuccess) { rc = TSVD_ERR_HIP; break; }
    const int64_t rows = (b == nbatch - 1) ? last_rows : R;
    const SyrkPlan& sp = (b == nbatch - 1) ? sp_last : sp_full;
    if ((rc = syrk_launch(mode, 0, buf[slot], rows, n, n, sp, partial, B, ldb, b > 0 ? 1 : 0, s))) break;
    if (hipEventRecord(consumed[slot], s) != hipSuccess) { rc = TSVD_ERR_HIP; break; }
  }
  if (rc) { cleanup(); return from_internal(ctx, rc, "pinned Gram pass"); }
  hipEventRecord(ctx->ev[1], s);
  // ---- prefetch the first batches of pass 2 while the power iteration runs
  const int64_t pre = nbatch < Q ? nbatch : Q;
  for (int64_t b = 0; b < pre && !rc; b++) rc = copy_batch(b, (int)(b % Q), true);
  if (rc) { cleanup(); return from_internal(ctx, rc, "prefetch"); }
  st = run_power(ctx, bump, B, 0, d, ldb, k, o, V, ldv, pp, d_status, d_iters, d_lambda, d_fixed, s);
  if (st) { cleanup(); return st; }
  hipEventRecord(ctx->ev[2], s);
  int hs[4];
  if (hipMemcpyAsync(hs, d_status, 16, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    cleanup();
    return fail(ctx, TSVD_ERR_HIP, "status readback: %s", hipGetErrorString(hipGetLastError()));
  }
  if (hs[2] != 0) {
    hipStreamSynchronize(cs);
    cleanup();
    if (hs[2] == 1) return fail(ctx, TSVD_ERR_INTERNAL, "power iteration: a bounded wait timed out");
    if (hs[2] == 2) return fail(ctx, TSVD_ERR_NONFINITE, "non-finite value in the Gram or the power iteration");
    return fail(ctx, TSVD_ERR_INVALID_ARG, "a start vector is zero");
  }
  const int kd = hs[0];
  // ---- pass 2: U = A V (FP64), column sums of squares per row tile
  int64_t tile_off = 0;
  for (int64_t b = 0; b < nbatch && !rc && kd > 0; b++) {
    const int slot = (int)(b % Q);
    if (b >= pre && (rc = copy_batch(b, slot, true))) break;
    if (hipStreamWaitEvent(s, copied[slot], 0) != hipSuccess) { rc = TSVD_ERR_HIP; break; }
    const int64_t r0 = b * R;
    const int64_t rows = (b == nbatch - 1) ? last_rows : R;
    if ((rc = finish_gemm_launch(0, 0, buf[slot], rows, n, n, V, ldv, kd, U + r0, ldu, ssq + tile_off * kd, s))) break;
    tile_off += (rows + 127) / 128;
    if (hipEventRecord(consumed[slot], s) != hipSuccess) { rc = TSVD_ERR_HIP; break; }
  }
  if (!rc && kd > 0) rc = finish_sigma_launch(ssq, tile_off, kd, S, s);
  if (!rc && kd > 0) rc = finish_scale_sign_launch(U, ldu, m, S, V, ldv, n, U, ldu, m, kd, 1, ssq + tiles_total * k, s);
  hipEventRecord(ctx->ev[3], s);
  if (!rc && (hipStreamSynchronize(s) != hipSuccess || hipStreamSynchronize(cs) != hipSuccess)) rc = TSVD_ERR_HIP;
  cleanup();
  if (rc) return from_internal(ctx, rc, "pinned finish pass");
  std::vector<int> hit(k);
  std::vector<double> hl(k);
  if (hipMemcpy(hit.data(), d_iters, (size_t)k * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(hl.data(), d_lambda, (size_t)k * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(ctx, TSVD_ERR_HIP, "readback");
  if (info) {
    info->k_done = kd;
    info->converged = hs[1];
    info->rank_deficient = hs[3];
    info->branch_right = 1;
    if (info->iters) memcpy(info->iters, hit.data(), (size_t)k * 4);
    if (info->lambda) memcpy(info->lambda, hl.data(), (size_t)k * 8);
    float t;
    hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1]); info->t_gram_ms = t;
    hipEventElapsedTime(&t, ctx->ev[1], ctx->ev[2]); info->t_eig_ms = t;
    hipEventElapsedTime(&t, ctx->ev[2], ctx->ev[3]); info->t_final_ms = t;
    hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[3]); info->t_total_ms = t;
    info->workspace_bytes = (int64_t)need;
    info->h2d_bytes = (int64_t)(m * n * 4) * (kd > 0 ? 2 : 1);
    info->latency_ms = 0;
  }
  if (!hs[1] && !o->fixed_iters && o->eps > 0)
    return fail(ctx, TSVD_ERR_NOT_CONVERGED, "some triplet reached max_iter");
  return TSVD_OK;
}

tsvd_status tsvd_dense(tsvd_ctx* ctx, const void* A, int32_t dtype, int32_t loc, int64_t m, int64_t n, int64_t lda,
                       const tsvd_opts* o, double* U, int64_t ldu, double* S, double* V, int64_t ldv,
                       tsvd_info* info, void* stream_) {
  if (!ctx) return TSVD_ERR_INVALID_ARG;
  if (!A || !o || !U || !S || !V || !o->v0) return fail(ctx, TSVD_ERR_INVALID_ARG, "null pointer");
  if (m < 1 || n < 1 || lda < n) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad shape m=%lld n=%lld lda=%lld",
                                              (long long)m, (long long)n, (long long)lda);
  if (ldu < m || ldv < n) return fail(ctx, TSVD_ERR_INVALID_ARG, "ldu < m or ldv < n");
  const int64_t mn = m < n ? m : n;
  const int k = o->k == -1 ? (int)mn : o->k;
  if (k < 1 || k > mn) return fail(ctx, TSVD_ERR_INVALID_ARG, "k=%d outside [1, min(m, n)=%lld]", o->k, (long long)mn);
  if (o->branch != 0 && o->branch != 1) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad branch");
  if (o->rows_per_block < 0) return fail(ctx, TSVD_ERR_INVALID_ARG, "rows_per_block < 0");
  if (o->fixed_iters)
    for (int l = 0; l < k; l++)
      if (o->fixed_iters[l] < 1) return fail(ctx, TSVD_ERR_INVALID_ARG, "fixed_iters[%d] < 1", l);
  if (loc != TSVD_LOC_DEVICE && loc != TSVD_LOC_PINNED_HOST) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad loc");
  const int mode = gram_mode(o->gram, dtype);
  tsvd_status st = check_mode(ctx, mode, dtype);
  if (st) return st;
  if (loc == TSVD_LOC_PINNED_HOST)
    return dense_pinned(ctx, (const float*)A, m, n, lda, o, k, mode, U, ldu, S, V, ldv, info, (hipStream_t)stream_);
  hipSetDevice(ctx->device);
  hipStream_t stream = (hipStream_t)stream_;

  const bool right = right_side(m, n, o->branch);
  const int side = right ? TSVD_SIDE_RIGHT : TSVD_SIDE_LEFT;
  const int64_t d = right ? n : m;
  const int64_t K = right ? m : n;
  const int is_f64 = mode == MODE_FP64;
  const int eb = is_f64 ? 8 : 4;
  const int64_t ldb = (d + 3) & ~3;

  SyrkPlan sp;
  syrk_plan(mode, d, K, o->rows_per_block, ctx->num_cu, &sp, ctx->tuning.gram_tile, ctx->tuning.gram_chunks);
  PowerPlan pp;
  if (power_plan(eb, (int)d, k, ctx->num_cu, ctx->max_lds, ctx->tuning.power_blocks, &pp))
    return fail(ctx, TSVD_ERR_UNSUPPORTED, "d=%lld too large for the LDS-resident iterate", (long long)d);
  const size_t b_bytes = align256((size_t)d * ldb * eb);
  const size_t fin_bytes = align256((size_t)finish_workspace_doubles(m, n, side, k) * 8);
  const size_t need = b_bytes + align256(sp.partial_bytes) + power_ws_bytes(pp, k) + fin_bytes + 4096;
  st = ensure_ws(ctx, need, o->hbm_budget);
  if (st) return st;
  Bump bump(ctx->ws, ctx->ws_bytes);
  void* B = bump.take(b_bytes);
  void* partial = bump.take(sp.partial_bytes);
  double* ssq = (double*)bump.take(fin_bytes);
  int* d_status = (int*)bump.take(256);
  int* d_iters = (int*)bump.take((size_t)k * 4);
  double* d_lambda = (double*)bump.take((size_t)k * 8);
  int* d_fixed = (int*)bump.take((size_t)k * 4);

  double* X = right ? V : U;
  const int64_t ldx = right ? ldv : ldu;
  double* W = right ? U : V;
  const int64_t ldw = right ? ldu : ldv;
  const int64_t Mw = right ? m : n;

  if (hipEventRecord(ctx->ev[0], stream) != hipSuccess) return fail(ctx, TSVD_ERR_HIP, "event");
  if (zero_cols_launch(U, ldu, m, k, stream) || zero_cols_launch(V, ldv, n, k, stream) ||
      zero_cols_launch(S, k, k, 1, stream))
    return fail(ctx, TSVD_ERR_HIP, "clear outputs");
  int rc = syrk_launch(mode, side, A, m, n, lda, sp, partial, B, ldb, 0, stream);
  if (rc) return from_internal(ctx, rc, "gram");
  hipEventRecord(ctx->ev[1], stream);
  st = run_power(ctx, bump, B, is_f64, d, ldb, k, o, X, ldx, pp, d_status, d_iters, d_lambda, d_fixed, stream);
  if (st) return st;
  hipEventRecord(ctx->ev[2], stream);
  int hs[4];
  if (hipMemcpyAsync(hs, d_status, 16, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return fail(ctx, TSVD_ERR_HIP, "status readback: %s", hipGetErrorString(hipGetLastError()));
  if (hs[2] == 1) return fail(ctx, TSVD_ERR_INTERNAL, "power iteration: a bounded wait timed out");
  if (hs[2] == 2) return fail(ctx, TSVD_ERR_NONFINITE, "non-finite value in the Gram or the power iteration");
  if (hs[2] == 3) return fail(ctx, TSVD_ERR_INVALID_ARG, "a start vector is zero");
  const int kd = hs[0];
  if (kd > 0) {
    rc = finish_launch(is_f64, side, A, m, n, lda, X, ldx, kd, W, ldw, S, ssq, stream);
    if (rc) return from_internal(ctx, rc, "finish");
    rc = finish_scale_sign_launch(W, ldw, Mw, S, V, ldv, n, U, ldu, m, kd, 1, ssq + finish_tiles(m, n, side) * k,
                                  stream);
    if (rc) return from_internal(ctx, rc, "finish scale/sign");
  }
  hipEventRecord(ctx->ev[3], stream);
  std::vector<int> hit(k);
  std::vector<double> hl(k);
  if (hipMemcpyAsync(hit.data(), d_iters, (size_t)k * 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipMemcpyAsync(hl.data(), d_lambda, (size_t)k * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return fail(ctx, TSVD_ERR_HIP, "readback: %s", hipGetErrorString(hipGetLastError()));
  if (info) {
    info->k_done = kd;
    info->converged = hs[1];
    info->rank_deficient = hs[3];
    info->branch_right = right ? 1 : 0;
    if (info->iters) memcpy(info->iters, hit.data(), (size_t)k * 4);
    if (info->lambda) memcpy(info->lambda, hl.data(), (size_t)k * 8);
    float t;
    hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1]); info->t_gram_ms = t;
    hipEventElapsedTime(&t, ctx->ev[1], ctx->ev[2]); info->t_eig_ms = t;
    hipEventElapsedTime(&t, ctx->ev[2], ctx->ev[3]); info->t_final_ms = t;
    hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[3]); info->t_total_ms = t;
    info->workspace_bytes = (int64_t)need;
    info->h2d_bytes = 0;
    info->latency_ms = 0;
  }
  if (!hs[1] && !o->fixed_iters && o->eps > 0)
    return fail(ctx, TSVD_ERR_NOT_CONVERGED, "some triplet reached max_iter");
  return TSVD_OK;
}

// ---------------------------------------------------------------------------
// sparse path
// ---------------------------------------------------------------------------
}  // extern "C"

struct tsvd_csr {
  int device = 0;
  int64_t m = 0, n = 0, nnz = 0;
  const int64_t* rowptr = nullptr;
  const int32_t* col = nullptr;
  const float* val = nullptr;
  int64_t* colptr = nullptr;  // owned CSC copy
  int32_t* rowidx = nullptr;
  float* cval = nullptr;
  // owned sliced tiles of A (from the CSR) and of A^T (from the CSC): dir 0 / 1
  tsvd::TilePlan tp[2] = {};
  int64_t* tptr[2] = {nullptr, nullptr};
  uint32_t* tkey[2] = {nullptr, nullptr};
  float* tval[2] = {nullptr, nullptr};
};

namespace {
// y = A x (dir 0) or A^T x (dir 1) through the sliced tiles
int csr_product(const tsvd_csr* c, int dir, const void* x, int x_is_f64, double* y, float* yf, hipStream_t s) {
  return spmv_tiles_launch(c->tp[dir], c->tptr[dir], c->tkey[dir], c->tval[dir], dir == 0 ? c->m : c->n, x, x_is_f64,
                           y, yf, s);
}
}  // namespace

extern "C" {

tsvd_status tsvd_csr_create(tsvd_ctx* ctx, int64_t m, int64_t n, int64_t nnz, const int64_t* rowptr,
                            const int32_t* col, const float* val, tsvd_csr** out, void* stream_) {
  if (!ctx) return TSVD_ERR_INVALID_ARG;
  if (!out) return fail(ctx, TSVD_ERR_INVALID_ARG, "null out");
  *out = nullptr;
  if (m < 1 || n < 1 || nnz < 0) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad shape m=%lld n=%lld nnz=%lld",
                                              (long long)m, (long long)n, (long long)nnz);
  if (n > 0x7fffffffLL || m > 0x7fffffffLL) return fail(ctx, TSVD_ERR_UNSUPPORTED, "int32 indices need m, n < 2^31");
  if (!rowptr || (nnz > 0 && (!col || !val))) return fail(ctx, TSVD_ERR_INVALID_ARG, "null pointer");
  hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream_;
  int* d_bad = nullptr;
  if (hipMalloc(&d_bad, 256) != hipSuccess) return fail(ctx, TSVD_ERR_OUT_OF_MEMORY, "hipMalloc");
  int rc = csr_validate(rowptr, col, m, n, nnz, d_bad, s);
  int hbad = 0;
  if (rc == 0 && (hipMemcpyAsync(&hbad, d_bad, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                  hipStreamSynchronize(s) != hipSuccess))
    rc = TSVD_ERR_HIP;
  hipFree(d_bad);
  if (rc) return from_internal(ctx, rc, "csr validation");
  if (hbad) return fail(ctx, TSVD_ERR_INVALID_ARG, "CSR structure invalid (flags %d: 1 row pointers, 2 ends, 4 columns)",
                        hbad);
  tsvd_csr* c = new tsvd_csr();
  c->device = ctx->device;
  c->m = m; c->n = n; c->nnz = nnz;
  c->rowptr = rowptr; c->col = col; c->val = val;
  void* scratch = nullptr;
  if (hipMalloc(&c->colptr, (size_t)(n + 1) * 8) != hipSuccess ||
      hipMalloc(&c->rowidx, (size_t)(nnz > 0 ? nnz : 1) * 4) != hipSuccess ||
      hipMalloc(&c->cval, (size_t)(nnz > 0 ? nnz : 1) * 4) != hipSuccess ||
      hipMalloc(&scratch, csc_build_scratch_bytes(n)) != hipSuccess) {
    (void)hipGetLastError();
    hipFree(scratch);
    tsvd_csr_destroy(c);
    return fail(ctx, TSVD_ERR_OUT_OF_MEMORY, "allocating the CSC copy (%lld nonzeros)", (long long)nnz);
  }
  rc = csc_build(rowptr, col, val, m, n, nnz, c->colptr, c->rowidx, c->cval, scratch, s);
  if (rc == 0 && hipStreamSynchronize(s) != hipSuccess) rc = TSVD_ERR_HIP;
  hipFree(scratch);
  if (rc) {
    tsvd_csr_destroy(c);
    return from_internal(ctx, rc, "CSC build");
  }
  // sliced tiles for both products: A from the CSR, A^T from the CSC
  for (int dir = 0; dir < 2; dir++) {
    const int64_t rows = dir == 0 ? m : n, cols = dir == 0 ? n : m;
    if (tiles_plan(rows, cols, ctx->num_cu, ctx->tuning.sparse_row_bits, ctx->tuning.sparse_col_bits, &c->tp[dir])) {
      tsvd_csr_destroy(c);
      return fail(ctx, TSVD_ERR_INVALID_ARG, "sparse tile bits out of range");
    }
    const int64_t nt = c->tp[dir].nchunks * c->tp[dir].nslices;
    void* tscr = nullptr;
    if (hipMalloc(&c->tptr[dir], (size_t)(nt + 1) * 8) != hipSuccess ||
        hipMalloc(&c->tkey[dir], (size_t)(nnz > 0 ? nnz : 1) * 4) != hipSuccess ||
        hipMalloc(&c->tval[dir], (size_t)(nnz > 0 ? nnz : 1) * 4) != hipSuccess ||
        hipMalloc(&tscr, tiles_scratch_bytes(c->tp[dir])) != hipSuccess) {
      (void)hipGetLastError();
      hipFree(tscr);
      tsvd_csr_destroy(c);
      return fail(ctx, TSVD_ERR_OUT_OF_MEMORY, "allocating the sparse tiles (%lld nonzeros)", (long long)nnz);
    }
    rc = dir == 0 ? tiles_build(rowptr, col, val, m, nnz, c->tp[0], c->tptr[0], c->tkey[0], c->tval[0], tscr, s)
                  : tiles_build(c->colptr, c->rowidx, c->cval, n, nnz, c->tp[1], c->tptr[1], c->tkey[1], c->tval[1],
                                tscr, s);
    if (rc == 0 && hipStreamSynchronize(s) != hipSuccess) rc = TSVD_ERR_HIP;
    hipFree(tscr);
    if (rc) {
      tsvd_csr_destroy(c);
      return from_internal(ctx, rc, "tile build");
    }
  }
  *out = c;
  return TSVD_OK;
}

void tsvd_csr_destroy(tsvd_csr* c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  hipFree(c->colptr);
  for (int dir = 0; dir < 2; dir++) {
    hipFree(c->tptr[dir]);
    hipFree(c->tkey[dir]);
    hipFree(c->tval[dir]);
  }
  hipFree(c->rowidx);
  hipFree(c->cval);
  delete c;
}

tsvd_status tsvd_csr_get_csc(tsvd_ctx* ctx, const tsvd_csr* c, int64_t* colptr, int32_t* rowidx, float* val,
                             void* stream) {
  if (!ctx) return TSVD_ERR_INVALID_ARG;
  if (!c || !colptr || (c->nnz > 0 && (!rowidx || !val))) return fail(ctx, TSVD_ERR_INVALID_ARG, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(colptr, c->colptr, (size_t)(c->n + 1) * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      (c->nnz > 0 && (hipMemcpyAsync(rowidx, c->rowidx, (size_t)c->nnz * 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                      hipMemcpyAsync(val, c->cval, (size_t)c->nnz * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)))
    return fail(ctx, TSVD_ERR_HIP, "copy CSC");
  return TSVD_OK;
}

tsvd_status tsvd_spmv(tsvd_ctx* ctx, const tsvd_csr* c, int32_t trans, const void* x, int32_t x_dtype, double* y,
                      void* stream) {
  if (!ctx) return TSVD_ERR_INVALID_ARG;
  if (!c || !x || !y) return fail(ctx, TSVD_ERR_INVALID_ARG, "null pointer");
  if (trans != 0 && trans != 1) return fail(ctx, TSVD_ERR_INVALID_ARG, "trans must be 0 or 1");
  if (x_dtype != TSVD_F32 && x_dtype != TSVD_F64) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad x dtype");
  hipSetDevice(ctx->device);
  int rc = csr_product(c, trans, x, x_dtype == TSVD_F64, y, nullptr, (hipStream_t)stream);
  return from_internal(ctx, rc, "spmv");
}

tsvd_status tsvd_sparse(tsvd_ctx* ctx, const tsvd_csr* c, const tsvd_opts* o, double* U, int64_t ldu, double* S,
                        double* V, int64_t ldv, tsvd_info* info, void* stream_) {
  if (!ctx) return TSVD_ERR_INVALID_ARG;
  if (!c || !o || !U || !S || !V || !o->v0) return fail(ctx, TSVD_ERR_INVALID_ARG, "null pointer");
  const int64_t m = c->m, n = c->n;
  if (ldu < m || ldv < n) return fail(ctx, TSVD_ERR_INVALID_ARG, "ldu < m or ldv < n");
  const int64_t mn = m < n ? m : n;
  const int k = o->k == -1 ? (int)mn : o->k;
  if (k < 1 || k > mn) return fail(ctx, TSVD_ERR_INVALID_ARG, "k=%d outside [1, min(m, n)=%lld]", o->k, (long long)mn);
  if (o->branch != 0 && o->branch != 1) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad branch");
  if (o->fixed_iters)
    for (int l = 0; l < k; l++)
      if (o->fixed_iters[l] < 1) return fail(ctx, TSVD_ERR_INVALID_ARG, "fixed_iters[%d] < 1", l);
  hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream_;
  const bool right = right_side(m, n, o->branch);
  const int64_t d = right ? n : m, e = right ? m : n;
  double* X = right ? V : U;
  const int64_t ldx = right ? ldv : ldu;
  double* W = right ? U : V;
  const int64_t ldw = right ? ldu : ldv;
  const int max_iter = o->max_iter > 0 ? o->max_iter : 10000;

  const int64_t nb = proj_blocks(d > e ? d : e);
  const size_t need = align256((size_t)d * 8) * 2 + align256((size_t)d * 4) + align256((size_t)e * 4) +
                      align256((size_t)nb * (k + 2) * 8) + align256((size_t)(k + 8) * 8) * 2 + 4096;
  tsvd_status st = ensure_ws(ctx, need, o->hbm_budget);
  if (st) return st;
  Bump bump(ctx->ws, ctx->ws_bytes);
  double* x = (double*)bump.take((size_t)d * 8);    // current unit iterate (FP64)
  double* w = (double*)bump.take((size_t)d * 8);    // product, projected in place
  float* xf = (float*)bump.take((size_t)d * 4);     // FP32 copy gathered by the first product
  float* tf = (float*)bump.take((size_t)e * 4);     // intermediate A x (or A^T x) in FP32
  double* partial = (double*)bump.take((size_t)std::max<int64_t>(nb * (k + 2), 2 * (int64_t)k) * 8);
  double* coef = (double*)bump.take((size_t)(k + 8) * 8);
  double* scal = (double*)bump.take((size_t)(k + 8) * 8);

  // right branch: t = A x, w = A^T t; left branch: t = A^T x, w = A t
  const int dir1 = right ? 0 : 1, dir2 = right ? 1 : 0;

  hipEventRecord(ctx->ev[0], s);
  if (zero_cols_launch(U, ldu, m, k, s) || zero_cols_launch(V, ldv, n, k, s) || zero_cols_launch(S, k, k, 1, s))
    return fail(ctx, TSVD_ERR_HIP, "clear outputs");
  hipEventRecord(ctx->ev[1], s);
  std::vector<int> iters(k, 0);
  std::vector<double> lams(k, 0.0);
  bool all_conv = true, rankdef = false;
  int kdone = k;
  int rc = 0;
  for (int l = 0; l < k && !rc && !rankdef; l++) {
    // start vector: x = v0_l / ||v0_l||, then x <- x - X (X^T x) (projected once, not renormalised)
    const double* v0 = o->v0 + (int64_t)l * d;
    if ((rc = sumsq_launch(v0, d, partial, scal, s))) break;
    if ((rc = start_scale_launch(v0, d, scal, x, s))) break;
    if (l > 0) {
      if ((rc = proj_partials_launch(X, ldx, l, x, x, d, partial, coef, s))) break;
      if ((rc = proj_apply_launch(X, ldx, l, coef, x, d, partial, scal + 1, s))) break;
    }
    if ((rc = to_float_launch(x, d, xf, s))) break;
    const int fixed = o->fixed_iters ? o->fixed_iters[l] : (o->eps <= 0.0 ? max_iter : 0);
    int it = 0;
    double nrm = 0.0;
    bool conv = false;
    while (true) {
      if ((rc = csr_product(c, dir1, xf, 0, nullptr, tf, s))) break;
      if ((rc = csr_product(c, dir2, tf, 0, w, nullptr, s))) break;
      it++;
      if ((rc = proj_partials_launch(X, ldx, l, w, x, d, partial, coef, s))) break;
      if ((rc = proj_apply_launch(X, ldx, l, coef, w, d, partial, scal, s))) break;
      double h[2];
      if (hipMemcpyAsync(&h[0], scal, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipMemcpyAsync(&h[1], coef + l + 1, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        rc = TSVD_ERR_HIP;
        break;
      }
      nrm = sqrt(h[0]);
      if (!std::isfinite(nrm)) return fail(ctx, TSVD_ERR_NONFINITE, "non-finite value in the sparse product");
      if (nrm == 0.0) { rankdef = true; kdone = l; break; }
      bool stop;
      if (fixed > 0) { stop = it >= fixed; conv = true; }
      else {
        conv = fabs(h[1]) / nrm >= 1.0 - o->eps;
        stop = conv || it >= max_iter;
      }
      if ((rc = normalize_launch(w, d, 1.0 / nrm, x, xf, s))) break;
      if (stop) break;
    }
    if (rc || rankdef) break;
    if (!conv) all_conv = false;
    iters[l] = it;
    lams[l] = nrm;
    // FP64 re-orthogonalisation against the earlier columns, then store column l
    if (l > 0) {
      if ((rc = proj_partials_launch(X, ldx, l, x, x, d, partial, coef, s))) break;
      if ((rc = proj_apply_launch(X, ldx, l, coef, x, d, partial, scal, s))) break;
    } else if ((rc = sumsq_launch(x, d, partial, scal, s))) break;
    double hn;
    if (hipMemcpyAsync(&hn, scal, 8, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
      rc = TSVD_ERR_HIP;
      break;
    }
    if (!(hn > 0.0)) { rankdef = true; kdone = l; break; }
    if ((rc = normalize_launch(x, d, 1.0 / sqrt(hn), X + (int64_t)l * ldx, nullptr, s))) break;
  }
  if (rc) return from_internal(ctx, rc, "sparse power iteration");
  hipEventRecord(ctx->ev[2], s);
  // finish: W[:, j] = A X[:, j] (right) or A^T X[:, j] (left) with FP64 input,
  // sigma_j = ||W[:, j]||, then scale and sign convention
  for (int j = 0; j < kdone && !rc; j++) {
    double* wj = W + (int64_t)j * ldw;
    rc = csr_product(c, dir1, X + (int64_t)j * ldx, 1, wj, nullptr, s);
    if (!rc) rc = sumsq_launch(wj, e, partial, S + j, s);
  }
  if (!rc && kdone > 0) rc = sqrt_inplace_launch(S, kdone, s);
  if (!rc && kdone > 0) rc = finish_scale_sign_launch(W, ldw, e, S, V, ldv, n, U, ldu, m, kdone, 1, partial, s);
  if (rc) return from_internal(ctx, rc, "sparse finish");
  hipEventRecord(ctx->ev[3], s);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(ctx, TSVD_ERR_HIP, "sync");
  if (info) {
    info->k_done = kdone;
    info->converged = all_conv ? 1 : 0;
    info->rank_deficient = rankdef ? 1 : 0;
    info->branch_right = right ? 1 : 0;
    if (info->iters) memcpy(info->iters, iters.data(), (size_t)k * 4);
    if (info->lambda) memcpy(info->lambda, lams.data(), (size_t)k * 8);
    float t;
    info->t_gram_ms = 0.0;
    hipEventElapsedTime(&t, ctx->ev[1], ctx->ev[2]); info->t_eig_ms = t;
    hipEventElapsedTime(&t, ctx->ev[2], ctx->ev[3]); info->t_final_ms = t;
    hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[3]); info->t_total_ms = t;
    info->workspace_bytes = (int64_t)need;
    info->h2d_bytes = 0;
    info->latency_ms = 0;
  }
  if (!all_conv && !o->fixed_iters && o->eps > 0)
    return fail(ctx, TSVD_ERR_NOT_CONVERGED, "some triplet reached max_iter");
  return TSVD_OK;
}

}  // extern "C"
