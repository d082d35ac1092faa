// C-ABI implementation: context, workspace, argument checks and the dense
// driver that chains Gram -> power iteration -> FP64 finishing pass
// (Algorithm 1 with Algorithm 2 on the Gram of Algorithm 3).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/tsvd.h"
#include "common.h"

#include "internal.h"

namespace tsvd {

static thread_local std::string g_hip_msg;

int hip_fail(hipError_t e, const char* what, const char* file, int line) {
  char buf[512];
  snprintf(buf, sizeof buf, "HIP error '%s' (%d) in %s at %s:%d", hipGetErrorString(e), (int)e, what, file, line);
  g_hip_msg = buf;
  return TSVD_ERR_HIP;
}

}  // namespace tsvd

using namespace tsvd;

struct tsvd_ctx {
  int device = 0;
  int num_cu = 0;
  size_t max_lds = 0;
  std::string last_error;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace {

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

struct Bump {
  char* base;
  size_t off = 0;
  size_t cap;
  explicit Bump(void* b, size_t c) : base((char*)b), cap(c) {}
  void* take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    void* p = base + off;
    off += bytes;
    return p;
  }
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

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

}  // namespace

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

void tsvd_opts_default(tsvd_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof *o);
  o->k = -1;
  o->eps = 1e-8;
  o->max_iter = 10000;
  o->gram = TSVD_GRAM_AUTO;
  o->queue_depth = 2;
}

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
  syrk_plan(mode, d, K, rows_per_block, ctx->num_cu, &sp);
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
  if (hipMemsetAsync(d_status, 0, 16, stream) != hipSuccess) return fail(ctx, TSVD_ERR_HIP, "memset status");
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
  if (power_plan(is_f64 ? 8 : 4, (int)d, k, ctx->num_cu, ctx->max_lds, 0, &pp))
    return fail(ctx, TSVD_ERR_UNSUPPORTED, "d=%lld too large for the LDS-resident iterate", (long long)d);
  tsvd_status st = ensure_ws(ctx, power_ws_bytes(pp, k), o->hbm_budget);
  if (st) return st;
  Bump bump(ctx->ws, ctx->ws_bytes);
  int* d_status = (int*)bump.take(256);
  int* d_iters = (int*)bump.take((size_t)k * 4);
  double* d_lambda = (double*)bump.take((size_t)k * 8);
  int* d_fixed = (int*)bump.take((size_t)k * 4);
  if (hipMemset2DAsync(X, ldx * 8, 0, d * 8, k, stream) != hipSuccess) return fail(ctx, TSVD_ERR_HIP, "memset X");
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
  rc = finish_scale_sign_launch(W, ldw, M, S, nullptr, 0, 0, nullptr, 0, 0, k, 0, (hipStream_t)stream);
  return from_internal(ctx, rc, "finish scale");
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
  if (loc != TSVD_LOC_DEVICE) return fail(ctx, TSVD_ERR_UNSUPPORTED, "pinned-host input is not built in yet");
  const int mode = gram_mode(o->gram, dtype);
  tsvd_status st = check_mode(ctx, mode, dtype);
  if (st) return st;
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
  syrk_plan(mode, d, K, o->rows_per_block, ctx->num_cu, &sp);
  PowerPlan pp;
  if (power_plan(eb, (int)d, k, ctx->num_cu, ctx->max_lds, 0, &pp))
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
  if (hipMemset2DAsync(U, ldu * 8, 0, m * 8, k, stream) != hipSuccess ||
      hipMemset2DAsync(V, ldv * 8, 0, n * 8, k, stream) != hipSuccess ||
      hipMemsetAsync(S, 0, (size_t)k * 8, stream) != hipSuccess)
    return fail(ctx, TSVD_ERR_HIP, "memset outputs");
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
    rc = finish_scale_sign_launch(W, ldw, Mw, S, V, ldv, n, U, ldu, m, kd, 1, stream);
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
  }
  if (!hs[1] && !o->fixed_iters && o->eps > 0)
    return fail(ctx, TSVD_ERR_NOT_CONVERGED, "some triplet reached max_iter");
  return TSVD_OK;
}

}  // extern "C"
