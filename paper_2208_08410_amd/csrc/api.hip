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
#include "implicit.h"

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
  if (t->sparse_row_bits < 0 || t->sparse_row_bits > 11 || t->sparse_col_bits < 0 || t->sparse_col_bits > 31 ||
      t->sparse_row_bits + t->sparse_col_bits > 32)
    return fail(ctx, TSVD_ERR_INVALID_ARG, "sparse tile bits out of range (rows <= 11, rows + cols <= 32)");
  if (t->team_kib != 0 && (t->team_kib < 8 || t->team_kib > 65536))
    return fail(ctx, TSVD_ERR_INVALID_ARG, "team_kib must be 0 or in [8, 65536]");
  if (t->group_kchunk != 0 && (t->group_kchunk < 32 || t->group_kchunk > (1 << 20)))
    return fail(ctx, TSVD_ERR_INVALID_ARG, "group_kchunk must be 0 or in [32, 2^20]");
  if (t->power_path != 0 && t->power_path != 1) return fail(ctx, TSVD_ERR_INVALID_ARG, "power_path must be 0 or 1");
  for (int c = 0; c < TSVD_GRAM_CLASSES; c++) {
    if (t->group_tile[c] != 0 && t->group_tile[c] != 64 && t->group_tile[c] != 128)
      return fail(ctx, TSVD_ERR_INVALID_ARG, "group_tile[%d] must be 0, 64 or 128", c);
    if (t->group_kchunk_cls[c] != 0 && (t->group_kchunk_cls[c] < 32 || t->group_kchunk_cls[c] > (1 << 20)))
      return fail(ctx, TSVD_ERR_INVALID_ARG, "group_kchunk_cls[%d] must be 0 or in [32, 2^20]", c);
  }
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

namespace {
bool ws_fits(tsvd_ctx* ctx, size_t need, int64_t budget);  // below
}  // namespace

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
  syrk_plan(mode, d, K, rows_per_block, ctx->num_cu, &sp, ctx->tuning.gram_tile, ctx->tuning.gram_chunks, 1);
  // the BF16 planes of the two-pass form need 4 B per element of A on top of
  // the partial tiles; without room for them the one-pass kernel runs
  if (sp.packed && !ws_fits(ctx, align256(sp.partial_bytes), 0))
    syrk_plan(mode, d, K, rows_per_block, ctx->num_cu, &sp, ctx->tuning.gram_tile, ctx->tuning.gram_chunks, 0);
  st = ensure_ws(ctx, align256(sp.partial_bytes), 0);
  if (st) return st;
  int rc = syrk_launch(mode, side, A, m, n, lda, sp, ctx->ws, B, ldb, accumulate, (hipStream_t)stream);
  return from_internal(ctx, rc, "tsvd_gram_dense");
}

// ---------------------------------------------------------------------------
// power phase on an explicit Gram in the workspace: the on-chip persistent
// kernel when its plan fits (and the tuning allows it), else the host-driven
// loop of HBM-streamed products B x with deflation by projection
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

struct PhaseResult {
  int kd = 0, conv = 1, rankdef = 0;
  std::vector<int> iters;
  std::vector<double> lams;
};

size_t power_ws_bytes(const PowerPlan& pp, int k) {
  const size_t words = pp.xex_words + pp.pex_words + pp.vex_words + pp.wex_words;
  return align256(words * 8) + align256((size_t)pp.G * 2 * (k + 2) * 8) + 4 * 256 + align256((size_t)k * 4) +
         align256((size_t)k * 8) + align256((size_t)k * 4) + 1024;
}

// plans the on-chip kernel; false when the loop must run instead
bool plan_onchip(tsvd_ctx* ctx, int eb, int64_t d, int k, PowerPlan* pp) {
  if (ctx->tuning.power_path != 0 || d > 0x7fffffffLL) return false;
  return power_plan(eb, (int)d, k, ctx->num_cu, ctx->max_lds, ctx->tuning.power_blocks, pp) == 0;
}

size_t phase_ws_bytes(bool onchip, const PowerPlan& pp, int64_t d, int k) {
  return onchip ? power_ws_bytes(pp, k) : loop_ws_bytes(d, k);
}

// true when `need` bytes of workspace fit hbm_budget and the device's memory
bool ws_fits(tsvd_ctx* ctx, size_t need, int64_t budget) {
  if (budget > 0 && (int64_t)need > budget) return false;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return true;
  }
  return need <= fr + ctx->ws_bytes;
}

tsvd_status power_phase(tsvd_ctx* ctx, Bump& bump, bool onchip, const PowerPlan& pp, void* B, int is_f64, int64_t d,
                        int64_t ldb, int k, const tsvd_opts* o, double* X, int64_t ldx, PhaseResult* pr,
                        hipStream_t stream) {
  pr->iters.assign(k, 0);
  pr->lams.assign(k, 0.0);
  if (!onchip) {
    LoopWs lw = loop_ws_take(bump, d, k);
    GramOp op;
    op.B = B;
    op.b_f64 = is_f64;
    op.d = d;
    op.ldb = ldb;
    DeviceFactor fac(X, ldx, d);
    PowerLoopResult r;
    int rc = implicit_power(op, fac, o, k, d, lw, &r, stream);
    if (rc) return from_internal(ctx, rc, "power iteration (streamed Gram)");
    if (r.nonfinite) return fail(ctx, TSVD_ERR_NONFINITE, "non-finite value in the Gram or the power iteration");
    pr->kd = r.kdone;
    pr->conv = r.all_conv ? 1 : 0;
    pr->rankdef = r.rankdef ? 1 : 0;
    pr->iters = r.iters;
    pr->lams = r.lams;
    return TSVD_OK;
  }
  int* d_status = (int*)bump.take(256);
  int* d_iters = (int*)bump.take((size_t)k * 4);
  double* d_lambda = (double*)bump.take((size_t)k * 8);
  int* d_fixed = (int*)bump.take((size_t)k * 4);
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
  if (rc) return from_internal(ctx, rc, "power iteration");
  int hs[4];
  if (hipMemcpyAsync(hs, d_status, 16, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipMemcpyAsync(pr->iters.data(), d_iters, (size_t)k * 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipMemcpyAsync(pr->lams.data(), d_lambda, (size_t)k * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return fail(ctx, TSVD_ERR_HIP, "power status readback: %s", hipGetErrorString(hipGetLastError()));
  if (hs[2] == 1) return fail(ctx, TSVD_ERR_INTERNAL, "power iteration: a bounded wait timed out");
  if (hs[2] == 2) return fail(ctx, TSVD_ERR_NONFINITE, "non-finite value in the Gram or the power iteration");
  if (hs[2] == 3) return fail(ctx, TSVD_ERR_INVALID_ARG, "a start vector is zero");
  pr->kd = hs[0];
  pr->conv = hs[1];
  pr->rankdef = hs[3];
  return TSVD_OK;
}

void fill_info(tsvd_info* info, const PhaseResult& pr, int k, bool right, tsvd_ctx* ctx, size_t need, int64_t h2d) {
  if (!info) return;
  info->k_done = pr.kd;
  info->converged = pr.conv;
  info->rank_deficient = pr.rankdef;
  info->branch_right = right ? 1 : 0;
  if (info->iters) memcpy(info->iters, pr.iters.data(), (size_t)k * 4);
  if (info->lambda) memcpy(info->lambda, pr.lams.data(), (size_t)k * 8);
  float t;
  hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1]); info->t_gram_ms = t;
  hipEventElapsedTime(&t, ctx->ev[1], ctx->ev[2]); info->t_eig_ms = t;
  hipEventElapsedTime(&t, ctx->ev[2], ctx->ev[3]); info->t_final_ms = t;
  hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[3]); info->t_total_ms = t;
  info->workspace_bytes = (int64_t)need;
  info->h2d_bytes = h2d;
  info->latency_ms = 0;
  info->t_stream_copy_ms = 0;
  info->t_stream_compute_ms = 0;
  info->t_stream_overlap_ms = 0;
}

tsvd_status not_converged(tsvd_ctx* ctx, const PhaseResult& pr, const tsvd_opts* o) {
  if (!pr.conv && !o->fixed_iters && o->eps > 0) return fail(ctx, TSVD_ERR_NOT_CONVERGED, "some triplet reached max_iter");
  return TSVD_OK;
}

}  // namespace

extern "C" {

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
  const bool onchip = plan_onchip(ctx, is_f64 ? 8 : 4, d, k, &pp);
  const size_t need = phase_ws_bytes(onchip, pp, d, k) + 1024;
  tsvd_status st = ensure_ws(ctx, need, o->hbm_budget);
  if (st) return st;
  Bump bump(ctx->ws, ctx->ws_bytes);
  if (int rc = zero_cols_launch(X, ldx, d, k, stream)) return from_internal(ctx, rc, "clear X");
  PhaseResult pr;
  st = power_phase(ctx, bump, onchip, pp, B, is_f64, d, ldb, k, o, X, ldx, &pr, stream);
  if (st) return st;
  if (info) {
    info->k_done = pr.kd;
    info->converged = pr.conv;
    info->rank_deficient = pr.rankdef;
    info->branch_right = 1;
    info->latency_ms = 0;
    info->t_stream_copy_ms = 0;
    info->t_stream_compute_ms = 0;
    info->t_stream_overlap_ms = 0;
    info->workspace_bytes = (int64_t)need;
    if (info->iters) memcpy(info->iters, pr.iters.data(), (size_t)k * 4);
    if (info->lambda) memcpy(info->lambda, pr.lams.data(), (size_t)k * 8);
  }
  return not_converged(ctx, pr, o);
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

}  // extern "C"

namespace {

// Dense t-SVD without the Gram: Algorithm 2's product applied as
// A^T (A x) (or A (A^T x)) every iteration (Equation 2 evaluated right to
// left).  A in HBM (any dtype, both branches) or FP32 A in pinned host memory
// (streamed once per iteration: row batches for the right branch, pitched
// column batches for the left).  The iterated factor may sit in pinned host
// memory (A in HBM only).
tsvd_status dense_implicit(tsvd_ctx* ctx, const void* A, int32_t dtype, int32_t loc, int64_t m, int64_t n, int64_t lda,
                           const tsvd_opts* o, int k, double* U, int64_t ldu, double* S, double* V, int64_t ldv,
                           tsvd_info* info, hipStream_t s) {
  const bool right = right_side(m, n, o->branch);
  const int side = right ? TSVD_SIDE_RIGHT : TSVD_SIDE_LEFT;
  const int64_t d = right ? n : m, e = right ? m : n;
  const bool pinned = loc == TSVD_LOC_PINNED_HOST;
  const bool host_x = o->factor_loc == TSVD_LOC_PINNED_HOST;
  if (pinned && dtype != TSVD_F32) return fail(ctx, TSVD_ERR_UNSUPPORTED, "pinned-host A is FP32");
  if (pinned && host_x) return fail(ctx, TSVD_ERR_UNSUPPORTED, "with A streamed from the host the factor stays on the device");
  const int Q = o->queue_depth > 0 ? o->queue_depth : 2;
  if (Q > 16 || o->factor_batches < 0) return fail(ctx, TSVD_ERR_INVALID_ARG, "queue_depth or factor_batches");
  const int is_f64 = dtype == TSVD_F64;
  double* X = right ? V : U;
  const int64_t ldx = right ? ldv : ldu;
  double* W = right ? U : V;
  const int64_t ldw = right ? ldu : ldv;
  if (host_x) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, X) != hipSuccess || attr.type != hipMemoryTypeHost) {
      (void)hipGetLastError();
      return fail(ctx, TSVD_ERR_INVALID_ARG, "factor_loc = PINNED_HOST needs %s in pinned host memory",
                  right ? "V" : "U");
    }
  }
  if (pinned) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, A) != hipSuccess || attr.type != hipMemoryTypeHost) {
      (void)hipGetLastError();
      return fail(ctx, TSVD_ERR_INVALID_ARG, "A is not pinned host memory (allocate it with hipHostMalloc / pin_memory)");
    }
  }
  // batch rows (right) or columns (left) of a pinned A: rows_per_block rounded
  // up to 128, or 4 GiB worth rounded down to 128
  int64_t R = 0;
  if (pinned) {
    R = o->rows_per_block > 0 ? ((o->rows_per_block + 127) / 128) * 128 : (((int64_t)4 << 30) / (d * 4)) / 128 * 128;
    if (R < 128) R = 128;
    if (R > e) R = e;
  }
  const int64_t nbatch = pinned ? (e + R - 1) / R : 0;
  const int Qa = pinned ? (int)std::min<int64_t>(Q, nbatch) : 0;
  const size_t buf_bytes = pinned ? align256((size_t)R * d * 4) : 0;
  const size_t op_bytes =
      align256((size_t)(pinned ? PinnedDenseOp::ws_doubles(m, n, R, right) : DenseOp::ws_doubles(m, n)) * 8);
  const int64_t tiles_total = pinned ? (e + 127) / 128 + nbatch : finish_tiles(m, n, side);
  const size_t fin_bytes = align256((size_t)(tiles_total + 2) * k * 8);
  const int64_t RX = host_x ? HostFactor::round_rows(d, o->factor_batches > 0 ? o->factor_batches : 1) : 0;
  const int Qx = host_x ? (int)std::min<int64_t>(Q, (d + RX - 1) / RX) : 0;
  const size_t slot_bytes = host_x ? align256((size_t)RX * k * 8) : 0;
  const size_t need = loop_ws_bytes(d, k) + (size_t)Qa * buf_bytes + op_bytes + fin_bytes + align256((size_t)d * 8) +
                      (size_t)Qx * slot_bytes + 4096;
  tsvd_status st = ensure_ws(ctx, need, o->hbm_budget);
  if (st) return st;
  Bump bump(ctx->ws, ctx->ws_bytes);
  LoopWs lw = loop_ws_take(bump, d, k);
  float* bufs[16];
  for (int q = 0; q < Qa; q++) bufs[q] = (float*)bump.take(buf_bytes);
  double* opws = (double*)bump.take(op_bytes);
  double* ssq = (double*)bump.take(fin_bytes);
  double* tmp = (double*)bump.take((size_t)d * 8);
  double* slots[16];
  for (int q = 0; q < Qx; q++) slots[q] = (double*)bump.take(slot_bytes);

  DenseOp dop;
  PinnedDenseOp pop;
  if (pinned) {
    if (pop.init((const float*)A, m, n, lda, R, Qa, bufs, opws, ctx->copy_stream, right))
      return fail(ctx, TSVD_ERR_HIP, "batch pipeline events");
  } else {
    dop.setup(A, is_f64, m, n, lda, right, opws);
  }
  ImplicitOp& op = pinned ? (ImplicitOp&)pop : (ImplicitOp&)dop;
  DeviceFactor dfac(X, ldx, d);
  HostFactor hfac;
  if (host_x && hfac.init(X, ldx, d, RX, Qx, k, slots, ctx->copy_stream))
    return fail(ctx, TSVD_ERR_HIP, "factor pipeline events");
  Factor& fac = host_x ? (Factor&)hfac : (Factor&)dfac;

  hipEventRecord(ctx->ev[0], s);
  if (zero_cols_launch(W, ldw, e, k, s) || zero_cols_launch(S, k, k, 1, s) ||
      (!host_x && zero_cols_launch(X, ldx, d, k, s)))
    return fail(ctx, TSVD_ERR_HIP, "clear outputs");
  if (host_x) {
    if (hipStreamSynchronize(s) != hipSuccess) return fail(ctx, TSVD_ERR_HIP, "sync");
    for (int j = 0; j < k; j++) memset(X + (int64_t)j * ldx, 0, (size_t)d * 8);
  }
  hipEventRecord(ctx->ev[1], s);
  PowerLoopResult r;
  int rc = implicit_power(op, fac, o, k, d, lw, &r, s);
  if (rc) return from_internal(ctx, rc, "implicit power iteration");
  if (r.nonfinite) return fail(ctx, TSVD_ERR_NONFINITE, "non-finite value in a product or a norm");
  const int kd = r.kdone;
  hipEventRecord(ctx->ev[2], s);
  if (kd > 0) {
    if (host_x) {
      rc = finish_host_factor(op, X, ldx, d, W, ldw, e, S, kd, right, tmp, lw.partial, s);
    } else if (pinned) {
      int64_t tiles = 0;
      rc = pop.finish(X, ldx, kd, W, ldw, ssq, &tiles, s);
      if (!rc) rc = finish_sigma_launch(ssq, tiles, kd, S, s);
      if (!rc) rc = finish_scale_sign_launch(W, ldw, e, S, V, ldv, n, U, ldu, m, kd, 1, ssq + tiles_total * k, s);
    } else {
      rc = finish_launch(is_f64, side, A, m, n, lda, X, ldx, kd, W, ldw, S, ssq, s);
      if (!rc)
        rc = finish_scale_sign_launch(W, ldw, e, S, V, ldv, n, U, ldu, m, kd, 1, ssq + finish_tiles(m, n, side) * k, s);
    }
    if (rc) return from_internal(ctx, rc, "finish");
  }
  hipEventRecord(ctx->ev[3], s);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(ctx, TSVD_ERR_HIP, "sync");
  PhaseResult pr;
  pr.kd = kd;
  pr.conv = r.all_conv ? 1 : 0;
  pr.rankdef = r.rankdef ? 1 : 0;
  pr.iters = r.iters;
  pr.lams = r.lams;
  fill_info(info, pr, k, right, ctx, need, op.h2d_bytes() + fac.h2d_bytes());
  if (info) info->t_gram_ms = 0.0;  // no Gram phase: the interval before the loop only clears the outputs
  return not_converged(ctx, pr, o);
}

// Dense t-SVD of an FP32 A held in pinned host memory (Algorithm 3's
// out-of-memory batching).  A is streamed in batches along the Gram's
// contraction: row batches for the A^T A branch, column batches (pitched 2-D
// copies) for the A A^T branch, through `queue_depth` device buffers: the copy
// stream fills buffer b % Q while the compute stream runs the Gram (pass 1) or
// the FP64 finishing product (pass 2: the rows of U, or of V, that the batch
// owns) on the previous batch; events order reuse.  The power iteration runs
// on the device-resident Gram between the passes, overlapped with the first
// copies of pass 2.  auto_method: fall back to the implicit product when the
// Gram's workspace does not fit.
tsvd_status dense_pinned(tsvd_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda, const tsvd_opts* o, int k,
                         int mode, bool auto_method, double* U, int64_t ldu, double* S, double* V, int64_t ldv,
                         tsvd_info* info, hipStream_t s) {
  const bool right = right_side(m, n, o->branch);
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, A) != hipSuccess || attr.type != hipMemoryTypeHost) {
    (void)hipGetLastError();
    return fail(ctx, TSVD_ERR_INVALID_ARG, "A is not pinned host memory (allocate it with hipHostMalloc / pin_memory)");
  }
  const int Q = o->queue_depth >= 2 ? o->queue_depth : 2;
  if (Q > 16) return fail(ctx, TSVD_ERR_INVALID_ARG, "queue_depth > 16");
  // d: Gram dimension; L: length of the streamed (contraction) dimension
  const int64_t d = right ? n : m, L = right ? m : n;
  const int64_t ldb = (d + 3) & ~3;
  const bool explicit_rows = o->rows_per_block > 0;
  // batch length: rows_per_block rounded up to a multiple of 128 (the
  // finishing pass's row tile), or 4 GiB worth of rows (columns) rounded down
  // to one
  int64_t R = explicit_rows ? ((o->rows_per_block + 127) / 128) * 128 : (((int64_t)4 << 30) / (d * 4)) / 128 * 128;
  if (R < 128) R = 128;
  if (R > L) R = L;
  const int64_t nbatch = (L + R - 1) / R;
  // Gram plan per batch (one chunk per batch when the batch size is given, so
  // the result is bitwise that of the in-HBM path with the same rows_per_block)
  SyrkPlan sp_full, sp_last;
  const int64_t last_rows = L - (nbatch - 1) * R;
  syrk_plan(mode, d, R, explicit_rows ? R : 0, ctx->num_cu, &sp_full, ctx->tuning.gram_tile, ctx->tuning.gram_chunks);
  syrk_plan(mode, d, last_rows, explicit_rows ? last_rows : 0, ctx->num_cu, &sp_last, ctx->tuning.gram_tile,
            ctx->tuning.gram_chunks);
  const size_t part_bytes = sp_full.partial_bytes > sp_last.partial_bytes ? sp_full.partial_bytes : sp_last.partial_bytes;
  PowerPlan pp;
  const bool onchip = plan_onchip(ctx, 4, d, k, &pp);
  const int64_t tiles_total = (L + 127) / 128 + nbatch;  // finish row tiles, one partial tile per batch at most
  const size_t buf_bytes = align256((size_t)R * d * 4);
  const size_t b_bytes = align256((size_t)d * ldb * 4);
  const size_t ssq_bytes = align256((size_t)(tiles_total + 2) * k * 8);
  const size_t need =
      (size_t)Q * buf_bytes + b_bytes + align256(part_bytes) + phase_ws_bytes(onchip, pp, d, k) + ssq_bytes + 4096;
  if (auto_method && !ws_fits(ctx, need, o->hbm_budget))
    return dense_implicit(ctx, A, TSVD_F32, TSVD_LOC_PINNED_HOST, m, n, lda, o, k, U, ldu, S, V, ldv, info, s);
  tsvd_status st = ensure_ws(ctx, need, o->hbm_budget);
  if (st) return st;
  Bump bump(ctx->ws, ctx->ws_bytes);
  float* buf[16];
  for (int q = 0; q < Q; q++) buf[q] = (float*)bump.take(buf_bytes);
  void* B = bump.take(b_bytes);
  void* partial = bump.take(part_bytes);
  double* ssq = (double*)bump.take(ssq_bytes);

  hipEvent_t copied[16], consumed[16];
  int made = 0;
  auto cleanup = [&]() {
    for (int i = 0; i < made; i++) {
      (void)hipEventDestroy(copied[i]);
      (void)hipEventDestroy(consumed[i]);
    }
  };
  for (; made < Q; made++) {
    if (hipEventCreateWithFlags(&copied[made], hipEventDisableTiming) != hipSuccess) { cleanup(); return fail(ctx, TSVD_ERR_HIP, "event"); }
    if (hipEventCreateWithFlags(&consumed[made], hipEventDisableTiming) != hipSuccess) {
      (void)hipEventDestroy(copied[made]);
      cleanup();
      return fail(ctx, TSVD_ERR_HIP, "event");
    }
  }
  hipStream_t cs = ctx->copy_stream;
  int rc = 0;
  // batch b: rows [r0, r0 + len) of A (a len x n block, pitch n) or its
  // columns [r0, r0 + len) (an m x len block, pitch len)
  auto copy_batch = [&](int64_t b, int slot, bool wait_slot) -> int {
    const int64_t r0 = b * R;
    const int64_t len = (b == nbatch - 1) ? last_rows : R;
    if (wait_slot && hipStreamWaitEvent(cs, consumed[slot], 0) != hipSuccess) return TSVD_ERR_HIP;
    const hipError_t e = right ? hipMemcpy2DAsync(buf[slot], (size_t)n * 4, A + r0 * lda, (size_t)lda * 4, (size_t)n * 4,
                                                  (size_t)len, hipMemcpyHostToDevice, cs)
                               : hipMemcpy2DAsync(buf[slot], (size_t)len * 4, A + r0, (size_t)lda * 4, (size_t)len * 4,
                                                  (size_t)m, hipMemcpyHostToDevice, cs);
    if (e != hipSuccess) return TSVD_ERR_HIP;
    if (hipEventRecord(copied[slot], cs) != hipSuccess) return TSVD_ERR_HIP;
    return 0;
  };

  // per-batch timing of the Gram pass (copy and compute intervals on their
  // streams), when the caller asks for info
  std::vector<hipEvent_t> tev;
  if (info) {
    tev.resize((size_t)nbatch * 4, nullptr);
    for (auto& e : tev)
      if (hipEventCreate(&e) != hipSuccess) {
        for (auto& f : tev)
          if (f) (void)hipEventDestroy(f);
        cleanup();
        return fail(ctx, TSVD_ERR_HIP, "timing events");
      }
  }
  auto cleanup_all = [&]() {
    for (auto& f : tev) (void)hipEventDestroy(f);
    tev.clear();
    cleanup();
  };
  hipEventRecord(ctx->ev[0], s);
  if (hipStreamWaitEvent(cs, ctx->ev[0], 0) != hipSuccess) { cleanup_all(); return fail(ctx, TSVD_ERR_HIP, "wait"); }
  if (zero_cols_launch(U, ldu, m, k, s) || zero_cols_launch(V, ldv, n, k, s) || zero_cols_launch(S, k, k, 1, s)) {
    cleanup_all();
    return fail(ctx, TSVD_ERR_HIP, "clear outputs");
  }
  // ---- pass 1: B = sum_b A_b^T A_b (or A_b A_b^T for column batches)
  for (int64_t b = 0; b < nbatch && !rc; b++) {
    const int slot = (int)(b % Q);
    if (b >= Q && hipStreamWaitEvent(cs, consumed[slot], 0) != hipSuccess) { rc = TSVD_ERR_HIP; break; }
    if (!tev.empty() && hipEventRecord(tev[4 * b], cs) != hipSuccess) { rc = TSVD_ERR_HIP; break; }
    if ((rc = copy_batch(b, slot, false))) break;
    if (!tev.empty() && hipEventRecord(tev[4 * b + 1], cs) != hipSuccess) { rc = TSVD_ERR_HIP; break; }
    if (hipStreamWaitEvent(s, copied[slot], 0) != hipSuccess) { rc = TSVD_ERR_HIP; break; }
    const int64_t len = (b == nbatch - 1) ? last_rows : R;
    const SyrkPlan& sp = (b == nbatch - 1) ? sp_last : sp_full;
    if (!tev.empty() && hipEventRecord(tev[4 * b + 2], s) != hipSuccess) { rc = TSVD_ERR_HIP; break; }
    rc = right ? syrk_launch(mode, 0, buf[slot], len, n, n, sp, partial, B, ldb, b > 0 ? 1 : 0, s)
               : syrk_launch(mode, 1, buf[slot], m, len, len, sp, partial, B, ldb, b > 0 ? 1 : 0, s);
    if (rc) break;
    if (!tev.empty() && hipEventRecord(tev[4 * b + 3], s) != hipSuccess) { rc = TSVD_ERR_HIP; break; }
    if (hipEventRecord(consumed[slot], s) != hipSuccess) { rc = TSVD_ERR_HIP; break; }
  }
  if (rc) { cleanup_all(); return from_internal(ctx, rc, "pinned Gram pass"); }
  hipEventRecord(ctx->ev[1], s);
  // ---- prefetch the first batches of pass 2 while the power iteration runs
  const int64_t pre = nbatch < Q ? nbatch : Q;
  for (int64_t b = 0; b < pre && !rc; b++) rc = copy_batch(b, (int)(b % Q), true);
  if (rc) { cleanup(); return from_internal(ctx, rc, "prefetch"); }
  PhaseResult pr;
  st = right ? power_phase(ctx, bump, onchip, pp, B, 0, d, ldb, k, o, V, ldv, &pr, s)
             : power_phase(ctx, bump, onchip, pp, B, 0, d, ldb, k, o, U, ldu, &pr, s);
  if (st) {
    (void)hipStreamSynchronize(cs);
    cleanup_all();
    return st;
  }
  hipEventRecord(ctx->ev[2], s);
  const int kd = pr.kd;
  // ---- pass 2: U = A V (or V = A^T U) in FP64, the batch's rows of it;
  // column sums of squares per row tile
  int64_t tile_off = 0;
  for (int64_t b = 0; b < nbatch && !rc && kd > 0; b++) {
    const int slot = (int)(b % Q);
    if (b >= pre && (rc = copy_batch(b, slot, true))) break;
    if (hipStreamWaitEvent(s, copied[slot], 0) != hipSuccess) { rc = TSVD_ERR_HIP; break; }
    const int64_t r0 = b * R;
    const int64_t len = (b == nbatch - 1) ? last_rows : R;
    rc = right ? finish_gemm_launch(0, 0, buf[slot], len, n, n, V, ldv, kd, U + r0, ldu, ssq + tile_off * kd, s)
               : finish_gemm_launch(0, 1, buf[slot], m, len, len, U, ldu, kd, V + r0, ldv, ssq + tile_off * kd, s);
    if (rc) break;
    tile_off += (len + 127) / 128;
    if (hipEventRecord(consumed[slot], s) != hipSuccess) { rc = TSVD_ERR_HIP; break; }
  }
  if (!rc && kd > 0) rc = finish_sigma_launch(ssq, tile_off, kd, S, s);
  if (!rc && kd > 0)
    rc = right ? finish_scale_sign_launch(U, ldu, m, S, V, ldv, n, U, ldu, m, kd, 1, ssq + tiles_total * k, s)
               : finish_scale_sign_launch(V, ldv, n, S, V, ldv, n, U, ldu, m, kd, 1, ssq + tiles_total * k, s);
  hipEventRecord(ctx->ev[3], s);
  if (!rc && (hipStreamSynchronize(s) != hipSuccess || hipStreamSynchronize(cs) != hipSuccess)) rc = TSVD_ERR_HIP;
  double copy_ms = 0.0, comp_ms = 0.0, overlap_ms = 0.0;
  if (!rc && !tev.empty()) {
    // intervals relative to ev[0]; each stream's intervals are disjoint and in order
    std::vector<float> t(tev.size());
    for (size_t i = 0; i < tev.size(); i++) hipEventElapsedTime(&t[i], ctx->ev[0], tev[i]);
    size_t j = 0;
    for (int64_t b = 0; b < nbatch; b++) {
      const double c0 = t[4 * b], c1 = t[4 * b + 1];
      copy_ms += c1 - c0;
      comp_ms += t[4 * b + 3] - t[4 * b + 2];
      while (j < (size_t)nbatch && t[4 * j + 3] <= c0) j++;
      for (size_t q = j; q < (size_t)nbatch && t[4 * q + 2] < c1; q++)
        overlap_ms += std::max(0.0, std::min(c1, (double)t[4 * q + 3]) - std::max(c0, (double)t[4 * q + 2]));
    }
  }
  cleanup_all();
  if (rc) return from_internal(ctx, rc, "pinned finish pass");
  fill_info(info, pr, k, right, ctx, need, (int64_t)(m * n * 4) * (kd > 0 ? 2 : 1));
  if (info) {
    info->t_stream_copy_ms = copy_ms;
    info->t_stream_compute_ms = comp_ms;
    info->t_stream_overlap_ms = overlap_ms;
  }
  return not_converged(ctx, pr, o);
}

}  // namespace

extern "C" {

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
  if (o->method < TSVD_METHOD_AUTO || o->method > TSVD_METHOD_IMPLICIT)
    return fail(ctx, TSVD_ERR_INVALID_ARG, "bad method %d", o->method);
  if (o->factor_loc != TSVD_LOC_DEVICE && o->factor_loc != TSVD_LOC_PINNED_HOST)
    return fail(ctx, TSVD_ERR_INVALID_ARG, "bad factor_loc");
  if (o->factor_loc == TSVD_LOC_PINNED_HOST && o->method == TSVD_METHOD_GRAM)
    return fail(ctx, TSVD_ERR_INVALID_ARG, "a pinned-host factor needs the implicit product (method IMPLICIT or AUTO)");
  hipSetDevice(ctx->device);
  hipStream_t stream = (hipStream_t)stream_;
  if (o->method == TSVD_METHOD_IMPLICIT || o->factor_loc == TSVD_LOC_PINNED_HOST)
    return dense_implicit(ctx, A, dtype, loc, m, n, lda, o, k, U, ldu, S, V, ldv, info, stream);
  const int mode = gram_mode(o->gram, dtype);
  tsvd_status st = check_mode(ctx, mode, dtype);
  if (st) return st;
  const bool auto_method = o->method == TSVD_METHOD_AUTO;
  if (loc == TSVD_LOC_PINNED_HOST)
    return dense_pinned(ctx, (const float*)A, m, n, lda, o, k, mode, auto_method, U, ldu, S, V, ldv, info, stream);

  const bool right = right_side(m, n, o->branch);
  const int side = right ? TSVD_SIDE_RIGHT : TSVD_SIDE_LEFT;
  const int64_t d = right ? n : m;
  const int64_t K = right ? m : n;
  const int is_f64 = mode == MODE_FP64;
  const int eb = is_f64 ? 8 : 4;
  const int64_t ldb = (d + 3) & ~3;

  SyrkPlan sp;
  syrk_plan(mode, d, K, o->rows_per_block, ctx->num_cu, &sp, ctx->tuning.gram_tile, ctx->tuning.gram_chunks, 1);
  PowerPlan pp;
  const bool onchip = plan_onchip(ctx, eb, d, k, &pp);
  const size_t b_bytes = align256((size_t)d * ldb * eb);
  const size_t fin_bytes = align256((size_t)finish_workspace_doubles(m, n, side, k) * 8);
  size_t need = b_bytes + align256(sp.partial_bytes) + phase_ws_bytes(onchip, pp, d, k) + fin_bytes + 4096;
  if (sp.packed && !ws_fits(ctx, need, o->hbm_budget)) {
    // no room for the BF16 planes of the two-pass Gram: the one-pass kernel
    syrk_plan(mode, d, K, o->rows_per_block, ctx->num_cu, &sp, ctx->tuning.gram_tile, ctx->tuning.gram_chunks, 0);
    need = b_bytes + align256(sp.partial_bytes) + phase_ws_bytes(onchip, pp, d, k) + fin_bytes + 4096;
  }
  if (auto_method && !ws_fits(ctx, need, o->hbm_budget))
    return dense_implicit(ctx, A, dtype, loc, m, n, lda, o, k, U, ldu, S, V, ldv, info, stream);
  st = ensure_ws(ctx, need, o->hbm_budget);
  if (st) return st;
  Bump bump(ctx->ws, ctx->ws_bytes);
  void* B = bump.take(b_bytes);
  void* partial = bump.take(sp.partial_bytes);
  double* ssq = (double*)bump.take(fin_bytes);

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
  PhaseResult pr;
  st = power_phase(ctx, bump, onchip, pp, B, is_f64, d, ldb, k, o, X, ldx, &pr, stream);
  if (st) return st;
  hipEventRecord(ctx->ev[2], stream);
  const int kd = pr.kd;
  if (kd > 0) {
    rc = finish_launch(is_f64, side, A, m, n, lda, X, ldx, kd, W, ldw, S, ssq, stream);
    if (rc) return from_internal(ctx, rc, "finish");
    rc = finish_scale_sign_launch(W, ldw, Mw, S, V, ldv, n, U, ldu, m, kd, 1, ssq + finish_tiles(m, n, side) * k,
                                  stream);
    if (rc) return from_internal(ctx, rc, "finish scale/sign");
  }
  hipEventRecord(ctx->ev[3], stream);
  if (hipStreamSynchronize(stream) != hipSuccess)
    return fail(ctx, TSVD_ERR_HIP, "sync: %s", hipGetErrorString(hipGetLastError()));
  fill_info(info, pr, k, right, ctx, need, 0);
  return not_converged(ctx, pr, o);
}

}  // extern "C"
