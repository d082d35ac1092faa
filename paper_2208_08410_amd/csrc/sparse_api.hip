// C-ABI implementation of the sparse path: CSR registration (CSC transpose
// and sliced tiles built on the device, or built batch by batch into pinned
// host memory and streamed to the device for every product), the two sparse
// products, and the t-SVD of Algorithm 1 with the implicit deflated product of
// Equation 2 / Algorithm 4 in factored form.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/tsvd.h"
#include "common.h"
#include "ctx.h"
#include "implicit.h"
#include "internal.h"

using namespace tsvd;

struct tsvd_csr {
  int device = 0;
  int64_t m = 0, n = 0, nnz = 0;
  int loc = TSVD_LOC_DEVICE;
  const int64_t* rowptr = nullptr;
  const int32_t* col = nullptr;
  const float* val = nullptr;
  int64_t* colptr = nullptr;  // owned CSC copy (device handles)
  int32_t* rowidx = nullptr;
  float* cval = nullptr;
  // owned sliced tiles of A (from the CSR) and of A^T (from the CSC): dir 0 / 1.
  // tptr is always on the device; keys and values are device arrays for a
  // device handle and pinned host arrays for a pinned one.
  TilePlan tp[2] = {};
  int64_t* tptr[2] = {nullptr, nullptr};
  uint32_t* tkey[2] = {nullptr, nullptr};
  float* tval[2] = {nullptr, nullptr};
  // pinned handles: batch b of direction dir covers row chunks
  // [bchunk[dir][b], bchunk[dir][b + 1]) and entries [bentry[dir][b],
  // bentry[dir][b + 1]) of the host tile arrays
  std::vector<int64_t> bchunk[2];
  std::vector<int64_t> bentry[2];
  int Q = 0;
  int64_t slot_entries = 0;
  uint32_t* skey[16] = {};
  float* sval[16] = {};
  hipStream_t cs = nullptr;
  hipEvent_t copied[16] = {}, consumed[16] = {}, start_ev = nullptr;
  bool used[16] = {};
  int made = 0;
  int64_t h2d = 0;
};

namespace {

// y = A x (dir 0) or A^T x (dir 1) through the sliced tiles
int csr_product(tsvd_csr* c, int dir, const void* x, int x_is_f64, double* y, float* yf, hipStream_t s) {
  const int64_t rows = dir == 0 ? c->m : c->n;
  if (c->loc == TSVD_LOC_DEVICE)
    return spmv_tiles_launch(c->tp[dir], c->tptr[dir], c->tkey[dir], c->tval[dir], rows, x, x_is_f64, y, yf, 0, 0,
                             c->tp[dir].nchunks, s);
  // pinned: batch b of row chunks is copied into slot b % Q while the previous
  // batch's product runs; the rows of y it covers are written by that product
  TSVD_HIP_TRY(hipEventRecord(c->start_ev, s));  // x is ready on s
  TSVD_HIP_TRY(hipStreamWaitEvent(c->cs, c->start_ev, 0));
  const std::vector<int64_t>& bc = c->bchunk[dir];
  for (size_t b = 0; b + 1 < bc.size(); b++) {
    const int q = (int)(b % c->Q);
    const int64_t c0 = bc[b], c1 = bc[b + 1];
    const int64_t e0 = c->bentry[dir][b], e1 = c->bentry[dir][b + 1];
    if (c->used[q]) TSVD_HIP_TRY(hipStreamWaitEvent(c->cs, c->consumed[q], 0));
    if (e1 > e0) {
      TSVD_HIP_TRY(hipMemcpyAsync(c->skey[q], c->tkey[dir] + e0, (size_t)(e1 - e0) * 4, hipMemcpyHostToDevice, c->cs));
      TSVD_HIP_TRY(hipMemcpyAsync(c->sval[q], c->tval[dir] + e0, (size_t)(e1 - e0) * 4, hipMemcpyHostToDevice, c->cs));
    }
    TSVD_HIP_TRY(hipEventRecord(c->copied[q], c->cs));
    TSVD_HIP_TRY(hipStreamWaitEvent(s, c->copied[q], 0));
    if (int rc = spmv_tiles_launch(c->tp[dir], c->tptr[dir], c->skey[q], c->sval[q], rows, x, x_is_f64, y, yf, e0, c0,
                                   c1 - c0, s))
      return rc;
    TSVD_HIP_TRY(hipEventRecord(c->consumed[q], s));
    c->used[q] = true;
    c->h2d += (e1 - e0) * 8;
  }
  return 0;
}

// Algorithm 2's operator on the sparse matrix: right branch z = A^T (A x),
// left z = A (A^T x); FP32 x and intermediate, FP64 accumulation and result
struct SparseOp : ImplicitOp {
  tsvd_csr* c;
  int dir1, dir2;
  float* tf;
  int64_t h2d0;
  SparseOp(tsvd_csr* c_, bool right, float* tf_) : c(c_), dir1(right ? 0 : 1), dir2(right ? 1 : 0), tf(tf_), h2d0(c_->h2d) {}
  int apply(const double* x, const float* xf, double* z, hipStream_t s) override {
    if (int rc = csr_product(c, dir1, xf, 0, nullptr, tf, s)) return rc;
    return csr_product(c, dir2, tf, 0, z, nullptr, s);
  }
  int first(const double* x, double* w, hipStream_t s) override { return csr_product(c, dir1, x, 1, w, nullptr, s); }
  int64_t h2d_bytes() const override { return c->h2d - h2d0; }
};

// greedy batches of whole row chunks holding at most `cap` entries each (a
// chunk larger than cap gets a batch of its own); ent(c) = entries of chunk c
template <typename F>
void chunk_batches(int64_t nchunks, int64_t cap, F ent, std::vector<int64_t>* bc, std::vector<int64_t>* be) {
  bc->assign(1, 0);
  be->assign(1, 0);
  int64_t cur = 0, e = 0;
  for (int64_t ch = 0; ch < nchunks; ch++) {
    const int64_t k = ent(ch);
    if (ch > bc->back() && cur + k > cap) {
      bc->push_back(ch);
      be->push_back(e);
      cur = 0;
    }
    cur += k;
    e += k;
  }
  bc->push_back(nchunks);
  be->push_back(e);
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
  (void)hipFree(d_bad);
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
    (void)hipFree(scratch);
    tsvd_csr_destroy(c);
    return fail(ctx, TSVD_ERR_OUT_OF_MEMORY, "allocating the CSC copy (%lld nonzeros)", (long long)nnz);
  }
  rc = csc_build(rowptr, col, val, m, n, nnz, c->colptr, c->rowidx, c->cval, scratch, s);
  if (rc == 0 && hipStreamSynchronize(s) != hipSuccess) rc = TSVD_ERR_HIP;
  (void)hipFree(scratch);
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
      (void)hipFree(tscr);
      tsvd_csr_destroy(c);
      return fail(ctx, TSVD_ERR_OUT_OF_MEMORY, "allocating the sparse tiles (%lld nonzeros)", (long long)nnz);
    }
    rc = dir == 0 ? tiles_build(rowptr, col, val, m, nnz, c->tp[0], c->tptr[0], c->tkey[0], c->tval[0], tscr, s)
                  : tiles_build(c->colptr, c->rowidx, c->cval, n, nnz, c->tp[1], c->tptr[1], c->tkey[1], c->tval[1],
                                tscr, s);
    if (rc == 0 && hipStreamSynchronize(s) != hipSuccess) rc = TSVD_ERR_HIP;
    (void)hipFree(tscr);
    if (rc) {
      tsvd_csr_destroy(c);
      return from_internal(ctx, rc, "tile build");
    }
  }
  *out = c;
  return TSVD_OK;
}

tsvd_status tsvd_csr_create_pinned(tsvd_ctx* ctx, int64_t m, int64_t n, int64_t nnz, const int64_t* rowptr,
                                   const int32_t* col, const float* val, int64_t batch_bytes, int32_t queue_depth,
                                   tsvd_csr** out, void* stream_) {
  if (!ctx) return TSVD_ERR_INVALID_ARG;
  if (!out) return fail(ctx, TSVD_ERR_INVALID_ARG, "null out");
  *out = nullptr;
  if (m < 1 || n < 1 || nnz < 0) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad shape m=%lld n=%lld nnz=%lld",
                                              (long long)m, (long long)n, (long long)nnz);
  if (n > 0x7fffffffLL || m > 0x7fffffffLL) return fail(ctx, TSVD_ERR_UNSUPPORTED, "int32 indices need m, n < 2^31");
  if (!rowptr || (nnz > 0 && (!col || !val))) return fail(ctx, TSVD_ERR_INVALID_ARG, "null pointer");
  if (batch_bytes < 0 || queue_depth < 0 || queue_depth > 16)
    return fail(ctx, TSVD_ERR_INVALID_ARG, "batch_bytes < 0 or queue_depth outside [0, 16]");
  for (const void* p : {(const void*)rowptr, (const void*)col, (const void*)val}) {
    if (!p) continue;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess || attr.type != hipMemoryTypeHost) {
      (void)hipGetLastError();
      return fail(ctx, TSVD_ERR_INVALID_ARG, "the CSR arrays must be pinned host memory");
    }
  }
  if (rowptr[0] != 0 || rowptr[m] != nnz)
    return fail(ctx, TSVD_ERR_INVALID_ARG, "CSR structure invalid (flags 2: ends)");
  hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream_;
  tsvd_csr* c = new tsvd_csr();
  c->device = ctx->device;
  c->loc = TSVD_LOC_PINNED_HOST;
  c->m = m; c->n = n; c->nnz = nnz;
  c->rowptr = rowptr; c->col = col; c->val = val;
  c->Q = queue_depth > 0 ? queue_depth : 2;
  const int64_t cap = std::max<int64_t>(1, (batch_bytes > 0 ? batch_bytes : ((int64_t)512 << 20)) / 8);
  for (int dir = 0; dir < 2; dir++) {
    const int64_t rows = dir == 0 ? m : n, cols = dir == 0 ? n : m;
    if (tiles_plan(rows, cols, ctx->num_cu, ctx->tuning.sparse_row_bits, ctx->tuning.sparse_col_bits, &c->tp[dir])) {
      tsvd_csr_destroy(c);
      return fail(ctx, TSVD_ERR_INVALID_ARG, "sparse tile bits out of range");
    }
  }
  // row pointers at chunk boundaries must be monotone before the host sizes copies by them
  const int rb0 = c->tp[0].rbits;
  for (int64_t ch = 0; ch < c->tp[0].nchunks; ch++) {
    const int64_t a = rowptr[ch << rb0], b = rowptr[std::min(m, (ch + 1) << rb0)];
    if (a < 0 || b < a || b > nnz) {
      tsvd_csr_destroy(c);
      return fail(ctx, TSVD_ERR_INVALID_ARG, "CSR structure invalid (flags 1: row pointers)");
    }
  }
  chunk_batches(c->tp[0].nchunks, cap,
                [&](int64_t ch) { return rowptr[std::min(m, (ch + 1) << rb0)] - rowptr[ch << rb0]; }, &c->bchunk[0],
                &c->bentry[0]);
  // ---- device staging for the build
  int64_t max_rows = 1, max_ent0 = 1, max_ch = 1;
  for (size_t b = 0; b + 1 < c->bchunk[0].size(); b++) {
    const int64_t r0 = c->bchunk[0][b] << rb0, r1 = std::min(m, c->bchunk[0][b + 1] << rb0);
    max_rows = std::max(max_rows, r1 - r0);
    max_ent0 = std::max(max_ent0, c->bentry[0][b + 1] - c->bentry[0][b]);
    max_ch = std::max(max_ch, c->bchunk[0][b + 1] - c->bchunk[0][b]);
  }
  int rc = 0;
  const int64_t ns0 = c->tp[0].nslices, ns1 = c->tp[1].nslices;
  int64_t *d_rp_raw = nullptr, *d_rp = nullptr, *d_colptr = nullptr, *d_tptr_b = nullptr, *d_sub = nullptr;
  int32_t* d_col = nullptr;
  float* d_val = nullptr;
  unsigned long long *d_cnt = nullptr, *d_bsum = nullptr;
  int* d_bad = nullptr;
  std::vector<void*> staged;
  auto dalloc = [&](void** p, size_t bytes) {
    if (rc) return;
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      rc = TSVD_ERR_OUT_OF_MEMORY;
      return;
    }
    staged.push_back(*p);
  };
  auto release = [&]() {
    (void)hipStreamSynchronize(s);
    for (void* p : staged) (void)hipFree(p);
    staged.clear();
  };
  dalloc((void**)&d_rp_raw, (size_t)(max_rows + 1) * 8);
  dalloc((void**)&d_rp, (size_t)(max_rows + 1) * 8);
  dalloc((void**)&d_col, (size_t)max_ent0 * 4);
  dalloc((void**)&d_val, (size_t)max_ent0 * 4);
  dalloc((void**)&d_cnt, (size_t)(n + 1) * 8);
  dalloc((void**)&d_bsum, (size_t)((n + 1023) / 1024 + 2) * 8);
  dalloc((void**)&d_colptr, (size_t)(n + 1) * 8);
  dalloc((void**)&d_bad, 256);
  if (!rc) {
    for (int dir = 0; dir < 2; dir++) {
      if (hipMalloc(&c->tptr[dir], (size_t)(c->tp[dir].nchunks * c->tp[dir].nslices + 1) * 8) != hipSuccess ||
          hipHostMalloc((void**)&c->tkey[dir], (size_t)std::max<int64_t>(nnz, 1) * 4, 0) != hipSuccess ||
          hipHostMalloc((void**)&c->tval[dir], (size_t)std::max<int64_t>(nnz, 1) * 4, 0) != hipSuccess) {
        (void)hipGetLastError();
        rc = TSVD_ERR_OUT_OF_MEMORY;
      }
    }
  }
  if (rc) {
    release();
    tsvd_csr_destroy(c);
    return fail(ctx, TSVD_ERR_OUT_OF_MEMORY, "allocating the staging and host tile arrays (%lld nonzeros)",
                (long long)nnz);
  }
  // tile staging, sized below for the larger direction
  uint32_t* d_tkey = nullptr;
  float* d_tval = nullptr;
  void* d_tscr = nullptr;
  int hbad = 0;
  auto upload_rows = [&](size_t b) -> int {  // row batch b of the CSR -> d_rp (rebased), d_col, d_val
    const int64_t r0 = c->bchunk[0][b] << rb0, r1 = std::min(m, c->bchunk[0][b + 1] << rb0);
    const int64_t e0 = c->bentry[0][b], e1 = c->bentry[0][b + 1];
    TSVD_HIP_TRY(hipMemcpyAsync(d_rp_raw, rowptr + r0, (size_t)(r1 - r0 + 1) * 8, hipMemcpyHostToDevice, s));
    if (e1 > e0) {
      TSVD_HIP_TRY(hipMemcpyAsync(d_col, col + e0, (size_t)(e1 - e0) * 4, hipMemcpyHostToDevice, s));
      TSVD_HIP_TRY(hipMemcpyAsync(d_val, val + e0, (size_t)(e1 - e0) * 4, hipMemcpyHostToDevice, s));
    }
    return rebase_launch(d_rp_raw, r1 - r0 + 1, d_rp, s);
  };
  // ---- pass 1: tiles of A, batch by batch; column counts on the way
  rc = zero_bytes_launch(d_cnt, (size_t)(n + 1) * 8, s);
  if (!rc) {
    dalloc((void**)&d_tkey, (size_t)max_ent0 * 4);
    dalloc((void**)&d_tval, (size_t)max_ent0 * 4);
    TilePlan tb = c->tp[0];
    tb.nchunks = max_ch;
    dalloc(&d_tscr, tiles_scratch_bytes(tb));
    dalloc((void**)&d_tptr_b, (size_t)(max_ch * ns0 + 1) * 8);
  }
  for (size_t b = 0; !rc && b + 1 < c->bchunk[0].size(); b++) {
    const int64_t c0 = c->bchunk[0][b], c1 = c->bchunk[0][b + 1];
    const int64_t r0 = c0 << rb0, r1 = std::min(m, c1 << rb0);
    const int64_t e0 = c->bentry[0][b], ent = c->bentry[0][b + 1] - e0;
    if ((rc = upload_rows(b))) break;
    // the structure is checked before anything indexes through it
    if ((rc = csr_validate(d_rp, d_col, r1 - r0, n, ent, d_bad, s))) break;
    if (hipMemcpyAsync(&hbad, d_bad, 4, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
      rc = TSVD_ERR_HIP;
      break;
    }
    if (hbad) break;
    if ((rc = csc_count_launch(d_col, ent, d_cnt, s))) break;
    TilePlan tb = c->tp[0];
    tb.nchunks = c1 - c0;
    if ((rc = tiles_build(d_rp, d_col, d_val, r1 - r0, ent, tb, d_tptr_b, d_tkey, d_tval, d_tscr, s))) break;
    if ((rc = offset_launch(d_tptr_b, (c1 - c0) * ns0 + 1, e0, c->tptr[0] + c0 * ns0, s))) break;
    if (ent > 0 && (hipMemcpyAsync(c->tkey[0] + e0, d_tkey, (size_t)ent * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipMemcpyAsync(c->tval[0] + e0, d_tval, (size_t)ent * 4, hipMemcpyDeviceToHost, s) != hipSuccess)) {
      rc = TSVD_ERR_HIP;
      break;
    }
    if (hipStreamSynchronize(s) != hipSuccess) {  // the staging is reused by the next batch
      rc = TSVD_ERR_HIP;
      break;
    }
  }
  if (!rc && hbad) {
    release();
    tsvd_csr_destroy(c);
    return fail(ctx, TSVD_ERR_INVALID_ARG, "CSR structure invalid (flags %d: 1 row pointers, 2 ends, 4 columns)", hbad);
  }
  // ---- column pointers, then tiles of A^T: per batch of A^T row chunks
  // (columns [j0, j1) of A), the whole CSR is streamed again and the entries
  // of those columns are gathered into a CSC of the sub-matrix, sorted by row
  std::vector<int64_t> colptr_h;
  if (!rc) rc = scan_counts(d_cnt, n, d_bsum, d_colptr, nnz, s);
  if (!rc) {
    colptr_h.resize(n + 1);
    if (hipMemcpyAsync(colptr_h.data(), d_colptr, (size_t)(n + 1) * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      rc = TSVD_ERR_HIP;
  }
  const int rb1 = c->tp[1].rbits;
  int64_t max_ent1 = 1, max_ch1 = 1, max_cols = 1;
  if (!rc) {
    chunk_batches(c->tp[1].nchunks, cap,
                  [&](int64_t ch) { return colptr_h[std::min(n, (ch + 1) << rb1)] - colptr_h[ch << rb1]; },
                  &c->bchunk[1], &c->bentry[1]);
    for (size_t b = 0; b + 1 < c->bchunk[1].size(); b++) {
      const int64_t j0 = c->bchunk[1][b] << rb1, j1 = std::min(n, c->bchunk[1][b + 1] << rb1);
      max_cols = std::max(max_cols, j1 - j0);
      max_ent1 = std::max(max_ent1, c->bentry[1][b + 1] - c->bentry[1][b]);
      max_ch1 = std::max(max_ch1, c->bchunk[1][b + 1] - c->bchunk[1][b]);
    }
  }
  int32_t* d_rowidx = nullptr;
  float* d_cval = nullptr;
  unsigned long long* d_fill = nullptr;
  if (!rc) {  // tile staging of pass 1 -> sized for A^T's batches
    (void)hipStreamSynchronize(s);
    for (void** p : {(void**)&d_tkey, (void**)&d_tval, &d_tscr, (void**)&d_tptr_b}) {
      staged.erase(std::remove(staged.begin(), staged.end(), *p), staged.end());
      (void)hipFree(*p);
      *p = nullptr;
    }
    TilePlan tb = c->tp[1];
    tb.nchunks = max_ch1;
    dalloc((void**)&d_tkey, (size_t)max_ent1 * 4);
    dalloc((void**)&d_tval, (size_t)max_ent1 * 4);
    dalloc(&d_tscr, tiles_scratch_bytes(tb));
    dalloc((void**)&d_tptr_b, (size_t)(max_ch1 * ns1 + 1) * 8);
  }
  dalloc((void**)&d_rowidx, (size_t)max_ent1 * 4);
  dalloc((void**)&d_cval, (size_t)max_ent1 * 4);
  dalloc((void**)&d_fill, (size_t)max_cols * 8);
  dalloc((void**)&d_sub, (size_t)(max_cols + 1) * 8);
  for (size_t b = 0; !rc && b + 1 < c->bchunk[1].size(); b++) {
    const int64_t c0 = c->bchunk[1][b], c1 = c->bchunk[1][b + 1];
    const int64_t j0 = c0 << rb1, j1 = std::min(n, c1 << rb1);
    const int64_t f0 = c->bentry[1][b], ent = c->bentry[1][b + 1] - f0;
    if ((rc = rebase_launch(d_colptr + j0, j1 - j0 + 1, d_sub, s))) break;
    if ((rc = zero_bytes_launch(d_fill, (size_t)(j1 - j0) * 8, s))) break;
    for (size_t rbt = 0; !rc && rbt + 1 < c->bchunk[0].size(); rbt++) {
      const int64_t r0 = c->bchunk[0][rbt] << rb0, r1 = std::min(m, c->bchunk[0][rbt + 1] << rb0);
      if ((rc = upload_rows(rbt))) break;
      rc = csc_fill_range_launch(d_rp, d_col, d_val, r1 - r0, r0, j0, j1, d_sub, d_fill, d_rowidx, d_cval, s);
    }
    if (rc) break;
    if ((rc = csc_sort_launch(d_sub, j1 - j0, d_rowidx, d_cval, s))) break;
    TilePlan tb = c->tp[1];
    tb.nchunks = c1 - c0;
    if ((rc = tiles_build(d_sub, d_rowidx, d_cval, j1 - j0, ent, tb, d_tptr_b, d_tkey, d_tval, d_tscr, s))) break;
    if ((rc = offset_launch(d_tptr_b, (c1 - c0) * ns1 + 1, f0, c->tptr[1] + c0 * ns1, s))) break;
    if (ent > 0 && (hipMemcpyAsync(c->tkey[1] + f0, d_tkey, (size_t)ent * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipMemcpyAsync(c->tval[1] + f0, d_tval, (size_t)ent * 4, hipMemcpyDeviceToHost, s) != hipSuccess)) {
      rc = TSVD_ERR_HIP;
      break;
    }
    if (hipStreamSynchronize(s) != hipSuccess) rc = TSVD_ERR_HIP;
  }
  release();
  if (rc) {
    tsvd_csr_destroy(c);
    if (rc == TSVD_ERR_OUT_OF_MEMORY) return fail(ctx, TSVD_ERR_OUT_OF_MEMORY, "allocating the build staging");
    return from_internal(ctx, rc, "pinned tile build");
  }
  // ---- the streaming pipeline: Q device slots of the largest batch, events, a copy stream
  c->slot_entries = std::max(max_ent0, max_ent1);
  for (int q = 0; q < c->Q; q++) {
    if (hipMalloc(&c->skey[q], (size_t)c->slot_entries * 4) != hipSuccess ||
        hipMalloc(&c->sval[q], (size_t)c->slot_entries * 4) != hipSuccess) {
      (void)hipGetLastError();
      tsvd_csr_destroy(c);
      return fail(ctx, TSVD_ERR_OUT_OF_MEMORY, "allocating %d streaming slots of %lld entries", c->Q,
                  (long long)c->slot_entries);
    }
  }
  bool ok = hipStreamCreateWithFlags(&c->cs, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&c->start_ev, hipEventDisableTiming) == hipSuccess;
  for (; ok && c->made < c->Q; c->made++) {
    if (hipEventCreateWithFlags(&c->copied[c->made], hipEventDisableTiming) != hipSuccess) { ok = false; break; }
    if (hipEventCreateWithFlags(&c->consumed[c->made], hipEventDisableTiming) != hipSuccess) {
      (void)hipEventDestroy(c->copied[c->made]);
      ok = false;
      break;
    }
  }
  if (!ok) {
    tsvd_csr_destroy(c);
    return fail(ctx, TSVD_ERR_HIP, "streaming pipeline");
  }
  *out = c;
  return TSVD_OK;
}

tsvd_status tsvd_csr_info(const tsvd_csr* c, int32_t* loc, int64_t* batches, int64_t* device_bytes) {
  if (!c) return TSVD_ERR_INVALID_ARG;
  if (loc) *loc = c->loc;
  if (batches) *batches = c->loc == TSVD_LOC_PINNED_HOST ? (int64_t)(c->bchunk[0].size() - 1) : 0;
  if (device_bytes) {
    int64_t b = 0;
    for (int dir = 0; dir < 2; dir++) b += (c->tp[dir].nchunks * c->tp[dir].nslices + 1) * 8;
    if (c->loc == TSVD_LOC_DEVICE) b += c->nnz * 8 * 2 + c->nnz * 8 + (c->n + 1) * 8;
    else b += (int64_t)c->Q * c->slot_entries * 8;
    *device_bytes = b;
  }
  return TSVD_OK;
}

void tsvd_csr_destroy(tsvd_csr* c) {
  if (!c) return;
  hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(c->colptr);
  (void)hipFree(c->rowidx);
  (void)hipFree(c->cval);
  for (int dir = 0; dir < 2; dir++) {
    (void)hipFree(c->tptr[dir]);
    if (c->loc == TSVD_LOC_DEVICE) {
      (void)hipFree(c->tkey[dir]);
      (void)hipFree(c->tval[dir]);
    } else {
      (void)hipHostFree(c->tkey[dir]);
      (void)hipHostFree(c->tval[dir]);
    }
  }
  for (int q = 0; q < 16; q++) {
    (void)hipFree(c->skey[q]);
    (void)hipFree(c->sval[q]);
  }
  for (int q = 0; q < c->made; q++) {
    (void)hipEventDestroy(c->copied[q]);
    (void)hipEventDestroy(c->consumed[q]);
  }
  if (c->start_ev) (void)hipEventDestroy(c->start_ev);
  if (c->cs) (void)hipStreamDestroy(c->cs);
  delete c;
}

tsvd_status tsvd_csr_get_csc(tsvd_ctx* ctx, const tsvd_csr* c, int64_t* colptr, int32_t* rowidx, float* val,
                             void* stream) {
  if (!ctx) return TSVD_ERR_INVALID_ARG;
  if (!c || !colptr || (c->nnz > 0 && (!rowidx || !val))) return fail(ctx, TSVD_ERR_INVALID_ARG, "null pointer");
  if (!c->colptr) return fail(ctx, TSVD_ERR_UNSUPPORTED, "a pinned-host handle keeps no CSC copy");
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
  int rc = csr_product(const_cast<tsvd_csr*>(c), trans, x, x_dtype == TSVD_F64, y, nullptr, (hipStream_t)stream);
  return from_internal(ctx, rc, "spmv");
}

tsvd_status tsvd_sparse(tsvd_ctx* ctx, const tsvd_csr* cc, const tsvd_opts* o, double* U, int64_t ldu, double* S,
                        double* V, int64_t ldv, tsvd_info* info, void* stream_) {
  if (!ctx) return TSVD_ERR_INVALID_ARG;
  tsvd_csr* c = const_cast<tsvd_csr*>(cc);
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
  if (o->factor_loc != TSVD_LOC_DEVICE && o->factor_loc != TSVD_LOC_PINNED_HOST)
    return fail(ctx, TSVD_ERR_INVALID_ARG, "bad factor_loc");
  const bool host_x = o->factor_loc == TSVD_LOC_PINNED_HOST;
  const int Q = o->queue_depth > 0 ? o->queue_depth : 2;
  if (host_x && (Q > 16 || o->factor_batches < 0)) return fail(ctx, TSVD_ERR_INVALID_ARG, "queue_depth or factor_batches");
  hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream_;
  const bool right = right_side(m, n, o->branch);
  const int64_t d = right ? n : m, e = right ? m : n;
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
  const int64_t R = host_x ? HostFactor::round_rows(d, o->factor_batches > 0 ? o->factor_batches : 1) : 0;
  const int Qx = host_x ? (int)std::min<int64_t>(Q, (d + R - 1) / R) : 0;  // no more slots than batches
  const size_t slot_bytes = host_x ? align256((size_t)R * k * 8) : 0;
  const size_t need = loop_ws_bytes(d, k) + align256((size_t)e * 4) + align256((size_t)d * 8) + Qx * slot_bytes + 4096;
  tsvd_status st = ensure_ws(ctx, need, o->hbm_budget);
  if (st) return st;
  Bump bump(ctx->ws, ctx->ws_bytes);
  LoopWs lw = loop_ws_take(bump, d, k);
  float* tf = (float*)bump.take((size_t)e * 4);    // intermediate A x (or A^T x) in FP32
  double* tmp = (double*)bump.take((size_t)d * 8); // a factor column on its way to the finishing product
  double* slots[16];
  for (int q = 0; q < Qx; q++) slots[q] = (double*)bump.take(slot_bytes);

  SparseOp op(c, right, tf);
  DeviceFactor dfac(X, ldx, d);
  HostFactor hfac;
  if (host_x && hfac.init(X, ldx, d, R, Qx, k, slots, ctx->copy_stream))
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
  if (rc) return from_internal(ctx, rc, "sparse power iteration");
  if (r.nonfinite) return fail(ctx, TSVD_ERR_NONFINITE, "non-finite value in the sparse product");
  const int kdone = r.kdone;
  hipEventRecord(ctx->ev[2], s);
  // finish: W[:, j] = A X[:, j] (right) or A^T X[:, j] (left) with FP64 input,
  // sigma_j = ||W[:, j]||, then scale and sign convention
  if (host_x) {
    rc = finish_host_factor(op, X, ldx, d, W, ldw, e, S, kdone, right, tmp, lw.partial, s);
  } else {
    for (int j = 0; j < kdone && !rc; j++) {
      double* wj = W + (int64_t)j * ldw;
      rc = op.first(X + (int64_t)j * ldx, wj, s);
      if (!rc) rc = sumsq_launch(wj, e, lw.partial, S + j, s);
    }
    if (!rc && kdone > 0) rc = sqrt_inplace_launch(S, kdone, s);
    if (!rc && kdone > 0) rc = finish_scale_sign_launch(W, ldw, e, S, V, ldv, n, U, ldu, m, kdone, 1, lw.partial, s);
  }
  if (rc) return from_internal(ctx, rc, "sparse finish");
  hipEventRecord(ctx->ev[3], s);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(ctx, TSVD_ERR_HIP, "sync");
  if (info) {
    info->k_done = kdone;
    info->converged = r.all_conv ? 1 : 0;
    info->rank_deficient = r.rankdef ? 1 : 0;
    info->branch_right = right ? 1 : 0;
    if (info->iters) memcpy(info->iters, r.iters.data(), (size_t)k * 4);
    if (info->lambda) memcpy(info->lambda, r.lams.data(), (size_t)k * 8);
    float t;
    info->t_gram_ms = 0.0;
    hipEventElapsedTime(&t, ctx->ev[1], ctx->ev[2]); info->t_eig_ms = t;
    hipEventElapsedTime(&t, ctx->ev[2], ctx->ev[3]); info->t_final_ms = t;
    hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[3]); info->t_total_ms = t;
    info->workspace_bytes = (int64_t)need;
    info->h2d_bytes = op.h2d_bytes() + fac.h2d_bytes();
    info->latency_ms = 0;
    info->t_stream_copy_ms = 0;
    info->t_stream_compute_ms = 0;
    info->t_stream_overlap_ms = 0;
  }
  if (!r.all_conv && !o->fixed_iters && o->eps > 0)
    return fail(ctx, TSVD_ERR_NOT_CONVERGED, "some triplet reached max_iter");
  return TSVD_OK;
}

}  // extern "C"
