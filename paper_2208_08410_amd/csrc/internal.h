// Internal host-side interfaces between the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tsvd {

enum { MODE_FP64 = 0, MODE_FP32 = 1, MODE_BF16X3 = 2 };

// ---- Gram (syrk.hip)
struct SyrkPlan {
  int BM, nt, T, S, xcd_map;
  int64_t kchunk, partial_elems;
  size_t partial_bytes;   // workspace of the launch: partial tiles (+ the BF16 planes when packed)
  int packed;             // BF16X3, 256-wide tiles: split pass into k-packed planes, then direct-to-LDS tiles
  int64_t dp, Kp;         // packed: Gram dimension and contraction length padded (256, 32)
  size_t plane_off;       // packed: byte offset of the hi plane in the workspace
};
// packed_ok: the two-pass BF16X3 form may be chosen (A resident in HBM and
// room for 4 B per element of planes)
int syrk_plan(int mode, int64_t d, int64_t K, int64_t rows_per_block, int num_cu, SyrkPlan* p, int tile = 0,
              int chunks = 0, int packed_ok = 0);
int syrk_launch(int mode, int side, const void* A, int64_t m, int64_t n, int64_t lda, const SyrkPlan& p,
                void* partial, void* B, int64_t ldb, int accumulate, hipStream_t stream);

// one problem's Gram in the batched engine
struct GramJob {
  const void* A;
  int64_t m, n, lda;
  int side;              // 0: A^T A, 1: A A^T
  int nt, T, S;
  int64_t kchunk;
  int vec_ok;
  int mode;              // MODE_BF16X3 or MODE_FP32
  int bm, pad;           // triangle tile edge: 64 or 128
  void* partial;         // S * T * bm * bm floats
  void* B;               // d x d (ldb)
  int64_t ldb;
};


// ---- power iteration (power.hip)
struct PowerArgs {
  void* B;
  int64_t ldb;
  int d, k;
  double eps;
  int max_iter;
  const int* fixed_iters;   // device, k entries, or null
  const double* v0;         // device, k x d row-major
  double* X;                // device, d x k column-major
  int64_t ldx;
  double* lambda;           // device, k
  int* iters;               // device, k
  int* status;              // device: [0] k_done [1] all converged [2] error [3] rank deficient
  uint64_t* xex;            // 2 * dpad * WPE words
  uint64_t* pex;            // 2 * G * pw words
  uint64_t* vex;            // 2 * 2 * dpad words
  uint64_t* wex;            // 2 * 2 * dpad words
  int rpb, cache_rows, ldsB;
  int pw;                   // partial words per block (2 per double)
  int vec_ok;               // 16-byte loads allowed on B rows
  int64_t spin_limit;
  double* kscr;             // device, G * 2 * (k + 2) doubles (per-block scratch)
  int64_t xwords;           // words per parity of xex
  int64_t vstride;          // words per parity of vex / wex
};
struct PowerPlan {
  int G, rpb, cache_rows, ldsB, pw;
  size_t lds_bytes;
  size_t xex_words, pex_words, vex_words, wex_words;
};
enum { ERR_NONE = 0, ERR_SPIN = 1, ERR_NONFINITE = 2, ERR_BADSTART = 3 };
int power_plan(int dtype_bytes, int d, int k, int num_cu, size_t max_lds, int max_blocks_hint, PowerPlan* p);
int power_launch(int is_f64, const PowerPlan& p, PowerArgs a, hipStream_t stream);
// Batched engine (one persistent launch for a whole batch): an ordered list
// of work items, taken one per fetch in list order.  A problem's items are
// its Gram units (idx = chunk * T + tile of its GramJob), then its reductions
// (idx = triangle tile), then the G seats of its power team (idx = rank).
enum { ITEM_GRAM = 0, ITEM_REDUCE = 1, ITEM_POWER = 2 };
struct EngineItem {
  int type, p, idx, job;  // kind, problem, unit / tile / rank, the problem's GramJob
  int G, pad0, pad1, pad2;
};
// static LDS of the engine kernel (its dynamic LDS must leave room for it)
size_t engine_static_lds();
// ctr: 4 zeroed ints per problem (Gram units done, reductions done, seats
// taken) and then the list head; the launch zeroes [zero_base, zero_base +
// zero_words) first (ctr and the exchange buffers live there); grid
// workgroups, one per CU, all resident at once.  exit_flags (optional, grid
// ints in coherent pinned host memory): each workgroup stores exit_id into its
// entry when it leaves the launch
int engine_launch(const EngineItem* d_items, int nitems, const GramJob* d_jobs, const PowerArgs* d_probs, int* d_ctr,
                  int nprob, int grid, size_t lds_bytes, uint64_t* zero_base, size_t zero_words, hipStream_t stream,
                  int* exit_flags, int exit_id);


// ---- finishing pass (finish.hip)
// one problem of a grouped finishing pass (FP32 A); k = triplets found
struct FinishJob {
  const void* A;
  int64_t m, n, lda;
  int side, k;
  double* U;
  int64_t ldu;
  double* V;
  int64_t ldv;
  double* S;
  double* ssq;           // (nb + 2) * k: column sums per row tile, then 2 factors per column
  const int* kdone;      // device: triplets the power phase produced (columns to scale)
  int nb, pad;           // row tiles of the product
  int64_t ubegin;        // first workgroup in the product launch (nb * column blocks units)
  int64_t cbegin;        // first workgroup in the scale launch (k units)
};
// max_rows: the longest U or V column among the jobs (rows of the apply grid)
// zero fills (kernels, not runtime memsets)
int zero_cols_launch(double* p, int64_t ld, int64_t rows, int64_t cols, hipStream_t s);
int zero_bytes_launch(void* p, size_t bytes, hipStream_t s);
int finish_grouped_zero_launch(const FinishJob* d_jobs, int njobs, int64_t cols, hipStream_t s);
int finish_grouped_launch(int side, const FinishJob* d_jobs, int njobs, int64_t units, int64_t cols, int64_t max_rows,
                          hipStream_t s);
// row tiles of the finishing product; workspace = (tiles + 2) * k doubles:
// column sums of squares per tile, then the scale/sign factors
int64_t finish_tiles(int64_t m, int64_t n, int side);
int64_t finish_workspace_doubles(int64_t m, int64_t n, int side, int k);
int finish_gemm_launch(int is_f64, int side, const void* A, int64_t m, int64_t n, int64_t lda, const double* X,
                       int64_t ldx, int k, double* W, int64_t ldw, double* ssq, hipStream_t stream);
int finish_sigma_launch(const double* ssq, int64_t nb, int k, double* S, hipStream_t stream);
int finish_launch(int is_f64, int side, const void* A, int64_t m, int64_t n, int64_t lda, const double* X,
                  int64_t ldx, int k, double* W, int64_t ldw, double* S, double* ssq, hipStream_t stream);
// fac: 2k doubles of scratch
int finish_scale_sign_launch(double* W, int64_t ldw, int64_t Mw, const double* S, double* V, int64_t ldv, int64_t n,
                             double* U, int64_t ldu, int64_t m, int k, int do_sign, double* fac, hipStream_t stream);

// ---- sparse path (sparse.hip)
int csr_validate(const int64_t* rowptr, const int32_t* col, int64_t m, int64_t n, int64_t nnz, int* d_bad,
                 hipStream_t s);
size_t csc_build_scratch_bytes(int64_t n);
int csc_build(const int64_t* rowptr, const int32_t* col, const float* val, int64_t m, int64_t n, int64_t nnz,
              int64_t* colptr, int32_t* rowidx, float* cval, void* scratch, hipStream_t s);
// pieces of a batched CSC build (pinned-host matrices): column counts,
// scatter of one row batch's entries with columns in [j0, j1) into the
// sub-matrix's CSC, per-column sort by row, pointer rebasing and offsets
int csc_count_launch(const int32_t* col, int64_t nnz, unsigned long long* cnt, hipStream_t s);
int csc_fill_range_launch(const int64_t* rowptr, const int32_t* col, const float* val, int64_t rows, int64_t row0,
                          int64_t j0, int64_t j1, const int64_t* sub_ptr, unsigned long long* fill, int32_t* rowidx,
                          float* cval, hipStream_t s);
int csc_sort_launch(const int64_t* colptr, int64_t n, int32_t* rowidx, float* cval, hipStream_t s);
int rebase_launch(const int64_t* in, int64_t count, int64_t* out, hipStream_t s);
int offset_launch(const int64_t* in, int64_t count, int64_t add, int64_t* out, hipStream_t s);
// exclusive scan of n counts into out[0..n] (out[n] = total); bsum: (n + 1023) / 1024 + 1 entries
int scan_counts(const unsigned long long* cnt, int64_t n, unsigned long long* bsum, int64_t* out, int64_t total,
                hipStream_t s);

// ---- sliced tiles for the sparse products (tiles.hip)
struct TilePlan {
  int rbits, cbits;          // tile = 2^rbits rows x 2^cbits columns
  int64_t nchunks, nslices;  // row chunks, column slices
};
// rbits_hint / cbits_hint: 0 = library choice; returns -1 for an impossible request
int tiles_plan(int64_t rows, int64_t cols, int num_cu, int rbits_hint, int cbits_hint, TilePlan* t);
size_t tiles_scratch_bytes(const TilePlan& t);
// tptr: nchunks * nslices + 1 int64; key, tval: nnz each
int tiles_build(const int64_t* ptr, const int32_t* idx, const float* val, int64_t rows, int64_t nnz,
                const TilePlan& t, int64_t* tptr, uint32_t* key, float* tval, void* scratch, hipStream_t s);
// y = A x over row chunks [c0, c0 + nch); key / val hold the entries from
// tptr[c0 * nslices] on, whose absolute position is `base` (0 when the arrays
// hold the whole matrix)
int spmv_tiles_launch(const TilePlan& t, const int64_t* tptr, const uint32_t* key, const float* val, int64_t rows,
                      const void* x, int x_is_f64, double* y, float* yf, int64_t base, int64_t c0, int64_t nch,
                      hipStream_t s);
int64_t proj_blocks(int64_t d);
int proj_partials_launch(const double* V, int64_t ldv, int l, const double* w, const double* x, int64_t d,
                         double* partial, double* out, hipStream_t s);
int proj_apply_launch(const double* V, int64_t ldv, int l, const double* coef, double* w, int64_t d, double* partial,
                      double* out, hipStream_t s);
int sumsq_launch(const double* v, int64_t d, double* partial, double* out, hipStream_t s);
int normalize_launch(const double* z, int64_t d, double inv, double* x, float* xf, hipStream_t s);
int start_scale_launch(const double* v0, int64_t d, const double* ss, double* x, hipStream_t s);
int to_float_launch(const double* x, int64_t d, float* xf, hipStream_t s);
int sqrt_inplace_launch(double* v, int n, hipStream_t s);

}  // namespace tsvd
