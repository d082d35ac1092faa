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
  size_t partial_bytes;
};
int syrk_plan(int mode, int64_t d, int64_t K, int64_t rows_per_block, int num_cu, SyrkPlan* p);
int syrk_launch(int mode, int side, const void* A, int64_t m, int64_t n, int64_t lda, const SyrkPlan& p,
                void* partial, void* B, int64_t ldb, int accumulate, hipStream_t stream);

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
};
struct PowerPlan {
  int G, rpb, cache_rows, ldsB, pw;
  size_t lds_bytes;
  size_t xex_words, pex_words, vex_words, wex_words;
};
enum { ERR_NONE = 0, ERR_SPIN = 1, ERR_NONFINITE = 2, ERR_BADSTART = 3 };
int power_plan(int dtype_bytes, int d, int k, int num_cu, size_t max_lds, int max_blocks_hint, PowerPlan* p);
int power_launch(int is_f64, const PowerPlan& p, PowerArgs a, hipStream_t stream);

// ---- finishing pass (finish.hip)
int finish_workspace_doubles(int64_t m, int64_t n, int side, int k);
int finish_launch(int is_f64, int side, const void* A, int64_t m, int64_t n, int64_t lda, const double* X,
                  int64_t ldx, int k, double* W, int64_t ldw, double* S, double* ssq, hipStream_t stream);
int finish_scale_sign_launch(double* W, int64_t ldw, int64_t Mw, const double* S, double* V, int64_t ldv, int64_t n,
                             double* U, int64_t ldu, int64_t m, int k, int do_sign, hipStream_t stream);

}  // namespace tsvd
