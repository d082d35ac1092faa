// Host-driven power iteration with the deflated product applied as
// mat-vecs (Equation 2 in factored form, Algorithm 4), shared by every path
// whose Gram is not held on chip: sparse A (CSR tiles in HBM or streamed from
// pinned host memory), dense A applied implicitly (A^T (A x), when the Gram is
// too large to form), and a Gram in HBM too large for the on-chip power
// kernel.  The iterated factor X (V on the right branch, U on the left) lives
// on the device or in pinned host memory, where it is batched to the device
// for every projection (the paper's out-of-memory handling of the heavy
// co-factor, Sec. V-C).
#pragma once

#include <vector>

#include "ctx.h"
#include "internal.h"

namespace tsvd {

// z = B x for the undeflated symmetric operator of Algorithm 2 (B = A^T A on
// the right branch, A A^T on the left, or an explicit Gram).  x is the unit
// iterate in FP64 and its FP32 copy; z is FP64.
struct ImplicitOp {
  virtual ~ImplicitOp() {}
  virtual int apply(const double* x, const float* xf, double* z, hipStream_t s) = 0;
  // the finishing product of one FP64 column: w = A x (right branch) or
  // A^T x (left), FP64 (operators over an explicit Gram have none)
  virtual int first(const double* x, double* w, hipStream_t s) { return TSVD_ERR_UNSUPPORTED; }
  virtual int64_t h2d_bytes() const { return 0; }
};

// The iterated factor X (d x k, FP64, column-major) and the projection
// P = I - X_l X_l^T against its first l columns (Algorithm 1's deflation,
// read as a projection).
struct Factor {
  virtual ~Factor() {}
  // coef[j] = X[:, j] . w for j < l, coef[l] = w . w, coef[l + 1] = x . w
  virtual int dots(int l, const double* w, const double* x, double* partial, double* coef, hipStream_t s) = 0;
  // w -= X[:, :l] coef[:l]; out[0] = w . w afterwards
  virtual int subtract(int l, const double* coef, double* w, double* partial, double* out, hipStream_t s) = 0;
  // X[:, l] = x * inv (x may be scaled in place)
  virtual int store(int l, double* x, double inv, hipStream_t s) = 0;
  virtual int64_t h2d_bytes() const { return 0; }
};

// X in HBM (ldx >= d)
struct DeviceFactor : Factor {
  double* X;
  int64_t ldx, d;
  DeviceFactor(double* X_, int64_t ldx_, int64_t d_) : X(X_), ldx(ldx_), d(d_) {}
  int dots(int l, const double* w, const double* x, double* partial, double* coef, hipStream_t s) override;
  int subtract(int l, const double* coef, double* w, double* partial, double* out, hipStream_t s) override;
  int store(int l, double* x, double inv, hipStream_t s) override;
};

// X in pinned host memory.  Its rows are cut into batches of R rows (R a
// multiple of the projection kernels' 4096-row block, so every block sees the
// same rows as on the device and the sums are bitwise those of DeviceFactor);
// each projection pass copies batch b into device slot b % Q on the copy
// stream while the compute stream works on the previous slot, and events
// order the reuse of a slot.  While a triplet runs X does not change, so when
// every batch has its own slot (batches <= Q) each batch is copied once per
// triplet and then stays resident.
struct HostFactor : Factor {
  double* X;           // pinned host
  int64_t ldx, d;
  int64_t R;           // rows per batch
  int64_t nbatch;
  int Q;
  int kcap;            // columns a slot holds
  double* slot[16];    // device, R x kcap each (column stride R)
  hipStream_t cs = nullptr;
  hipEvent_t copied[16], consumed[16], stored = nullptr;
  int64_t slot_batch[16];
  int slot_cols[16];
  bool slot_used[16];
  bool wait_stored = false;
  int64_t h2d = 0;
  int made = 0;
  HostFactor() {}
  ~HostFactor() override;
  // rows_per_batch: R before rounding; returns 0 or TSVD_ERR_HIP
  int init(double* X_, int64_t ldx_, int64_t d_, int64_t R_, int Q_, int kcap_, double* const* slots, hipStream_t cs_);
  static int64_t round_rows(int64_t d, int64_t nb_wanted);
  int dots(int l, const double* w, const double* x, double* partial, double* coef, hipStream_t s) override;
  int subtract(int l, const double* coef, double* w, double* partial, double* out, hipStream_t s) override;
  int store(int l, double* x, double inv, hipStream_t s) override;
  int64_t h2d_bytes() const override { return h2d; }

 private:
  int ensure(int64_t b, int l, hipStream_t s, int* slot_out);
};

// z = B x with B an explicit d x d Gram in HBM (FP32 or FP64, row-major ldb):
// one HBM-bound stream over B per iteration, for Grams whose iterate does not
// fit the on-chip power kernel
struct GramOp : ImplicitOp {
  const void* B = nullptr;
  int b_f64 = 0;
  int64_t d = 0, ldb = 0;
  int apply(const double* x, const float* xf, double* z, hipStream_t s) override;
};

// z = A^T (A x) (right) or A (A^T x) (left) for a dense A in HBM: the Gram is
// never formed (the dense reading of Equation 2's right-to-left evaluation,
// for n too large to hold B)
struct DenseOp : ImplicitOp {
  const void* A = nullptr;
  int a_f64 = 0;
  int64_t m = 0, n = 0, lda = 0;
  bool right = true;
  // right: slabs of every row batch, side by side (n wide); left: slabs of
  // the m rows of one column batch (R wide), reused batch after batch
  int64_t slab_rows = 0, slabs = 0;
  double* part = nullptr;  // slabs x n
  double* t = nullptr;     // max(m, n)
  float* tf = nullptr;     // max(m, n) floats
  static int64_t ws_doubles(int64_t m, int64_t n);
  void setup(const void* A, int a_f64, int64_t m, int64_t n, int64_t lda, bool right, double* ws);
  int apply(const double* x, const float* xf, double* z, hipStream_t s) override;
  int first(const double* x, double* w, hipStream_t s) override;
};

// The same product for an FP32 A in pinned host memory (right branch): every
// product streams A once, in row batches through Q device buffers (batch b on
// the copy stream while the previous batch computes t_b = A_b x and its share
// of A_b^T t_b), so the host link bounds it (the paper's degree-1 dense case,
// the time/memory trade-off of Sec. IV's implicit product)
// A in pinned host memory, streamed once per product through Q device
// buffers: row batches A_b for the right branch (z = sum_b A_b^T (A_b x)),
// pitched column batches A_c for the left branch (z = sum_c A_c (A_c^T x)),
// the batches' contributions added in batch order.
struct PinnedDenseOp : ImplicitOp {
  const float* A = nullptr;
  int64_t m = 0, n = 0, lda = 0, R = 0, nbatch = 0;
  bool right = true;       // row batches (A^T A branch) or column batches (A A^T branch)
  int Q = 0;
  float* buf[16];
  hipStream_t cs = nullptr;
  hipEvent_t copied[16], consumed[16], start_ev;
  bool used[16];
  bool have_start = false;
  int made = 0;
  // right: slabs of every row batch, side by side (n wide); left: slabs of
  // the m rows of one column batch (R wide), reused batch after batch
  int64_t slab_rows = 0, slabs = 0;
  double* part = nullptr;
  double* t = nullptr;      // right: m (A x); left: R (one batch's A_c^T x)
  double* zpart = nullptr;  // left: nbatch x m (each batch's A_c t_c)
  int64_t h2d = 0;
  ~PinnedDenseOp() override;
  // R: rows (right) or columns (left) per batch
  static int64_t ws_doubles(int64_t m, int64_t n, int64_t R, bool right);
  int init(const float* A, int64_t m, int64_t n, int64_t lda, int64_t R, int Q, float* const* bufs, double* ws,
           hipStream_t cs, bool right);
  int apply(const double* x, const float* xf, double* z, hipStream_t s) override;
  // Algorithm 1's finishing product for all kd columns at once, one more pass
  // over A: W = A X (right: U = A V) or W = A^T X (left: V = A^T U), FP64,
  // with column sums of squares per 128-row tile of W in ssq; *tiles = the
  // tile count
  int finish(const double* X, int64_t ldx, int kd, double* W, int64_t ldw, double* ssq, int64_t* tiles, hipStream_t s);
  int64_t h2d_bytes() const override { return h2d; }
  int copy_batch(int64_t r0, int64_t len, int q, hipStream_t s);
};

// device workspace of implicit_power
struct LoopWs {
  double *x, *w;
  float* xf;
  double *partial, *coef, *scal;
};
size_t loop_ws_bytes(int64_t d, int k);
LoopWs loop_ws_take(Bump& b, int64_t d, int k);

struct PowerLoopResult {
  int kdone = 0;
  bool all_conv = true;
  bool rankdef = false;
  bool nonfinite = false;
  std::vector<int> iters;
  std::vector<double> lams;
};

// Algorithm 1's loop over triplets with Algorithm 2 on P B P for each:
// start x = P (v0_l / ||v0_l||); repeat w = P op(x), x = w / ||w|| until
// |x_old . x| >= 1 - eps (FP64; eps <= 0: max_iter iterations; fixed_iters:
// exactly that many); then x is re-orthogonalised in FP64 and stored as
// column l.  A zero product stops the run (rank deficiency).  Workspace (all
// device): x, w FP64 d; xf FP32 d; partial max(proj_blocks(d) (k + 2), 2k);
// coef, scal k + 8 each.  One small device-to-host read per iteration.
int implicit_power(ImplicitOp& op, Factor& fac, const tsvd_opts* o, int k, int64_t d, const LoopWs& ws,
                   PowerLoopResult* r, hipStream_t s);

// Algorithm 1's finishing step for a factor in pinned host memory, one column
// at a time: x_j is copied to `tmp` (d doubles), w_j = op.first(x_j) into W's
// column, S[j] = ||w_j||, then w_j /= S[j] and the sign convention is applied
// to w_j and x_j, and x_j is copied back.  W: DEVICE (ldw, e rows).
int finish_host_factor(ImplicitOp& op, double* Xh, int64_t ldx, int64_t d, double* W, int64_t ldw, int64_t e,
                       double* S, int kdone, bool right, double* tmp, double* partial, hipStream_t s);

// ---- dense mat-vec kernels (implicit.hip) --------------------------------
// y = A x for row-major A (rows x n, lda), FP64 accumulation; A FP32 or FP64,
// x FP32 or FP64; y FP64 and/or yf FP32 (either may be null)
int gemv_rows_launch(int a_f64, const void* A, int64_t rows, int64_t n, int64_t lda, const void* x, int x_f64,
                     double* y, float* yf, hipStream_t s);
// rows per slab of the transposed product (slab partials are summed in slab order)
int64_t gemv_cols_slab_rows(int64_t rows, int64_t n);
int64_t gemv_cols_slabs(int64_t rows, int64_t slab_rows);
// partial[s][j] = sum over the rows i of slab s of A[i, j] t[i] (partial: slabs x n FP64)
int gemv_cols_partial_launch(int a_f64, const void* A, int64_t rows, int64_t n, int64_t lda, const double* t,
                             int64_t slab_rows, double* partial, hipStream_t s);
// y[j] = sum_s partial[s][j] in slab order (y FP64 and/or yf FP32)
int reduce_slabs_launch(const double* partial, int64_t slabs, int64_t n, double* y, float* yf, hipStream_t s);

// projection pieces over a contiguous run of 4096-row blocks (sparse.hip):
// write block partials without the final reduction
int proj_partials_part_launch(const double* V, int64_t ldv, int l, const double* w, const double* x, int64_t rows,
                              double* partial, hipStream_t s);
int proj_apply_part_launch(const double* V, int64_t ldv, int l, const double* coef, double* w, int64_t rows,
                           double* partial, hipStream_t s);
int reduce_partials_launch(const double* partial, int64_t nb, int P, double* out, hipStream_t s);
constexpr int64_t kProjRows = 4096;

}  // namespace tsvd
