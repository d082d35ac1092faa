// Mat-vec kernels and the host-driven power loop for the paths whose Gram is
// not held on chip (see implicit.h): the deflated product of Equation 2 /
// Algorithm 4 applied right to left, one FP64-accumulated mat-vec at a time.
//
// Dense products are HBM-bound streams over A (or over an explicit Gram B):
// y = A x gives one row per wave (16-byte loads, four in flight per lane, the
// row's sum reduced over the wave in a fixed order); y = A^T t cuts the rows
// into slabs, each thread owns four adjacent columns of a slab and walks its
// rows, and the slab partials are summed in slab order by a second kernel, so
// every result is deterministic.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "common.h"
#include "implicit.h"

namespace tsvd {

// ---------------------------------------------------------------------------
// dense mat-vec kernels
// ---------------------------------------------------------------------------

__device__ __forceinline__ void load4(const float* p, double (&o)[4]) {
  const float4 v = *(const float4*)p;
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void load4(const double* p, double (&o)[4]) {
  const double2 a = *(const double2*)p;
  const double2 b = *(const double2*)(p + 2);
  o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}

constexpr int GR_WAVES = 4;  // rows per 256-thread block

// y[row] = sum_j A[row, j] x[j]; VEC: lda % 4 == 0 and A, x 16-byte aligned
template <typename AT, typename XT, bool VEC>
__global__ __launch_bounds__(256) void gemv_rows_kernel(const AT* __restrict__ A, int64_t rows, int64_t n, int64_t lda,
                                                        const XT* __restrict__ x, double* __restrict__ y,
                                                        float* __restrict__ yf) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * GR_WAVES + (threadIdx.x >> 6);
  if (row >= rows) return;  // wave-uniform
  const AT* a = A + row * lda;
  double s = 0.0;
  if (VEC) {
    const int64_t n4 = n >> 2;
    int64_t c = lane;
    for (; c + 192 < n4; c += 256) {
      double av[4][4], xv[4][4];
#pragma unroll
      for (int u = 0; u < 4; u++) load4(a + 4 * (c + 64 * u), av[u]);
#pragma unroll
      for (int u = 0; u < 4; u++) load4(x + 4 * (c + 64 * u), xv[u]);
#pragma unroll
      for (int u = 0; u < 4; u++)
#pragma unroll
        for (int e = 0; e < 4; e++) s = fma(av[u][e], xv[u][e], s);
    }
    for (; c < n4; c += 64) {
      double av[4], xv[4];
      load4(a + 4 * c, av);
      load4(x + 4 * c, xv);
#pragma unroll
      for (int e = 0; e < 4; e++) s = fma(av[e], xv[e], s);
    }
    const int64_t j = 4 * n4 + lane;
    if (j < n) s = fma((double)a[j], (double)x[j], s);
  } else {
    for (int64_t j = lane; j < n; j += 64) s = fma((double)a[j], (double)x[j], s);
  }
  s = wave_sum(s);
  if (lane == 0) {
    if (y) y[row] = s;
    if (yf) yf[row] = (float)s;
  }
}

// partial[slab][j] = sum_{i in slab} A[i, j] t[i]; four adjacent columns per
// thread, rows of the slab in order (four rows' loads in flight)
template <typename AT, bool VEC>
__global__ __launch_bounds__(256) void gemv_cols_partial_kernel(const AT* __restrict__ A, int64_t rows, int64_t n,
                                                                int64_t lda, const double* __restrict__ t,
                                                                int64_t slab_rows, double* __restrict__ partial) {
  const int64_t j0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  const int64_t slab = blockIdx.y;
  const int64_t i0 = slab * slab_rows;
  const int64_t i1 = i0 + slab_rows < rows ? i0 + slab_rows : rows;
  if (j0 >= n) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (VEC && j0 + 3 < n) {
    int64_t i = i0;
    for (; i + 3 < i1; i += 4) {
      double av[4][4];
#pragma unroll
      for (int u = 0; u < 4; u++) load4(A + (i + u) * lda + j0, av[u]);
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const double ti = t[i + u];
#pragma unroll
        for (int e = 0; e < 4; e++) acc[e] = fma(av[u][e], ti, acc[e]);
      }
    }
    for (; i < i1; i++) {
      double av[4];
      load4(A + i * lda + j0, av);
      const double ti = t[i];
#pragma unroll
      for (int e = 0; e < 4; e++) acc[e] = fma(av[e], ti, acc[e]);
    }
  } else {
    for (int64_t i = i0; i < i1; i++) {
      const double ti = t[i];
#pragma unroll
      for (int e = 0; e < 4; e++)
        if (j0 + e < n) acc[e] = fma((double)A[i * lda + j0 + e], ti, acc[e]);
    }
  }
  double* out = partial + slab * n + j0;
#pragma unroll
  for (int e = 0; e < 4; e++)
    if (j0 + e < n) out[e] = acc[e];
}

// y[j] = sum over slabs s (in order) of partial[s][j]
__global__ __launch_bounds__(256) void reduce_slabs_kernel(const double* __restrict__ partial, int64_t slabs, int64_t n,
                                                           double* __restrict__ y, float* __restrict__ yf) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  int64_t q = 0;
  for (; q + 3 < slabs; q += 4) {
    const double p0 = partial[q * n + j], p1 = partial[(q + 1) * n + j];
    const double p2 = partial[(q + 2) * n + j], p3 = partial[(q + 3) * n + j];
    s += p0;
    s += p1;
    s += p2;
    s += p3;
  }
  for (; q < slabs; q++) s += partial[q * n + j];
  if (y) y[j] = s;
  if (yf) yf[j] = (float)s;
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

int gemv_rows_launch(int a_f64, const void* A, int64_t rows, int64_t n, int64_t lda, const void* x, int x_f64,
                     double* y, float* yf, hipStream_t s) {
  if (rows <= 0) return 0;
  const bool vec = (lda % 4 == 0) && aligned16(A) && aligned16(x);
  const dim3 grid((unsigned)((rows + GR_WAVES - 1) / GR_WAVES)), block(256);
#define TSVD_GR(AT, XT)                                                                                       \
  do {                                                                                                        \
    if (vec)                                                                                                  \
      hipLaunchKernelGGL((gemv_rows_kernel<AT, XT, true>), grid, block, 0, s, (const AT*)A, rows, n, lda,     \
                         (const XT*)x, y, yf);                                                                \
    else                                                                                                      \
      hipLaunchKernelGGL((gemv_rows_kernel<AT, XT, false>), grid, block, 0, s, (const AT*)A, rows, n, lda,    \
                         (const XT*)x, y, yf);                                                                \
  } while (0)
  if (a_f64) {
    if (x_f64) TSVD_GR(double, double);
    else TSVD_GR(double, float);
  } else {
    if (x_f64) TSVD_GR(float, double);
    else TSVD_GR(float, float);
  }
#undef TSVD_GR
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int64_t gemv_cols_slab_rows(int64_t rows, int64_t n) {
  const int64_t xb = (n + 1023) / 1024;      // column blocks of 256 threads x 4 columns
  const int64_t want = (4096 + xb - 1) / xb;  // about 4096 workgroups
  int64_t sr = (rows + want - 1) / want;
  if (sr < 64) sr = 64;
  return sr;
}

int64_t gemv_cols_slabs(int64_t rows, int64_t slab_rows) { return rows <= 0 ? 0 : (rows + slab_rows - 1) / slab_rows; }

int gemv_cols_partial_launch(int a_f64, const void* A, int64_t rows, int64_t n, int64_t lda, const double* t,
                             int64_t slab_rows, double* partial, hipStream_t s) {
  const int64_t slabs = gemv_cols_slabs(rows, slab_rows);
  if (slabs == 0) return 0;
  if (slabs > 65535) return TSVD_ERR_INTERNAL;
  const bool vec = (lda % 4 == 0) && aligned16(A);
  const dim3 grid((unsigned)((n + 1023) / 1024), (unsigned)slabs), block(256);
  if (a_f64) {
    if (vec)
      hipLaunchKernelGGL((gemv_cols_partial_kernel<double, true>), grid, block, 0, s, (const double*)A, rows, n, lda, t,
                         slab_rows, partial);
    else
      hipLaunchKernelGGL((gemv_cols_partial_kernel<double, false>), grid, block, 0, s, (const double*)A, rows, n, lda,
                         t, slab_rows, partial);
  } else {
    if (vec)
      hipLaunchKernelGGL((gemv_cols_partial_kernel<float, true>), grid, block, 0, s, (const float*)A, rows, n, lda, t,
                         slab_rows, partial);
    else
      hipLaunchKernelGGL((gemv_cols_partial_kernel<float, false>), grid, block, 0, s, (const float*)A, rows, n, lda, t,
                         slab_rows, partial);
  }
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int reduce_slabs_launch(const double* partial, int64_t slabs, int64_t n, double* y, float* yf, hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(reduce_slabs_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, partial, slabs, n, y, yf);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

// ---------------------------------------------------------------------------
// factor storage
// ---------------------------------------------------------------------------

int DeviceFactor::dots(int l, const double* w, const double* x, double* partial, double* coef, hipStream_t s) {
  return proj_partials_launch(X, ldx, l, w, x, d, partial, coef, s);
}

int DeviceFactor::subtract(int l, const double* coef, double* w, double* partial, double* out, hipStream_t s) {
  return proj_apply_launch(X, ldx, l, coef, w, d, partial, out, s);
}

int DeviceFactor::store(int l, double* x, double inv, hipStream_t s) {
  return normalize_launch(x, d, inv, X + (int64_t)l * ldx, nullptr, s);
}

int64_t HostFactor::round_rows(int64_t d, int64_t nb_wanted) {
  if (nb_wanted < 1) nb_wanted = 1;
  int64_t r = (d + nb_wanted - 1) / nb_wanted;
  r = (r + kProjRows - 1) / kProjRows * kProjRows;
  return r < kProjRows ? kProjRows : r;
}

int HostFactor::init(double* X_, int64_t ldx_, int64_t d_, int64_t R_, int Q_, int kcap_, double* const* slots,
                     hipStream_t cs_) {
  X = X_;
  ldx = ldx_;
  d = d_;
  R = R_;
  nbatch = (d + R - 1) / R;
  Q = Q_;
  kcap = kcap_;
  cs = cs_;
  for (int q = 0; q < Q; q++) {
    slot[q] = slots[q];
    slot_batch[q] = -1;
    slot_cols[q] = 0;
    slot_used[q] = false;
  }
  if (hipEventCreateWithFlags(&stored, hipEventDisableTiming) != hipSuccess) return TSVD_ERR_HIP;
  for (; made < Q; made++) {
    if (hipEventCreateWithFlags(&copied[made], hipEventDisableTiming) != hipSuccess) return TSVD_ERR_HIP;
    if (hipEventCreateWithFlags(&consumed[made], hipEventDisableTiming) != hipSuccess) {
      (void)hipEventDestroy(copied[made]);
      return TSVD_ERR_HIP;
    }
  }
  return 0;
}

HostFactor::~HostFactor() {
  if (cs) (void)hipStreamSynchronize(cs);
  for (int q = 0; q < made; q++) {
    (void)hipEventDestroy(copied[q]);
    (void)hipEventDestroy(consumed[q]);
  }
  if (stored) (void)hipEventDestroy(stored);
}

// make batch b's first l columns available in a slot; the compute stream s
// waits for the copy
int HostFactor::ensure(int64_t b, int l, hipStream_t s, int* slot_out) {
  const int q = (int)(b % Q);
  *slot_out = q;
  if (slot_batch[q] == b && slot_cols[q] >= l) return 0;  // resident (stream order covers the earlier copy)
  const int64_t r0 = b * R;
  const int64_t rows = std::min(R, d - r0);
  if (wait_stored) {
    TSVD_HIP_TRY(hipStreamWaitEvent(cs, stored, 0));
    wait_stored = false;
  }
  if (slot_used[q]) TSVD_HIP_TRY(hipStreamWaitEvent(cs, consumed[q], 0));
  TSVD_HIP_TRY(hipMemcpy2DAsync(slot[q], (size_t)R * 8, X + r0, (size_t)ldx * 8, (size_t)rows * 8, (size_t)l,
                                hipMemcpyHostToDevice, cs));
  TSVD_HIP_TRY(hipEventRecord(copied[q], cs));
  TSVD_HIP_TRY(hipStreamWaitEvent(s, copied[q], 0));
  slot_batch[q] = b;
  slot_cols[q] = l;
  h2d += rows * l * 8;
  return 0;
}

int HostFactor::dots(int l, const double* w, const double* x, double* partial, double* coef, hipStream_t s) {
  if (l == 0) return proj_partials_launch(nullptr, 1, 0, w, x, d, partial, coef, s);
  const int P = l + 2;
  for (int64_t b = 0; b < nbatch; b++) {
    int q;
    if (int rc = ensure(b, l, s, &q)) return rc;
    const int64_t r0 = b * R, rows = std::min(R, d - r0);
    if (int rc = proj_partials_part_launch(slot[q], R, l, w + r0, x + r0, rows, partial + (r0 / kProjRows) * P, s))
      return rc;
    TSVD_HIP_TRY(hipEventRecord(consumed[q], s));
    slot_used[q] = true;
  }
  return reduce_partials_launch(partial, proj_blocks(d), P, coef, s);
}

int HostFactor::subtract(int l, const double* coef, double* w, double* partial, double* out, hipStream_t s) {
  if (l == 0) return proj_apply_launch(nullptr, 1, 0, coef, w, d, partial, out, s);
  for (int64_t b = 0; b < nbatch; b++) {
    int q;
    if (int rc = ensure(b, l, s, &q)) return rc;
    const int64_t r0 = b * R, rows = std::min(R, d - r0);
    if (int rc = proj_apply_part_launch(slot[q], R, l, coef, w + r0, rows, partial + r0 / kProjRows, s)) return rc;
    TSVD_HIP_TRY(hipEventRecord(consumed[q], s));
    slot_used[q] = true;
  }
  return reduce_partials_launch(partial, proj_blocks(d), 1, out, s);
}

int HostFactor::store(int l, double* x, double inv, hipStream_t s) {
  if (int rc = normalize_launch(x, d, inv, x, nullptr, s)) return rc;
  TSVD_HIP_TRY(hipMemcpyAsync(X + (int64_t)l * ldx, x, (size_t)d * 8, hipMemcpyDeviceToHost, s));
  TSVD_HIP_TRY(hipEventRecord(stored, s));
  wait_stored = true;
  for (int q = 0; q < Q; q++) slot_batch[q] = -1;  // the next projection has one more column
  return 0;
}

// ---------------------------------------------------------------------------
// the power loop
// ---------------------------------------------------------------------------

size_t loop_ws_bytes(int64_t d, int k) {
  const int64_t nb = proj_blocks(d);
  return align256((size_t)d * 8) * 2 + align256((size_t)d * 4) +
         align256((size_t)std::max<int64_t>(nb * (k + 2), 2 * (int64_t)k + 2) * 8) + align256((size_t)(k + 8) * 8) * 2 +
         1024;
}

LoopWs loop_ws_take(Bump& b, int64_t d, int k) {
  LoopWs w;
  const int64_t nb = proj_blocks(d);
  w.x = (double*)b.take((size_t)d * 8);
  w.w = (double*)b.take((size_t)d * 8);
  w.xf = (float*)b.take((size_t)d * 4);
  w.partial = (double*)b.take((size_t)std::max<int64_t>(nb * (k + 2), 2 * (int64_t)k + 2) * 8);
  w.coef = (double*)b.take((size_t)(k + 8) * 8);
  w.scal = (double*)b.take((size_t)(k + 8) * 8);
  return w;
}

int implicit_power(ImplicitOp& op, Factor& fac, const tsvd_opts* o, int k, int64_t d, const LoopWs& ws,
                   PowerLoopResult* r, hipStream_t s) {
  double *x = ws.x, *w = ws.w, *partial = ws.partial, *coef = ws.coef, *scal = ws.scal;
  float* xf = ws.xf;
  const int max_iter = o->max_iter > 0 ? o->max_iter : 10000;
  r->kdone = k;
  r->iters.assign(k, 0);
  r->lams.assign(k, 0.0);
  int rc = 0;
  for (int l = 0; l < k; l++) {
    // start vector: x = v0_l / ||v0_l||, then x <- P x (projected once, not renormalised)
    const double* v0 = o->v0 + (int64_t)l * d;
    if ((rc = sumsq_launch(v0, d, partial, scal, s))) return rc;
    if ((rc = start_scale_launch(v0, d, scal, x, s))) return rc;
    if (l > 0) {
      if ((rc = fac.dots(l, x, x, partial, coef, s))) return rc;
      if ((rc = fac.subtract(l, coef, x, partial, scal + 1, s))) return rc;
    }
    if ((rc = to_float_launch(x, d, xf, s))) return rc;
    const int fixed = o->fixed_iters ? o->fixed_iters[l] : (o->eps <= 0.0 ? max_iter : 0);
    int it = 0;
    double nrm = 0.0;
    bool conv = false;
    while (true) {
      if ((rc = op.apply(x, xf, w, s))) return rc;
      it++;
      if ((rc = fac.dots(l, w, x, partial, coef, s))) return rc;
      if ((rc = fac.subtract(l, coef, w, partial, scal, s))) return rc;
      double h[2];
      TSVD_HIP_TRY(hipMemcpyAsync(&h[0], scal, 8, hipMemcpyDeviceToHost, s));
      TSVD_HIP_TRY(hipMemcpyAsync(&h[1], coef + l + 1, 8, hipMemcpyDeviceToHost, s));
      TSVD_HIP_TRY(hipStreamSynchronize(s));
      nrm = sqrt(h[0]);
      if (!std::isfinite(nrm)) {
        r->nonfinite = true;
        return 0;
      }
      if (nrm == 0.0) {
        r->rankdef = true;
        r->kdone = l;
        return 0;
      }
      bool stop;
      if (fixed > 0) {
        stop = it >= fixed;
        conv = true;
      } else {
        conv = fabs(h[1]) / nrm >= 1.0 - o->eps;
        stop = conv || it >= max_iter;
      }
      if ((rc = normalize_launch(w, d, 1.0 / nrm, x, xf, s))) return rc;
      if (stop) break;
    }
    if (!conv) r->all_conv = false;
    r->iters[l] = it;
    r->lams[l] = nrm;
    // FP64 re-orthogonalisation against the earlier columns, then column l
    if (l > 0) {
      if ((rc = fac.dots(l, x, x, partial, coef, s))) return rc;
      if ((rc = fac.subtract(l, coef, x, partial, scal, s))) return rc;
    } else if ((rc = sumsq_launch(x, d, partial, scal, s))) {
      return rc;
    }
    double hn;
    TSVD_HIP_TRY(hipMemcpyAsync(&hn, scal, 8, hipMemcpyDeviceToHost, s));
    TSVD_HIP_TRY(hipStreamSynchronize(s));
    if (!(hn > 0.0)) {
      r->rankdef = true;
      r->kdone = l;
      return 0;
    }
    if ((rc = fac.store(l, x, 1.0 / sqrt(hn), s))) return rc;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// operators
// ---------------------------------------------------------------------------

int GramOp::apply(const double* x, const float* xf, double* z, hipStream_t s) {
  return b_f64 ? gemv_rows_launch(1, B, d, d, ldb, x, 1, z, nullptr, s)
               : gemv_rows_launch(0, B, d, d, ldb, xf, 0, z, nullptr, s);
}

int finish_host_factor(ImplicitOp& op, double* Xh, int64_t ldx, int64_t d, double* W, int64_t ldw, int64_t e,
                       double* S, int kdone, bool right, double* tmp, double* partial, hipStream_t s) {
  for (int j = 0; j < kdone; j++) {
    double* wj = W + (int64_t)j * ldw;
    TSVD_HIP_TRY(hipMemcpyAsync(tmp, Xh + (int64_t)j * ldx, (size_t)d * 8, hipMemcpyHostToDevice, s));
    if (int rc = op.first(tmp, wj, s)) return rc;
    if (int rc = sumsq_launch(wj, e, partial, S + j, s)) return rc;
    if (int rc = sqrt_inplace_launch(S + j, 1, s)) return rc;
    // one column: W aliases U (right) or V (left); the factor's column is tmp
    int rc = right ? finish_scale_sign_launch(wj, ldw, e, S + j, tmp, d, d, wj, ldw, e, 1, 1, partial + 4, s)
                   : finish_scale_sign_launch(wj, ldw, e, S + j, wj, ldw, e, tmp, d, d, 1, 1, partial + 4, s);
    if (rc) return rc;
    TSVD_HIP_TRY(hipMemcpyAsync(Xh + (int64_t)j * ldx, tmp, (size_t)d * 8, hipMemcpyDeviceToHost, s));
  }
  return 0;
}

int64_t DenseOp::ws_doubles(int64_t m, int64_t n) {
  const int64_t sr = gemv_cols_slab_rows(m, n);
  const int64_t mx = m > n ? m : n;
  return gemv_cols_slabs(m, sr) * n + 2 * mx + 64;
}

void DenseOp::setup(const void* A_, int a_f64_, int64_t m_, int64_t n_, int64_t lda_, bool right_, double* ws) {
  A = A_;
  a_f64 = a_f64_;
  m = m_;
  n = n_;
  lda = lda_;
  right = right_;
  slab_rows = gemv_cols_slab_rows(m, n);
  slabs = gemv_cols_slabs(m, slab_rows);
  part = ws;
  t = part + slabs * n;
  tf = (float*)(t + (m > n ? m : n));
}

int DenseOp::apply(const double* x, const float* xf, double* z, hipStream_t s) {
  if (right) {  // t = A x, z = A^T t
    if (int rc = gemv_rows_launch(a_f64, A, m, n, lda, a_f64 ? (const void*)x : (const void*)xf, a_f64, t, nullptr, s))
      return rc;
    if (int rc = gemv_cols_partial_launch(a_f64, A, m, n, lda, t, slab_rows, part, s)) return rc;
    return reduce_slabs_launch(part, slabs, n, z, nullptr, s);
  }
  // left: t = A^T x, z = A t
  if (int rc = gemv_cols_partial_launch(a_f64, A, m, n, lda, x, slab_rows, part, s)) return rc;
  if (int rc = reduce_slabs_launch(part, slabs, n, t, a_f64 ? nullptr : tf, s)) return rc;
  return gemv_rows_launch(a_f64, A, m, n, lda, a_f64 ? (const void*)t : (const void*)tf, a_f64, z, nullptr, s);
}

int DenseOp::first(const double* x, double* w, hipStream_t s) {
  if (right) return gemv_rows_launch(a_f64, A, m, n, lda, x, 1, w, nullptr, s);
  if (int rc = gemv_cols_partial_launch(a_f64, A, m, n, lda, x, slab_rows, part, s)) return rc;
  return reduce_slabs_launch(part, slabs, n, w, nullptr, s);
}

int64_t PinnedDenseOp::ws_doubles(int64_t m, int64_t n, int64_t R, bool right) {
  if (!right) {
    const int64_t nb = (n + R - 1) / R;
    const int64_t sl = gemv_cols_slabs(m, gemv_cols_slab_rows(m, R));
    return sl * R + R + nb * m + 64;
  }
  const int64_t nb = (m + R - 1) / R;
  const int64_t sr = gemv_cols_slab_rows(R, n);
  int64_t slabs = 0;
  for (int64_t b = 0; b < nb; b++) slabs += gemv_cols_slabs(std::min(R, m - b * R), sr);
  return slabs * n + m + 64;
}

int PinnedDenseOp::init(const float* A_, int64_t m_, int64_t n_, int64_t lda_, int64_t R_, int Q_, float* const* bufs,
                        double* ws, hipStream_t cs_, bool right_) {
  A = A_;
  m = m_;
  n = n_;
  lda = lda_;
  R = R_;
  right = right_;
  nbatch = right ? (m + R - 1) / R : (n + R - 1) / R;
  Q = Q_;
  cs = cs_;
  for (int q = 0; q < Q; q++) buf[q] = bufs[q];
  if (right) {
    slab_rows = gemv_cols_slab_rows(R, n);
    slabs = 0;
    for (int64_t b = 0; b < nbatch; b++) slabs += gemv_cols_slabs(std::min(R, m - b * R), slab_rows);
    part = ws;
    t = part + slabs * n;
  } else {
    // one batch's A_c^T x in slabs of the m rows, then A_c t_c per batch
    slab_rows = gemv_cols_slab_rows(m, R);
    slabs = gemv_cols_slabs(m, slab_rows);
    part = ws;
    t = part + slabs * R;
    zpart = t + R;
  }
  if (hipEventCreateWithFlags(&start_ev, hipEventDisableTiming) != hipSuccess) return TSVD_ERR_HIP;
  have_start = true;
  for (; made < Q; made++) {
    if (hipEventCreateWithFlags(&copied[made], hipEventDisableTiming) != hipSuccess) return TSVD_ERR_HIP;
    if (hipEventCreateWithFlags(&consumed[made], hipEventDisableTiming) != hipSuccess) {
      (void)hipEventDestroy(copied[made]);
      return TSVD_ERR_HIP;
    }
    used[made] = false;
  }
  return 0;
}

PinnedDenseOp::~PinnedDenseOp() {
  if (cs) (void)hipStreamSynchronize(cs);
  for (int q = 0; q < made; q++) {
    (void)hipEventDestroy(copied[q]);
    (void)hipEventDestroy(consumed[q]);
  }
  if (have_start) (void)hipEventDestroy(start_ev);
}

// batch [r0, r0 + len) of rows (right) or columns (left) into slot q on the
// copy stream, once the slot's previous batch is consumed; `s` waits for it
int PinnedDenseOp::copy_batch(int64_t r0, int64_t len, int q, hipStream_t s) {
  if (used[q]) TSVD_HIP_TRY(hipStreamWaitEvent(cs, consumed[q], 0));
  if (right)
    TSVD_HIP_TRY(hipMemcpy2DAsync(buf[q], (size_t)n * 4, A + r0 * lda, (size_t)lda * 4, (size_t)n * 4, (size_t)len,
                                  hipMemcpyHostToDevice, cs));
  else
    TSVD_HIP_TRY(hipMemcpy2DAsync(buf[q], (size_t)len * 4, A + r0, (size_t)lda * 4, (size_t)len * 4, (size_t)m,
                                  hipMemcpyHostToDevice, cs));
  TSVD_HIP_TRY(hipEventRecord(copied[q], cs));
  TSVD_HIP_TRY(hipStreamWaitEvent(s, copied[q], 0));
  return 0;
}

// one pass over A per product: batch b is copied into slot b % Q while the
// previous batch computes its contribution (right: t_b = A_b x and its slabs
// of A_b^T t_b; left: t_c = A_c^T x, then A_c t_c)
int PinnedDenseOp::apply(const double* x, const float* xf, double* z, hipStream_t s) {
  TSVD_HIP_TRY(hipEventRecord(start_ev, s));  // x is ready: the copies may start
  TSVD_HIP_TRY(hipStreamWaitEvent(cs, start_ev, 0));
  int64_t slab0 = 0;
  for (int64_t b = 0; b < nbatch; b++) {
    const int q = (int)(b % Q);
    const int64_t r0 = b * R, len = std::min(R, (right ? m : n) - r0);
    if (int rc = copy_batch(r0, len, q, s)) return rc;
    if (right) {
      if (int rc = gemv_rows_launch(0, buf[q], len, n, n, xf, 0, t + r0, nullptr, s)) return rc;
      if (int rc = gemv_cols_partial_launch(0, buf[q], len, n, n, t + r0, slab_rows, part + slab0 * n, s)) return rc;
      slab0 += gemv_cols_slabs(len, slab_rows);
    } else {
      if (int rc = gemv_cols_partial_launch(0, buf[q], m, len, len, x, slab_rows, part, s)) return rc;
      if (int rc = reduce_slabs_launch(part, slabs, len, t, nullptr, s)) return rc;
      if (int rc = gemv_rows_launch(0, buf[q], m, len, len, t, 1, zpart + b * m, nullptr, s)) return rc;
    }
    TSVD_HIP_TRY(hipEventRecord(consumed[q], s));
    used[q] = true;
    h2d += len * (right ? n : m) * 4;
  }
  return right ? reduce_slabs_launch(part, slabs, n, z, nullptr, s) : reduce_slabs_launch(zpart, nbatch, m, z, nullptr, s);
}

int PinnedDenseOp::finish(const double* X, int64_t ldx, int kd, double* W, int64_t ldw, double* ssq, int64_t* tiles,
                          hipStream_t s) {
  TSVD_HIP_TRY(hipEventRecord(start_ev, s));
  TSVD_HIP_TRY(hipStreamWaitEvent(cs, start_ev, 0));
  int64_t tile_off = 0;
  for (int64_t b = 0; b < nbatch; b++) {
    const int q = (int)(b % Q);
    const int64_t r0 = b * R, len = std::min(R, (right ? m : n) - r0);
    if (int rc = copy_batch(r0, len, q, s)) return rc;
    // the batch's rows of W: rows r0.. of U = A V, or of V = A^T U
    const int rc = right ? finish_gemm_launch(0, 0, buf[q], len, n, n, X, ldx, kd, W + r0, ldw, ssq + tile_off * kd, s)
                         : finish_gemm_launch(0, 1, buf[q], m, len, len, X, ldx, kd, W + r0, ldw, ssq + tile_off * kd, s);
    if (rc) return rc;
    TSVD_HIP_TRY(hipEventRecord(consumed[q], s));
    used[q] = true;
    tile_off += (len + 127) / 128;
    h2d += len * (right ? n : m) * 4;
  }
  *tiles = tile_off;
  return 0;
}

}  // namespace tsvd
