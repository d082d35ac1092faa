// Power iteration with deflation on a symmetric Gram matrix (Algorithm 2, run
// once per triplet as Algorithm 1 does), as ONE persistent cooperative launch.
//
// Layout: workgroup b owns the contiguous rows R_b of B (rpb rows).  The first
// cache_rows of them are kept in LDS for the whole launch; the rest are read
// from HBM/L2 every iteration.  Every workgroup keeps a copy of the current
// iterate x (the GEMV input) in LDS.
//
// One iteration of Algorithm 2 (v1 = B v0; v1 /= ||v1||; stop if
// |v0 . v1| >= 1 - eps):
//   y_R = B[R, :] x                      (FP64 accumulation)
//   publish y_R and the block partials  q_b = sum y_i^2, d_b = sum x_i y_i
//   gather every block's partials       -> ||y||^2, x . y  (fixed order: every
//                                          block takes the same decision)
//   gather y                            -> x = y / ||y|| for the next product
// Data and synchronisation travel together in tagged 64-bit words (see
// common.h), so an iteration costs one exchange and no grid barrier.
//
// Deflation (Algorithm 1 forms X = A - U S V^T and its Gram again for every
// triplet; Equations 1-3 expand that Gram).  With u_j sigma_j = A v_j the
// deflated Gram is exactly (I - V V^T) B (I - V V^T).  Here it is kept
// explicitly: after triplet l converges to v,
//   v <- v - V (V^T v), v <- v / ||v||        (FP64 re-orthogonalisation)
//   w = B v, alpha = v . w
//   B <- B - v w^T - w v^T + alpha v v^T     (= (I - v v^T) B (I - v v^T))
// The update is done in FP64 arithmetic on each workgroup's own rows (LDS or
// HBM) and rounded once to B's storage type.
#include <math.h>

#include "common.h"
#include "internal.h"

namespace tsvd {

template <typename BT> struct VecOf;
template <> struct VecOf<float> { static constexpr int N = 4; };
template <> struct VecOf<double> { static constexpr int N = 2; };

template <typename BT>
__device__ __forceinline__ void load_vec(const BT* p, double (&v)[VecOf<BT>::N]);
template <>
__device__ __forceinline__ void load_vec<float>(const float* p, double (&v)[4]) {
  float4 f = *(const float4*)p;
  v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
}
template <>
__device__ __forceinline__ void load_vec<double>(const double* p, double (&v)[2]) {
  double2 f = *(const double2*)p;
  v[0] = f.x; v[1] = f.y;
}

// y[li] = B row li . x for rows li in [begin, end) of one storage (LDS or HBM).
// Wave w takes rows begin + 16 g + 4 w + q, q < 4, processing 4 rows per pass so
// each x chunk read from LDS feeds 4 rows.
template <typename BT>
__device__ void gemv_range(const BT* rows, int64_t stride, int begin, int end, const BT* xs, int d, bool vec_ok,
                           double* yout) {
  constexpr int VN = VecOf<BT>::N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int dv = vec_ok ? (d / VN) * VN : 0;
  for (int g0 = begin; g0 < end; g0 += 16) {
    const int li0 = g0 + wave * 4;
    if (li0 >= end) continue;
    const int nr = min(4, end - li0);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const BT* rp[4];
#pragma unroll
    for (int q = 0; q < 4; q++) rp[q] = rows + (int64_t)(li0 + (q < nr ? q : 0)) * stride;
#pragma unroll 2
    for (int c = lane * VN; c < dv; c += 64 * VN) {
      double xv[VN];
      load_vec<BT>(xs + c, xv);
#pragma unroll
      for (int q = 0; q < 4; q++) {
        if (q < nr) {
          double bv[VN];
          load_vec<BT>(rp[q] + c, bv);
#pragma unroll
          for (int e = 0; e < VN; e++) acc[q] = fma(bv[e], xv[e], acc[q]);
        }
      }
    }
    for (int c = dv + lane; c < d; c += 64) {
      const double xv = (double)xs[c];
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (q < nr) acc[q] = fma((double)rp[q][c], xv, acc[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
      double s = wave_sum(acc[q]);
      if (lane == 0 && q < nr) yout[li0 + q] = s;
    }
  }
}

template <typename BT>
__device__ __forceinline__ void gemv_own(const PowerArgs& a, const BT* Bs, const BT* Bg, int nrows, const BT* xs,
                                         double* yout) {
  const int cr = min(a.cache_rows, nrows);
  gemv_range<BT>(Bs, a.ldsB, 0, cr, xs, a.d, true, yout);
  gemv_range<BT>(Bg + (int64_t)cr * a.ldb, a.ldb, 0, nrows - cr, xs, a.d, a.vec_ok != 0, yout + cr);
}

// Sum vals[0..P) over all G workgroups (published in the partial buffer under
// epoch ex); out[0..P) receives the totals, identical in every workgroup.
// Returns false (uniformly in the block) if a wait ran out of budget.
__device__ bool allreduce_blocks(uint64_t* pbuf, int pw, int G, uint32_t ex, const double* vals, int P, double* out,
                                 double* scratch, int* flag, int64_t spin_limit) {
  const int tid = threadIdx.x, b = blockIdx.x;
  for (int j = tid; j < P; j += 256) ll_store_f64(pbuf + (int64_t)b * pw + 2 * j, ex, vals[j]);
  if (tid == 0) *flag = 1;
  __syncthreads();
  for (int jb = 0; jb < P; jb += 256) {
    const int Pc = min(256, P - jb);
    const int NG = 256 / Pc;
    const int j = tid % Pc, gg = tid / Pc;
    double acc = 0.0;
    bool ok = true;
    if (gg < NG) {
      int64_t budget = spin_limit;
      for (int g0 = gg; g0 < G && ok; g0 += NG * 8) {
        uint64_t lo[8], hi[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
          const int g = g0 + NG * u;
          if (g < G) {
            const uint64_t* p = pbuf + (int64_t)g * pw + 2 * (jb + j);
            lo[u] = ll_load(p);
            hi[u] = ll_load(p + 1);
          } else {
            lo[u] = hi[u] = ((uint64_t)ex << 32);
          }
        }
        while (true) {
          bool all = true;
#pragma unroll
          for (int u = 0; u < 8; u++)
            all = all && ((uint32_t)(lo[u] >> 32) == ex) && ((uint32_t)(hi[u] >> 32) == ex);
          if (all) break;
          if (--budget <= 0) { ok = false; break; }
          __builtin_amdgcn_s_sleep(1);
#pragma unroll
          for (int u = 0; u < 8; u++) {
            const int g = g0 + NG * u;
            if (g < G) {
              const uint64_t* p = pbuf + (int64_t)g * pw + 2 * (jb + j);
              if ((uint32_t)(lo[u] >> 32) != ex) lo[u] = ll_load(p);
              if ((uint32_t)(hi[u] >> 32) != ex) hi[u] = ll_load(p + 1);
            }
          }
        }
        if (ok) {
#pragma unroll
          for (int u = 0; u < 8; u++)
            if (g0 + NG * u < G) acc += ll_join_f64(lo[u], hi[u]);
        }
      }
      scratch[gg * Pc + j] = acc;
    }
    if (!ok) *flag = 0;
    __syncthreads();
    if (tid < Pc) {
      double s = 0.0;
      for (int g = 0; g < NG; g++) s += scratch[g * Pc + tid];
      out[jb + tid] = s;
    }
    __syncthreads();
  }
  const bool res = *flag != 0;
  __syncthreads();
  return res;
}

// Publish own rows of a vector (FP64 values in `own`, rows r0..r0+nrows) as
// words of type BT (1 word per float, 2 per double).
template <typename BT>
__device__ __forceinline__ void publish_vec(uint64_t* buf, uint32_t ex, int r0, int nrows, const double* own,
                                            double scale) {
  for (int i = threadIdx.x; i < nrows; i += 256) {
    const double v = own[i] * scale;
    if constexpr (sizeof(BT) == 4) {
      ll_store(buf + (r0 + i), ex, __float_as_uint((float)v));
    } else {
      ll_store_f64(buf + 2 * (int64_t)(r0 + i), ex, v);
    }
  }
}

// Gather a published BT vector of length d into LDS dst (as BT), multiplying by
// scale.  Returns false (block-uniform) on a timed-out wait.
template <typename BT>
__device__ bool gather_vec(const uint64_t* buf, uint32_t ex, int d, BT* dst, double scale, int* flag,
                           int64_t spin_limit) {
  constexpr int WPE = sizeof(BT) / 4;
  if (threadIdx.x == 0) *flag = 1;
  __syncthreads();
  int64_t budget = spin_limit;
  uint32_t* raw = (uint32_t*)dst;
  bool ok = ll_read_words<16>(buf, (int64_t)d * WPE, ex, threadIdx.x, 256, budget,
                              [&](int64_t idx, uint32_t payload) { raw[idx] = payload; });
  if (!ok) *flag = 0;
  __syncthreads();
  const bool res = *flag != 0;
  if (res && scale != 1.0)
    for (int c = threadIdx.x; c < d; c += 256) dst[c] = (BT)((double)dst[c] * scale);
  __syncthreads();
  return res;
}

// Gather a published FP64 vector (2 words per element) into dst as BT.
template <typename BT>
__device__ bool gather_f64_as(const uint64_t* buf, uint32_t ex, int d, BT* dst, int* flag, int64_t spin_limit) {
  if (threadIdx.x == 0) *flag = 1;
  __syncthreads();
  int64_t budget = spin_limit;
  bool ok = true;
  constexpr int W = 8;
  for (int base = 0; base < d && ok; base += 256 * W) {
    uint64_t lo[W], hi[W];
#pragma unroll
    for (int j = 0; j < W; j++) {
      const int e = base + threadIdx.x + 256 * j;
      if (e < d) { lo[j] = ll_load(buf + 2 * (int64_t)e); hi[j] = ll_load(buf + 2 * (int64_t)e + 1); }
      else lo[j] = hi[j] = ((uint64_t)ex << 32);
    }
    while (true) {
      bool all = true;
#pragma unroll
      for (int j = 0; j < W; j++) all = all && ((uint32_t)(lo[j] >> 32) == ex) && ((uint32_t)(hi[j] >> 32) == ex);
      if (all) break;
      if (--budget <= 0) { ok = false; break; }
      __builtin_amdgcn_s_sleep(1);
#pragma unroll
      for (int j = 0; j < W; j++) {
        const int e = base + threadIdx.x + 256 * j;
        if (e < d) {
          if ((uint32_t)(lo[j] >> 32) != ex) lo[j] = ll_load(buf + 2 * (int64_t)e);
          if ((uint32_t)(hi[j] >> 32) != ex) hi[j] = ll_load(buf + 2 * (int64_t)e + 1);
        }
      }
    }
    if (ok) {
#pragma unroll
      for (int j = 0; j < W; j++) {
        const int e = base + threadIdx.x + 256 * j;
        if (e < d) dst[e] = (BT)ll_join_f64(lo[j], hi[j]);
      }
    }
  }
  if (!ok) *flag = 0;
  __syncthreads();
  const bool res = *flag != 0;
  __syncthreads();
  return res;
}

template <typename BT>
__global__ __launch_bounds__(256) void power_kernel(PowerArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int G = gridDim.x, b = blockIdx.x;
  const int d = a.d;
  const int dpad = (d + 3) & ~3;
  const int r0 = b * a.rpb;
  const int nrows = max(0, min(a.rpb, d - r0));
  const int rpbA = (a.rpb + 1) & ~1;

  // LDS carve (sizes mirrored by power_lds_fixed)
  double* yv = (double*)smem;           // own rows: y = B x
  double* xv = yv + rpbA;               // own rows: x (FP64)
  double* vv = xv + rpbA;               // own rows: v (FP64) at the end of a triplet
  double* wv = vv + rpbA;               // own rows: w = B v
  double* scratch = wv + rpbA;          // 256: allreduce scratch
  double* redw = scratch + 256;         // 8: block_sum scratch
  double* sv = redw + 8;                // 8: small values to publish
  double* st = sv + 8;                  // 16: small totals
  int* flag = (int*)(st + 16);          // block-uniform ok flag (2 doubles reserved)
  BT* xs = (BT*)(st + 18);              // dpad: iterate (GEMV input)
  BT* aux = xs + dpad;                  // dpad: w during deflation
  BT* Bs = aux + dpad;                  // cache_rows x ldsB
  BT* Bg = (BT*)a.B + (int64_t)r0 * a.ldb;
  double* kvals = a.kscr + (int64_t)b * 2 * (a.k + 2);  // per-block global scratch
  double* ktot = kvals + (a.k + 2);

  // one-time load of the cached rows
  const int cr = min(a.cache_rows, nrows);
  for (int li = 0; li < a.cache_rows; li++)
    for (int c = tid; c < a.ldsB; c += 256)
      Bs[li * a.ldsB + c] = (li < cr && c < d) ? Bg[(int64_t)li * a.ldb + c] : (BT)0;
  __syncthreads();

  uint32_t epoch = 0, nx = 0, np = 0;
  const int64_t xwords = (int64_t)dpad * (sizeof(BT) / 4);
  int err = ERR_NONE;
  int kdone = a.k;
  bool all_conv = true, rankdef = false;

  for (int l = 0; l < a.k; l++) {
    // ---- start vector x = v0_l / ||v0_l|| (every block computes the same norm)
    const double* v0 = a.v0 + (int64_t)l * d;
    double ss = 0.0;
    for (int c = tid; c < d; c += 256) ss = fma(v0[c], v0[c], ss);
    ss = block_sum(ss, redw, tid, 256);
    if (!isfinite(ss)) { err = ERR_NONFINITE; break; }
    if (!(ss > 0.0)) { err = ERR_BADSTART; break; }
    const double inv0 = 1.0 / sqrt(ss);
    for (int c = tid; c < dpad; c += 256) { xs[c] = c < d ? (BT)(v0[c] * inv0) : (BT)0; aux[c] = (BT)0; }
    for (int i = tid; i < nrows; i += 256) xv[i] = v0[r0 + i] * inv0;
    __syncthreads();

    const int fixed = a.fixed_iters ? a.fixed_iters[l] : (a.eps <= 0.0 ? a.max_iter : 0);
    int it = 0;
    double nrm = 0.0;
    bool conv = false;
    while (true) {
      gemv_own<BT>(a, Bs, Bg, nrows, xs, yv);
      __syncthreads();
      it++;
      if (tid == 0) {
        double q = 0.0, dd = 0.0;
        for (int i = 0; i < nrows; i++) { q = fma(yv[i], yv[i], q); dd = fma(xv[i], yv[i], dd); }
        sv[0] = q; sv[1] = dd;
      }
      __syncthreads();
      ++epoch;
      uint64_t* xb = a.xex + (int64_t)(nx & 1) * xwords; nx++;
      uint64_t* pb = a.pex + (int64_t)(np & 1) * G * a.pw; np++;
      publish_vec<BT>(xb, epoch, r0, nrows, yv, 1.0);
      if (!allreduce_blocks(pb, a.pw, G, epoch, sv, 2, st, scratch, flag, a.spin_limit)) { err = ERR_SPIN; break; }
      const double q = st[0], dd = st[1];
      nrm = sqrt(q);
      if (!isfinite(nrm)) { err = ERR_NONFINITE; break; }
      if (nrm == 0.0) { rankdef = true; kdone = l; break; }
      bool stop;
      if (fixed > 0) { stop = it >= fixed; conv = true; }
      else {
        conv = fabs(dd) / nrm >= 1.0 - a.eps;
        stop = conv || it >= a.max_iter;
      }
      const double inv = 1.0 / nrm;
      if (stop) {
        for (int i = tid; i < nrows; i += 256) vv[i] = yv[i] * inv;
        __syncthreads();
        break;
      }
      if (!gather_vec<BT>(xb, epoch, d, xs, inv, flag, a.spin_limit)) { err = ERR_SPIN; break; }
      for (int i = tid; i < nrows; i += 256) xv[i] = yv[i] * inv;
      __syncthreads();
    }
    if (err != ERR_NONE || rankdef) break;
    if (!conv) all_conv = false;

    // ---- FP64 re-orthogonalisation of v against X[:, 0..l)
    const int P = l + 1;  // c_j = X[:, j] . v (j < l) and ||v||^2 (j = l)
    for (int j = wave; j < P; j += 4) {
      double s = 0.0;
      for (int i = lane; i < nrows; i += 64) {
        const double xi = (j < l) ? a.X[(int64_t)j * a.ldx + r0 + i] : vv[i];
        s = fma(xi, vv[i], s);
      }
      s = wave_sum(s);
      if (lane == 0) kvals[j] = s;
    }
    __syncthreads();
    ++epoch;
    {
      uint64_t* pb = a.pex + (int64_t)(np & 1) * G * a.pw; np++;
      if (!allreduce_blocks(pb, a.pw, G, epoch, kvals, P, ktot, scratch, flag, a.spin_limit)) { err = ERR_SPIN; break; }
    }
    for (int i = tid; i < nrows; i += 256) {
      double v = vv[i];
      for (int j = 0; j < l; j++) v = fma(-a.X[(int64_t)j * a.ldx + r0 + i], ktot[j], v);
      vv[i] = v;
    }
    __syncthreads();
    {
      double s = 0.0;
      for (int i = tid; i < nrows; i += 256) s = fma(vv[i], vv[i], s);
      s = block_sum(s, redw, tid, 256);
      if (tid == 0) sv[2] = s;
      __syncthreads();
    }
    ++epoch;
    {
      uint64_t* pb = a.pex + (int64_t)(np & 1) * G * a.pw; np++;
      if (!allreduce_blocks(pb, a.pw, G, epoch, sv + 2, 1, st + 4, scratch, flag, a.spin_limit)) { err = ERR_SPIN; break; }
    }
    const double vn2 = st[4];
    if (!isfinite(vn2)) { err = ERR_NONFINITE; break; }
    if (!(vn2 > 0.0)) { rankdef = true; kdone = l; break; }
    const double vinv = 1.0 / sqrt(vn2);
    for (int i = tid; i < nrows; i += 256) {
      vv[i] *= vinv;
      a.X[(int64_t)l * a.ldx + r0 + i] = vv[i];
    }
    if (b == 0 && tid == 0) { a.lambda[l] = nrm; a.iters[l] = it; }
    __syncthreads();
    if (l + 1 >= a.k) break;

    // ---- deflation: w = B v, alpha = v.w, B <- B - v w^T - w v^T + alpha v v^T
    ++epoch;
    {
      uint64_t* vb = a.vex + (int64_t)(l & 1) * 2 * dpad;
      for (int i = tid; i < nrows; i += 256) ll_store_f64(vb + 2 * (int64_t)(r0 + i), epoch, vv[i]);
      if (!gather_f64_as<BT>(vb, epoch, d, xs, flag, a.spin_limit)) { err = ERR_SPIN; break; }
    }
    gemv_own<BT>(a, Bs, Bg, nrows, xs, wv);
    __syncthreads();
    if (tid == 0) {
      double al = 0.0;
      for (int i = 0; i < nrows; i++) al = fma(vv[i], wv[i], al);
      sv[3] = al;
    }
    __syncthreads();
    ++epoch;
    {
      uint64_t* wb = a.wex + (int64_t)(l & 1) * 2 * dpad;
      for (int i = tid; i < nrows; i += 256) ll_store_f64(wb + 2 * (int64_t)(r0 + i), epoch, wv[i]);
      uint64_t* pb = a.pex + (int64_t)(np & 1) * G * a.pw; np++;
      if (!allreduce_blocks(pb, a.pw, G, epoch, sv + 3, 1, st + 5, scratch, flag, a.spin_limit)) { err = ERR_SPIN; break; }
      if (!gather_f64_as<BT>(wb, epoch, d, aux, flag, a.spin_limit)) { err = ERR_SPIN; break; }
    }
    const double alpha = st[5];
    // own-row update, LDS rows then HBM rows
    for (int li = 0; li < nrows; li++) {
      const double vi = vv[li], wi = wv[li];
      BT* row = li < cr ? Bs + (int64_t)li * a.ldsB : Bg + (int64_t)li * a.ldb;
      for (int c = tid; c < d; c += 256) {
        const double vc = (double)xs[c], wc = (double)aux[c];
        double x = (double)row[c];
        x = fma(-vi, wc, x);
        x = fma(-wi, vc, x);
        x = fma(alpha * vi, vc, x);
        row[c] = (BT)x;
      }
    }
    __syncthreads();
  }

  if (b == 0 && tid == 0) {
    a.status[0] = kdone;
    a.status[1] = all_conv ? 1 : 0;
    a.status[3] = rankdef ? 1 : 0;
  }
  if (err != ERR_NONE && tid == 0) atomicMax(a.status + 2, err);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static size_t power_lds_fixed(int rpb, int dpad, int elem) {
  const int rpbA = (rpb + 1) & ~1;
  return (size_t)(4 * rpbA + 256 + 8 + 8 + 18) * 8 + (size_t)2 * dpad * elem;
}

int power_plan(int dtype_bytes, int d, int k, int num_cu, size_t max_lds, int max_blocks_hint, PowerPlan* p) {
  int G = num_cu;
  if (max_blocks_hint > 0 && max_blocks_hint < G) G = max_blocks_hint;
  const int min_rows = 4;
  if ((d + min_rows - 1) / min_rows < G) G = (d + min_rows - 1) / min_rows;
  if (G < 1) G = 1;
  p->G = G;
  p->rpb = (d + G - 1) / G;
  const int dpad = (d + 3) & ~3;
  p->ldsB = dpad;
  const size_t fixed = power_lds_fixed(p->rpb, dpad, dtype_bytes);
  if (fixed > max_lds) return -1;  // vector does not fit in LDS
  const size_t row_bytes = (size_t)dpad * dtype_bytes;
  int cache = (int)((max_lds - fixed) / row_bytes);
  if (cache > p->rpb) cache = p->rpb;
  if (cache < 0) cache = 0;
  p->cache_rows = cache;
  p->lds_bytes = fixed + (size_t)cache * row_bytes;
  // partial buffer holds up to k+1 doubles per block (re-orthogonalisation)
  p->pw = 2 * (k + 2);
  p->xex_words = (size_t)2 * dpad * (dtype_bytes / 4);
  p->pex_words = (size_t)2 * G * p->pw;
  p->vex_words = (size_t)2 * 2 * dpad;
  p->wex_words = (size_t)2 * 2 * dpad;
  return 0;
}

__global__ void zero_words_kernel(uint64_t* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

int power_launch(int is_f64, const PowerPlan& p, PowerArgs a, hipStream_t stream) {
  const size_t total = p.xex_words + p.pex_words + p.vex_words + p.wex_words;
  hipLaunchKernelGGL(zero_words_kernel, dim3(256), dim3(256), 0, stream, a.xex, total);
  TSVD_HIP_TRY(hipGetLastError());
  a.rpb = p.rpb; a.cache_rows = p.cache_rows; a.ldsB = p.ldsB; a.pw = p.pw;
  void* args[] = {&a};
  const void* fn = is_f64 ? (const void*)power_kernel<double> : (const void*)power_kernel<float>;
  TSVD_HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes));
  int per_cu = 0;
  TSVD_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, p.lds_bytes));
  if (per_cu < 1) return -2;
  TSVD_HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(p.G), dim3(256), args, p.lds_bytes, stream));
  return 0;
}

}  // namespace tsvd
