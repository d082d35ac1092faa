// Power iteration with deflation on a symmetric Gram matrix (Algorithm 2, run
// once per triplet as Algorithm 1 does), as ONE persistent launch.
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

#include <algorithm>
#include <type_traits>

#include "common.h"
#include "exchange.h"
#include "internal.h"
#include "syrk_dev.h"

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

// y[r] = scale * (B row r . x) for the NR rows r = first + 4q (q < NR) of one
// storage (LDS or HBM).  The body is straight-line (every load and FMA is
// unconditional), so the loads of UNR column steps are in flight together; a
// per-row predicate inside the loop would make the compiler wait for each LDS
// load on its own.  Each lane keeps one FMA chain per (row, vector component)
// in B's type (16 chains for FP32 and 4 rows: one wave per SIMD has no other
// wave to hide FMA and LDS latency behind), about d / 256 products per chain;
// chains and lanes are then added in FP64.
template <typename BT, int NR, int UNR>
__device__ __forceinline__ void gemv_rows(const BT* rows, int64_t stride, int first, const BT* xs, int d, int dv,
                                          double scale, double* yout) {
  constexpr int VN = VecOf<BT>::N;
  using VT = typename std::conditional<sizeof(BT) == 4, float4, double2>::type;
  const int lane = threadIdx.x & 63;
  const BT* rp[NR];
#pragma unroll
  for (int q = 0; q < NR; q++) rp[q] = rows + (int64_t)(first + 4 * q) * stride;
  BT acc[NR][VN];
#pragma unroll
  for (int q = 0; q < NR; q++)
#pragma unroll
    for (int e = 0; e < VN; e++) acc[q][e] = (BT)0;
#pragma unroll UNR
  for (int c = lane * VN; c < dv; c += 64 * VN) {
    const VT xv = *(const VT*)(xs + c);
    VT bv[NR];
#pragma unroll
    for (int q = 0; q < NR; q++) bv[q] = *(const VT*)(rp[q] + c);
#pragma unroll
    for (int q = 0; q < NR; q++) {
      if constexpr (VN == 4) {
        acc[q][0] = fma(bv[q].x, xv.x, acc[q][0]);
        acc[q][1] = fma(bv[q].y, xv.y, acc[q][1]);
        acc[q][2] = fma(bv[q].z, xv.z, acc[q][2]);
        acc[q][3] = fma(bv[q].w, xv.w, acc[q][3]);
      } else {
        acc[q][0] = fma(bv[q].x, xv.x, acc[q][0]);
        acc[q][1] = fma(bv[q].y, xv.y, acc[q][1]);
      }
    }
  }
  for (int c = dv + lane; c < d; c += 64) {
    const BT xv = xs[c];
#pragma unroll
    for (int q = 0; q < NR; q++) acc[q][0] = fma(rp[q][c], xv, acc[q][0]);
  }
#pragma unroll
  for (int q = 0; q < NR; q++) {
    double t = 0.0;
#pragma unroll
    for (int e = 0; e < VN; e++) t += (double)acc[q][e];
    const double sum = wave_sum(t);
    if (lane == 0) yout[first + 4 * q] = sum * scale;
  }
}

// y[li] = scale * (B row li . x) for rows li in [begin, end) of one storage.
// Rows are dealt to the 4 waves round-robin (wave w: begin + w + 4j); a wave
// takes up to 4 of its rows per pass so each x chunk read from LDS feeds them
// all.  The wave index is made explicitly uniform so the row-count dispatch is
// a scalar branch.
template <typename BT, int UNR = 2>
__device__ __forceinline__ void gemv_range(const BT* rows, int64_t stride, int begin, int end, const BT* xs, int d, bool vec_ok,
                           double scale, double* yout) {
  constexpr int VN = VecOf<BT>::N;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int dv = vec_ok ? (d / VN) * VN : 0;
  for (int first = begin + wave; first < end; first += 16) {
    const int nr = (end - first + 3) / 4;
    if (nr >= 4) gemv_rows<BT, 4, UNR>(rows, stride, first, xs, d, dv, scale, yout);
    else if (nr == 3) gemv_rows<BT, 3, UNR>(rows, stride, first, xs, d, dv, scale, yout);
    else if (nr == 2) gemv_rows<BT, 2, UNR>(rows, stride, first, xs, d, dv, scale, yout);
    else gemv_rows<BT, 1, UNR>(rows, stride, first, xs, d, dv, scale, yout);
  }
}

// Register-resident rows: wave w holds rows cr + w + 4q (q < RR) of its block,
// lane l keeping columns VN*l + 64*VN*s + e (s < NV, e < VN), zero beyond d.
template <typename BT, int NV, int RR>
struct RegRows {
  static constexpr int VN = VecOf<BT>::N;
  BT v[RR > 0 ? RR : 1][NV > 0 ? NV : 1][VN];
};

template <typename BT, int NV, int RR>
__device__ __forceinline__ void gemv_regrows(const RegRows<BT, NV, RR>& R, int cr, int nreg, const BT* xs,
                                             double scale, double* yout) {
  if constexpr (RR > 0 && NV > 0) {
    if (nreg <= 0) return;
    // per-lane partial sums in BT (16 products per chain at d = 4096),
    // summed across chains and lanes in FP64
    constexpr int VN = VecOf<BT>::N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    BT acc[RR][VN];  // one FMA chain per (row, component)
#pragma unroll
    for (int q = 0; q < RR; q++)
#pragma unroll
      for (int e = 0; e < VN; e++) acc[q][e] = (BT)0;
#pragma unroll
    for (int s = 0; s < NV; s++) {
      BT xv[VN];
      if constexpr (VN == 4) {
        const float4 f = *(const float4*)(xs + VN * lane + 64 * VN * s);
        xv[0] = f.x; xv[1] = f.y; xv[2] = f.z; xv[3] = f.w;
      } else {
        const double2 f = *(const double2*)(xs + VN * lane + 64 * VN * s);
        xv[0] = f.x; xv[1] = f.y;
      }
#pragma unroll
      for (int q = 0; q < RR; q++)
#pragma unroll
        for (int e = 0; e < VN; e++) acc[q][e] = fma(R.v[q][s][e], xv[e], acc[q][e]);
    }
#pragma unroll
    for (int q = 0; q < RR; q++) {
      const int li = wave + 4 * q;
      double t = 0.0;
#pragma unroll
      for (int e = 0; e < VN; e++) t += (double)acc[q][e];
      double sum = wave_sum(t);
      if (lane == 0 && li < nreg) yout[cr + li] = sum * scale;
    }
  }
}

// One pass over the iterate for all of a wave's resident rows, FP32 B: the
// RR register rows (cr + wave + 4q) and LR LDS rows (wave + 4j) of the block.
// Each 4-column chunk of x is read from LDS once per wave and feeds every row;
// the chunks of x and of the LDS rows are fetched two steps ahead, so a single
// wave per SIMD is not left waiting on LDS latency step by step.  Requires
// cr == 4 LR, nreg == 4 RR (or RR == 0) and ldsB == 256 NV (no ragged
// chunk).  Every row is summed exactly as gemv_rows / gemv_regrows sum it (one
// FMA chain per component over ascending chunks, then the components and the
// lanes in FP64), so the result is the same bit for bit.
template <int NV, int RR, int LR>
__device__ __forceinline__ void gemv_fused(const RegRows<float, NV, RR>& R, const float* Bs, int ldsB, int cr,
                                           const float* xs, double scale, double* yout) {
  constexpr int NRR = RR > 0 ? RR : 0;
  constexpr int D = 2;  // prefetch distance (chunks)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float* xp = xs + 4 * lane;
  const float* lp[LR];
#pragma unroll
  for (int j = 0; j < LR; j++) lp[j] = Bs + (wave + 4 * j) * ldsB + 4 * lane;
  float acc[NRR + LR][4];
#pragma unroll
  for (int q = 0; q < NRR + LR; q++)
#pragma unroll
    for (int e = 0; e < 4; e++) acc[q][e] = 0.0f;
  float4 xb[D], lb[D][LR];
#pragma unroll
  for (int t = 0; t < D; t++) {
    xb[t] = *(const float4*)(xp + 256 * t);
#pragma unroll
    for (int j = 0; j < LR; j++) lb[t][j] = *(const float4*)(lp[j] + 256 * t);
  }
#pragma unroll
  for (int sidx = 0; sidx < NV; sidx++) {
    const int slot = sidx % D;
    const float4 xv = xb[slot];
    float4 lv[LR];
#pragma unroll
    for (int j = 0; j < LR; j++) lv[j] = lb[slot][j];
    if (sidx + D < NV) {
      xb[slot] = *(const float4*)(xp + 256 * (sidx + D));
#pragma unroll
      for (int j = 0; j < LR; j++) lb[slot][j] = *(const float4*)(lp[j] + 256 * (sidx + D));
    }
    const float x4[4] = {xv.x, xv.y, xv.z, xv.w};
    if constexpr (RR > 0) {
#pragma unroll
      for (int q = 0; q < RR; q++)
#pragma unroll
        for (int e = 0; e < 4; e++) acc[q][e] = fma(R.v[q][sidx][e], x4[e], acc[q][e]);
    }
#pragma unroll
    for (int j = 0; j < LR; j++) {
      acc[NRR + j][0] = fma(lv[j].x, xv.x, acc[NRR + j][0]);
      acc[NRR + j][1] = fma(lv[j].y, xv.y, acc[NRR + j][1]);
      acc[NRR + j][2] = fma(lv[j].z, xv.z, acc[NRR + j][2]);
      acc[NRR + j][3] = fma(lv[j].w, xv.w, acc[NRR + j][3]);
    }
  }
  double t[NRR + LR];
#pragma unroll
  for (int q = 0; q < NRR + LR; q++) {
    t[q] = 0.0;
#pragma unroll
    for (int e = 0; e < 4; e++) t[q] += (double)acc[q][e];
  }
#pragma unroll
  for (int q = 0; q < NRR + LR; q++) t[q] = wave_sum(t[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NRR; q++) yout[cr + wave + 4 * q] = t[q] * scale;
#pragma unroll
    for (int j = 0; j < LR; j++) yout[wave + 4 * j] = t[NRR + j] * scale;
  }
}

// Sum vals[0..P) over all G workgroups (published in the partial buffer under
// epoch ex); out[0..P) receives the totals, identical in every workgroup.
// Returns false (uniformly in the block) if a wait ran out of budget.
__device__ __forceinline__ bool allreduce_blocks(uint64_t* pbuf, int pw, int b, int G, uint32_t ex, const double* vals, int P,
                                 double* out, double* scratch, int* flag, int64_t spin_limit) {
  const int tid = threadIdx.x;
  for (int w = tid; w < 2 * P; w += 256) ll_store(pbuf + (int64_t)b * pw + w, ex, f64_half(vals[w >> 1], w & 1));
  if (tid == 0) *flag = 1;
  __syncthreads();
  for (int jb = 0; jb < P; jb += 256) {
    const int Pc = min(256, P - jb);
    // thread (gg, j) = (tid / Pp, tid % Pp) with Pp the power of two >= Pc:
    // it sums output j over the workgroups g = gg, gg + NG, ...
    const int lg = Pc > 1 ? 32 - __clz(Pc - 1) : 0;
    const int Pp = 1 << lg, NG = 256 >> lg;
    const int j = tid & (Pp - 1), gg = tid >> lg;
    double acc = 0.0;
    bool ok = true;
    if (j < Pc) {
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
    }
    if (!ok) *flag = 0;
    // fixed-order tree over gg: a butterfly across the lanes of a wave that
    // hold the same j (Pp, 2 Pp, ... apart), then the per-wave partials (or,
    // for Pp >= 64, the per-group ones) in order
    for (int m = Pp; m < 64; m <<= 1) acc += __shfl_xor(acc, m, 64);
    const int nparts = Pp < 64 ? 4 : NG;
    const int part = Pp < 64 ? (tid >> 6) : gg;
    if (j < Pc && (Pp >= 64 || (tid & 63) < Pp)) scratch[part * Pp + j] = acc;
    __syncthreads();
    if (tid < Pc) {
      double s = 0.0;
      for (int q = 0; q < nparts; q++) s += scratch[q * Pp + tid];
      out[jb + tid] = s;
    }
    __syncthreads();
  }
  const bool res = *flag != 0;
  __syncthreads();
  return res;
}

// row[c] -= coef[li] * z[c] for rows li in [begin, end) of one storage (LDS or
// HBM) and columns c < d; z is a vector in LDS.  FP64 arithmetic, rounded once
// to B's type; the column loop is unrolled so that several row chunks are in
// flight.
template <typename BT>
__device__ __forceinline__ void deflate_rows(BT* rows, int64_t stride, int begin, int end, bool vec_ok, int d, const BT* z,
                             const double* coef) {
  constexpr int VN = VecOf<BT>::N;
  using VT = typename std::conditional<sizeof(BT) == 4, float4, double2>::type;
  const int tid = threadIdx.x;
  const int dv = vec_ok ? (d / VN) * VN : 0;
  for (int li = begin; li < end; li++) {
    BT* row = rows + (int64_t)li * stride;
    const double ci = coef[li];
#pragma unroll 4
    for (int c = tid * VN; c < dv; c += 256 * VN) {
      VT r = *(const VT*)(row + c);
      const VT zz = *(const VT*)(z + c);
      if constexpr (VN == 4) {
        r.x = (BT)fma(-ci, (double)zz.x, (double)r.x);
        r.y = (BT)fma(-ci, (double)zz.y, (double)r.y);
        r.z = (BT)fma(-ci, (double)zz.z, (double)r.z);
        r.w = (BT)fma(-ci, (double)zz.w, (double)r.w);
      } else {
        r.x = (BT)fma(-ci, (double)zz.x, (double)r.x);
        r.y = (BT)fma(-ci, (double)zz.y, (double)r.y);
      }
      *(VT*)(row + c) = r;
    }
    for (int c = dv + tid; c < d; c += 256) row[c] = (BT)fma(-ci, (double)z[c], (double)row[c]);
  }
}

// The same update on the register rows (columns c >= d keep their zeros).
template <typename BT, int NV, int RR>
__device__ __forceinline__ void deflate_regrows(RegRows<BT, NV, RR>& R, int cr, int nreg, int d, const BT* z,
                                                const double* coef) {
  if constexpr (RR > 0 && NV > 0) {
    if (nreg <= 0) return;
    constexpr int VN = VecOf<BT>::N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < RR; q++) {
      const int li = wave + 4 * q;
      const double ci = li < nreg ? coef[cr + li] : 0.0;
#pragma unroll
      for (int s = 0; s < NV; s++) {
        BT zv[VN];
        if constexpr (VN == 4) {
          const float4 f = *(const float4*)(z + VN * lane + 64 * VN * s);
          zv[0] = f.x; zv[1] = f.y; zv[2] = f.z; zv[3] = f.w;
        } else {
          const double2 f = *(const double2*)(z + VN * lane + 64 * VN * s);
          zv[0] = f.x; zv[1] = f.y;
        }
#pragma unroll
        for (int e = 0; e < VN; e++) {
          const int c = VN * lane + 64 * VN * s + e;
          const BT nv = (BT)fma(-ci, (double)zv[e], (double)R.v[q][s][e]);
          R.v[q][s][e] = c < d ? nv : R.v[q][s][e];
        }
      }
    }
  }
}

template <typename BT, int NV, int RR>
__device__ __forceinline__ void load_regrows(RegRows<BT, NV, RR>& R, const BT* Bg, int64_t ldb, int cr, int nreg,
                                             int d) {
  if constexpr (RR > 0 && NV > 0) {
    constexpr int VN = VecOf<BT>::N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < RR; q++) {
      const bool live = wave + 4 * q < nreg;
      const BT* row = Bg + (int64_t)(cr + wave + 4 * q) * ldb;
#pragma unroll
      for (int s = 0; s < NV; s++)
#pragma unroll
        for (int e = 0; e < VN; e++) {
          const int c = VN * lane + 64 * VN * s + e;
          R.v[q][s][e] = (live && c < d) ? row[c] : (BT)0;
        }
    }
  }
}

// One problem solved by a team of G workgroups (this one is member b).  The
// exchange counters persist across problems solved by the same team.  Returns
// the error code this workgroup met (ERR_NONE on success).
template <typename BT, int NV, int RR>
__device__ __forceinline__ int solve_problem(const PowerArgs& a, int b, int G, unsigned char* smem, uint32_t& epoch, uint32_t& nx,
                              uint32_t& np) {
  constexpr int VN = VecOf<BT>::N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
  double* redw = scratch + 256;         // 8: block_sum / tree scratch
  double* sv = redw + 8;                // 8: small values to publish
  double* st = sv + 8;                  // 16: small totals
  int* flag = (int*)(st + 16);          // block-uniform ok flag (2 doubles reserved)
  BT* xs = (BT*)(st + 18);              // dpad: iterate (GEMV input), zero padded
  BT* Bs = xs + dpad;                   // cache_rows x ldsB
  BT* Bg = (BT*)a.B + (int64_t)r0 * a.ldb;
  double* kvals = a.kscr + (int64_t)b * 2 * (a.k + 2);  // per-block global scratch
  double* ktot = kvals + (a.k + 2);

  // row classes: [0, cr) in LDS, [cr, cr + nreg) in registers, the rest read from B
  const int cr = min(a.cache_rows, nrows);
  const int nreg = (RR > 0 && NV > 0) ? min(4 * RR, nrows - cr) : 0;
  const int g0 = cr + nreg;
  // the single-pass product serves the common shapes: FP32 B, every chunk of x
  // full, 4 or 8 LDS rows and all register rows present
  int fused = 0;
  if constexpr (sizeof(BT) == 4 && RR > 0 && NV > 0) {
    if (a.ldsB == 256 * NV && nreg == 4 * RR && (cr == 4 || cr == 8)) fused = cr / 4;
  }

  // one-time loads
  for (int li = 0; li < a.cache_rows; li++)
    for (int c = tid; c < a.ldsB; c += 256)
      Bs[li * a.ldsB + c] = (li < cr && c < d) ? Bg[(int64_t)li * a.ldb + c] : (BT)0;
  __syncthreads();

  const int64_t xwords = a.xwords;
  int err = ERR_NONE;
  int kdone = a.k;
  bool all_conv = true, rankdef = false;
  // register rows stay resident for the whole launch and are deflated in place
  RegRows<BT, NV, RR> R;
  load_regrows<BT, NV, RR>(R, Bg, a.ldb, cr, nreg, d);

  for (int l = 0; l < a.k; l++) {
    // ---- start vector x = v0_l / ||v0_l|| (every block computes the same norm)
    const double* v0 = a.v0 + (int64_t)l * d;
    double ss = 0.0;
#pragma unroll 8
    for (int c = tid; c < d; c += 256) ss = fma(v0[c], v0[c], ss);
    ss = block_sum(ss, redw, tid, 256);
    if (!isfinite(ss)) { err = ERR_NONFINITE; break; }
    if (!(ss > 0.0)) { err = ERR_BADSTART; break; }
    const double inv0 = 1.0 / sqrt(ss);
#pragma unroll 8
    for (int c = tid; c < dpad; c += 256) xs[c] = c < d ? (BT)(v0[c] * inv0) : (BT)0;
    for (int i = tid; i < nrows; i += 256) xv[i] = v0[r0 + i] * inv0;
    __syncthreads();

    const int fixed = a.fixed_iters ? a.fixed_iters[l] : (a.eps <= 0.0 ? a.max_iter : 0);
    int it = 0;
    double nrm = 0.0;
    bool conv = false;
    // x_t = scale * xs: xs holds x_0, then the gathered y_t as published; the
    // normalisation 1 / ||y_t|| is applied to the next product's row sums
    // instead of to the iterate (the same value without a pass over xs)
    double scale = 1.0;
    while (true) {
      // ---- y = B x on the block's rows
      bool one_pass = false;
      if constexpr (sizeof(BT) == 4 && RR > 0 && NV > 0) {
        if (fused == 2) { gemv_fused<NV, RR, 2>(R, Bs, a.ldsB, cr, xs, scale, yv); one_pass = true; }
        else if (fused == 1) { gemv_fused<NV, RR, 1>(R, Bs, a.ldsB, cr, xs, scale, yv); one_pass = true; }
      }
      if (!one_pass) {
        gemv_regrows<BT, NV, RR>(R, cr, nreg, xs, scale, yv);
        gemv_range<BT, 4>(Bs, a.ldsB, 0, cr, xs, d, true, scale, yv);
      }
      gemv_range<BT, (RR > 0 ? 2 : 8)>(Bg, a.ldb, g0, nrows, xs, d, a.vec_ok != 0, scale, yv);
      __syncthreads();
      it++;
      // ---- publish y (own rows) and the block partials ||y_R||^2, x_R . y_R
      ++epoch;
      uint64_t* xb = a.xex + (int64_t)(nx & 1) * xwords; nx++;
      uint64_t* pb = a.pex + (int64_t)(np & 1) * G * a.pw; np++;
      publish_rows<BT>(xb, epoch, r0, nrows, yv);
      if (wave == 3) {
        double q = 0.0, dd = 0.0;
        for (int i = lane; i < nrows; i += 64) { q = fma(yv[i], yv[i], q); dd = fma(xv[i], yv[i], dd); }
        q = wave_sum(q);
        dd = wave_sum(dd);
        // the four words (q lo/hi, dd lo/hi) go out in one store instruction:
        // a wave's device-scope stores become visible one after another
        if (lane < 4) ll_store(pb + 4 * (int64_t)b + lane, epoch, f64_half(lane < 2 ? q : dd, lane & 1));
      }
      // ---- one wait for every block's y and partials
      double q, dd;
      // (the widest register-row configuration has no registers to spare for W = 16)
      const bool got = (NV <= 16 && d * (int)(sizeof(BT) / 4) > 256 * 8)
                           ? gather_iteration<BT, 16>(xb, pb, epoch, d, b, G, xs, redw, flag, a.spin_limit, q, dd)
                           : gather_iteration<BT, 8>(xb, pb, epoch, d, b, G, xs, redw, flag, a.spin_limit, q, dd);
      if (!got) { err = ERR_SPIN; break; }
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
      // x_{t+1} = y / ||y||: xs keeps y, the next row sums are scaled by 1 / ||y||
      scale = inv;
      for (int i = tid; i < nrows; i += 256) xv[i] = yv[i] * inv;
      __syncthreads();
    }
    if (err != ERR_NONE || rankdef) break;
    if (!conv) all_conv = false;

    // ---- FP64 re-orthogonalisation of v against X[:, 0..l)
    const int P = l + 1;  // c_j = X[:, j] . v (j < l) and ||v||^2 (j = l)
    {
      // wave w takes j = w, w + 4, ...; JB of them per pass so that their X
      // loads are in flight together (j >= l reads a valid column and is
      // replaced by v)
      constexpr int JB = 8;
      const int jmax = l > 0 ? l - 1 : 0;
      for (int j0 = wave; j0 < P; j0 += 4 * JB) {
        double sj[JB];
#pragma unroll
        for (int u = 0; u < JB; u++) sj[u] = 0.0;
        for (int i = lane; i < nrows; i += 64) {
          const double vi = vv[i];
          double xj[JB];
#pragma unroll
          for (int u = 0; u < JB; u++) xj[u] = a.X[(int64_t)min(j0 + 4 * u, jmax) * a.ldx + r0 + i];
#pragma unroll
          for (int u = 0; u < JB; u++) sj[u] = fma(j0 + 4 * u < l ? xj[u] : vi, vi, sj[u]);
        }
#pragma unroll
        for (int u = 0; u < JB; u++) {
          const double t = wave_sum(sj[u]);
          if (lane == 0 && j0 + 4 * u < P) kvals[j0 + 4 * u] = t;
        }
      }
    }
    __syncthreads();
    ++epoch;
    {
      uint64_t* pb = a.pex + (int64_t)(np & 1) * G * a.pw; np++;
      if (!allreduce_blocks(pb, a.pw, b, G, epoch, kvals, P, ktot, scratch, flag, a.spin_limit)) { err = ERR_SPIN; break; }
    }
    if (nrows <= 128) {
      // v_i -= sum_j X[i][j] c_j with the j range split over parts = 256 / nrows
      // threads per row (their loads in flight together), parts added in order
      const int parts = nrows > 0 ? 256 / nrows : 1;
      const int i = nrows > 0 ? tid % nrows : 0, part = nrows > 0 ? tid / nrows : 0;
      double acc = 0.0;
      if (part < parts) {
#pragma unroll 4
        for (int j = part; j < l; j += parts) acc = fma(a.X[(int64_t)j * a.ldx + r0 + i], ktot[j], acc);
        scratch[part * nrows + i] = acc;
      }
      __syncthreads();
      if (tid < nrows) {
        double t = 0.0;
        for (int p2 = 0; p2 < parts; p2++) t += scratch[p2 * nrows + tid];
        vv[tid] -= t;
      }
    } else {
      for (int i = tid; i < nrows; i += 256) {
        double v = vv[i];
#pragma unroll 8
        for (int j = 0; j < l; j++) v = fma(-a.X[(int64_t)j * a.ldx + r0 + i], ktot[j], v);
        vv[i] = v;
      }
    }
    __syncthreads();

    // ---- publish v' = v - X c (own rows) with the block partial ||v'_R||^2:
    // one wait brings every block v' (the GEMV input of the deflation) and
    // ||v'||^2; 1 / ||v'|| is then applied to the row sums and coefficients
    constexpr int WG = (NV <= 16) ? 16 : 8;  // gather width (registers permitting)
    ++epoch;
    const uint32_t vep = epoch;
    uint64_t* vb = a.vex + (int64_t)(l & 1) * a.vstride;
    double vn2;
    {
      uint64_t* pb = a.pex + (int64_t)(np & 1) * G * a.pw; np++;
      publish_rows<BT>(vb, vep, r0, nrows, vv);
      if (wave == 3) {
        double q = 0.0;
        for (int i = lane; i < nrows; i += 64) q = fma(vv[i], vv[i], q);
        q = wave_sum(q);
        if (lane < 4) ll_store(pb + 4 * (int64_t)b + lane, vep, f64_half(lane < 2 ? q : 0.0, lane & 1));
      }
      double d0;
      if (!gather_iteration<BT, WG>(vb, pb, vep, d, b, G, xs, redw, flag, a.spin_limit, vn2, d0)) { err = ERR_SPIN; break; }
    }
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

    // ---- deflation: w = B v, alpha = v.w, B <- B - v w^T - beta v^T with
    // beta = w - alpha v (= (I - v v^T) B (I - v v^T)); xs holds v' = v ||v'||
    gemv_regrows<BT, NV, RR>(R, cr, nreg, xs, vinv, wv);
    gemv_range<BT, 4>(Bs, a.ldsB, 0, cr, xs, d, true, vinv, wv);
    gemv_range<BT, (RR > 0 ? 2 : 8)>(Bg, a.ldb, g0, nrows, xs, d, a.vec_ok != 0, vinv, wv);
    __syncthreads();
    // publish w (own rows) with the block partial alpha_R = v_R . w_R
    ++epoch;
    const uint32_t wep = epoch;
    uint64_t* wb = a.wex + (int64_t)(l & 1) * a.vstride;
    double alpha;
    {
      uint64_t* pb = a.pex + (int64_t)(np & 1) * G * a.pw; np++;
      publish_rows<BT>(wb, wep, r0, nrows, wv);
      if (wave == 3) {
        double q = 0.0;
        for (int i = lane; i < nrows; i += 64) q = fma(vv[i], wv[i], q);
        q = wave_sum(q);
        if (lane < 4) ll_store(pb + 4 * (int64_t)b + lane, wep, f64_half(lane < 2 ? q : 0.0, lane & 1));
      }
      double d0;
      if (!gather_iteration<BT, WG>(wb, pb, wep, d, b, G, xs, redw, flag, a.spin_limit, alpha, d0)) { err = ERR_SPIN; break; }
    }
    // Own-row update in two phases that each read one vector from LDS, each
    // done in FP64 and rounded to B's type: first B -= v w^T with xs = w, then
    // B -= beta v^T with xs = v' read again from its published words (beta is
    // scaled by 1 / ||v'||)
    deflate_rows<BT>(Bs, a.ldsB, 0, cr, true, d, xs, vv);
    deflate_regrows<BT, NV, RR>(R, cr, nreg, d, xs, vv);
    deflate_rows<BT>(Bg, a.ldb, g0, nrows, a.vec_ok != 0, d, xs, vv);
    for (int i = tid; i < nrows; i += 256) xv[i] = (wv[i] - alpha * vv[i]) * vinv;
    __syncthreads();
    {
      double q0, d0;
      if (!gather_iteration<BT, WG>(vb, vb, vep, d, b, 0, xs, redw, flag, a.spin_limit, q0, d0)) { err = ERR_SPIN; break; }
    }
    deflate_rows<BT>(Bs, a.ldsB, 0, cr, true, d, xs, xv);
    deflate_regrows<BT, NV, RR>(R, cr, nreg, d, xs, xv);
    deflate_rows<BT>(Bg, a.ldb, g0, nrows, a.vec_ok != 0, d, xs, xv);
    __syncthreads();
  }

  if (b == 0 && tid == 0) {
    a.status[0] = kdone;
    a.status[1] = all_conv ? 1 : 0;
    a.status[3] = rankdef ? 1 : 0;
  }
  if (err != ERR_NONE && tid == 0) atomicMax(a.status + 2, err);
  return err;
}

// Out-of-line entry into solve_problem for the batched kernel: each register
// variant keeps its own register allocation (inlined together they spill);
// the call's register saves happen once per problem, not per iteration.
template <typename BT, int NV, int RR>
__device__ __attribute__((noinline)) int solve_problem_call(const PowerArgs& a, int b, int G, unsigned char* smem,
                                                            uint32_t* epoch, uint32_t* nx, uint32_t* np) {
  return solve_problem<BT, NV, RR>(a, b, G, smem, *epoch, *nx, *np);
}

// Single problem: the whole grid is one team.
template <typename BT, int NV, int RR>
__global__ __launch_bounds__(256, 1) void power_kernel(PowerArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t epoch = 0, nx = 0, np = 0;
  solve_problem<BT, NV, RR>(a, blockIdx.x, gridDim.x, smem, epoch, nx, np);
}

// ---------------------------------------------------------------------------
// Batched engine: one persistent launch runs a whole batch (every problem's
// Gram units, their reduction into the problem's B, and its power iteration)
// from one list of work items that its workgroups take one fetch at a time,
// in list order.  The list holds, problem after problem in the power queue's
// order, the problem's Gram units, then its reductions, then the G seats of
// its team, so the Gram work of later problems runs beside the power teams of
// earlier ones.  Every wait is on items earlier in the list, which were taken
// by workgroups that are running and never wait on later items, so the list
// drains (and every wait is bounded besides).  Completions are published
// with a device-scope release (the fence writes the unit's stores back past
// the XCD's L2) and observed with an acquire load, so a reduction reads every
// partial tile and a team reads all of its B.  The arithmetic of each unit,
// reduction and team is the stand-alone kernels', so results do not change.
// ---------------------------------------------------------------------------
// Poll with relaxed loads (an acquire load per poll would invalidate the
// XCD's L2 on every poll, under the running teams' feet) and acquire once.
__device__ __forceinline__ bool wait_count(const int* c, int target, int64_t spin) {
  int64_t budget = spin;
  while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (--budget <= 0) return false;
    __builtin_amdgcn_s_sleep(2);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

__device__ __forceinline__ void count_done(int* c) {
  __hip_atomic_fetch_add(c, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// one Gram work unit of a batched problem (tile edge BM)
template <int BM>
__device__ __forceinline__ void engine_gram_unit(const GramJob& j, const SyrkArgs& a, int s, int t,
                                                 unsigned char* smem) {
  if (j.mode == MODE_BF16X3) {
    if (j.side == 0) syrk_unit<MODE_BF16X3, 0, BM>(a, s, t, smem);
    else syrk_unit<MODE_BF16X3, 1, BM>(a, s, t, smem);
  } else {
    if (j.side == 0) syrk_unit<MODE_FP32, 0, BM>(a, s, t, smem);
    else syrk_unit<MODE_FP32, 1, BM>(a, s, t, smem);
  }
}

// reduction of one triangle tile's chunk partials into B, 32 x 32 at a time
template <int BM>
__device__ __forceinline__ void engine_reduce_tile(const GramJob& j, int tile, unsigned char* smem) {
  constexpr int SUBS = (BM / 32) * (BM / 32);
  const int64_t d = j.side == 0 ? j.n : j.m;
  for (int sub = 0; sub < SUBS; sub++) {
    syrk_reduce_unit<float, BM>((const float*)j.partial, j.T, j.S, d, (float*)j.B, j.ldb, 0, tile * SUBS + sub, smem);
    __syncthreads();
  }
}

__global__ __launch_bounds__(256, 1) void batch_engine_kernel(const EngineItem* items, int nitems,
                                                              const GramJob* jobs, const PowerArgs* probs, int* ctr,
                                                              int nprob, int64_t spin, int* exit_flags, int exit_id) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_t, s_ok;
  int* head = ctr + 4 * nprob;
  while (true) {
    if (threadIdx.x == 0) s_t = atomicAdd(head, 1);
    __syncthreads();
    const int t = s_t;
    if (t >= nitems) {
      if (threadIdx.x == 0 && exit_flags)
        __hip_atomic_store(exit_flags + blockIdx.x, exit_id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      return;
    }
    const EngineItem it = items[t];
    int* pc = ctr + 4 * it.p;
    const GramJob& j = jobs[it.job];
    if (it.type == ITEM_GRAM) {
      const SyrkArgs a = job_args(j);
      const int s = it.idx / j.T, tt = it.idx % j.T;
      if (j.bm == 64) engine_gram_unit<64>(j, a, s, tt, smem);
      else engine_gram_unit<128>(j, a, s, tt, smem);
      __syncthreads();
      if (threadIdx.x == 0) count_done(pc + 0);
    } else if (it.type == ITEM_REDUCE) {
      if (threadIdx.x == 0) s_ok = wait_count(pc + 0, j.S * j.T, spin) ? 1 : 0;
      __syncthreads();
      if (s_ok) {
        if (j.bm == 64) engine_reduce_tile<64>(j, it.idx, smem);
        else engine_reduce_tile<128>(j, it.idx, smem);
      } else if (threadIdx.x == 0) {
        atomicMax(probs[it.p].status + 2, (int)ERR_SPIN);
      }
      if (threadIdx.x == 0) count_done(pc + 1);
    } else {
      // a seat of the problem's team: wait for the whole team and for B
      if (threadIdx.x == 0) {
        atomicAdd(pc + 2, 1);
        s_ok = (wait_count(pc + 2, it.G, spin) && wait_count(pc + 1, j.T, spin)) ? 1 : 0;
      }
      __syncthreads();
      const PowerArgs a = probs[it.p];
      if (!s_ok) {
        if (threadIdx.x == 0) atomicMax(a.status + 2, (int)ERR_SPIN);
        __syncthreads();
        continue;
      }
      uint32_t epoch = 0, nx = 0, np = 0;
      const int d = a.d;
      if (d <= 1024) solve_problem_call<float, 4, 4>(a, it.idx, it.G, smem, &epoch, &nx, &np);
      else if (d <= 2048) solve_problem_call<float, 8, 4>(a, it.idx, it.G, smem, &epoch, &nx, &np);
      else if (d <= 4096) solve_problem_call<float, 16, 2>(a, it.idx, it.G, smem, &epoch, &nx, &np);
      else if (d <= 8192) solve_problem_call<float, 32, 1>(a, it.idx, it.G, smem, &epoch, &nx, &np);
      else solve_problem_call<float, 0, 0>(a, it.idx, it.G, smem, &epoch, &nx, &np);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static size_t power_lds_fixed(int rpb, int dpad, int elem) {
  const int rpbA = (rpb + 1) & ~1;
  return (size_t)(4 * rpbA + 256 + 8 + 8 + 18) * 8 + (size_t)dpad * elem;
}

// register-row configuration for an FP32 Gram of dimension d
static void reg_config(int d, int* NV, int* RR) {
  if (d <= 1024) { *NV = 4; *RR = 4; }
  else if (d <= 2048) { *NV = 8; *RR = 4; }
  else if (d <= 4096) { *NV = 16; *RR = 2; }
  else if (d <= 8192) { *NV = 32; *RR = 1; }
  else { *NV = 0; *RR = 0; }
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
  if (fixed > max_lds) return -1;  // the iterate does not fit in LDS
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

// compute units of the current device (cached per device)
static int max_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) { (void)hipGetLastError(); return 1 << 20; }
  if (cus[dev] == 0) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) {
      (void)hipGetLastError();
      return 1 << 20;
    }
    cus[dev] = c;
  }
  return cus[dev];
}

__global__ void zero_words_kernel(uint64_t* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

static const void* pick_kernel(int is_f64, int d) {
  if (is_f64) return (const void*)power_kernel<double, 0, 0>;
  int NV, RR;
  reg_config(d, &NV, &RR);
  switch (NV) {
    case 4: return (const void*)power_kernel<float, 4, 4>;
    case 8: return (const void*)power_kernel<float, 8, 4>;
    case 16: return (const void*)power_kernel<float, 16, 2>;
    case 32: return (const void*)power_kernel<float, 32, 1>;
    default: return (const void*)power_kernel<float, 0, 0>;
  }
}

int power_launch(int is_f64, const PowerPlan& p, PowerArgs a, hipStream_t stream) {
  const size_t total = p.xex_words + p.pex_words + p.vex_words + p.wex_words;
  hipLaunchKernelGGL(zero_words_kernel, dim3(256), dim3(256), 0, stream, a.xex, total);
  TSVD_HIP_TRY(hipGetLastError());
  a.rpb = p.rpb; a.cache_rows = p.cache_rows; a.ldsB = p.ldsB; a.pw = p.pw;
  a.xwords = (int64_t)p.ldsB * (is_f64 ? 2 : 1);
  a.vstride = (int64_t)2 * p.ldsB;
  void* args[] = {&a};
  const void* fn = pick_kernel(is_f64, a.d);
  TSVD_HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes));
  int per_cu = 0;
  TSVD_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, p.lds_bytes));
  if (per_cu < 1) return -2;
  // An ordinary launch: G <= CUs x per_cu, so every workgroup is resident at
  // once on an otherwise idle device (the kernel's waits are bounded: a member
  // that cannot start in time makes the call fail, never hang).  The runtime's
  // cooperative-launch path is not used; it added nothing but a launch check.
  if ((int64_t)p.G > (int64_t)per_cu * max_cus()) return -2;
  TSVD_HIP_TRY(hipLaunchKernel(fn, dim3(p.G), dim3(256), args, p.lds_bytes, stream));
  return 0;
}

size_t engine_static_lds() {
  static size_t bytes = (size_t)-1;
  if (bytes == (size_t)-1) {
    hipFuncAttributes attr;
    bytes = hipFuncGetAttributes(&attr, (const void*)batch_engine_kernel) == hipSuccess ? attr.sharedSizeBytes : 256;
    (void)hipGetLastError();
  }
  return bytes;
}

int engine_launch(const EngineItem* d_items, int nitems, const GramJob* d_jobs, const PowerArgs* d_probs, int* d_ctr,
                  int nprob, int grid, size_t lds_bytes, uint64_t* zero_base, size_t zero_words, hipStream_t stream,
                  int* exit_flags, int exit_id) {
  if (grid <= 0 || nitems <= 0) return 0;
  if (zero_words) {
    hipLaunchKernelGGL(zero_words_kernel, dim3(256), dim3(256), 0, stream, zero_base, zero_words);
    TSVD_HIP_TRY(hipGetLastError());
  }
  // a Gram unit's LDS (both stages of both panels) must fit as well
  lds_bytes = std::max(lds_bytes, std::max(SyrkCfg<MODE_BF16X3>::LDS, SyrkCfg<MODE_FP32>::LDS));
  const void* fn = (const void*)batch_engine_kernel;
  TSVD_HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
  int per_cu = 0;
  TSVD_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds_bytes));
  if (per_cu < 1) return -2;
  // all workgroups resident at once (teams wait for their members)
  if ((int64_t)grid > (int64_t)per_cu * max_cus()) return -2;
  int64_t spin = (int64_t)1 << 26;
  void* args[] = {(void*)&d_items, (void*)&nitems, (void*)&d_jobs, (void*)&d_probs, (void*)&d_ctr,
                  (void*)&nprob,   (void*)&spin,   (void*)&exit_flags, (void*)&exit_id};
  TSVD_HIP_TRY(hipLaunchKernel(fn, dim3(grid), dim3(256), args, lds_bytes, stream));
  return 0;
}

}  // namespace tsvd
