// Gram product on MFMA (Algorithm 2's B = X^T X / X X^T, formed as Algorithm 3's
// sum of block products).
//
// Work unit = (triangle tile t, contraction chunk s).  A work unit computes the
// BM x BM product of two column panels of A (side RIGHT: B[I,J] = A[:,I]^T A[:,J]
// over rows of the chunk) or two row panels (side LEFT: B[I,J] = A[I,:] A[J,:]^T
// over columns of the chunk) and stores it as a partial tile.  Only tiles with
// I >= J are computed (the symmetric half: the reduced task list of the paper's
// Gram task scheduling).  A second kernel sums the chunk partials in a fixed
// order and writes both triangles of B, so results do not depend on scheduling.
//
// Operands are staged through LDS "k-contiguous" ([panel column][k]) so that an
// MFMA lane reads its consecutive-k operand slice with one wide LDS load; for a
// row-major A on side RIGHT the transpose happens in registers on the way in.
//
// Modes:
//   MODE_BF16X3: a = hi + lo with hi = bf16_rn(a), lo = bf16_rn(a - hi), done in
//                registers while staging (HBM traffic stays 4 B per element);
//                tile += hi^T hi + hi^T lo + lo^T hi on v_mfma_f32_32x32x16_bf16.
//   MODE_FP32:   v_mfma_f32_32x32x2f32.
//   MODE_FP64:   v_mfma_f64_16x16x4f64 (FP64 A).
//
// XCD-aware mapping: workgroups are dispatched round-robin over the 8 XCDs, so
// when the chunk count is a multiple of 8, XCD x is given chunks x, x+8, ...
// for every tile; the workgroups resident on one XCD then read the same rows of
// A at about the same time and share them through that XCD's L2.
#include <cmath>

#include "common.h"
#include "internal.h"

namespace tsvd {

template <int MODE> struct SyrkCfg;
template <> struct SyrkCfg<MODE_BF16X3> {
  static constexpr int BM = 128, BK = 32, LDK = BK + 8;  // LDS row of bf16
  using AT = float; using OT = float;
};
template <> struct SyrkCfg<MODE_FP32> {
  static constexpr int BM = 128, BK = 32, LDK = BK + 4;  // LDS row of float
  using AT = float; using OT = float;
};
template <> struct SyrkCfg<MODE_FP64> {
  static constexpr int BM = 64, BK = 16, LDK = BK + 2;   // LDS row of double
  using AT = double; using OT = double;
};

struct SyrkArgs {
  const void* A;
  int64_t m, n, lda;
  int64_t d;        // Gram dimension (n for RIGHT, m for LEFT)
  int64_t K;        // contraction length (m for RIGHT, n for LEFT)
  int64_t kchunk;   // contraction elements per chunk
  int nt, T, S;     // tiles per side, triangle tiles, chunks
  int xcd_map;
  int vec_ok;       // A and lda allow 16-byte vector loads
  void* partial;    // S * T * BM * BM elements of OT
};

__device__ __forceinline__ void tri_tile(int t, int& ti, int& tj) {
  // lower-triangle tiles enumerated row by row: t = ti*(ti+1)/2 + tj, tj <= ti
  int r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= t) r++;
  while (r * (r + 1) / 2 > t) r--;
  ti = r;
  tj = t - r * (r + 1) / 2;
}

__device__ __forceinline__ void unit_of(const SyrkArgs& a, int b, int& s, int& t) {
  if (a.xcd_map) {
    int x = b & 7, local = b >> 3;
    s = x + 8 * (local / a.T);
    t = local % a.T;
  } else {
    s = b / a.T;
    t = b % a.T;
  }
}

// position of contraction index k inside an LDS row, so that the values an MFMA
// lane consumes on successive k-steps are contiguous
template <int MODE> __device__ __forceinline__ int kpos(int k);
template <> __device__ __forceinline__ int kpos<MODE_BF16X3>(int k) { return k; }
template <> __device__ __forceinline__ int kpos<MODE_FP32>(int k) { return (k & 1) * 16 + (k >> 1); }
template <> __device__ __forceinline__ int kpos<MODE_FP64>(int k) { return (k & 3) * 4 + (k >> 2); }

__device__ __forceinline__ void split_bf16(float a, __bf16& hi, __bf16& lo) {
  hi = (__bf16)a;                 // round to nearest even
  float r = a - (float)hi;        // exact in FP32
  lo = (__bf16)r;
}

// ---------------------------------------------------------------------------
// BF16X3 staging: 4 consecutive k for one LDS column per 8-byte LDS store.
// ---------------------------------------------------------------------------
template <int SIDE>
__device__ __forceinline__ void load_panel_bf16(const SyrkArgs& a, int64_t c0, int64_t k0, int64_t kend,
                                                float (&v)[4][4]) {
  const float* A = (const float*)a.A;
  const int tid = threadIdx.x;
  if (SIDE == 0) {
    // rows k (contraction) x columns c of A; thread covers 4 rows x 4 columns
    const int rg = tid & 7, cg = tid >> 3;
    const int64_t c = c0 + 4 * cg;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int64_t k = k0 + 4 * rg + j;
      const float* p = A + k * a.lda + c;
      if (k < kend && a.vec_ok && c + 3 < a.d) {
        float4 f = *(const float4*)p;
        v[j][0] = f.x; v[j][1] = f.y; v[j][2] = f.z; v[j][3] = f.w;
      } else {
#pragma unroll
        for (int i = 0; i < 4; i++) v[j][i] = (k < kend && c + i < a.d) ? p[i] : 0.0f;
      }
    }
  } else {
    // rows c of A (panel rows) x columns k (contraction); thread covers 4 rows x 4 k
    const int kg = tid & 7, rr = tid >> 3;
    const int64_t k = k0 + 4 * kg;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int64_t c = c0 + rr + 32 * q;
      const float* p = A + c * a.lda + k;
      if (c < a.d && a.vec_ok && k + 3 < kend) {
        float4 f = *(const float4*)p;
        v[q][0] = f.x; v[q][1] = f.y; v[q][2] = f.z; v[q][3] = f.w;
      } else {
#pragma unroll
        for (int i = 0; i < 4; i++) v[q][i] = (c < a.d && k + i < kend) ? p[i] : 0.0f;
      }
    }
  }
}

template <int SIDE>
__device__ __forceinline__ void store_panel_bf16(__bf16* hi, __bf16* lo, const float (&v)[4][4]) {
  constexpr int LDK = SyrkCfg<MODE_BF16X3>::LDK;
  const int tid = threadIdx.x;
  if (SIDE == 0) {
    const int rg = tid & 7, cg = tid >> 3;
#pragma unroll
    for (int i = 0; i < 4; i++) {          // column 4cg+i holds k = 4rg..4rg+3 = v[0..3][i]
      bf16x4 h, l;
#pragma unroll
      for (int j = 0; j < 4; j++) { __bf16 x, y; split_bf16(v[j][i], x, y); h[j] = x; l[j] = y; }
      const int off = (4 * cg + i) * LDK + 4 * rg;
      *(bf16x4*)(hi + off) = h;
      *(bf16x4*)(lo + off) = l;
    }
  } else {
    const int kg = tid & 7, rr = tid >> 3;
#pragma unroll
    for (int q = 0; q < 4; q++) {          // panel row rr+32q holds k = 4kg..4kg+3 = v[q][0..3]
      bf16x4 h, l;
#pragma unroll
      for (int j = 0; j < 4; j++) { __bf16 x, y; split_bf16(v[q][j], x, y); h[j] = x; l[j] = y; }
      const int off = (rr + 32 * q) * LDK + 4 * kg;
      *(bf16x4*)(hi + off) = h;
      *(bf16x4*)(lo + off) = l;
    }
  }
}

// ---------------------------------------------------------------------------
// FP32 / FP64 staging: element-wise (these modes are bound by the slower MFMA).
// ---------------------------------------------------------------------------
template <int MODE, int SIDE>
__device__ __forceinline__ void load_panel_elem(const SyrkArgs& a, int64_t c0, int64_t k0, int64_t kend,
                                                typename SyrkCfg<MODE>::AT (&v)[SyrkCfg<MODE>::BM * SyrkCfg<MODE>::BK / 256]) {
  using Cfg = SyrkCfg<MODE>;
  using AT = typename Cfg::AT;
  constexpr int E = Cfg::BM * Cfg::BK / 256;
  const AT* A = (const AT*)a.A;
#pragma unroll
  for (int e = 0; e < E; e++) {
    const int f = threadIdx.x + 256 * e;
    int c, kk;
    if (SIDE == 0) { c = f % Cfg::BM; kk = f / Cfg::BM; }
    else { kk = f % Cfg::BK; c = f / Cfg::BK; }
    const int64_t gc = c0 + c, gk = k0 + kk;
    bool ok = gc < a.d && gk < kend;
    v[e] = ok ? (SIDE == 0 ? A[gk * a.lda + gc] : A[gc * a.lda + gk]) : (AT)0;
  }
}

template <int MODE, int SIDE>
__device__ __forceinline__ void store_panel_elem(typename SyrkCfg<MODE>::AT* s,
                                                 const typename SyrkCfg<MODE>::AT (&v)[SyrkCfg<MODE>::BM * SyrkCfg<MODE>::BK / 256]) {
  using Cfg = SyrkCfg<MODE>;
  constexpr int E = Cfg::BM * Cfg::BK / 256;
#pragma unroll
  for (int e = 0; e < E; e++) {
    const int f = threadIdx.x + 256 * e;
    int c, kk;
    if (SIDE == 0) { c = f % Cfg::BM; kk = f / Cfg::BM; }
    else { kk = f % Cfg::BK; c = f / Cfg::BK; }
    s[c * Cfg::LDK + kpos<MODE>(kk)] = v[e];
  }
}

// ---------------------------------------------------------------------------
// Partial-tile kernel
// ---------------------------------------------------------------------------
template <int MODE, int SIDE>
__device__ __forceinline__ void syrk_unit(const SyrkArgs& a, int s, int t) {
  using Cfg = SyrkCfg<MODE>;
  using AT = typename Cfg::AT;
  using OT = typename Cfg::OT;
  constexpr int BM = Cfg::BM, BK = Cfg::BK, LDK = Cfg::LDK;

  int ti, tj;
  tri_tile(t, ti, tj);
  const bool diag = (ti == tj);
  const int64_t k0 = (int64_t)s * a.kchunk;
  const int64_t kend = k0 + a.kchunk < a.K ? k0 + a.kchunk : a.K;
  const int64_t cI = (int64_t)ti * BM, cJ = (int64_t)tj * BM;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // 2 x 2 waves, each (BM/2) x (BM/2)
  OT* out = (OT*)a.partial + ((int64_t)s * a.T + t) * BM * BM;
  const int nk = (int)((kend - k0 + BK - 1) / BK);

  if constexpr (MODE == MODE_BF16X3) {
    // LDS: [stage][panel I/J][hi/lo][BM][LDK] bf16
    __shared__ __bf16 lds[2][2][2][BM * LDK];
    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int j = 0; j < 2; j++)
#pragma unroll
        for (int e = 0; e < 16; e++) acc[i][j][e] = 0.0f;

    float vi[4][4], vj[4][4];
    if (nk > 0) {
      load_panel_bf16<SIDE>(a, cI, k0, kend, vi);
      if (!diag) load_panel_bf16<SIDE>(a, cJ, k0, kend, vj);
      store_panel_bf16<SIDE>(lds[0][0][0], lds[0][0][1], vi);
      if (!diag) store_panel_bf16<SIDE>(lds[0][1][0], lds[0][1][1], vj);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; kt++) {
      const int cur = kt & 1;
      const bool more = kt + 1 < nk;
      if (more) {
        const int64_t kb = k0 + (int64_t)(kt + 1) * BK;
        load_panel_bf16<SIDE>(a, cI, kb, kend, vi);
        if (!diag) load_panel_bf16<SIDE>(a, cJ, kb, kend, vj);
      }
      const __bf16* Ih = lds[cur][0][0];
      const __bf16* Il = lds[cur][0][1];
      const __bf16* Jh = diag ? Ih : lds[cur][1][0];
      const __bf16* Jl = diag ? Il : lds[cur][1][1];
#pragma unroll
      for (int ks = 0; ks < BK; ks += 16) {
        bf16x8 ah[2], al[2], bh[2], bl[2];
        const int kofs = ks + 8 * (lane >> 5);
#pragma unroll
        for (int i = 0; i < 2; i++) {
          const int r = wm * 64 + i * 32 + (lane & 31);
          ah[i] = *(const bf16x8*)(Ih + r * LDK + kofs);
          al[i] = *(const bf16x8*)(Il + r * LDK + kofs);
        }
#pragma unroll
        for (int j = 0; j < 2; j++) {
          const int c = wn * 64 + j * 32 + (lane & 31);
          bh[j] = *(const bf16x8*)(Jh + c * LDK + kofs);
          bl[j] = *(const bf16x8*)(Jl + c * LDK + kofs);
        }
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
          for (int j = 0; j < 2; j++) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          }
      }
      if (more) {
        store_panel_bf16<SIDE>(lds[cur ^ 1][0][0], lds[cur ^ 1][0][1], vi);
        if (!diag) store_panel_bf16<SIDE>(lds[cur ^ 1][1][0], lds[cur ^ 1][1][1], vj);
      }
      __syncthreads();
    }
    // 32x32 accumulator layout: item e -> row (e/4)*8 + (lane/32)*4 + e%4, col lane%32
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int j = 0; j < 2; j++)
#pragma unroll
        for (int e = 0; e < 16; e++) {
          const int r = wm * 64 + i * 32 + (e >> 2) * 8 + (lane >> 5) * 4 + (e & 3);
          const int c = wn * 64 + j * 32 + (lane & 31);
          out[r * BM + c] = acc[i][j][e];
        }
  } else if constexpr (MODE == MODE_FP32) {
    __shared__ float lds[2][2][BM * LDK];
    constexpr int E = BM * BK / 256;
    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int j = 0; j < 2; j++)
#pragma unroll
        for (int e = 0; e < 16; e++) acc[i][j][e] = 0.0f;
    float vi[E], vj[E];
    if (nk > 0) {
      load_panel_elem<MODE, SIDE>(a, cI, k0, kend, vi);
      if (!diag) load_panel_elem<MODE, SIDE>(a, cJ, k0, kend, vj);
      store_panel_elem<MODE, SIDE>(lds[0][0], vi);
      if (!diag) store_panel_elem<MODE, SIDE>(lds[0][1], vj);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; kt++) {
      const int cur = kt & 1;
      const bool more = kt + 1 < nk;
      if (more) {
        const int64_t kb = k0 + (int64_t)(kt + 1) * BK;
        load_panel_elem<MODE, SIDE>(a, cI, kb, kend, vi);
        if (!diag) load_panel_elem<MODE, SIDE>(a, cJ, kb, kend, vj);
      }
      const float* I = lds[cur][0];
      const float* J = diag ? I : lds[cur][1];
      // lane half h consumes k = 2*s + h for s = 0..15: stored at h*16 + s
      const int h = lane >> 5;
      float av[2][16], bv[2][16];
#pragma unroll
      for (int i = 0; i < 2; i++) {
        const int r = wm * 64 + i * 32 + (lane & 31);
#pragma unroll
        for (int q = 0; q < 4; q++) {
          float4 f = *(const float4*)(I + r * LDK + h * 16 + 4 * q);
          av[i][4 * q] = f.x; av[i][4 * q + 1] = f.y; av[i][4 * q + 2] = f.z; av[i][4 * q + 3] = f.w;
        }
      }
#pragma unroll
      for (int j = 0; j < 2; j++) {
        const int c = wn * 64 + j * 32 + (lane & 31);
#pragma unroll
        for (int q = 0; q < 4; q++) {
          float4 f = *(const float4*)(J + c * LDK + h * 16 + 4 * q);
          bv[j][4 * q] = f.x; bv[j][4 * q + 1] = f.y; bv[j][4 * q + 2] = f.z; bv[j][4 * q + 3] = f.w;
        }
      }
#pragma unroll
      for (int ss = 0; ss < 16; ss++)
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
          for (int j = 0; j < 2; j++)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i][ss], bv[j][ss], acc[i][j], 0, 0, 0);
      if (more) {
        store_panel_elem<MODE, SIDE>(lds[cur ^ 1][0], vi);
        if (!diag) store_panel_elem<MODE, SIDE>(lds[cur ^ 1][1], vj);
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int j = 0; j < 2; j++)
#pragma unroll
        for (int e = 0; e < 16; e++) {
          const int r = wm * 64 + i * 32 + (e >> 2) * 8 + (lane >> 5) * 4 + (e & 3);
          const int c = wn * 64 + j * 32 + (lane & 31);
          out[r * BM + c] = acc[i][j][e];
        }
  } else {
    // FP64: BM = 64, waves 2 x 2 of 32 x 32, MFMA tiles 16 x 16 x 4
    __shared__ double lds[2][2][BM * LDK];
    constexpr int E = BM * BK / 256;
    doublex4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int j = 0; j < 2; j++)
#pragma unroll
        for (int e = 0; e < 4; e++) acc[i][j][e] = 0.0;
    double vi[E], vj[E];
    if (nk > 0) {
      load_panel_elem<MODE, SIDE>(a, cI, k0, kend, vi);
      if (!diag) load_panel_elem<MODE, SIDE>(a, cJ, k0, kend, vj);
      store_panel_elem<MODE, SIDE>(lds[0][0], vi);
      if (!diag) store_panel_elem<MODE, SIDE>(lds[0][1], vj);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; kt++) {
      const int cur = kt & 1;
      const bool more = kt + 1 < nk;
      if (more) {
        const int64_t kb = k0 + (int64_t)(kt + 1) * BK;
        load_panel_elem<MODE, SIDE>(a, cI, kb, kend, vi);
        if (!diag) load_panel_elem<MODE, SIDE>(a, cJ, kb, kend, vj);
      }
      const double* I = lds[cur][0];
      const double* J = diag ? I : lds[cur][1];
      // lane quarter q consumes k = 4*s + q for s = 0..3: stored at q*4 + s
      const int q = lane >> 4;
      double av[2][4], bv[2][4];
#pragma unroll
      for (int i = 0; i < 2; i++) {
        const int r = wm * 32 + i * 16 + (lane & 15);
#pragma unroll
        for (int ss = 0; ss < 4; ss++) av[i][ss] = I[r * LDK + q * 4 + ss];
      }
#pragma unroll
      for (int j = 0; j < 2; j++) {
        const int c = wn * 32 + j * 16 + (lane & 15);
#pragma unroll
        for (int ss = 0; ss < 4; ss++) bv[j][ss] = J[c * LDK + q * 4 + ss];
      }
#pragma unroll
      for (int ss = 0; ss < 4; ss++)
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
          for (int j = 0; j < 2; j++)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][ss], bv[j][ss], acc[i][j], 0, 0, 0);
      if (more) {
        store_panel_elem<MODE, SIDE>(lds[cur ^ 1][0], vi);
        if (!diag) store_panel_elem<MODE, SIDE>(lds[cur ^ 1][1], vj);
      }
      __syncthreads();
    }
    // 16x16 FP64 accumulator layout: item e -> row 4e + lane/16, col lane%16
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int j = 0; j < 2; j++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int r = wm * 32 + i * 16 + 4 * e + (lane >> 4);
          const int c = wn * 32 + j * 16 + (lane & 15);
          out[r * BM + c] = acc[i][j][e];
        }
  }
}

template <int MODE, int SIDE>
__global__ __launch_bounds__(256) void syrk_partial_kernel(SyrkArgs a) {
  int s, t;
  unit_of(a, blockIdx.x, s, t);
  syrk_unit<MODE, SIDE>(a, s, t);
}

// ---------------------------------------------------------------------------
// BF16X3 partial tiles of 256 x 256 with 8 waves (2 x 4, each 128 x 64 as
// 4 x 2 MFMA 32x32x16 blocks).  Per k-step a wave reads 12 fragments for 24
// MFMAs (half the LDS traffic per MFMA of the 128-tile kernel); the two LDS
// stages take the whole 160 KB, so one workgroup runs per CU.
// ---------------------------------------------------------------------------
constexpr int BIG_BM = 256, BIG_BK = 32, BIG_LDK = BIG_BK + 8;
constexpr size_t BIG_LDS = (size_t)2 * 2 * 2 * BIG_BM * BIG_LDK * 2;  // stages x panels x hi/lo x rows x LDK x 2 B

template <int SIDE>
__device__ __forceinline__ void big_load(const SyrkArgs& a, int64_t c0, int64_t k0, int64_t kend, float (&v)[4][4]) {
  const float* A = (const float*)a.A;
  const int tid = threadIdx.x;
  if (SIDE == 0) {
    const int rg = tid & 7, cg = tid >> 3;  // 8 row groups x 64 column groups
    const int64_t c = c0 + 4 * cg;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int64_t k = k0 + 4 * rg + j;
      const float* p = A + k * a.lda + c;
      if (k < kend && a.vec_ok && c + 3 < a.d) {
        const float4 f = *(const float4*)p;
        v[j][0] = f.x; v[j][1] = f.y; v[j][2] = f.z; v[j][3] = f.w;
      } else {
#pragma unroll
        for (int i = 0; i < 4; i++) v[j][i] = (k < kend && c + i < a.d) ? p[i] : 0.0f;
      }
    }
  } else {
    const int kg = tid & 7, rr = tid >> 3;  // 8 k groups x 64 rows (x 4 passes)
    const int64_t k = k0 + 4 * kg;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int64_t c = c0 + rr + 64 * q;
      const float* p = A + c * a.lda + k;
      if (c < a.d && a.vec_ok && k + 3 < kend) {
        const float4 f = *(const float4*)p;
        v[q][0] = f.x; v[q][1] = f.y; v[q][2] = f.z; v[q][3] = f.w;
      } else {
#pragma unroll
        for (int i = 0; i < 4; i++) v[q][i] = (c < a.d && k + i < kend) ? p[i] : 0.0f;
      }
    }
  }
}

template <int SIDE>
__device__ __forceinline__ void big_store(__bf16* hi, __bf16* lo, const float (&v)[4][4]) {
  const int tid = threadIdx.x;
  if (SIDE == 0) {
    const int rg = tid & 7, cg = tid >> 3;
#pragma unroll
    for (int i = 0; i < 4; i++) {
      bf16x4 h, l;
#pragma unroll
      for (int j = 0; j < 4; j++) { __bf16 x, y; split_bf16(v[j][i], x, y); h[j] = x; l[j] = y; }
      const int off = (4 * cg + i) * BIG_LDK + 4 * rg;
      *(bf16x4*)(hi + off) = h;
      *(bf16x4*)(lo + off) = l;
    }
  } else {
    const int kg = tid & 7, rr = tid >> 3;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      bf16x4 h, l;
#pragma unroll
      for (int j = 0; j < 4; j++) { __bf16 x, y; split_bf16(v[q][j], x, y); h[j] = x; l[j] = y; }
      const int off = (rr + 64 * q) * BIG_LDK + 4 * kg;
      *(bf16x4*)(hi + off) = h;
      *(bf16x4*)(lo + off) = l;
    }
  }
}

template <int SIDE>
__global__ __launch_bounds__(512, 1) void syrk_bf16x3_big_kernel(SyrkArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16* lds = (__bf16*)smem;  // [stage][panel][hi/lo][BM * LDK]
  auto at = [&](int stage, int panel, int part) { return lds + ((stage * 2 + panel) * 2 + part) * BIG_BM * BIG_LDK; };
  int s, t, ti, tj;
  unit_of(a, blockIdx.x, s, t);
  tri_tile(t, ti, tj);
  const bool diag = (ti == tj);
  const int64_t k0 = (int64_t)s * a.kchunk;
  const int64_t kend = k0 + a.kchunk < a.K ? k0 + a.kchunk : a.K;
  const int64_t cI = (int64_t)ti * BIG_BM, cJ = (int64_t)tj * BIG_BM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;  // 2 x 4 waves, each 128 x 64
  float* out = (float*)a.partial + ((int64_t)s * a.T + t) * BIG_BM * BIG_BM;
  const int nk = (int)((kend - k0 + BIG_BK - 1) / BIG_BK);

  floatx16 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
      for (int e = 0; e < 16; e++) acc[i][j][e] = 0.0f;

  float vi[4][4], vj[4][4];
  if (nk > 0) {
    big_load<SIDE>(a, cI, k0, kend, vi);
    if (!diag) big_load<SIDE>(a, cJ, k0, kend, vj);
    big_store<SIDE>(at(0, 0, 0), at(0, 0, 1), vi);
    if (!diag) big_store<SIDE>(at(0, 1, 0), at(0, 1, 1), vj);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; kt++) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) {
      const int64_t kb = k0 + (int64_t)(kt + 1) * BIG_BK;
      big_load<SIDE>(a, cI, kb, kend, vi);
      if (!diag) big_load<SIDE>(a, cJ, kb, kend, vj);
    }
    const __bf16* Ih = at(cur, 0, 0);
    const __bf16* Il = at(cur, 0, 1);
    const __bf16* Jh = diag ? Ih : at(cur, 1, 0);
    const __bf16* Jl = diag ? Il : at(cur, 1, 1);
#pragma unroll
    for (int ks = 0; ks < BIG_BK; ks += 16) {
      bf16x8 ah[4], al[4], bh[2], bl[2];
      const int kofs = ks + 8 * (lane >> 5);
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int r = wm * 128 + i * 32 + (lane & 31);
        ah[i] = *(const bf16x8*)(Ih + r * BIG_LDK + kofs);
        al[i] = *(const bf16x8*)(Il + r * BIG_LDK + kofs);
      }
#pragma unroll
      for (int j = 0; j < 2; j++) {
        const int c = wn * 64 + j * 32 + (lane & 31);
        bh[j] = *(const bf16x8*)(Jh + c * BIG_LDK + kofs);
        bl[j] = *(const bf16x8*)(Jl + c * BIG_LDK + kofs);
      }
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
    if (more) {
      big_store<SIDE>(at(cur ^ 1, 0, 0), at(cur ^ 1, 0, 1), vi);
      if (!diag) big_store<SIDE>(at(cur ^ 1, 1, 0), at(cur ^ 1, 1, 1), vj);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
      for (int e = 0; e < 16; e++) {
        const int r = wm * 128 + i * 32 + (e >> 2) * 8 + (lane >> 5) * 4 + (e & 3);
        const int c = wn * 64 + j * 32 + (lane & 31);
        out[r * BIG_BM + c] = acc[i][j][e];
      }
}

// ---------------------------------------------------------------------------
// Reduction of chunk partials into the full symmetric B.
// One workgroup per 32x32 sub-tile of a triangle tile; sums the S partials in
// chunk order, then writes the sub-tile and (through LDS) its transpose, both
// coalesced.  Sub-tiles strictly above the diagonal of a diagonal tile are
// skipped; on diagonal sub-tiles only the lower half is taken from the sums.
// ---------------------------------------------------------------------------
template <typename OT, int BM>
__device__ __forceinline__ void syrk_reduce_unit(const OT* partial, int T, int S, int64_t d, OT* B, int64_t ldb,
                                                 int accumulate, int unit) {
  constexpr int SUB = BM / 32;
  const int t = unit / (SUB * SUB);
  const int sub = unit % (SUB * SUB);
  const int sr = sub / SUB, sc = sub % SUB;
  int ti, tj;
  tri_tile(t, ti, tj);
  if (ti == tj && sr < sc) return;
  __shared__ OT tile[32][33];
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)ti * BM + sr * 32, col0 = (int64_t)tj * BM + sc * 32;
  const bool dsub = (ti == tj && sr == sc);
#pragma unroll
  for (int e = 0; e < 4; e++) {
    const int idx = tid + 256 * e;  // 0..1023
    const int r = idx >> 5, c = idx & 31;
    const int64_t off = (int64_t)(sr * 32 + r) * BM + sc * 32 + c;
    OT acc = 0;
    for (int s = 0; s < S; s++) acc += partial[((int64_t)s * T + t) * BM * BM + off];
    const int64_t gr = row0 + r, gc = col0 + c;
    if (accumulate && gr < d && gc < d) acc += B[gr * ldb + gc];
    tile[r][c] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 4; e++) {
    const int idx = tid + 256 * e;
    const int r = idx >> 5, c = idx & 31;
    const int64_t gr = row0 + r, gc = col0 + c;
    // lower/direct part
    if (gr < d && gc < d && (!dsub || r >= c)) B[gr * ldb + gc] = tile[r][c];
    // mirrored part: B[col0 + r][row0 + c] = tile[c][r]; on a diagonal sub-tile
    // only the strict upper half is filled this way
    const int64_t mr = col0 + r, mc = row0 + c;
    if (mr < d && mc < d && (!dsub || c > r)) B[mr * ldb + mc] = tile[c][r];
  }
}

template <typename OT, int BM>
__global__ __launch_bounds__(256) void syrk_reduce_kernel(const OT* partial, int T, int S, int64_t d, OT* B,
                                                          int64_t ldb, int accumulate) {
  syrk_reduce_unit<OT, BM>(partial, T, S, d, B, ldb, accumulate, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Grouped Gram for a batch of problems (128 tiles, FP32 or BF16X3): workgroup
// ids are dealt to problems by prefix sums of their unit counts.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_job(const GramJob* jobs, int njobs, int64_t u, bool reduce) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((reduce ? jobs[mid].rbegin : jobs[mid].ubegin) <= u) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ SyrkArgs job_args(const GramJob& j) {
  SyrkArgs a;
  a.A = j.A; a.m = j.m; a.n = j.n; a.lda = j.lda;
  a.d = j.side == 0 ? j.n : j.m;
  a.K = j.side == 0 ? j.m : j.n;
  a.kchunk = j.kchunk; a.nt = j.nt; a.T = j.T; a.S = j.S; a.xcd_map = 0;
  a.vec_ok = j.vec_ok;
  a.partial = j.partial;
  return a;
}

// all jobs of one launch share the side (one LDS layout per kernel)
template <int MODE, int SIDE>
__global__ __launch_bounds__(256) void syrk_grouped_kernel(const GramJob* jobs, int njobs) {
  const int jb = find_job(jobs, njobs, blockIdx.x, false);
  const GramJob& j = jobs[jb];
  const SyrkArgs a = job_args(j);
  const int u = (int)(blockIdx.x - j.ubegin);
  syrk_unit<MODE, SIDE>(a, u / j.T, u % j.T);
}

__global__ __launch_bounds__(256) void syrk_grouped_reduce_kernel(const GramJob* jobs, int njobs) {
  const int jb = find_job(jobs, njobs, blockIdx.x, true);
  const GramJob& j = jobs[jb];
  syrk_reduce_unit<float, 128>((const float*)j.partial, j.T, j.S, j.side == 0 ? j.n : j.m, (float*)j.B, j.ldb, 0,
                               (int)(blockIdx.x - j.rbegin));
}

int syrk_grouped_launch(int mode, int side, const GramJob* d_jobs, int njobs, int64_t units, int64_t runits,
                        hipStream_t s) {
  if (njobs <= 0) return 0;
  const dim3 g((unsigned)units), blk(256);
  if (mode == MODE_BF16X3) {
    if (side == 0) hipLaunchKernelGGL((syrk_grouped_kernel<MODE_BF16X3, 0>), g, blk, 0, s, d_jobs, njobs);
    else hipLaunchKernelGGL((syrk_grouped_kernel<MODE_BF16X3, 1>), g, blk, 0, s, d_jobs, njobs);
  } else {
    if (side == 0) hipLaunchKernelGGL((syrk_grouped_kernel<MODE_FP32, 0>), g, blk, 0, s, d_jobs, njobs);
    else hipLaunchKernelGGL((syrk_grouped_kernel<MODE_FP32, 1>), g, blk, 0, s, d_jobs, njobs);
  }
  TSVD_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(syrk_grouped_reduce_kernel, dim3((unsigned)runits), dim3(256), 0, s, d_jobs, njobs);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
int syrk_plan(int mode, int64_t d, int64_t K, int64_t rows_per_block, int num_cu, SyrkPlan* p, int tile,
              int chunks) {
  // BF16X3 uses 256-wide tiles for large Grams unless told otherwise
  if (mode == MODE_BF16X3 && tile == 0) tile = d >= 1024 ? 256 : 128;
  const int BM = (mode == MODE_FP64) ? 64 : (mode == MODE_BF16X3 && tile == 256 ? 256 : 128);
  const int BK = (mode == MODE_FP64) ? 16 : 32;
  p->BM = BM;
  p->nt = (int)((d + BM - 1) / BM);
  p->T = p->nt * (p->nt + 1) / 2;
  int64_t S;
  if (rows_per_block > 0) {
    S = (K + rows_per_block - 1) / rows_per_block;
  } else if (chunks > 0) {
    S = chunks;
  } else {
    const int64_t target = (BM == 256 ? 8 : 4) * (int64_t)num_cu;  // workgroups per CU: 1 for 256 tiles, 2 else
    S = (target + p->T - 1) / p->T;
    if (S > 1) S = ((S + 7) / 8) * 8;  // whole XCD rounds; a Gram with enough tiles takes one chunk
    const int64_t maxS = (K + 4 * BK - 1) / (4 * BK);  // at least 4 k-stages per chunk
    if (BM == 256 && S > 1) {
      // one 256-tile workgroup per CU: take up to two more XCD rounds of
      // chunks if that fills the last wave of workgroups (T x S close to a
      // multiple of the CU count; at 136 tiles 24 chunks fill 98 % against
      // 94 % for 16, 0.3 ms less at 200,000 x 4,096 with the reduction)
      auto fill = [&](int64_t s) {
        const double w = (double)p->T * (double)s / num_cu;
        return w / std::ceil(w);
      };
      int64_t best = S;
      if (fill(S) < 0.97)
        for (int64_t c = S + 8; c <= S + 16 && c <= maxS && c <= 256; c += 8)
          if (fill(c) >= 0.97 || fill(c) > fill(best) + 0.02) { best = c; if (fill(c) >= 0.97) break; }
      S = best;
    }
    if (S > maxS) S = maxS;
    if (S > 256) S = 256;
    if (S < 1) S = 1;
  }
  if (K == 0) S = 1;
  p->S = (int)S;
  p->kchunk = K > 0 ? (K + S - 1) / S : 1;
  if (rows_per_block > 0) p->kchunk = rows_per_block;
  // round chunk to the k-stage so only the last chunk is ragged
  p->kchunk = ((p->kchunk + BK - 1) / BK) * BK;
  p->S = (int)(K > 0 ? (K + p->kchunk - 1) / p->kchunk : 1);
  p->xcd_map = (p->S % 8 == 0) ? 1 : 0;
  p->partial_elems = (int64_t)p->S * p->T * BM * BM;
  p->partial_bytes = (size_t)p->partial_elems * (mode == MODE_FP64 ? 8 : 4);
  return 0;
}

int syrk_launch(int mode, int side, const void* A, int64_t m, int64_t n, int64_t lda, const SyrkPlan& p,
                void* partial, void* B, int64_t ldb, int accumulate, hipStream_t stream) {
  SyrkArgs a;
  a.A = A; a.m = m; a.n = n; a.lda = lda;
  a.d = side == 0 ? n : m;
  a.K = side == 0 ? m : n;
  a.kchunk = p.kchunk; a.nt = p.nt; a.T = p.T; a.S = p.S; a.xcd_map = p.xcd_map;
  a.vec_ok = (((uintptr_t)A & 15) == 0) && (lda % 4 == 0);
  a.partial = partial;
  const int grid = p.T * p.S;
  if (mode == MODE_BF16X3 && p.BM == 256) {
    const void* fn = side == 0 ? (const void*)syrk_bf16x3_big_kernel<0> : (const void*)syrk_bf16x3_big_kernel<1>;
    TSVD_HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)BIG_LDS));
    if (side == 0) hipLaunchKernelGGL((syrk_bf16x3_big_kernel<0>), dim3(grid), dim3(512), BIG_LDS, stream, a);
    else hipLaunchKernelGGL((syrk_bf16x3_big_kernel<1>), dim3(grid), dim3(512), BIG_LDS, stream, a);
  } else if (mode == MODE_BF16X3) {
    if (side == 0) hipLaunchKernelGGL((syrk_partial_kernel<MODE_BF16X3, 0>), dim3(grid), dim3(256), 0, stream, a);
    else hipLaunchKernelGGL((syrk_partial_kernel<MODE_BF16X3, 1>), dim3(grid), dim3(256), 0, stream, a);
  } else if (mode == MODE_FP32) {
    if (side == 0) hipLaunchKernelGGL((syrk_partial_kernel<MODE_FP32, 0>), dim3(grid), dim3(256), 0, stream, a);
    else hipLaunchKernelGGL((syrk_partial_kernel<MODE_FP32, 1>), dim3(grid), dim3(256), 0, stream, a);
  } else {
    if (side == 0) hipLaunchKernelGGL((syrk_partial_kernel<MODE_FP64, 0>), dim3(grid), dim3(256), 0, stream, a);
    else hipLaunchKernelGGL((syrk_partial_kernel<MODE_FP64, 1>), dim3(grid), dim3(256), 0, stream, a);
  }
  TSVD_HIP_TRY(hipGetLastError());
  const int SUB = p.BM / 32;
  const int rgrid = p.T * SUB * SUB;
  if (mode == MODE_FP64)
    hipLaunchKernelGGL((syrk_reduce_kernel<double, 64>), dim3(rgrid), dim3(256), 0, stream, (const double*)partial,
                       p.T, p.S, a.d, (double*)B, ldb, accumulate);
  else if (p.BM == 256)
    hipLaunchKernelGGL((syrk_reduce_kernel<float, 256>), dim3(rgrid), dim3(256), 0, stream, (const float*)partial,
                       p.T, p.S, a.d, (float*)B, ldb, accumulate);
  else
    hipLaunchKernelGGL((syrk_reduce_kernel<float, 128>), dim3(rgrid), dim3(256), 0, stream, (const float*)partial,
                       p.T, p.S, a.d, (float*)B, ldb, accumulate);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace tsvd
