// Device-side pieces of the Gram product shared by the Gram launches and the
// batched engine: the per-mode tile configurations, the work-unit mapping,
// the staging of panels (with the BF16X3 hi/lo split) and the work units
// themselves.  A unit's LDS comes from the caller (a static buffer of the
// stand-alone kernels, the dynamic LDS of the batched engine).
#pragma once

#include "common.h"
#include "internal.h"

namespace tsvd {

// BM: triangle tile edge.  BF16X3 and FP32 take 128 (the stand-alone 128-tile
// launch and the batched engine) or 64 (the engine, for small Gram
// dimensions); a tile's partial sums do not depend on its edge, because every
// element is accumulated over the same contraction steps in the same order.
template <int MODE, int BM_ = (MODE == MODE_FP64 ? 64 : 128)> struct SyrkCfg;
template <int BM_> struct SyrkCfg<MODE_BF16X3, BM_> {
  static_assert(BM_ == 64 || BM_ == 128, "BF16X3 tile edge");
  static constexpr int BM = BM_, BK = 32, LDK = BK + 8;  // LDS row of bf16
  using AT = float; using OT = float;
  static constexpr size_t LDS = (size_t)2 * 2 * 2 * BM * LDK * 2;  // stages x panels x hi/lo
};
template <int BM_> struct SyrkCfg<MODE_FP32, BM_> {
  static_assert(BM_ == 64 || BM_ == 128, "FP32 tile edge");
  static constexpr int BM = BM_, BK = 32, LDK = BK + 4;  // LDS row of float
  using AT = float; using OT = float;
  static constexpr size_t LDS = (size_t)2 * 2 * BM * LDK * 4;      // stages x panels
};
template <int BM_> struct SyrkCfg<MODE_FP64, BM_> {
  static_assert(BM_ == 64, "FP64 tile edge");
  static constexpr int BM = 64, BK = 16, LDK = BK + 2;   // LDS row of double
  using AT = double; using OT = double;
  static constexpr size_t LDS = (size_t)2 * 2 * BM * LDK * 8;
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
// A thread holds 4 k x CW columns (SIDE 0) or BM/32 panel rows x 4 k (SIDE 1)
// in v; with BM = 64 only the first half of v's inner (SIDE 0) or outer
// (SIDE 1) index is used.
// ---------------------------------------------------------------------------
template <int SIDE, int BM = 128>
__device__ __forceinline__ void load_panel_bf16(const SyrkArgs& a, int64_t c0, int64_t k0, int64_t kend,
                                                float (&v)[4][4]) {
  const float* A = (const float*)a.A;
  const int tid = threadIdx.x;
  if (SIDE == 0) {
    // rows k (contraction) x columns c of A; thread covers 4 rows x CW columns
    constexpr int CW = BM / 32;
    const int rg = tid & 7, cg = tid >> 3;
    const int64_t c = c0 + CW * cg;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int64_t k = k0 + 4 * rg + j;
      const float* p = A + k * a.lda + c;
      if (k < kend && a.vec_ok && c + CW - 1 < a.d) {
        if constexpr (CW == 4) {
          float4 f = *(const float4*)p;
          v[j][0] = f.x; v[j][1] = f.y; v[j][2] = f.z; v[j][3] = f.w;
        } else {
          float2 f = *(const float2*)p;
          v[j][0] = f.x; v[j][1] = f.y;
        }
      } else {
#pragma unroll
        for (int i = 0; i < CW; i++) v[j][i] = (k < kend && c + i < a.d) ? p[i] : 0.0f;
      }
    }
  } else {
    // rows c of A (panel rows) x columns k (contraction); thread covers BM/32 rows x 4 k
    const int kg = tid & 7, rr = tid >> 3;
    const int64_t k = k0 + 4 * kg;
#pragma unroll
    for (int q = 0; q < BM / 32; q++) {
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

template <int SIDE, int BM = 128>
__device__ __forceinline__ void store_panel_bf16(__bf16* hi, __bf16* lo, const float (&v)[4][4]) {
  constexpr int LDK = SyrkCfg<MODE_BF16X3, BM>::LDK;
  const int tid = threadIdx.x;
  if (SIDE == 0) {
    constexpr int CW = BM / 32;
    const int rg = tid & 7, cg = tid >> 3;
#pragma unroll
    for (int i = 0; i < CW; i++) {         // column CW*cg+i holds k = 4rg..4rg+3 = v[0..3][i]
      bf16x4 h, l;
#pragma unroll
      for (int j = 0; j < 4; j++) { __bf16 x, y; split_bf16(v[j][i], x, y); h[j] = x; l[j] = y; }
      const int off = (CW * cg + i) * LDK + 4 * rg;
      *(bf16x4*)(hi + off) = h;
      *(bf16x4*)(lo + off) = l;
    }
  } else {
    const int kg = tid & 7, rr = tid >> 3;
#pragma unroll
    for (int q = 0; q < BM / 32; q++) {    // panel row rr+32q holds k = 4kg..4kg+3 = v[q][0..3]
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
template <int MODE, int SIDE, int BM = SyrkCfg<MODE>::BM>
__device__ __forceinline__ void load_panel_elem(const SyrkArgs& a, int64_t c0, int64_t k0, int64_t kend,
                                                typename SyrkCfg<MODE, BM>::AT (&v)[BM * SyrkCfg<MODE, BM>::BK / 256]) {
  using Cfg = SyrkCfg<MODE, BM>;
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

template <int MODE, int SIDE, int BM = SyrkCfg<MODE>::BM>
__device__ __forceinline__ void store_panel_elem(typename SyrkCfg<MODE, BM>::AT* s,
                                                 const typename SyrkCfg<MODE, BM>::AT (&v)[BM * SyrkCfg<MODE, BM>::BK / 256]) {
  using Cfg = SyrkCfg<MODE, BM>;
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
template <int MODE, int SIDE, int BM_ = SyrkCfg<MODE>::BM>
__device__ __forceinline__ void syrk_unit(const SyrkArgs& a, int s, int t, unsigned char* smem) {
  using Cfg = SyrkCfg<MODE, BM_>;
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
  constexpr int WT = BM / 64;                 // 32 x 32 MFMA tiles per wave and dimension (BF16X3, FP32)
  OT* out = (OT*)a.partial + ((int64_t)s * a.T + t) * BM * BM;
  const int nk = (int)((kend - k0 + BK - 1) / BK);

  if constexpr (MODE == MODE_BF16X3) {
    // LDS: [stage][panel I/J][hi/lo][BM][LDK] bf16
    __bf16 (*lds)[2][2][BM * LDK] = reinterpret_cast<__bf16 (*)[2][2][BM * LDK]>(smem);
    floatx16 acc[WT][WT];
#pragma unroll
    for (int i = 0; i < WT; i++)
#pragma unroll
      for (int j = 0; j < WT; j++)
#pragma unroll
        for (int e = 0; e < 16; e++) acc[i][j][e] = 0.0f;

    float vi[4][4], vj[4][4];
    if (nk > 0) {
      load_panel_bf16<SIDE, BM>(a, cI, k0, kend, vi);
      if (!diag) load_panel_bf16<SIDE, BM>(a, cJ, k0, kend, vj);
      store_panel_bf16<SIDE, BM>(lds[0][0][0], lds[0][0][1], vi);
      if (!diag) store_panel_bf16<SIDE, BM>(lds[0][1][0], lds[0][1][1], vj);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; kt++) {
      const int cur = kt & 1;
      const bool more = kt + 1 < nk;
      if (more) {
        const int64_t kb = k0 + (int64_t)(kt + 1) * BK;
        load_panel_bf16<SIDE, BM>(a, cI, kb, kend, vi);
        if (!diag) load_panel_bf16<SIDE, BM>(a, cJ, kb, kend, vj);
      }
      const __bf16* Ih = lds[cur][0][0];
      const __bf16* Il = lds[cur][0][1];
      const __bf16* Jh = diag ? Ih : lds[cur][1][0];
      const __bf16* Jl = diag ? Il : lds[cur][1][1];
#pragma unroll
      for (int ks = 0; ks < BK; ks += 16) {
        bf16x8 ah[WT], al[WT], bh[WT], bl[WT];
        const int kofs = ks + 8 * (lane >> 5);
#pragma unroll
        for (int i = 0; i < WT; i++) {
          const int r = wm * (BM / 2) + i * 32 + (lane & 31);
          ah[i] = *(const bf16x8*)(Ih + r * LDK + kofs);
          al[i] = *(const bf16x8*)(Il + r * LDK + kofs);
        }
#pragma unroll
        for (int j = 0; j < WT; j++) {
          const int c = wn * (BM / 2) + j * 32 + (lane & 31);
          bh[j] = *(const bf16x8*)(Jh + c * LDK + kofs);
          bl[j] = *(const bf16x8*)(Jl + c * LDK + kofs);
        }
#pragma unroll
        for (int i = 0; i < WT; i++)
#pragma unroll
          for (int j = 0; j < WT; j++) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          }
      }
      if (more) {
        store_panel_bf16<SIDE, BM>(lds[cur ^ 1][0][0], lds[cur ^ 1][0][1], vi);
        if (!diag) store_panel_bf16<SIDE, BM>(lds[cur ^ 1][1][0], lds[cur ^ 1][1][1], vj);
      }
      __syncthreads();
    }
    // 32x32 accumulator layout: item e -> row (e/4)*8 + (lane/32)*4 + e%4, col lane%32
#pragma unroll
    for (int i = 0; i < WT; i++)
#pragma unroll
      for (int j = 0; j < WT; j++)
#pragma unroll
        for (int e = 0; e < 16; e++) {
          const int r = wm * (BM / 2) + i * 32 + (e >> 2) * 8 + (lane >> 5) * 4 + (e & 3);
          const int c = wn * (BM / 2) + j * 32 + (lane & 31);
          out[r * BM + c] = acc[i][j][e];
        }
  } else if constexpr (MODE == MODE_FP32) {
    float (*lds)[2][BM * LDK] = reinterpret_cast<float (*)[2][BM * LDK]>(smem);
    constexpr int E = BM * BK / 256;
    floatx16 acc[WT][WT];
#pragma unroll
    for (int i = 0; i < WT; i++)
#pragma unroll
      for (int j = 0; j < WT; j++)
#pragma unroll
        for (int e = 0; e < 16; e++) acc[i][j][e] = 0.0f;
    float vi[E], vj[E];
    if (nk > 0) {
      load_panel_elem<MODE, SIDE, BM>(a, cI, k0, kend, vi);
      if (!diag) load_panel_elem<MODE, SIDE, BM>(a, cJ, k0, kend, vj);
      store_panel_elem<MODE, SIDE, BM>(lds[0][0], vi);
      if (!diag) store_panel_elem<MODE, SIDE, BM>(lds[0][1], vj);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; kt++) {
      const int cur = kt & 1;
      const bool more = kt + 1 < nk;
      if (more) {
        const int64_t kb = k0 + (int64_t)(kt + 1) * BK;
        load_panel_elem<MODE, SIDE, BM>(a, cI, kb, kend, vi);
        if (!diag) load_panel_elem<MODE, SIDE, BM>(a, cJ, kb, kend, vj);
      }
      const float* I = lds[cur][0];
      const float* J = diag ? I : lds[cur][1];
      // lane half h consumes k = 2*s + h for s = 0..15: stored at h*16 + s
      const int h = lane >> 5;
      float av[WT][16], bv[WT][16];
#pragma unroll
      for (int i = 0; i < WT; i++) {
        const int r = wm * (BM / 2) + i * 32 + (lane & 31);
#pragma unroll
        for (int q = 0; q < 4; q++) {
          float4 f = *(const float4*)(I + r * LDK + h * 16 + 4 * q);
          av[i][4 * q] = f.x; av[i][4 * q + 1] = f.y; av[i][4 * q + 2] = f.z; av[i][4 * q + 3] = f.w;
        }
      }
#pragma unroll
      for (int j = 0; j < WT; j++) {
        const int c = wn * (BM / 2) + j * 32 + (lane & 31);
#pragma unroll
        for (int q = 0; q < 4; q++) {
          float4 f = *(const float4*)(J + c * LDK + h * 16 + 4 * q);
          bv[j][4 * q] = f.x; bv[j][4 * q + 1] = f.y; bv[j][4 * q + 2] = f.z; bv[j][4 * q + 3] = f.w;
        }
      }
#pragma unroll
      for (int ss = 0; ss < 16; ss++)
#pragma unroll
        for (int i = 0; i < WT; i++)
#pragma unroll
          for (int j = 0; j < WT; j++)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i][ss], bv[j][ss], acc[i][j], 0, 0, 0);
      if (more) {
        store_panel_elem<MODE, SIDE, BM>(lds[cur ^ 1][0], vi);
        if (!diag) store_panel_elem<MODE, SIDE, BM>(lds[cur ^ 1][1], vj);
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < WT; i++)
#pragma unroll
      for (int j = 0; j < WT; j++)
#pragma unroll
        for (int e = 0; e < 16; e++) {
          const int r = wm * (BM / 2) + i * 32 + (e >> 2) * 8 + (lane >> 5) * 4 + (e & 3);
          const int c = wn * (BM / 2) + j * 32 + (lane & 31);
          out[r * BM + c] = acc[i][j][e];
        }
  } else {
    // FP64: BM = 64, waves 2 x 2 of 32 x 32, MFMA tiles 16 x 16 x 4
    double (*lds)[2][BM * LDK] = reinterpret_cast<double (*)[2][BM * LDK]>(smem);
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


// ---------------------------------------------------------------------------
// Reduction of chunk partials into the full symmetric B.
// One workgroup per 32x32 sub-tile of a triangle tile; sums the S partials in
// chunk order, then writes the sub-tile and (through LDS) its transpose, both
// coalesced.  Sub-tiles strictly above the diagonal of a diagonal tile are
// skipped; on diagonal sub-tiles only the lower half is taken from the sums.
// ---------------------------------------------------------------------------
template <typename OT, int BM>
__device__ __forceinline__ void syrk_reduce_unit(const OT* partial, int T, int S, int64_t d, OT* B, int64_t ldb,
                                                 int accumulate, int unit, unsigned char* smem) {
  constexpr int SUB = BM / 32;
  const int t = unit / (SUB * SUB);
  const int sub = unit % (SUB * SUB);
  const int sr = sub / SUB, sc = sub % SUB;
  int ti, tj;
  tri_tile(t, ti, tj);
  if (ti == tj && sr < sc) return;
  OT (*tile)[33] = reinterpret_cast<OT (*)[33]>(smem);
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

}  // namespace tsvd
