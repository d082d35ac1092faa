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
#include "syrk_dev.h"

namespace tsvd {

template <int MODE, int SIDE>
__global__ __launch_bounds__(256) void syrk_partial_kernel(SyrkArgs a) {
  __shared__ __align__(16) unsigned char smem[SyrkCfg<MODE>::LDS];
  int s, t;
  unit_of(a, blockIdx.x, s, t);
  syrk_unit<MODE, SIDE>(a, s, t, smem);
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
// BF16X3 Gram of 256-wide tiles over an A resident in HBM, in two passes.
// Pass 1 (split_pack_kernel) reads A once and writes its hi and lo parts as
// two BF16 planes in a k-packed layout: plane[g * dp + c] is the 16-byte chunk
// of the 8 contraction indices 8g .. 8g + 7 of Gram index c, zero beyond K and
// d, so the planes need no bounds checks.  Pass 2 (syrk_packed_kernel) loads
// those chunks straight into LDS with global_load_lds_dwordx4 (no register
// staging and no split in its loop), four 16-wide k-stages ahead.  The LDS
// layout of a stage is the planes' layout, which is also what an MFMA lane
// reads: 8 consecutive k of one row in one 16-byte load, 32 rows of one
// 16-byte group contiguous (conflict-free).  Per 16 k the tile takes the big
// kernel's products in the big kernel's order, so its partial tiles are the
// same bits.
// ---------------------------------------------------------------------------
constexpr int PK_BK = 16, PK_NS = 4;                           // k per stage, stages in flight
constexpr int PK_BUF = (PK_BK / 8) * BIG_BM * 16;              // one plane of one panel per stage (8 KB)
constexpr int PK_STAGE = 4 * PK_BUF;                           // I hi, I lo, J hi, J lo
constexpr size_t PK_LDS = (size_t)PK_NS * PK_STAGE;            // 128 KB

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

template <int SIDE>
__global__ __launch_bounds__(256) void split_pack_kernel(const float* A, int64_t lda, int64_t d, int64_t K, int64_t dp,
                                                         int64_t ng, int vec_ok, bf16x8* H, bf16x8* L) {
  const int64_t t = blockIdx.x * 256ll + threadIdx.x;
  if (SIDE == 0) {
    // rows k of A are the contraction: a thread splits 4 columns of 8 rows
    const int64_t nc4 = dp / 4;
    if (t >= ng * nc4) return;
    const int64_t g = t / nc4, c = 4 * (t % nc4);
    float v[8][4];
#pragma unroll
    for (int e = 0; e < 8; e++) {
      const int64_t k = 8 * g + e;
      const float* p = A + k * lda + c;
      if (k < K && vec_ok && c + 3 < d) {
        const float4 f = *(const float4*)p;
        v[e][0] = f.x; v[e][1] = f.y; v[e][2] = f.z; v[e][3] = f.w;
      } else {
#pragma unroll
        for (int i = 0; i < 4; i++) v[e][i] = (k < K && c + i < d) ? p[i] : 0.0f;
      }
    }
#pragma unroll
    for (int i = 0; i < 4; i++) {
      bf16x8 h, l;
#pragma unroll
      for (int e = 0; e < 8; e++) { __bf16 x, y; split_bf16(v[e][i], x, y); h[e] = x; l[e] = y; }
      H[g * dp + c + i] = h;
      L[g * dp + c + i] = l;
    }
  } else {
    // columns of A are the contraction: a thread splits 4 groups of 8 of one row
    const int64_t ng4 = (ng + 3) / 4;
    if (t >= ng4 * dp) return;
    const int64_t c = t % dp, g0 = 4 * (t / dp);
#pragma unroll
    for (int gi = 0; gi < 4; gi++) {
      const int64_t g = g0 + gi;
      if (g >= ng) break;
      float v[8];
      const float* p = A + c * lda + 8 * g;
      if (c < d && vec_ok && 8 * g + 7 < K) {
        const float4 f0 = *(const float4*)p, f1 = *(const float4*)(p + 4);
        v[0] = f0.x; v[1] = f0.y; v[2] = f0.z; v[3] = f0.w; v[4] = f1.x; v[5] = f1.y; v[6] = f1.z; v[7] = f1.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; e++) v[e] = (c < d && 8 * g + e < K) ? p[e] : 0.0f;
      }
      bf16x8 h, l;
#pragma unroll
      for (int e = 0; e < 8; e++) { __bf16 x, y; split_bf16(v[e], x, y); h[e] = x; l[e] = y; }
      H[g * dp + c] = h;
      L[g * dp + c] = l;
    }
  }
}

struct PackArgs {
  const bf16x8* H;
  const bf16x8* L;
  int64_t dp, Kp, kchunk;
  int nt, T, S, xcd_map;
  float* partial;
};

// s_waitcnt vmcnt(N) alone (the other counters at their maxima)
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x70 | 0xF00);
}
// keeps the compiler from moving memory operations across the hardware barrier
__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

template <bool DIAG>
__device__ __forceinline__ void packed_tile(const PackArgs& a, unsigned char* smem, int s, int ti, int tj) {
  constexpr int NBUF = DIAG ? 2 : 4;                 // a diagonal tile needs panel I only
  constexpr int IPB = (PK_BK / 8) * BIG_BM / 64;     // wave-loads per buffer and stage
  constexpr int LPW = NBUF * IPB / 8;                // per wave and stage
  static_assert(NBUF * IPB % 8 == 0, "loads per wave");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave >> 2, wn = wave & 3;           // 2 x 4 waves, each 128 x 64
  const int64_t k0 = (int64_t)s * a.kchunk;
  const int64_t kend = k0 + a.kchunk < a.Kp ? k0 + a.kchunk : a.Kp;
  const int nk = (int)((kend - k0) / PK_BK);
  const int64_t cI = (int64_t)ti * BIG_BM, cJ = (int64_t)tj * BIG_BM;

  // stage kt into LDS slot `slot`: wave-load u covers 64 consecutive chunks
  // (one 1 KB run in the plane and in LDS; lane i lands at offset 16 i)
  auto issue = [&](int kt, int slot) {
    const int64_t gb = (k0 + (int64_t)kt * PK_BK) / 8;
#pragma unroll
    for (int i = 0; i < LPW; i++) {
      const int u = wave * LPW + i;
      const int b = u / IPB, r = u % IPB;
      const int q = r * 64 + lane;
      const int g = q / BIG_BM, c = q % BIG_BM;
      const bf16x8* src = ((b & 1) ? a.L : a.H) + (gb + g) * a.dp + ((b < 2) ? cI : cJ) + c;
      unsigned char* dst = smem + slot * PK_STAGE + b * PK_BUF + r * 1024;
      __builtin_amdgcn_global_load_lds((glb_void_t*)src, (lds_void_t*)dst, 16, 0, 0);
    }
  };

  floatx16 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
      for (int e = 0; e < 16; e++) acc[i][j][e] = 0.0f;

#pragma unroll
  for (int st = 0; st < PK_NS - 1; st++)
    if (st < nk) issue(st, st);
  for (int kt = 0; kt < nk; kt++) {
    // this wave's loads of stage kt are done once at most the later stages'
    // are outstanding; the barrier then makes every wave's visible, and every
    // wave is past its reads of the slot refilled below
    if (kt + PK_NS - 2 < nk) wait_vmcnt<LPW * (PK_NS - 2)>();
    else wait_vmcnt<0>();
    compiler_fence();
    __builtin_amdgcn_s_barrier();
    compiler_fence();
    if (kt + PK_NS - 1 < nk) issue(kt + PK_NS - 1, (kt + PK_NS - 1) % PK_NS);
    const unsigned char* base = smem + (kt % PK_NS) * PK_STAGE;
    const __bf16* Ih = (const __bf16*)base;
    const __bf16* Il = (const __bf16*)(base + PK_BUF);
    const __bf16* Jh = DIAG ? Ih : (const __bf16*)(base + 2 * PK_BUF);
    const __bf16* Jl = DIAG ? Il : (const __bf16*)(base + 3 * PK_BUF);
    const int g = lane >> 5;
    bf16x8 ah[4], al[4], bh[2], bl[2];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int r = wm * 128 + i * 32 + (lane & 31);
      ah[i] = *(const bf16x8*)(Ih + (g * BIG_BM + r) * 8);
      al[i] = *(const bf16x8*)(Il + (g * BIG_BM + r) * 8);
    }
#pragma unroll
    for (int j = 0; j < 2; j++) {
      const int c = wn * 64 + j * 32 + (lane & 31);
      bh[j] = *(const bf16x8*)(Jh + (g * BIG_BM + c) * 8);
      bl[j] = *(const bf16x8*)(Jl + (g * BIG_BM + c) * 8);
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
  wait_vmcnt<0>();  // no load into LDS may outlive the workgroup
  float* out = a.partial + ((int64_t)s * a.T + (ti * (ti + 1) / 2 + tj)) * BIG_BM * BIG_BM;
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

__global__ __launch_bounds__(512, 1) void syrk_packed_kernel(PackArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  int s, t;
  if (a.xcd_map) {
    const int x = blockIdx.x & 7, local = blockIdx.x >> 3;
    s = x + 8 * (local / a.T);
    t = local % a.T;
  } else {
    s = blockIdx.x / a.T;
    t = blockIdx.x % a.T;
  }
  int ti, tj;
  tri_tile(t, ti, tj);
  if (ti == tj) packed_tile<true>(a, smem, s, ti, tj);
  else packed_tile<false>(a, smem, s, ti, tj);
}

template <typename OT, int BM>
__global__ __launch_bounds__(256) void syrk_reduce_kernel(const OT* partial, int T, int S, int64_t d, OT* B,
                                                          int64_t ldb, int accumulate) {
  __shared__ __align__(16) unsigned char smem[32 * 33 * sizeof(OT)];
  syrk_reduce_unit<OT, BM>(partial, T, S, d, B, ldb, accumulate, blockIdx.x, smem);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
int syrk_plan(int mode, int64_t d, int64_t K, int64_t rows_per_block, int num_cu, SyrkPlan* p, int tile,
              int chunks, int packed_ok) {
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
  p->packed = 0;
  p->dp = p->Kp = 0;
  p->plane_off = 0;
  if (packed_ok && mode == MODE_BF16X3 && BM == 256 && rows_per_block <= 0 && K > 0) {
    // the chunks end on 32-row boundaries and the last one starts below K, so
    // every stage of every chunk lies inside the planes' Kp rows
    p->packed = 1;
    p->dp = (int64_t)p->nt * BIG_BM;
    p->Kp = ((K + 31) / 32) * 32;
    p->plane_off = (p->partial_bytes + 255) & ~(size_t)255;
    p->partial_bytes = p->plane_off + (size_t)4 * p->Kp * p->dp;  // hi and lo, 2 B each
  }
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
  if (p.packed) {
    const int64_t ng = p.Kp / 8;
    bf16x8* H = (bf16x8*)((char*)partial + p.plane_off);
    bf16x8* L = H + ng * p.dp;
    const int64_t nthr = side == 0 ? ng * (p.dp / 4) : ((ng + 3) / 4) * p.dp;
    const dim3 sg((unsigned)((nthr + 255) / 256));
    if (side == 0) hipLaunchKernelGGL((split_pack_kernel<0>), sg, dim3(256), 0, stream, (const float*)A, lda, a.d, a.K, p.dp, ng, a.vec_ok, H, L);
    else hipLaunchKernelGGL((split_pack_kernel<1>), sg, dim3(256), 0, stream, (const float*)A, lda, a.d, a.K, p.dp, ng, a.vec_ok, H, L);
    TSVD_HIP_TRY(hipGetLastError());
    PackArgs pa;
    pa.H = H; pa.L = L; pa.dp = p.dp; pa.Kp = p.Kp; pa.kchunk = p.kchunk;
    pa.nt = p.nt; pa.T = p.T; pa.S = p.S; pa.xcd_map = p.xcd_map; pa.partial = (float*)partial;
    TSVD_HIP_TRY(hipFuncSetAttribute((const void*)syrk_packed_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)PK_LDS));
    hipLaunchKernelGGL(syrk_packed_kernel, dim3(grid), dim3(512), PK_LDS, stream, pa);
  } else if (mode == MODE_BF16X3 && p.BM == 256) {
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
