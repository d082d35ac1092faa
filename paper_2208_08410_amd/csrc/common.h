// Shared device/host helpers for the gfx950 t-SVD kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsvd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Tagged-word exchange between workgroups of one persistent launch.
//
// A value is published as one or two 64-bit words: the high 32 bits carry the
// exchange's epoch, the low 32 bits the payload (a float, or one half of a
// double).  An aligned 64-bit store is single-copy atomic, so a reader that
// sees the expected epoch in a word also sees that word's payload: data and
// synchronisation travel together and no separate barrier is needed.  Stores
// and loads are agent-scope atomics so they are coherent across XCDs.
// Every wait is bounded; a reader that runs out of budget reports failure
// and the kernel exits through its error path.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void ll_store(uint64_t* p, uint32_t epoch, uint32_t payload) {
  uint64_t w = ((uint64_t)epoch << 32) | (uint64_t)payload;
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t ll_load(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void ll_store_f64(uint64_t* p, uint32_t epoch, double v) {
  uint64_t b = __double_as_longlong(v);
  ll_store(p, epoch, (uint32_t)b);
  ll_store(p + 1, epoch, (uint32_t)(b >> 32));
}

// low (half = 0) or high (half = 1) 32 bits of a double, as published by ll_store_f64
__device__ __forceinline__ uint32_t f64_half(double v, int half) {
  const uint64_t b = __double_as_longlong(v);
  return half ? (uint32_t)(b >> 32) : (uint32_t)b;
}

__device__ __forceinline__ double ll_join_f64(uint64_t lo, uint64_t hi) {
  return __longlong_as_double((long long)(((hi & 0xffffffffull) << 32) | (lo & 0xffffffffull)));
}

// Read `count` words starting at p into out[] (payloads), waiting until every
// word carries `epoch`.  Each thread of the block reads words tid, tid + nthr,
// ...; loads are issued W at a time so their latencies overlap.  Returns false
// if the spin budget ran out.
template <int W, typename F>
__device__ __forceinline__ bool ll_read_words(const uint64_t* p, int64_t count, uint32_t epoch, int tid, int nthr,
                                              int64_t& budget, F&& consume) {
  for (int64_t base = 0; base < count; base += (int64_t)nthr * W) {
    uint64_t w[W];
#pragma unroll
    for (int j = 0; j < W; j++) {
      int64_t idx = base + tid + (int64_t)nthr * j;
      w[j] = idx < count ? ll_load(p + idx) : ((uint64_t)epoch << 32);
    }
    while (true) {
      bool all = true;
#pragma unroll
      for (int j = 0; j < W; j++) all = all && ((uint32_t)(w[j] >> 32) == epoch);
      if (all) break;
      if (--budget <= 0) return false;
      __builtin_amdgcn_s_sleep(1);
#pragma unroll
      for (int j = 0; j < W; j++) {
        int64_t idx = base + tid + (int64_t)nthr * j;
        if ((uint32_t)(w[j] >> 32) != epoch) w[j] = ll_load(p + idx);
      }
    }
#pragma unroll
    for (int j = 0; j < W; j++) {
      int64_t idx = base + tid + (int64_t)nthr * j;
      if (idx < count) consume(idx, (uint32_t)w[j]);
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// Deterministic reductions (fixed association order, result taken from lane 0)
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Cross-lane reductions on DPP (data-parallel primitives: a lane reads another
// lane's register inside the VALU instruction), which are much cheaper than
// shuffles through the LDS permute unit.  A double moves as two 32-bit halves.
// Controls (GFX9 family): 0x4E quad_perm [2,3,0,1], 0xB1 quad_perm [1,0,3,2],
// 0x111 + s row_shr:s, 0x130 wave_shl:1, 0x140 row_mirror, 0x141
// row_half_mirror, 0x142 row_bcast:15, 0x143 row_bcast:31.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK, bool BOUND_ZERO>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int tlo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xF, BOUND_ZERO);
  const int thi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xF, BOUND_ZERO);
  return __hiloint2double(thi, tlo);
}
template <int CTRL, int ROW_MASK, bool BOUND_ZERO>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xF, BOUND_ZERO);
}
// the key of another lane, with "no lane" (out of row, or a row left out of
// ROW_MASK) reading as -1: keys travel as key + 1 so that 0 means "none"
template <int CTRL, int ROW_MASK, bool BOUND_ZERO>
__device__ __forceinline__ int dpp_key(int key) {
  return (int)((unsigned)dpp_i32<CTRL, ROW_MASK, BOUND_ZERO>((int)((unsigned)key + 1u)) - 1u);
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes in a fixed order (pairs, quads, 8, 16, then rows);
// every lane returns the total.  The first four patterns give every lane a
// source inside its row, so they take bound_ctrl (no "old" operand to set up).
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1, 0xF, true>(v);   // lane ^ 1
  v += dpp_f64<0x4E, 0xF, true>(v);   // lane ^ 2
  v += dpp_f64<0x141, 0xF, true>(v);  // mirror within 8: other quad
  v += dpp_f64<0x140, 0xF, true>(v);  // mirror within 16: other half row
  v += dpp_f64<0x142, 0xA, false>(v);  // row 1 += row 0, row 3 += row 2
  v += dpp_f64<0x143, 0xC, false>(v);  // rows 2, 3 += lane 31 (rows 0 + 1)
  return readlane_f64(v, 63);
}

// Inclusive scan of p over lanes, restarted wherever key changes; keys must be
// non-decreasing over the lanes (equal keys contiguous).  Lane i receives the
// sum of p over the lanes j <= i with key[j] == key[i].
__device__ __forceinline__ double wave_seg_scan(double p, int key) {
  // within rows of 16: Hillis-Steele with shifts 1, 2, 4, 8 (lanes shifted in
  // from before the row start read 0 / key -1, which never matches)
  {
    const double t = dpp_f64<0x111, 0xF, true>(p);
    const int k = dpp_key<0x111, 0xF, true>(key);
    if (k == key) p += t;
  }
  {
    const double t = dpp_f64<0x112, 0xF, true>(p);
    const int k = dpp_key<0x112, 0xF, true>(key);
    if (k == key) p += t;
  }
  {
    const double t = dpp_f64<0x114, 0xF, true>(p);
    const int k = dpp_key<0x114, 0xF, true>(key);
    if (k == key) p += t;
  }
  {
    const double t = dpp_f64<0x118, 0xF, true>(p);
    const int k = dpp_key<0x118, 0xF, true>(key);
    if (k == key) p += t;
  }
  // across rows: a segment that reaches a row's start continues the previous
  // row's last lane (keys are sorted, so equal keys mean the lanes between
  // all belong to that segment)
  {
    const double t = dpp_f64<0x142, 0xA, false>(p);
    const int k = dpp_key<0x142, 0xA, false>(key);
    if (((threadIdx.x >> 4) & 1) && k == key) p += t;
  }
  {
    const double t = dpp_f64<0x143, 0xC, false>(p);
    const int k = dpp_key<0x143, 0xC, false>(key);
    if (((threadIdx.x >> 5) & 1) && k == key) p += t;
  }
  return p;
}

// key of lane + 1 (lane 63 reads -1)
__device__ __forceinline__ int next_lane_key(int key) { return dpp_key<0x130, 0xF, true>(key); }

// Sum of one double per thread over a block of nthr (multiple of 64) threads;
// red must hold nthr/64 doubles.  Every thread returns the same value.
__device__ __forceinline__ double block_sum(double v, double* red, int tid, int nthr) {
  v = wave_sum(v);
  int lane = tid & (kWave - 1), w = tid / kWave;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nthr / kWave; i++) s += red[i];
  __syncthreads();
  return s;
}

}  // namespace tsvd

// ---------------------------------------------------------------------------
// Host-side error plumbing shared by the translation units.
// ---------------------------------------------------------------------------
#define TSVD_HIP_TRY(expr)                                                   \
  do {                                                                       \
    hipError_t _e = (expr);                                                  \
    if (_e != hipSuccess) return ::tsvd::hip_fail(_e, #expr, __FILE__, __LINE__); \
  } while (0)

namespace tsvd {
int hip_fail(hipError_t e, const char* what, const char* file, int line);  // records message, returns TSVD_ERR_HIP
}
