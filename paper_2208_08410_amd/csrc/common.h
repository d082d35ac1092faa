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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
  return v;  // valid in lane 0
}

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
