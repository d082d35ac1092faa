// Iteration exchange of the persistent power-iteration kernel: every
// workgroup publishes its own rows of a vector and gathers everyone's rows
// plus two partial sums per workgroup, in tagged 64-bit words (common.h).
// Shared by the kernel and by the benchmark driver's exchange-latency probe,
// which times this code on its own (no products) as the floor of an
// iteration.
#pragma once

#include "common.h"

namespace tsvd {

// Publish own rows r0 + i (i < nrows) of a vector in B's type: one word per
// FP32 element, two (low, high half) per FP64 element, each thread storing
// one word so that a wave's words leave in one store instruction.
template <typename BT>
__device__ __forceinline__ void publish_rows(uint64_t* buf, uint32_t ep, int r0, int nrows, const double* v) {
  if constexpr (sizeof(BT) == 4) {
    for (int i = threadIdx.x; i < nrows; i += 256) ll_store(buf + r0 + i, ep, __float_as_uint((float)v[i]));
  } else {
    for (int w = threadIdx.x; w < 2 * nrows; w += 256) ll_store(buf + 2 * (int64_t)r0 + w, ep, f64_half(v[w >> 1], w & 1));
  }
}

// Iteration exchange: wait until every y word of this epoch (rotated start per
// block to spread the requests over memory channels) and every block's two
// partials are published; y lands in xs (raw), partials are summed with a
// fixed-shape tree.  With G = 0 only the vector is gathered (q = dd = 0).
// Returns false (block-uniform) on a timed-out wait.
// W words per thread per round: 16 puts up to 4096 words in flight at once
// (one round for a 4096-entry FP32 iterate), 8 keeps registers for smaller d.
template <typename BT, int W>
__device__ __forceinline__ bool gather_iteration(const uint64_t* xb, const uint64_t* pb, uint32_t ex, int d, int b, int G, BT* xs,
                                 double* red, int* flag, int64_t spin_limit, double& q, double& dd) {
  constexpr int WPE = sizeof(BT) / 4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int count = d * WPE;
  const int rot = (int)(((int64_t)b * 1031) % count);
  uint32_t* raw = (uint32_t*)xs;
  int64_t budget = spin_limit;
  bool ok = true;
  double pq = 0.0, pd = 0.0;
  for (int base = 0; base < count && ok; base += 256 * W) {
    uint64_t w[W];
    uint64_t pw4[4];
    const bool first = base == 0;
#pragma unroll
    for (int j = 0; j < W; j++) {
      const int i = base + tid + 256 * j;
      int ii = i + rot;
      if (ii >= count) ii -= count;
      w[j] = i < count ? ll_load(xb + ii) : ((uint64_t)ex << 32);
    }
#pragma unroll
    for (int j = 0; j < 4; j++) pw4[j] = (first && tid < G) ? ll_load(pb + 4 * (int64_t)tid + j) : ((uint64_t)ex << 32);
    while (true) {
      bool all = true;
#pragma unroll
      for (int j = 0; j < W; j++) all = all && ((uint32_t)(w[j] >> 32) == ex);
#pragma unroll
      for (int j = 0; j < 4; j++) all = all && ((uint32_t)(pw4[j] >> 32) == ex);
      if (all) break;
      if (--budget <= 0) { ok = false; break; }
      __builtin_amdgcn_s_sleep(1);
#pragma unroll
      for (int j = 0; j < W; j++) {
        const int i = base + tid + 256 * j;
        int ii = i + rot;
        if (ii >= count) ii -= count;
        if (i < count && (uint32_t)(w[j] >> 32) != ex) w[j] = ll_load(xb + ii);
      }
#pragma unroll
      for (int j = 0; j < 4; j++)
        if (first && tid < G && (uint32_t)(pw4[j] >> 32) != ex) pw4[j] = ll_load(pb + 4 * (int64_t)tid + j);
    }
    if (ok) {
#pragma unroll
      for (int j = 0; j < W; j++) {
        const int i = base + tid + 256 * j;
        int ii = i + rot;
        if (ii >= count) ii -= count;
        if (i < count) raw[ii] = (uint32_t)w[j];
      }
      if (first && tid < G) { pq = ll_join_f64(pw4[0], pw4[1]); pd = ll_join_f64(pw4[2], pw4[3]); }
    }
  }
  if (tid == 0) *flag = 1;
  __syncthreads();
  if (!ok) *flag = 0;
  pq = wave_sum(pq);
  pd = wave_sum(pd);
  if (lane == 0) { red[wave] = pq; red[4 + wave] = pd; }
  __syncthreads();
  q = (red[0] + red[1]) + (red[2] + red[3]);
  dd = (red[4] + red[5]) + (red[6] + red[7]);
  const bool res = *flag != 0;
  __syncthreads();
  return res;
}

}  // namespace tsvd
