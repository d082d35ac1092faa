// Sliced tile format for the sparse products (the SpMV pair of Equation 2 /
// Algorithm 4 evaluated in factored form).
//
// A compressed-row matrix (CSR of A, or the CSC of A read as the CSR of A^T)
// is cut into tiles of 2^rbits rows x 2^cbits columns.  Tile (c, s) holds the
// entries of row chunk c in column slice s, in row order (the original order
// within a row), each as one 32-bit key (row_local << cbits | col_local) and
// its FP32 value; tptr[c * nslices + s] is the tile's first entry.
//
// y = A x then runs one workgroup per row chunk, accumulating the chunk's y in
// LDS (FP64) while it walks the slices in order.  All workgroups walk the
// slices in the same order, so at any time the x gathers of the chip hit a
// few 1 MiB slices that sit in L2, instead of a 200 MB vector scattered
// over HBM: random gathers that miss L2 run at a fraction of the rate of those
// that hit it.  Keys and values are streamed once with non-temporal loads.
//
// Products are exact in FP64; the sums use a fixed order (a segmented scan
// over 64 lanes on DPP, then per-wave boundary rows added by one thread in
// wave order), so results are deterministic.
#include "../../include/tsvd.h"
#include "common.h"
#include "internal.h"

namespace tsvd {

// ---- build --------------------------------------------------------------

// counts[c * ns + s] = entries of row chunk c in slice s
__global__ __launch_bounds__(256) void tile_count_kernel(const int64_t* ptr, const int32_t* idx, int64_t rows,
                                                         int rbits, int cbits, int64_t ns,
                                                         unsigned long long* counts) {
  extern __shared__ unsigned int hist[];  // ns entries
  const int64_t c = blockIdx.x;
  for (int64_t s = threadIdx.x; s < ns; s += 256) hist[s] = 0;
  __syncthreads();
  const int64_t r0 = c << rbits, r1 = min(rows, (c + 1) << rbits);
  for (int64_t e = ptr[r0] + threadIdx.x; e < ptr[r1]; e += 256) atomicAdd(&hist[idx[e] >> cbits], 1u);
  __syncthreads();
  for (int64_t s = threadIdx.x; s < ns; s += 256) counts[c * ns + s] = hist[s];
}

// Stable bucketing of one row chunk's entries into its slices, SG slices at a
// time: thread t owns a contiguous range of the chunk's rows; it counts its
// entries per slice, the counts are scanned over threads (in thread order),
// and each thread then writes its entries in order.  The result is in row
// order inside every tile.
constexpr int TG = 64;  // slices per group (LDS: TG x 256 counters)
__global__ __launch_bounds__(256) void tile_fill_kernel(const int64_t* ptr, const int32_t* idx, const float* val,
                                                        int64_t rows, int rbits, int cbits, int64_t ns,
                                                        const int64_t* tptr, uint32_t* key, float* tval) {
  __shared__ unsigned int cnt[TG][257];
  const int64_t c = blockIdx.x;
  const int t = threadIdx.x;
  const int64_t r0 = c << rbits, r1 = min(rows, (c + 1) << rbits);
  const int64_t nr = r1 - r0;
  const int64_t ra = r0 + (nr * t) / 256, rb = r0 + (nr * (t + 1)) / 256;  // this thread's rows
  const uint32_t cmask = (cbits >= 32) ? 0xffffffffu : ((1u << cbits) - 1u);
  for (int64_t g0 = 0; g0 < ns; g0 += TG) {
    const int64_t g1 = min(ns, g0 + TG);
    for (int s = 0; s < TG; s++) cnt[s][t] = 0;
    __syncthreads();
    for (int64_t e = ptr[ra]; e < ptr[rb]; e++) {
      const int64_t s = idx[e] >> cbits;
      if (s >= g0 && s < g1) cnt[s - g0][t]++;
    }
    __syncthreads();
    // exclusive scan over threads for each slice of the group (one thread per slice)
    if (t < g1 - g0) {
      unsigned int run = 0;
      for (int u = 0; u < 256; u++) {
        const unsigned int v = cnt[t][u];
        cnt[t][u] = run;
        run += v;
      }
    }
    __syncthreads();
    for (int64_t r = ra; r < rb; r++) {
      const uint32_t rl = (uint32_t)(r - r0);
      for (int64_t e = ptr[r]; e < ptr[r + 1]; e++) {
        const int32_t col = idx[e];
        const int64_t s = col >> cbits;
        if (s < g0 || s >= g1) continue;
        const int64_t pos = tptr[c * ns + s] + cnt[s - g0][t]++;
        key[pos] = (rl << cbits) | ((uint32_t)col & cmask);
        tval[pos] = val[e];
      }
    }
    __syncthreads();
  }
}

// ---- product ------------------------------------------------------------

constexpr int TW = 8;  // waves per workgroup of the tiled product: one row chunk each
constexpr int kMaxRowBits = 11;  // TW x 2^bits doubles of LDS: 128 KiB at most

// y = A x over row chunks [c0, c0 + nch): wave w of workgroup g owns chunk
// c0 + TW g + w and accumulates that chunk's y in its own FP64 slice of LDS
// while it walks the column slices in order.  No other wave touches the
// slice; the waves only meet at one barrier per column slice, which keeps
// their gathers in the same slice of x.  The loop is software-pipelined over tiles:
// while a tile's x gathers are in flight, the keys and values of the next
// tile and the pointer of the one after are already being loaded, so a tile
// costs one dependent round trip (the gathers) instead of three.  Within a
// tile the entries are in row order; 64-entry chunks are reduced with a
// segmented scan over the lanes (skipped when a chunk's rows are all
// distinct, the common case at C4's density), and every lane that ends a
// segment adds its sum to LDS with one FP64 LDS add (one lane per row per
// instruction; the instructions of a wave execute in order), so the sums have
// a fixed order and the result is deterministic.  At 5e7 x 5e7 with 2.5e9
// nonzeros: 16.3 ms per product with 1024-row chunks and 2^18-column slices
// (2^17: 22.6 ms, 2^19: 36.6 ms; 2^11-row chunks 22.1 ms, 2^9 24.3 ms; 16
// waves per workgroup 19.2 ms; free-running waves without the per-slice
// barrier 37-38 ms; a read-modify-write instead of the LDS add 16.7 ms).
constexpr int UC = 8;  // 64-entry chunks of a tile held in registers (the rest of a longer tile loops)

template <typename XT>
__device__ __forceinline__ void tile_chunks(double* yl, int lane, int64_t e_begin, int64_t b, int cbits, uint32_t cmask,
                                            const uint32_t (&kk)[UC], const float (&vv)[UC], const XT (&xx)[UC]) {
#pragma unroll
  for (int u = 0; u < UC; u++) {
    const int64_t e0 = e_begin + 64 * u;
    if (e0 >= b) break;  // uniform
    const bool valid = e0 + lane < b;
    const int nvalid = (int)min((int64_t)64, b - e0);
    int row = 0x7fffffff;
    double p = 0.0;
    if (valid) {
      row = (int)(kk[u] >> cbits);
      p = (double)vv[u] * (double)xx[u];
    }
    // rows are sorted, so a chunk whose rows are all distinct needs no scan
    const int rn = next_lane_key(row);
    const bool distinct = __builtin_amdgcn_ballot_w64(valid && lane < nvalid - 1 && rn == row) == 0;
    if (!distinct) p = wave_seg_scan(p, row);
    // the last lane of each segment in this chunk adds it (a segment that
    // continues into the next chunk is added in two parts, in order)
    if (valid && (lane == nvalid - 1 || rn != row)) atomicAdd(yl + row, p);  // ds_add_f64: one lane per row
  }
}

template <typename XT>
__global__ __launch_bounds__(TW * 64) void spmv_tiles_kernel(const int64_t* __restrict__ tptr,
                                                         const uint32_t* __restrict__ key,
                                                         const float* __restrict__ val, int64_t rows, int rbits,
                                                         int cbits, int64_t ns, const XT* __restrict__ x, double* y,
                                                         float* yf, int64_t base, int64_t c0, int64_t nch) {
  extern __shared__ double ylds[];  // TW x 2^rbits
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t cl0 = (int64_t)blockIdx.x * TW + wave;
  const bool active = cl0 < nch;  // a wave past the last chunk only keeps step with the others
  const int64_t cl = active ? cl0 : nch - 1;
  const int64_t c = c0 + cl;
  const int RH = 1 << rbits;
  double* yl = ylds + (size_t)wave * RH;
  const int64_t r0 = c << rbits;
  const int nrow = (int)min((int64_t)RH, rows - r0);
  const uint32_t cmask = (cbits >= 32) ? 0xffffffffu : ((1u << cbits) - 1u);
  for (int i = lane; i < RH; i += 64) yl[i] = 0.0;
  const int64_t* tp = tptr + c * ns;
  // pipeline state: the current tile [a, b) with its first UC chunks' keys and
  // values in registers, and the end of the next tile
  int64_t a = tp[0] - base, b = tp[1] - base;
  int64_t bn = ns > 1 ? tp[2] - base : b;
  if (!active) a = b = bn = 0;
  uint32_t kk[UC];
  float vv[UC];
#pragma unroll
  for (int u = 0; u < UC; u++) {
    const int64_t e = a + 64 * u + lane;
    kk[u] = e < b ? __builtin_nontemporal_load(key + e) : 0u;
    vv[u] = e < b ? __builtin_nontemporal_load(val + e) : 0.f;
  }
  for (int64_t s = 0; s < ns; s++) {
    const XT* xs = x + (s << cbits);
    XT xx[UC];
#pragma unroll
    for (int u = 0; u < UC; u++) xx[u] = (a + 64 * u + lane < b) ? xs[kk[u] & cmask] : (XT)0;
    // next tile's keys and values, and the pointer after it, while the gathers fly
    uint32_t kn[UC];
    float vn[UC];
#pragma unroll
    for (int u = 0; u < UC; u++) {
      const int64_t e = b + 64 * u + lane;
      kn[u] = e < bn ? __builtin_nontemporal_load(key + e) : 0u;
      vn[u] = e < bn ? __builtin_nontemporal_load(val + e) : 0.f;
    }
    const int64_t bnn = !active ? 0 : (s + 2 < ns ? tp[s + 3] - base : bn);
    tile_chunks<XT>(yl, lane, a, b, cbits, cmask, kk, vv, xx);
    // a tile longer than UC chunks: the rest, UC chunks at a time, unpipelined
    for (int64_t s0 = a + 64 * UC; s0 < b; s0 += 64 * UC) {
      uint32_t k2[UC];
      float v2[UC];
      XT x2[UC];
#pragma unroll
      for (int u = 0; u < UC; u++) {
        const int64_t e = s0 + 64 * u + lane;
        k2[u] = e < b ? __builtin_nontemporal_load(key + e) : 0u;
        v2[u] = e < b ? __builtin_nontemporal_load(val + e) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < UC; u++) x2[u] = (s0 + 64 * u + lane < b) ? xs[k2[u] & cmask] : (XT)0;
      tile_chunks<XT>(yl, lane, s0, b, cbits, cmask, k2, v2, x2);
    }
#pragma unroll
    for (int u = 0; u < UC; u++) {
      kk[u] = kn[u];
      vv[u] = vn[u];
    }
    a = b;
    b = bn;
    bn = bnn;
    // the waves of a workgroup walk the slices in step, so their x gathers
    // fall in the same slice of x, which stays in L2 (free-running waves
    // drift apart and the slices they touch no longer fit)
    __syncthreads();
  }
  if (!active) return;
  for (int i = lane; i < nrow; i += 64) {
    const double v = yl[i];
    if (y) y[r0 + i] = v;
    if (yf) yf[r0 + i] = (float)v;
  }
}

}  // namespace tsvd

namespace tsvd {

static int ceil_log2(int64_t v) {
  int b = 0;
  while (((int64_t)1 << b) < v) b++;
  return b;
}

int tiles_plan(int64_t rows, int64_t cols, int num_cu, int rbits_hint, int cbits_hint, TilePlan* t) {
  int rb = rbits_hint;
  if (rb <= 0) {  // 32 .. 1024-row chunks, about two workgroups of TW chunks per CU (64 KiB of LDS each)
    rb = 10;
    while (rb > 5 && (rows >> rb) < 2 * TW * (int64_t)num_cu) rb--;
  }
  int cb = cbits_hint > 0 ? cbits_hint : 18;  // 1 MiB FP32 slices of x (measured best of 2^18 / 2^19)
  const int lc = ceil_log2(cols);
  if (cb > lc) cb = lc > 0 ? lc : 1;
  if (cb < lc - 14) cb = lc - 14;  // at most 16384 slices (tile_count_kernel's LDS histogram)
  if (rb < 1 || rb > kMaxRowBits || cb < 1 || rb + cb > 32) return -1;
  t->rbits = rb;
  t->cbits = cb;
  t->nchunks = (rows + ((int64_t)1 << rb) - 1) >> rb;
  t->nslices = (cols + ((int64_t)1 << cb) - 1) >> cb;
  return 0;
}

size_t tiles_scratch_bytes(const TilePlan& t) {
  const int64_t nt = t.nchunks * t.nslices;
  return (size_t)(nt + 1) * 8 + (size_t)((nt + 1023) / 1024 + 1) * 8 + 256;
}

int tiles_build(const int64_t* ptr, const int32_t* idx, const float* val, int64_t rows, int64_t nnz,
                const TilePlan& t, int64_t* tptr, uint32_t* key, float* tval, void* scratch, hipStream_t s) {
  const int64_t nt = t.nchunks * t.nslices;
  unsigned long long* counts = (unsigned long long*)scratch;
  unsigned long long* bsum = counts + (nt + 1);
  hipLaunchKernelGGL(tile_count_kernel, dim3((unsigned)t.nchunks), dim3(256), (size_t)t.nslices * 4, s, ptr, idx, rows,
                     t.rbits, t.cbits, t.nslices, counts);
  TSVD_HIP_TRY(hipGetLastError());
  if (int rc = scan_counts(counts, nt, bsum, tptr, nnz, s)) return rc;
  hipLaunchKernelGGL(tile_fill_kernel, dim3((unsigned)t.nchunks), dim3(256), 0, s, ptr, idx, val, rows, t.rbits,
                     t.cbits, t.nslices, tptr, key, tval);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int spmv_tiles_launch(const TilePlan& t, const int64_t* tptr, const uint32_t* key, const float* val, int64_t rows,
                      const void* x, int x_is_f64, double* y, float* yf, int64_t base, int64_t c0, int64_t nch,
                      hipStream_t s) {
  if (nch <= 0) return 0;
  if (c0 < 0 || c0 + nch > t.nchunks) return TSVD_ERR_INTERNAL;
  const size_t lds = ((size_t)TW << t.rbits) * 8;
  const unsigned grid = (unsigned)((nch + TW - 1) / TW);
  static bool attr_set = false;  // up to 128 KiB of dynamic LDS for 2^11-row chunks
  if (!attr_set) {
    TSVD_HIP_TRY(hipFuncSetAttribute((const void*)spmv_tiles_kernel<float>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)((size_t)TW << kMaxRowBits) * 8));
    TSVD_HIP_TRY(hipFuncSetAttribute((const void*)spmv_tiles_kernel<double>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)((size_t)TW << kMaxRowBits) * 8));
    attr_set = true;
  }
  if (x_is_f64)
    hipLaunchKernelGGL((spmv_tiles_kernel<double>), dim3(grid), dim3(TW * 64), lds, s, tptr, key, val, rows, t.rbits,
                       t.cbits, t.nslices, (const double*)x, y, yf, base, c0, nch);
  else
    hipLaunchKernelGGL((spmv_tiles_kernel<float>), dim3(grid), dim3(TW * 64), lds, s, tptr, key, val, rows, t.rbits,
                       t.cbits, t.nslices, (const float*)x, y, yf, base, c0, nch);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace tsvd
