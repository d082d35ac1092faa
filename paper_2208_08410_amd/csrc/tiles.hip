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

constexpr int TW = 8;  // waves per workgroup of the tiled product
template <typename XT>
__global__ __launch_bounds__(TW * 64) void spmv_tiles_kernel(const int64_t* tptr, const uint32_t* key, const float* val,
                                                         int64_t rows, int rbits, int cbits, int64_t ns, const XT* x,
                                                         double* y, float* yf, int64_t base, int64_t c_off) {
  extern __shared__ double yl[];  // 2^rbits
  __shared__ int brow[2 * TW];
  __shared__ double bval[2 * TW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t c = blockIdx.x + c_off;
  const int RH = 1 << rbits;
  const int64_t r0 = (int64_t)c << rbits;
  const int nrow = (int)min((int64_t)RH, rows - r0);
  const uint32_t cmask = (cbits >= 32) ? 0xffffffffu : ((1u << cbits) - 1u);
  for (int i = threadIdx.x; i < RH; i += TW * 64) yl[i] = 0.0;
  __syncthreads();
  for (int64_t s = 0; s < ns; s++) {
    const int64_t a = tptr[c * ns + s] - base, b = tptr[c * ns + s + 1] - base;  // entries of this batch's arrays
    const int64_t n = b - a;
    if (n == 0) continue;  // uniform
    const XT* xs = x + (s << cbits);
    const int64_t wa = a + (n * wave) / TW, wb = a + (n * (wave + 1)) / TW;
    // left boundary: the wave's first row (may continue the previous wave's
    // range); right boundary: its last open segment
    int first_row = -1;
    if (wa < wb) first_row = (int)(__builtin_nontemporal_load(key + wa) >> cbits);
    int carry_row = -1;  // wave-uniform: the open segment at the end of the last chunk
    double carry = 0.0;
    double left = 0.0;   // the first segment's sum, held by the one lane that closed it
    // UC chunks of 64 entries per step: their keys, values and x gathers are
    // all issued before the first scan, so each wave keeps UC independent
    // gathers in flight; the chunks are then reduced in order.  With 8, a
    // wave's share of a tile at density 1e-6 (about 270 entries) takes one
    // step instead of two (A x at 5e7 x 5e7: 27.1 -> 25.2 ms; 5 does as well)
    constexpr int UC = 8;
    for (int64_t s0 = wa; s0 < wb; s0 += 64 * UC) {
      uint32_t kk[UC];
      float vv[UC];
      XT xx[UC];
#pragma unroll
      for (int u = 0; u < UC; u++) {
        const int64_t e = s0 + 64 * u + lane;
        kk[u] = e < wb ? __builtin_nontemporal_load(key + e) : 0u;
        vv[u] = e < wb ? __builtin_nontemporal_load(val + e) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < UC; u++) xx[u] = (s0 + 64 * u + lane < wb) ? xs[kk[u] & cmask] : (XT)0;
#pragma unroll
      for (int u = 0; u < UC; u++) {
        const int64_t e0 = s0 + 64 * u;
        if (e0 >= wb) break;  // uniform
        const int64_t e = e0 + lane;
        const bool valid = e < wb;
        const int nvalid = (int)min((int64_t)64, wb - e0);
        int row = 0x7fffffff;
        double p = 0.0;
        if (valid) {
          row = (int)(kk[u] >> cbits);
          p = (double)vv[u] * (double)xx[u];
        }
        // the open segment ended exactly at the last chunk's end: close it
        if (carry_row >= 0 && __builtin_amdgcn_readlane(row, 0) != carry_row) {
          if (lane == 0) {
            if (carry_row == first_row) left = carry;
            else yl[carry_row] += carry;  // interior row: no other wave holds it
          }
          carry_row = -1;
          carry = 0.0;
        }
        // segmented inclusive scan (rows are sorted, so equal rows are contiguous)
        p = wave_seg_scan(p, row);
        if (row == carry_row) p += carry;  // the segment continued from the last chunk
        const int rn = next_lane_key(row);
        if (valid && lane < nvalid - 1 && rn != row) {  // a segment ends inside this chunk
          if (row == first_row) left = p;  // only the first segment has first_row
          else yl[row] += p;
        }
        carry_row = __builtin_amdgcn_readlane(row, nvalid - 1);
        carry = readlane_f64(p, nvalid - 1);
      }
    }
    // boundary rows: the first segment (left) and the open last one (right);
    // they are added by one thread in wave order after the tile
    const double lsum = wave_sum(left);  // one lane holds it, the others 0: exact
    if (lane == 0) {
      const bool whole = carry_row >= 0 && carry_row == first_row;
      brow[2 * wave] = wa < wb ? first_row : -1;
      bval[2 * wave] = whole ? carry : lsum;
      brow[2 * wave + 1] = (carry_row >= 0 && !whole) ? carry_row : -1;
      bval[2 * wave + 1] = carry;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int j = 0; j < 2 * TW; j++)
        if (brow[j] >= 0) yl[brow[j]] += bval[j];
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < nrow; i += TW * 64) {
    if (y) y[r0 + i] = yl[i];
    if (yf) yf[r0 + i] = (float)yl[i];
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
  if (rb <= 0) {  // about 2 chunks per CU, 32 .. 8192 rows (64 KiB of LDS: 2 workgroups of 8 waves per CU)
    rb = 13;
    while (rb > 5 && (rows >> rb) < 2 * (int64_t)num_cu) rb--;
  }
  int cb = cbits_hint > 0 ? cbits_hint : 18;  // 1 MiB FP32 slices of x (measured best of 2^18 / 2^19)
  const int lc = ceil_log2(cols);
  if (cb > lc) cb = lc > 0 ? lc : 1;
  if (cb < lc - 14) cb = lc - 14;  // at most 16384 slices (tile_count_kernel's LDS histogram)
  if (rb < 1 || rb > 13 || cb < 1 || rb + cb > 32) return -1;
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
  const size_t lds = ((size_t)1 << t.rbits) * 8;
  if (x_is_f64)
    hipLaunchKernelGGL((spmv_tiles_kernel<double>), dim3((unsigned)nch), dim3(TW * 64), lds, s, tptr, key, val, rows,
                       t.rbits, t.cbits, t.nslices, (const double*)x, y, yf, base, c0);
  else
    hipLaunchKernelGGL((spmv_tiles_kernel<float>), dim3((unsigned)nch), dim3(TW * 64), lds, s, tptr, key, val, rows,
                       t.rbits, t.cbits, t.nslices, (const float*)x, y, yf, base, c0);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace tsvd
