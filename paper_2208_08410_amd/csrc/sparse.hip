// Sparse path: the implicit deflated product of Equation 2 / Algorithm 4 in
// factored form, z = P A^T (A (P x)) with P = I - V V^T, for a CSR matrix.
// B = A^T A is never formed; each power iteration is one CSR SpMV (t = A x),
// one CSC SpMV (w = A^T t, the transpose kept as a CSC copy so both products
// are gather-only, with no atomics) and an FP64 projection.
//
// Kernels:
//   csr_validate_kernel   checks row pointers and column indices before any
//                         product touches memory through them
//   csc_count/scan/fill   builds the CSC copy (counting sort by column);
//   csc_sort_kernel       orders rows inside each column so sums are
//                         deterministic
//   proj_partials_kernel  block partials of V^T w, ||w||^2 and x . w
//   proj_apply_kernel     z = w - V c, partial ||z||^2
//   normalize_kernel      x = z / ||z|| (FP64) and its FP32 copy
//   reduce_partials       fixed-order sum of block partials (one block)
#include "common.h"
#include "internal.h"
#include "implicit.h"

namespace tsvd {

// ---------------------------------------------------------------------------
// validation and CSC construction
// ---------------------------------------------------------------------------
__global__ void csr_validate_kernel(const int64_t* rowptr, const int32_t* col, int64_t m, int64_t n, int64_t nnz,
                                    int* bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = tid; i < m; i += stride) {
    const int64_t a = rowptr[i], b = rowptr[i + 1];
    if (a > b || a < 0 || b > nnz) atomicOr(bad, 1);
  }
  if (tid == 0 && (rowptr[0] != 0 || rowptr[m] != nnz)) atomicOr(bad, 2);
  for (int64_t e = tid; e < nnz; e += stride) {
    const int32_t c = col[e];
    if (c < 0 || (int64_t)c >= n) atomicOr(bad, 4);
  }
}

__global__ void csc_count_kernel(const int32_t* col, int64_t nnz, unsigned long long* cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride)
    atomicAdd(cnt + col[e], 1ull);
}

// exclusive scan of n counts into colptr[0..n] (three passes: block sums, scan
// of block sums in one block, add-back)
constexpr int SCAN_B = 1024;  // elements per block in pass 1/3
__global__ void scan_block_sums_kernel(const unsigned long long* cnt, int64_t n, unsigned long long* bsum) {
  __shared__ unsigned long long s[256];
  const int64_t base = (int64_t)blockIdx.x * SCAN_B;
  unsigned long long t = 0;
  for (int i = threadIdx.x; i < SCAN_B; i += 256)
    if (base + i < n) t += cnt[base + i];
  s[threadIdx.x] = t;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = s[0];
}

__global__ void scan_bsums_kernel(unsigned long long* bsum, int64_t nb) {
  if (threadIdx.x != 0) return;
  unsigned long long run = 0;
  for (int64_t b = 0; b < nb; b++) {
    const unsigned long long v = bsum[b];
    bsum[b] = run;
    run += v;
  }
}

__global__ void scan_apply_kernel(const unsigned long long* cnt, int64_t n, const unsigned long long* bsum,
                                  int64_t* colptr, int64_t total) {
  __shared__ unsigned long long s[SCAN_B];
  const int64_t base = (int64_t)blockIdx.x * SCAN_B;
  for (int i = threadIdx.x; i < SCAN_B; i += 256) s[i] = (base + i < n) ? cnt[base + i] : 0ull;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long run = bsum[blockIdx.x];
    for (int i = 0; i < SCAN_B; i++) {
      const unsigned long long v = s[i];
      s[i] = run;
      run += v;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < SCAN_B; i += 256)
    if (base + i < n) colptr[base + i] = (int64_t)s[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) colptr[n] = total;
}

// scatter entries into their column (positions within a column in arbitrary
// order; csc_sort_kernel fixes the order afterwards)
__global__ void csc_fill_kernel(const int64_t* rowptr, const int32_t* col, const float* val, int64_t m,
                                const int64_t* colptr, unsigned long long* fill, int32_t* rowidx, float* cval) {
  // one 64-lane wave per row
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
  for (int64_t r = wave; r < m; r += nw) {
    for (int64_t e = rowptr[r] + lane; e < rowptr[r + 1]; e += 64) {
      const int32_t c = col[e];
      const unsigned long long p = atomicAdd(fill + c, 1ull);
      const int64_t pos = colptr[c] + (int64_t)p;
      rowidx[pos] = (int32_t)r;
      cval[pos] = val[e];
    }
  }
}

// the entries of a batch of rows whose column lies in [j0, j1), scattered
// into their column of the sub-matrix A[:, j0:j1] (CSC, column pointers
// sub_ptr relative to its first entry); rows are numbered from row0
__global__ void csc_fill_range_kernel(const int64_t* rowptr, const int32_t* col, const float* val, int64_t rows,
                                      int64_t row0, int64_t j0, int64_t j1, const int64_t* sub_ptr,
                                      unsigned long long* fill, int32_t* rowidx, float* cval) {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
  for (int64_t r = wave; r < rows; r += nw) {
    for (int64_t e = rowptr[r] + lane; e < rowptr[r + 1]; e += 64) {
      const int64_t c = col[e];
      if (c < j0 || c >= j1) continue;
      const unsigned long long p = atomicAdd(fill + (c - j0), 1ull);
      const int64_t pos = sub_ptr[c - j0] + (int64_t)p;
      rowidx[pos] = (int32_t)(row0 + r);
      cval[pos] = val[e];
    }
  }
}

// out[i] = in[i] - in[0] for i < count (pointer arrays of a batch made relative to its first entry)
__global__ void rebase_kernel(const int64_t* in, int64_t count, int64_t* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t b = in[0];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) out[i] = in[i] - b;
}

// out[i] = in[i] + add
__global__ void offset_kernel(const int64_t* in, int64_t count, int64_t add, int64_t* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) out[i] = in[i] + add;
}

// insertion sort of each column's (row, value) pairs by row; one thread per
// column (columns hold a few dozen entries in the target workloads).
__global__ void csc_sort_kernel(const int64_t* colptr, int64_t n, int32_t* rowidx, float* cval) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
    const int64_t a = colptr[c], b = colptr[c + 1];
    for (int64_t i = a + 1; i < b; i++) {
      const int32_t r = rowidx[i];
      const float v = cval[i];
      int64_t j = i - 1;
      while (j >= a && rowidx[j] > r) {
        rowidx[j + 1] = rowidx[j];
        cval[j + 1] = cval[j];
        j--;
      }
      rowidx[j + 1] = r;
      cval[j + 1] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// projection pieces (FP64)
// ---------------------------------------------------------------------------
constexpr int PB = 256;        // threads per block
constexpr int PROWS = 4096;    // vector entries per block in the partial kernels

// partial[b][j] = sum_{i in block b} V[i, j] w[i] (j < l); partial[b][l] =
// sum w_i^2; partial[b][l+1] = sum x_i w_i.  One wave per column j (strided),
// fixed order inside the block.
__global__ __launch_bounds__(PB) void proj_partials_kernel(const double* V, int64_t ldv, int l, const double* w,
                                                           const double* x, int64_t d, double* partial) {
  const int64_t i0 = (int64_t)blockIdx.x * PROWS;
  const int64_t i1 = i0 + PROWS < d ? i0 + PROWS : d;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int P = l + 2;
  for (int j = wave; j < P; j += PB / 64) {
    double s = 0.0;
    for (int64_t i = i0 + lane; i < i1; i += 64) {
      const double wi = w[i];
      const double a = j < l ? V[(int64_t)j * ldv + i] : (j == l ? wi : x[i]);
      s = fma(a, wi, s);
    }
    s = wave_sum(s);
    if (lane == 0) partial[(int64_t)blockIdx.x * P + j] = s;
  }
}

// out[j] = sum_b partial[b][j] (one block of 256 threads).  Up to 256 outputs
// per pass; each output's sum is split over 256 / outputs threads that add
// strided partials (loads in flight together), and the thread sums are added
// in thread order: a fixed association, independent of timing.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double* partial, int64_t nb, int P, double* out) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  for (int j0 = 0; j0 < P; j0 += 256) {
    const int pc = P - j0 < 256 ? P - j0 : 256;
    const int per = 256 / pc;
    const int j = tid % pc, part = tid / pc;
    double s = 0.0;
    if (part < per) {
#pragma unroll 8
      for (int64_t b = part; b < nb; b += per) s += partial[b * P + j0 + j];
    }
    red[tid] = s;
    __syncthreads();
    if (tid < pc) {
      double t = 0.0;
      for (int q = 0; q < per; q++) t += red[q * pc + tid];
      out[j0 + tid] = t;
    }
    __syncthreads();
  }
}

// z = w - V c (c = coef[0..l)); partial[b] = sum z_i^2 over the block's rows
__global__ __launch_bounds__(PB) void proj_apply_kernel(const double* V, int64_t ldv, int l, const double* coef,
                                                        double* w, int64_t d, double* partial) {
  const int64_t i0 = (int64_t)blockIdx.x * PROWS;
  const int64_t i1 = i0 + PROWS < d ? i0 + PROWS : d;
  __shared__ double red[PB / 64];
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += PB) {
    double z = w[i];
    for (int j = 0; j < l; j++) z = fma(-V[(int64_t)j * ldv + i], coef[j], z);
    w[i] = z;
    s = fma(z, z, s);
  }
  s = block_sum(s, red, threadIdx.x, PB);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// x = z * inv (FP64) and xf = (float)x
__global__ void normalize_kernel(const double* z, int64_t d, double inv, double* x, float* xf) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d; i += stride) {
    const double v = z[i] * inv;
    x[i] = v;
    if (xf) xf[i] = (float)v;
  }
}

// x = v0_l / ||v0_l|| with ||v0_l|| from scal[0] (a sum of squares)
__global__ void start_scale_kernel(const double* v0, int64_t d, const double* ss, double* x) {
  const double inv = 1.0 / sqrt(ss[0]);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d; i += stride) x[i] = v0[i] * inv;
}

__global__ __launch_bounds__(PB) void sumsq_partial_kernel(const double* v, int64_t d, double* partial) {
  const int64_t i0 = (int64_t)blockIdx.x * PROWS;
  const int64_t i1 = i0 + PROWS < d ? i0 + PROWS : d;
  __shared__ double red[PB / 64];
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += PB) s = fma(v[i], v[i], s);
  s = block_sum(s, red, threadIdx.x, PB);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void to_float_kernel(const double* x, int64_t d, float* xf) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d; i += stride) xf[i] = (float)x[i];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static int grid_for(int64_t work, int per_block, int cap = 1 << 20) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

int csr_validate(const int64_t* rowptr, const int32_t* col, int64_t m, int64_t n, int64_t nnz, int* d_bad,
                 hipStream_t s) {
  if (int rc = zero_bytes_launch(d_bad, sizeof(int), s)) return rc;
  hipLaunchKernelGGL(csr_validate_kernel, dim3(grid_for(m > nnz ? m : nnz, 256, 65536)), dim3(256), 0, s, rowptr,
                     col, m, n, nnz, d_bad);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

size_t csc_build_scratch_bytes(int64_t n) {
  const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
  return (size_t)(n + 1) * 8 * 2 + (size_t)(nb + 1) * 8 + 1024;
}

int scan_counts(const unsigned long long* cnt, int64_t n, unsigned long long* bsum, int64_t* out, int64_t total,
                hipStream_t s) {
  const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
  if (nb > 0) {
    hipLaunchKernelGGL(scan_block_sums_kernel, dim3((unsigned)nb), dim3(256), 0, s, cnt, n, bsum);
    hipLaunchKernelGGL(scan_bsums_kernel, dim3(1), dim3(64), 0, s, bsum, nb);
    hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(256), 0, s, cnt, n, bsum, out, total);
  }
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int csc_build(const int64_t* rowptr, const int32_t* col, const float* val, int64_t m, int64_t n, int64_t nnz,
              int64_t* colptr, int32_t* rowidx, float* cval, void* scratch, hipStream_t s) {
  unsigned long long* cnt = (unsigned long long*)scratch;
  unsigned long long* fill = cnt + (n + 1);
  unsigned long long* bsum = fill + (n + 1);
  const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
  if (int rc = zero_bytes_launch(cnt, (size_t)(n + 1) * 8 * 2, s)) return rc;
  hipLaunchKernelGGL(csc_count_kernel, dim3(grid_for(nnz, 256, 65536)), dim3(256), 0, s, col, nnz, cnt);
  hipLaunchKernelGGL(scan_block_sums_kernel, dim3((unsigned)nb), dim3(256), 0, s, cnt, n, bsum);
  hipLaunchKernelGGL(scan_bsums_kernel, dim3(1), dim3(64), 0, s, bsum, nb);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(256), 0, s, cnt, n, bsum, colptr, nnz);
  hipLaunchKernelGGL(csc_fill_kernel, dim3(grid_for(m * 64, 256, 65536)), dim3(256), 0, s, rowptr, col, val, m,
                     colptr, fill, rowidx, cval);
  hipLaunchKernelGGL(csc_sort_kernel, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, colptr, n, rowidx, cval);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int csc_count_launch(const int32_t* col, int64_t nnz, unsigned long long* cnt, hipStream_t s) {
  if (nnz <= 0) return 0;
  hipLaunchKernelGGL(csc_count_kernel, dim3(grid_for(nnz, 256, 65536)), dim3(256), 0, s, col, nnz, cnt);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int csc_fill_range_launch(const int64_t* rowptr, const int32_t* col, const float* val, int64_t rows, int64_t row0,
                          int64_t j0, int64_t j1, const int64_t* sub_ptr, unsigned long long* fill, int32_t* rowidx,
                          float* cval, hipStream_t s) {
  if (rows <= 0) return 0;
  hipLaunchKernelGGL(csc_fill_range_kernel, dim3(grid_for(rows * 64, 256, 65536)), dim3(256), 0, s, rowptr, col, val,
                     rows, row0, j0, j1, sub_ptr, fill, rowidx, cval);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int csc_sort_launch(const int64_t* colptr, int64_t n, int32_t* rowidx, float* cval, hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(csc_sort_kernel, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, colptr, n, rowidx, cval);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int rebase_launch(const int64_t* in, int64_t count, int64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(rebase_kernel, dim3(grid_for(count, 256, 65536)), dim3(256), 0, s, in, count, out);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int offset_launch(const int64_t* in, int64_t count, int64_t add, int64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(offset_kernel, dim3(grid_for(count, 256, 65536)), dim3(256), 0, s, in, count, add, out);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int64_t proj_blocks(int64_t d) { return (d + PROWS - 1) / PROWS; }

int proj_partials_launch(const double* V, int64_t ldv, int l, const double* w, const double* x, int64_t d,
                         double* partial, double* out, hipStream_t s) {
  const int64_t nb = proj_blocks(d);
  hipLaunchKernelGGL(proj_partials_kernel, dim3((unsigned)nb), dim3(PB), 0, s, V, ldv, l, w, x, d, partial);
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, s, partial, nb, l + 2, out);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int proj_apply_launch(const double* V, int64_t ldv, int l, const double* coef, double* w, int64_t d, double* partial,
                      double* out, hipStream_t s) {
  const int64_t nb = proj_blocks(d);
  hipLaunchKernelGGL(proj_apply_kernel, dim3((unsigned)nb), dim3(PB), 0, s, V, ldv, l, coef, w, d, partial);
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, s, partial, nb, 1, out);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int proj_partials_part_launch(const double* V, int64_t ldv, int l, const double* w, const double* x, int64_t rows,
                              double* partial, hipStream_t s) {
  static_assert(PROWS == kProjRows, "host batches of the factor align with the projection blocks");
  hipLaunchKernelGGL(proj_partials_kernel, dim3((unsigned)proj_blocks(rows)), dim3(PB), 0, s, V, ldv, l, w, x, rows,
                     partial);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int proj_apply_part_launch(const double* V, int64_t ldv, int l, const double* coef, double* w, int64_t rows,
                           double* partial, hipStream_t s) {
  hipLaunchKernelGGL(proj_apply_kernel, dim3((unsigned)proj_blocks(rows)), dim3(PB), 0, s, V, ldv, l, coef, w, rows,
                     partial);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int reduce_partials_launch(const double* partial, int64_t nb, int P, double* out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, s, partial, nb, P, out);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int sumsq_launch(const double* v, int64_t d, double* partial, double* out, hipStream_t s) {
  const int64_t nb = proj_blocks(d);
  hipLaunchKernelGGL(sumsq_partial_kernel, dim3((unsigned)nb), dim3(PB), 0, s, v, d, partial);
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, s, partial, nb, 1, out);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int normalize_launch(const double* z, int64_t d, double inv, double* x, float* xf, hipStream_t s) {
  hipLaunchKernelGGL(normalize_kernel, dim3(grid_for(d, 256, 65536)), dim3(256), 0, s, z, d, inv, x, xf);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int start_scale_launch(const double* v0, int64_t d, const double* ss, double* x, hipStream_t s) {
  hipLaunchKernelGGL(start_scale_kernel, dim3(grid_for(d, 256, 65536)), dim3(256), 0, s, v0, d, ss, x);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

__global__ void sqrt_inplace_kernel(double* v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = sqrt(v[i]);
}

int sqrt_inplace_launch(double* v, int n, hipStream_t s) {
  hipLaunchKernelGGL(sqrt_inplace_kernel, dim3((n + 255) / 256), dim3(256), 0, s, v, n);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int to_float_launch(const double* x, int64_t d, float* xf, hipStream_t s) {
  hipLaunchKernelGGL(to_float_kernel, dim3(grid_for(d, 256, 65536)), dim3(256), 0, s, x, d, xf);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace tsvd
