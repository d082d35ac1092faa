// Finishing pass of Algorithm 1 for all triplets at once, in FP64:
//   side RIGHT: U_raw = A V      (u = A v, sigma = ||u||, u = u / sigma)
//   side LEFT:  V_raw = A^T U    (v = A^T u, sigma = ||v||, v = v / sigma)
// The product runs on v_mfma_f64_16x16x4f64; each workgroup also emits the
// partial column sums of squares of its rows, which a second kernel adds in
// workgroup order (deterministic) to give sigma.  A last kernel divides by
// sigma and applies the sign convention (largest-|.| entry of each v positive).
#include <algorithm>

#include "common.h"
#include "internal.h"

namespace tsvd {

constexpr int FBM = 128;  // output rows per workgroup
constexpr int FBN = 64;   // output columns per workgroup
constexpr int FBK = 32;   // contraction per stage (8 MFMA k-steps)
constexpr int FLDA = FBK + 1;  // LDS row of A (elements): odd stride spreads rows over banks
constexpr int FLDX = FBK + 1;  // LDS row of X (doubles)

// W[M x N] (column-major, ldw) = op(A) X, X is K x N column-major (ldx).
// side 0: op(A) = A (M = m, K = n); side 1: op(A) = A^T (M = n, K = m).
// A tile (128 x 32) and X tile (32 x 64) are staged through LDS, the next
// stage's loads in flight (16-byte loads when vec) while this stage's 64
// v_mfma_f64_16x16x4f64 per wave run.  A is converted to FP64 on the way to
// the MFMA, so each product a_ik x_kj is exact and only the accumulation rounds.
template <typename AT, int SIDE>
__device__ __forceinline__ void finish_gemm_unit(const AT* A, int64_t lda, int64_t M, int64_t K, const double* X,
                                                 int64_t ldx, int N, double* W, int64_t ldw, double* ssq, int bx,
                                                 int by, bool vec) {
  __shared__ AT As[2][FBM * FLDA];
  __shared__ double Xs[2][FBN * FLDX];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m0 = (int64_t)bx * FBM;
  const int j0 = by * FBN;
  const int nk = (int)((K + FBK - 1) / FBK);
  constexpr int VA = sizeof(AT) == 4 ? 4 : 2;     // elements per 16-byte load of A
  constexpr int NA = FBM * FBK / VA / 256;        // A vectors per thread per stage (4 or 8)
  constexpr int NX = FBN * FBK / 2 / 256;         // X double2 per thread per stage (4)

  AT av[NA][VA];
  double xv[NX][2];
  // A vector f: side 0 -> row r = f / (FBK/VA), k = (f % (FBK/VA)) * VA (k-contiguous in A)
  //             side 1 -> k = f / (FBM/VA), r = (f % (FBM/VA)) * VA (r-contiguous in A)
  auto load = [&](int kt) {
    const int64_t k0 = (int64_t)kt * FBK;
#pragma unroll
    for (int e = 0; e < NA; e++) {
      const int f = tid + 256 * e;
      int r, kk;
      if (SIDE == 0) { r = f / (FBK / VA); kk = (f % (FBK / VA)) * VA; }
      else { kk = f / (FBM / VA); r = (f % (FBM / VA)) * VA; }
      const int64_t gr = m0 + r, gk = k0 + kk;
      if (SIDE == 0) {
        const AT* p = A + gr * lda + gk;
        if (vec && gr < M && gk + VA <= K) {
          if constexpr (VA == 4) { const float4 t = *(const float4*)p; av[e][0] = t.x; av[e][1] = t.y; av[e][2] = t.z; av[e][3] = t.w; }
          else { const double2 t = *(const double2*)p; av[e][0] = t.x; av[e][1] = t.y; }
        } else {
#pragma unroll
          for (int u = 0; u < VA; u++) av[e][u] = (gr < M && gk + u < K) ? p[u] : (AT)0;
        }
      } else {
        const AT* p = A + gk * lda + gr;
        if (vec && gk < K && gr + VA <= M) {
          if constexpr (VA == 4) { const float4 t = *(const float4*)p; av[e][0] = t.x; av[e][1] = t.y; av[e][2] = t.z; av[e][3] = t.w; }
          else { const double2 t = *(const double2*)p; av[e][0] = t.x; av[e][1] = t.y; }
        } else {
#pragma unroll
          for (int u = 0; u < VA; u++) av[e][u] = (gk < K && gr + u < M) ? p[u] : (AT)0;
        }
      }
    }
#pragma unroll
    for (int e = 0; e < NX; e++) {
      const int f = tid + 256 * e;
      const int j = f / (FBK / 2), kk = (f % (FBK / 2)) * 2;
      const int64_t gk = k0 + kk;
      const double* p = X + (int64_t)(j0 + j) * ldx + gk;
      const bool colok = j0 + j < N;
      if (colok && gk + 2 <= K && (((uintptr_t)p & 15) == 0)) {
        const double2 t = *(const double2*)p;
        xv[e][0] = t.x; xv[e][1] = t.y;
      } else {
        xv[e][0] = (colok && gk < K) ? p[0] : 0.0;
        xv[e][1] = (colok && gk + 1 < K) ? p[1] : 0.0;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < NA; e++) {
      const int f = tid + 256 * e;
      if (SIDE == 0) {
        const int r = f / (FBK / VA), kk = (f % (FBK / VA)) * VA;
#pragma unroll
        for (int u = 0; u < VA; u++) As[buf][r * FLDA + kk + u] = av[e][u];
      } else {
        const int kk = f / (FBM / VA), r = (f % (FBM / VA)) * VA;
#pragma unroll
        for (int u = 0; u < VA; u++) As[buf][(r + u) * FLDA + kk] = av[e][u];
      }
    }
#pragma unroll
    for (int e = 0; e < NX; e++) {
      const int f = tid + 256 * e;
      const int j = f / (FBK / 2), kk = (f % (FBK / 2)) * 2;
      Xs[buf][j * FLDX + kk] = xv[e][0];
      Xs[buf][j * FLDX + kk + 1] = xv[e][1];
    }
  };

  doublex4 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 4; j++)
#pragma unroll
      for (int e = 0; e < 4; e++) acc[i][j][e] = 0.0;

  if (nk > 0) { load(0); store(0); }
  __syncthreads();
  const int q = lane >> 4, l16 = lane & 15;
  for (int kt = 0; kt < nk; kt++) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) load(kt + 1);
#pragma unroll
    for (int t = 0; t < FBK / 4; t++) {
      double a[2], x[4];
#pragma unroll
      for (int i = 0; i < 2; i++) a[i] = (double)As[cur][(wave * 32 + i * 16 + l16) * FLDA + 4 * t + q];
#pragma unroll
      for (int j = 0; j < 4; j++) x[j] = Xs[cur][(j * 16 + l16) * FLDX + 4 * t + q];
#pragma unroll
      for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], x[j], acc[i][j], 0, 0, 0);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
  }

  // write W and the per-column sums of squares of this row tile
  __shared__ double colss[4][FBN];
  double ss[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 4; j++)
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int64_t r = m0 + wave * 32 + i * 16 + 4 * e + (lane >> 4);
        const int c = j0 + j * 16 + (lane & 15);
        const double v = acc[i][j][e];
        if (r < M && c < N) {
          W[(int64_t)c * ldw + r] = v;
          ss[j] = fma(v, v, ss[j]);
        }
      }
#pragma unroll
  for (int j = 0; j < 4; j++) {
    double v = ss[j];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (lane < 16) colss[wave][j * 16 + lane] = v;
  }
  __syncthreads();
  if (tid < FBN && j0 + tid < N) {
    const double t = colss[0][tid] + colss[1][tid] + colss[2][tid] + colss[3][tid];
    ssq[(int64_t)bx * N + j0 + tid] = t;
  }
}

template <typename AT, int SIDE>
__global__ __launch_bounds__(256) void finish_gemm_kernel(const AT* A, int64_t lda, int64_t M, int64_t K,
                                                          const double* X, int64_t ldx, int N, double* W,
                                                          int64_t ldw, double* ssq, int vec) {
  finish_gemm_unit<AT, SIDE>(A, lda, M, K, X, ldx, N, W, ldw, ssq, blockIdx.x, blockIdx.y, vec != 0);
}

// sigma_j = sqrt(sum over row tiles of ssq[b][j]): one workgroup per column,
// thread t adds tiles t, t + 256, ... in order, then a fixed-shape tree.
__device__ __forceinline__ void sigma_column(const double* ssq, int64_t nb, int N, int j, double* S) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double t = 0.0;
  for (int64_t b = tid; b < nb; b += 256) t += ssq[b * N + j];
  red[tid] = t;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) S[j] = sqrt(red[0]);
}

__global__ __launch_bounds__(256) void finish_sigma_kernel(const double* ssq, int64_t nb, int N, double* S) {
  sigma_column(ssq, nb, N, blockIdx.x, S);
}

// Column factors: fac[2j] multiplies W[:, j] (1/sigma_j, negated when the
// column's sign flips; 0 when sigma_j = 0), fac[2j+1] multiplies the iterate
// column X[:, j] (+1 or -1).  The sign convention makes the largest-|.| entry
// of v_j positive (ties: lowest index); v is X (v_from_w = 0, the right
// branch) or the scaled W (v_from_w = 1, the left branch, where W = V).
__device__ __forceinline__ void sign_column(const double* W, int64_t ldw, const double* S, const double* X,
                                            int64_t ldx, int64_t n, int v_from_w, int do_sign, int j, double* fac) {
  const int tid = threadIdx.x;
  const double s = S[j];
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
  if (!do_sign) {
    if (tid == 0) { fac[2 * j] = inv; fac[2 * j + 1] = 1.0; }
    return;
  }
  const double* v = v_from_w ? W + (int64_t)j * ldw : X + (int64_t)j * ldx;
  const double sc = v_from_w ? inv : 1.0;
  double best = -1.0, bval = 0.0;
  int64_t bi = 0;
  for (int64_t i = tid; i < n; i += 256) {
    const double val = v[i] * sc;
    const double a = fabs(val);
    if (a > best) { best = a; bi = i; bval = val; }
  }
  __shared__ double sb[256], sv[256];
  __shared__ int64_t si[256];
  sb[tid] = best; si[tid] = bi; sv[tid] = bval;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) {
      const double ob = sb[tid + off];
      const int64_t oi = si[tid + off];
      if (ob > sb[tid] || (ob == sb[tid] && oi < si[tid])) { sb[tid] = ob; si[tid] = oi; sv[tid] = sv[tid + off]; }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const bool flip = sv[0] < 0.0;
    fac[2 * j] = flip ? -inv : inv;
    fac[2 * j + 1] = flip ? -1.0 : 1.0;
  }
}

__global__ __launch_bounds__(256) void finish_sign_kernel(const double* W, int64_t ldw, const double* S,
                                                          const double* X, int64_t ldx, int64_t n, int v_from_w,
                                                          int do_sign, double* fac) {
  sign_column(W, ldw, S, X, ldx, n, v_from_w, do_sign, blockIdx.x, fac);
}

// W[:, j] *= fac[2j] (rows < Mw; exact zeros when sigma_j = 0) and
// X[:, j] *= fac[2j+1] when that is -1 (rows < Mx); grid (row chunks, columns).
constexpr int APPLY_ROWS = 2048;
__device__ __forceinline__ void apply_column(double* W, int64_t ldw, int64_t Mw, double* X, int64_t ldx, int64_t Mx,
                                             const double* fac, int j, int64_t chunk) {
  const double f = fac[2 * j], g = fac[2 * j + 1];
  const int64_t r0 = chunk * APPLY_ROWS;
  double* w = W + (int64_t)j * ldw;
  for (int64_t i = r0 + threadIdx.x; i < min(Mw, r0 + APPLY_ROWS); i += 256) w[i] = f != 0.0 ? w[i] * f : 0.0;
  if (X && g < 0.0) {
    double* x = X + (int64_t)j * ldx;
    for (int64_t i = r0 + threadIdx.x; i < min(Mx, r0 + APPLY_ROWS); i += 256) x[i] = -x[i];
  }
}

__global__ __launch_bounds__(256) void finish_apply_kernel(double* W, int64_t ldw, int64_t Mw, double* X, int64_t ldx,
                                                           int64_t Mx, const double* fac) {
  apply_column(W, ldw, Mw, X, ldx, Mx, fac, blockIdx.y, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Grouped finishing pass for a batch (FP32 A): one launch for the products of
// every problem (units = row tiles x column blocks), one for sigma (a block per
// problem), one for scale and signs (a block per column of each problem).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_fjob(const FinishJob* jobs, int njobs, int64_t u, int which) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t b = which == 0 ? jobs[mid].ubegin : jobs[mid].cbegin;
    if (b <= u) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int SIDE>
__global__ __launch_bounds__(256) void finish_grouped_gemm_kernel(const FinishJob* jobs, int njobs) {
  const int jb = find_fjob(jobs, njobs, blockIdx.x, 0);
  const FinishJob& j = jobs[jb];
  const int u = (int)(blockIdx.x - j.ubegin);
  const int64_t M = SIDE == 0 ? j.m : j.n, K = SIDE == 0 ? j.n : j.m;
  const double* X = SIDE == 0 ? j.V : j.U;
  const int64_t ldx = SIDE == 0 ? j.ldv : j.ldu;
  double* W = SIDE == 0 ? j.U : j.V;
  const int64_t ldw = SIDE == 0 ? j.ldu : j.ldv;
  const bool vec = (((uintptr_t)j.A & 15) == 0) && (j.lda % 4 == 0);
  finish_gemm_unit<float, SIDE>((const float*)j.A, j.lda, M, K, X, ldx, j.k, W, ldw, j.ssq, u % j.nb, u / j.nb, vec);
}

// workgroup -> (job, column) through cbegin
__global__ __launch_bounds__(256) void finish_grouped_sigma_kernel(const FinishJob* jobs, int njobs) {
  const FinishJob& j = jobs[find_fjob(jobs, njobs, blockIdx.x, 1)];
  sigma_column(j.ssq, j.nb, j.k, (int)(blockIdx.x - j.cbegin), j.S);
}

__global__ __launch_bounds__(256) void finish_grouped_sign_kernel(const FinishJob* jobs, int njobs) {
  const FinishJob& j = jobs[find_fjob(jobs, njobs, blockIdx.x, 1)];
  const int c = (int)(blockIdx.x - j.cbegin);
  if (c >= *j.kdone) return;
  double* fac = j.ssq + (int64_t)j.nb * j.k;
  if (j.side == 0) sign_column(j.U, j.ldu, j.S, j.V, j.ldv, j.n, 0, 1, c, fac);
  else sign_column(j.V, j.ldv, j.S, j.U, j.ldu, j.n, 1, 1, c, fac);
}

// grid (row chunks of the longest column, total columns)
__global__ __launch_bounds__(256) void finish_grouped_apply_kernel(const FinishJob* jobs, int njobs) {
  const FinishJob& j = jobs[find_fjob(jobs, njobs, blockIdx.y, 1)];
  const int c = (int)(blockIdx.y - j.cbegin);
  if (c >= *j.kdone) return;
  const double* fac = j.ssq + (int64_t)j.nb * j.k;
  if (j.side == 0) apply_column(j.U, j.ldu, j.m, j.V, j.ldv, j.n, fac, c, blockIdx.x);
  else apply_column(j.V, j.ldv, j.n, j.U, j.ldu, j.m, fac, c, blockIdx.x);
}

// Zero fills.  The library clears device memory with these kernels rather
// than with runtime memsets, so that the work it puts on a caller's stream is
// kernels only (memset nodes recorded into a captured graph have given wrong
// results on replays here).
__global__ __launch_bounds__(256) void zero_cols_kernel(double* p, int64_t ld, int64_t rows, int64_t cols) {
  for (int64_t c = blockIdx.y; c < cols; c += gridDim.y)
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < rows; r += (int64_t)gridDim.x * 256) p[c * ld + r] = 0.0;
}

__global__ __launch_bounds__(256) void zero_words32_kernel(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0u;
}

int zero_cols_launch(double* p, int64_t ld, int64_t rows, int64_t cols, hipStream_t s) {
  if (!p || rows <= 0 || cols <= 0) return 0;
  const unsigned gx = (unsigned)std::min<int64_t>((rows + 255) / 256, 64);
  const unsigned gy = (unsigned)std::min<int64_t>(cols, 4096);
  hipLaunchKernelGGL(zero_cols_kernel, dim3(gx, gy), dim3(256), 0, s, p, ld, rows, cols);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int zero_bytes_launch(void* p, size_t bytes, hipStream_t s) {
  if (!p || bytes == 0) return 0;
  const int64_t n = (int64_t)((bytes + 3) / 4);  // callers pass multiples of 4 bytes
  hipLaunchKernelGGL(zero_words32_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, s,
                     (uint32_t*)p, n);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

// U[:, c], V[:, c] and S[c] of every column c of every job (grid: the group's
// columns), so that columns a problem does not produce read as zero.
__global__ __launch_bounds__(256) void finish_grouped_zero_kernel(const FinishJob* jobs, int njobs) {
  const FinishJob& j = jobs[find_fjob(jobs, njobs, blockIdx.x, 1)];
  const int64_t c = (int64_t)blockIdx.x - j.cbegin;
  double* u = j.U + c * j.ldu;
  double* v = j.V + c * j.ldv;
  for (int64_t r = threadIdx.x; r < j.m; r += 256) u[r] = 0.0;
  for (int64_t r = threadIdx.x; r < j.n; r += 256) v[r] = 0.0;
  if (threadIdx.x == 0) j.S[c] = 0.0;
}

int finish_grouped_zero_launch(const FinishJob* d_jobs, int njobs, int64_t cols, hipStream_t s) {
  if (njobs <= 0 || cols <= 0) return 0;
  hipLaunchKernelGGL(finish_grouped_zero_kernel, dim3((unsigned)cols), dim3(256), 0, s, d_jobs, njobs);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int finish_grouped_launch(int side, const FinishJob* d_jobs, int njobs, int64_t units, int64_t cols, int64_t max_rows,
                          hipStream_t s) {
  if (njobs <= 0) return 0;
  if (side == 0) hipLaunchKernelGGL(finish_grouped_gemm_kernel<0>, dim3((unsigned)units), dim3(256), 0, s, d_jobs, njobs);
  else hipLaunchKernelGGL(finish_grouped_gemm_kernel<1>, dim3((unsigned)units), dim3(256), 0, s, d_jobs, njobs);
  TSVD_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(finish_grouped_sigma_kernel, dim3((unsigned)cols), dim3(256), 0, s, d_jobs, njobs);
  TSVD_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(finish_grouped_sign_kernel, dim3((unsigned)cols), dim3(256), 0, s, d_jobs, njobs);
  TSVD_HIP_TRY(hipGetLastError());
  const unsigned chunks = (unsigned)((max_rows + APPLY_ROWS - 1) / APPLY_ROWS);
  hipLaunchKernelGGL(finish_grouped_apply_kernel, dim3(chunks, (unsigned)cols), dim3(256), 0, s, d_jobs, njobs);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int64_t finish_tiles(int64_t m, int64_t n, int side) {
  const int64_t M = side == 0 ? m : n;
  return (M + FBM - 1) / FBM;
}
int64_t finish_workspace_doubles(int64_t m, int64_t n, int side, int k) {
  return (finish_tiles(m, n, side) + 2) * k;  // column sums per row tile, then 2 factors per column
}

int finish_gemm_launch(int is_f64, int side, const void* A, int64_t m, int64_t n, int64_t lda, const double* X,
                       int64_t ldx, int k, double* W, int64_t ldw, double* ssq, hipStream_t stream) {
  const int64_t M = side == 0 ? m : n;
  const int64_t K = side == 0 ? n : m;
  const int64_t nb = (M + FBM - 1) / FBM;
  dim3 grid((unsigned)nb, (unsigned)((k + FBN - 1) / FBN));
  const int vec = (((uintptr_t)A & 15) == 0) && (lda % (is_f64 ? 2 : 4) == 0);
  if (is_f64) {
    if (side == 0)
      hipLaunchKernelGGL((finish_gemm_kernel<double, 0>), grid, dim3(256), 0, stream, (const double*)A, lda, M, K, X,
                         ldx, k, W, ldw, ssq, vec);
    else
      hipLaunchKernelGGL((finish_gemm_kernel<double, 1>), grid, dim3(256), 0, stream, (const double*)A, lda, M, K, X,
                         ldx, k, W, ldw, ssq, vec);
  } else {
    if (side == 0)
      hipLaunchKernelGGL((finish_gemm_kernel<float, 0>), grid, dim3(256), 0, stream, (const float*)A, lda, M, K, X,
                         ldx, k, W, ldw, ssq, vec);
    else
      hipLaunchKernelGGL((finish_gemm_kernel<float, 1>), grid, dim3(256), 0, stream, (const float*)A, lda, M, K, X,
                         ldx, k, W, ldw, ssq, vec);
  }
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int finish_sigma_launch(const double* ssq, int64_t nb, int k, double* S, hipStream_t stream) {
  if (k <= 0) return 0;
  hipLaunchKernelGGL(finish_sigma_kernel, dim3(k), dim3(256), 0, stream, ssq, nb, k, S);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

int finish_launch(int is_f64, int side, const void* A, int64_t m, int64_t n, int64_t lda, const double* X,
                  int64_t ldx, int k, double* W, int64_t ldw, double* S, double* ssq, hipStream_t stream) {
  int rc = finish_gemm_launch(is_f64, side, A, m, n, lda, X, ldx, k, W, ldw, ssq, stream);
  if (rc) return rc;
  const int64_t M = side == 0 ? m : n;
  return finish_sigma_launch(ssq, (M + FBM - 1) / FBM, k, S, stream);
}

int finish_scale_sign_launch(double* W, int64_t ldw, int64_t Mw, const double* S, double* V, int64_t ldv, int64_t n,
                             double* U, int64_t ldu, int64_t m, int k, int do_sign, double* fac, hipStream_t stream) {
  if (k <= 0) return 0;
  // W aliases U (right branch: the iterate X is V) or V (left branch: X is U)
  const bool w_is_v = (W == V);
  double* X = do_sign ? (w_is_v ? U : V) : nullptr;
  const int64_t ldx = w_is_v ? ldu : ldv, Mx = w_is_v ? m : n;
  hipLaunchKernelGGL(finish_sign_kernel, dim3(k), dim3(256), 0, stream, W, ldw, S, X, ldx, n, w_is_v ? 1 : 0, do_sign,
                     fac);
  TSVD_HIP_TRY(hipGetLastError());
  const int64_t rows = std::max(Mw, do_sign ? Mx : (int64_t)0);
  hipLaunchKernelGGL(finish_apply_kernel, dim3((unsigned)((rows + APPLY_ROWS - 1) / APPLY_ROWS), (unsigned)k), dim3(256),
                     0, stream, W, ldw, Mw, X, ldx, Mx, fac);
  TSVD_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace tsvd
