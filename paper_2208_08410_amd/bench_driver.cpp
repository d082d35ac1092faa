// Stand-alone driver for profiling the dense t-SVD through the C ABI, without
// Python in the process (rocprofv3 runs it directly).
//
//   tsvd_bench [m n k eps gram steps warmup seed copy_bytes]
//     gram: 1 = FP32, 2 = BF16X3; copy_bytes > 0 first runs the copy kernel
//     below once on that many bytes (a traffic-counter reference in the same
//     profiled process)
//   tsvd_bench copy BYTES [reps]
//     a plain device-to-device copy kernel of BYTES (multiple of 16), the
//     reference for scaling hardware traffic counters to bytes
//   tsvd_bench mfma
//     dense MFMA peak loops on every CU (BF16 32x32x16 and FP64 16x16x4, four
//     independent accumulators per wave): the measured roofline denominators
//   tsvd_bench exchange [d] [rounds]
//     the power kernel's per-iteration exchange alone (csrc/exchange.h: every
//     workgroup publishes its rows of a d-vector and two partial sums, then
//     gathers all of them), one workgroup per CU, no products: the latency
//     floor of one power iteration
//   tsvd_bench gather
//     random 4-byte gathers x[idx[i]] (idx uniform over a set of 2^k floats,
//     2^26 gathers, eight in flight per lane) for gathered sets from 1 MiB to
//     1 GiB: the gather ceiling of the sparse products once x leaves an XCD's
//     L2
//   tsvd_bench batch COUNT [steps warmup seed team_kib]
//     COUNT problems of the serving mix (m log-uniform in [1024, 65536], n in
//     [128, 4096], k in {8, 16, 32, 64}, s_i = 0.95^i, eps = 5e-8) solved by
//     one tsvd_dense_batched call per step, A resident in HBM
//
// A = H_L [diag(s); 0] H_R with s_i = 0.97^i and H_L, H_R products of two
// random Householder reflectors (exactly orthogonal), so the singular values
// are s; start vectors are N(0, 1) from a counter-based generator.  Prints one
// JSON line with per-step and per-phase times and the sigma error.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <chrono>
#include <vector>

#include "../include/tsvd.h"
#include "csrc/exchange.h"

static uint64_t splitmix(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
static double gauss(uint64_t seed, uint64_t i) {  // Box-Muller on two counter draws
  const double u1 = ((splitmix(seed * 0x100000001B3ull + 2 * i) >> 11) + 1.0) * (1.0 / 9007199254740993.0);
  const double u2 = (splitmix(seed * 0x100000001B3ull + 2 * i + 1) >> 11) * (1.0 / 9007199254740992.0);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

__global__ void copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx16_t __attribute__((ext_vector_type(16)));
typedef double doublex4_t __attribute__((ext_vector_type(4)));

// ITERS x 4 independent MFMA chains per wave; the results are stored so the
// work is not removed
template <int ITERS>
__global__ __launch_bounds__(256) void mfma_bf16_loop(float* out, float seed) {
  bf16x8_t a, b;
  for (int i = 0; i < 8; i++) { a[i] = (__bf16)(seed + 0.001f * threadIdx.x); b[i] = (__bf16)(seed - 0.002f * i); }
  floatx16_t c0 = {}, c1 = {}, c2 = {}, c3 = {};
  for (int it = 0; it < ITERS; it++) {
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c3, 0, 0, 0);
  }
  float s = 0;
  for (int e = 0; e < 16; e++) s += c0[e] + c1[e] + c2[e] + c3[e];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int ITERS>
__global__ __launch_bounds__(256) void mfma_f64_loop(double* out, double seed) {
  const double a = seed + 0.001 * threadIdx.x, b = seed - 0.002;
  doublex4_t c0 = {}, c1 = {}, c2 = {}, c3 = {};
  for (int it = 0; it < ITERS; it++) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c3, 0, 0, 0);
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = c0[0] + c1[1] + c2[2] + c3[3];
}

static int run_mfma() {
  int num_cu = 0;
  if (hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess) return 1;
  const int grid = num_cu * 8;  // 8 workgroups of 4 waves per CU: 8 waves per SIMD
  constexpr int ITERS = 4096;
  void* out;
  if (hipMalloc(&out, (size_t)grid * 256 * 8) != hipSuccess) return 1;
  hipEvent_t e0, e1;
  hipEventCreate(&e0); hipEventCreate(&e1);
  float best_bf16 = 1e30f, best_f64 = 1e30f;
  for (int r = 0; r < 4; r++) {
    hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(mfma_bf16_loop<ITERS>, dim3(grid), dim3(256), 0, nullptr, (float*)out, 1.0f + r);
    hipEventRecord(e1, nullptr);
    hipEventSynchronize(e1);
    float t;
    hipEventElapsedTime(&t, e0, e1);
    if (r > 0 && t < best_bf16) best_bf16 = t;
    hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(mfma_f64_loop<ITERS>, dim3(grid), dim3(256), 0, nullptr, (double*)out, 1.0 + r);
    hipEventRecord(e1, nullptr);
    hipEventSynchronize(e1);
    hipEventElapsedTime(&t, e0, e1);
    if (r > 0 && t < best_f64) best_f64 = t;
  }
  const double waves = (double)grid * 4;
  const double bf16_flops = waves * ITERS * 4 * (2.0 * 32 * 32 * 16);
  const double f64_flops = waves * ITERS * 4 * (2.0 * 16 * 16 * 4);
  printf("{\"mfma_bf16_tflops\": %.1f, \"mfma_f64_tflops\": %.2f, \"cus\": %d}\n", bf16_flops / (best_bf16 * 1e-3) / 1e12,
         f64_flops / (best_f64 * 1e-3) / 1e12, num_cu);
  fflush(stdout);
  hipFree(out);
  return 0;
}

// `rounds` iterations of the power kernel's exchange with nothing else: each
// workgroup owns ceil(d / G) entries, publishes them with its two partial
// sums, gathers the whole vector and every partial, and derives its next
// entries from what it gathered.  The dynamic LDS request matches the power
// kernel's (the CU's whole LDS) so that placement is one workgroup per CU.
__global__ __launch_bounds__(256, 1) void exchange_probe_kernel(uint64_t* xex, uint64_t* pex, int d, int rounds,
                                                                int64_t spin, int* err) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int G = gridDim.x, b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int dpad = (d + 3) & ~3;
  const int rpb = (d + G - 1) / G;
  const int r0 = b * rpb;
  const int nrows = max(0, min(rpb, d - r0));
  double* yv = (double*)smem;
  double* red = yv + ((rpb + 1) & ~1);
  int* flag = (int*)(red + 8);
  float* xs = (float*)(red + 10);
  for (int i = tid; i < nrows; i += 256) yv[i] = 1.0 + (r0 + i) * 1e-3;
  __syncthreads();
  for (int r = 1; r <= rounds; r++) {
    uint64_t* xb = xex + (int64_t)(r & 1) * dpad;
    uint64_t* pb = pex + (int64_t)(r & 1) * G * 4;
    tsvd::publish_rows<float>(xb, (uint32_t)r, r0, nrows, yv);
    if (wave == 3) {
      double q = 0.0, dd = 0.0;
      for (int i = lane; i < nrows; i += 64) { q = fma(yv[i], yv[i], q); dd += yv[i]; }
      q = tsvd::wave_sum(q);
      dd = tsvd::wave_sum(dd);
      if (lane < 4) tsvd::ll_store(pb + 4 * (int64_t)b + lane, (uint32_t)r, tsvd::f64_half(lane < 2 ? q : dd, lane & 1));
    }
    double q, dd;
    if (!tsvd::gather_iteration<float, 16>(xb, pb, (uint32_t)r, d, b, G, xs, red, flag, spin, q, dd)) {
      if (tid == 0) atomicMax(err, 1);
      return;
    }
    for (int i = tid; i < nrows; i += 256) yv[i] = (double)xs[r0 + i] / (1.0 + 1e-9 * q);
    __syncthreads();
  }
}

static int run_exchange(int d, int rounds) {
  int num_cu = 0, max_lds = 0;
  if (hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess ||
      hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, 0) != hipSuccess)
    return 1;
  if (d < 4 * num_cu || d > 16384 || rounds < 1) { fprintf(stderr, "exchange: need 4 * CUs <= d <= 16384\n"); return 2; }
  const int G = num_cu;
  const int dpad = (d + 3) & ~3;
  const size_t need = (size_t)(((d + G - 1) / G + 1) / 2 * 2 + 10) * 8 + (size_t)dpad * 4;
  size_t lds = (size_t)max_lds;
  if (lds > 160 * 1024) lds = 160 * 1024;
  if (need > lds) { fprintf(stderr, "exchange: LDS\n"); return 2; }
  const void* fn = (const void*)exchange_probe_kernel;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 1;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds) != hipSuccess || per_cu < 1) return 1;
  uint64_t *xex, *pex;
  int* err;
  const size_t xw = (size_t)2 * dpad, pw = (size_t)2 * G * 4;
  if (hipMalloc(&xex, xw * 8) || hipMalloc(&pex, pw * 8) || hipMalloc(&err, 4)) return 1;
  hipEvent_t e0, e1;
  hipEventCreate(&e0); hipEventCreate(&e1);
  int64_t spin = (int64_t)1 << 21;
  float best = 1e30f;
  for (int rep = 0; rep < 4; rep++) {
    const int R = rep == 0 ? 100 : rounds;  // the first launch warms up
    hipMemset(xex, 0, xw * 8);
    hipMemset(pex, 0, pw * 8);
    hipMemset(err, 0, 4);
    void* args[] = {(void*)&xex, (void*)&pex, (void*)&d, (void*)&R, (void*)&spin, (void*)&err};
    hipEventRecord(e0, nullptr);
    if (hipLaunchKernel(fn, dim3(G), dim3(256), args, lds, nullptr) != hipSuccess) return 1;
    hipEventRecord(e1, nullptr);
    hipEventSynchronize(e1);
    int herr = 0;
    hipMemcpy(&herr, err, 4, hipMemcpyDeviceToHost);
    if (herr) { fprintf(stderr, "exchange: a bounded wait timed out\n"); return 1; }
    float t;
    hipEventElapsedTime(&t, e0, e1);
    if (rep > 0 && t < best) best = t;
  }
  printf("{\"exchange_us_per_round\": %.3f, \"d\": %d, \"workgroups\": %d, \"rounds\": %d}\n",
         best * 1e3 / rounds, d, G, rounds);
  fflush(stdout);
  hipFree(xex); hipFree(pex); hipFree(err);
  return 0;
}

// sum of x[idx[i]] over a grid-stride range, 8 independent gathers per lane
__global__ __launch_bounds__(256) void gather_kernel(const float* __restrict__ x, const uint32_t* __restrict__ idx,
                                                     size_t n, float* out) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  float acc = 0.f;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 7 * stride < n; i += 8 * stride) {
    uint32_t j[8];
#pragma unroll
    for (int u = 0; u < 8; u++) j[u] = __builtin_nontemporal_load(idx + i + u * stride);
#pragma unroll
    for (int u = 0; u < 8; u++) acc += x[j[u]];
  }
  for (; i < n; i += stride) acc += x[idx[i]];
  if (acc == 12345.f) out[0] = acc;  // keeps the loads
}

static int run_gather() {
  const size_t n = (size_t)1 << 26;
  const int max_bits = 28;  // 2^28 floats = 1 GiB
  std::vector<uint32_t> hidx(n);
  float *x = nullptr, *out = nullptr;
  uint32_t* idx = nullptr;
  if (hipMalloc(&x, ((size_t)1 << max_bits) * 4) || hipMalloc(&idx, n * 4) || hipMalloc(&out, 64)) {
    fprintf(stderr, "device alloc\n");
    return 1;
  }
  (void)hipMemset(x, 0, ((size_t)1 << max_bits) * 4);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  printf("{\"gathers\": %zu, \"sets\": [", n);
  bool first = true;
  for (int bits = 18; bits <= max_bits; bits += 2) {
    const uint32_t mask = (1u << bits) - 1u;
    for (size_t i = 0; i < n; i++) hidx[i] = (uint32_t)(splitmix(((uint64_t)bits << 40) + i) & mask);  // < 2^bits
    (void)hipMemcpy(idx, hidx.data(), n * 4, hipMemcpyHostToDevice);
    const int grid = 256 * 32;
    hipLaunchKernelGGL(gather_kernel, dim3(grid), dim3(256), 0, 0, x, idx, n, out);
    float best = 1e30f;
    for (int r = 0; r < 5; r++) {
      (void)hipEventRecord(e0, 0);
      hipLaunchKernelGGL(gather_kernel, dim3(grid), dim3(256), 0, 0, x, idx, n, out);
      (void)hipEventRecord(e1, 0);
      (void)hipEventSynchronize(e1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      best = fminf(best, ms);
    }
    printf("%s{\"set_mib\": %.0f, \"ms\": %.4f, \"g_gathers_per_s\": %.1f}", first ? "" : ", ",
           ((size_t)1 << bits) * 4.0 / (1 << 20), best, n / (best * 1e-3) / 1e9);
    first = false;
  }
  printf("]}\n");
  fflush(stdout);
  (void)hipFree(x);
  (void)hipFree(idx);
  (void)hipFree(out);
  return 0;
}

static int run_copy(size_t bytes, int reps) {
  if (bytes == 0 || bytes % 16) { fprintf(stderr, "copy: BYTES must be a positive multiple of 16\n"); return 2; }
  void *a, *b;
  if (hipMalloc(&a, bytes) || hipMalloc(&b, bytes)) { fprintf(stderr, "device alloc\n"); return 1; }
  hipMemset(a, 0, bytes);
  hipEvent_t e0, e1;
  hipEventCreate(&e0); hipEventCreate(&e1);
  const size_t n = bytes / 16;
  float best = 1e30f;
  for (int r = 0; r < reps; r++) {
    hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(copy_kernel, dim3(4096), dim3(256), 0, nullptr, (const float4*)a, (float4*)b, n);
    hipEventRecord(e1, nullptr);
    hipEventSynchronize(e1);
    float t;
    hipEventElapsedTime(&t, e0, e1);
    if (t < best) best = t;
  }
  printf("{\"copy_bytes\": %zu, \"reps\": %d, \"best_ms\": %.4f, \"gbs\": %.1f}\n", bytes, reps, best,
         2.0 * bytes / (best * 1e-3) / 1e9);
  hipFree(a); hipFree(b);
  return 0;
}

// A = H_L [diag(s); 0] H_R (m >= n) into hA (row-major m x n FP32), with H_L,
// H_R products of two random Householder reflectors.
static void make_known(int64_t m, int64_t n, const std::vector<double>& s, uint64_t seed, float* hA) {
  // A = H_L [diag(s); 0] H_R, built row by row: row i of [diag(s); 0] H_R is
  // s_i * (row i of H_R) for i < n and 0 otherwise; H_L mixes rows through two
  // rank-1 corrections.
  std::vector<double> wl[2], wr[2];
  for (int r = 0; r < 2; r++) {
    wl[r].resize(m); wr[r].resize(n);
    double a = 0, b = 0;
    for (int64_t i = 0; i < m; i++) { wl[r][i] = gauss(seed + 11 + r, i); a += wl[r][i] * wl[r][i]; }
    for (int64_t j = 0; j < n; j++) { wr[r][j] = gauss(seed + 21 + r, j); b += wr[r][j] * wr[r][j]; }
    a = 1.0 / sqrt(a); b = 1.0 / sqrt(b);
    for (auto& x : wl[r]) x *= a;
    for (auto& x : wr[r]) x *= b;
  }
  // D H_R rows: R_i = s_i e_i^T (I - 2 w1 w1^T)(I - 2 w2 w2^T)
  // M0 = [D H_R; 0]; A = (I - 2 u1 u1^T)(I - 2 u2 u2^T) M0
  // c_r = u_r^T M0 (n-vectors) are needed for the left reflectors.
  auto row_dhr = [&](int64_t i, double* out) {  // i < n
    for (int64_t j = 0; j < n; j++) out[j] = (j == i) ? s[i] : 0.0;
    for (int r = 0; r < 2; r++) {
      double dot = 0;
      for (int64_t j = 0; j < n; j++) dot += out[j] * wr[r][j];
      for (int64_t j = 0; j < n; j++) out[j] -= 2.0 * dot * wr[r][j];
    }
  };
  std::vector<double> M0((size_t)n * n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) row_dhr(i, &M0[(size_t)i * n]);
  // A = L2 L1 M0 with L_r = I - 2 u_r u_r^T applied as L2 (L1 M0):
  // (L1 M0) = M0 - 2 u1 (u1^T M0); then L2 X = X - 2 u2 (u2^T X)
  std::vector<double> c1(n, 0.0), c2(n, 0.0);
  for (int64_t i = 0; i < n; i++)
    for (int64_t j = 0; j < n; j++) c1[j] += wl[0][i] * M0[(size_t)i * n + j];
  // u2^T (L1 M0) = u2^T M0 - 2 (u2.u1) c1
  double u21 = 0;
  for (int64_t i = 0; i < m; i++) u21 += wl[1][i] * wl[0][i];
  for (int64_t i = 0; i < n; i++)
    for (int64_t j = 0; j < n; j++) c2[j] += wl[1][i] * M0[(size_t)i * n + j];
  for (int64_t j = 0; j < n; j++) c2[j] -= 2.0 * u21 * c1[j];
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; i++) {
    for (int64_t j = 0; j < n; j++) {
      double x = i < n ? M0[(size_t)i * n + j] : 0.0;
      x -= 2.0 * wl[0][i] * c1[j];
      x -= 2.0 * wl[1][i] * c2[j];
      hA[(size_t)i * n + j] = (float)x;
    }
  }
}

static int run_batch(int count, int steps, int warmup, uint64_t seed, int team_kib) {
  std::vector<tsvd_problem> probs(count);
  std::vector<std::vector<double>> sv(count);
  std::vector<void*> bufs;
  for (int p = 0; p < count; p++) {
    const double lm = log(1024.0) + (log(65536.0) - log(1024.0)) * ((splitmix(seed * 977 + 4 * p) >> 11) * (1.0 / 9007199254740992.0));
    const double ln = log(128.0) + (log(4096.0) - log(128.0)) * ((splitmix(seed * 977 + 4 * p + 1) >> 11) * (1.0 / 9007199254740992.0));
    int64_t m = (int64_t)llround(exp(lm)), n = (int64_t)llround(exp(ln));
    const int ks[4] = {8, 16, 32, 64};
    int k = ks[splitmix(seed * 977 + 4 * p + 2) & 3];
    const bool right = m >= n;
    const int64_t M = right ? m : n, N = right ? n : m;  // build the tall orientation, transpose if wide
    const int64_t d = N;
    if (k > d) k = (int)d;
    sv[p].resize(d);
    for (int64_t i = 0; i < d; i++) sv[p][i] = pow(0.95, (double)i);
    std::vector<float> hT((size_t)M * N);
    make_known(M, N, sv[p], seed * 131 + p, hT.data());
    std::vector<float> hA((size_t)m * n);
    for (int64_t i = 0; i < m; i++)
      for (int64_t j = 0; j < n; j++) hA[(size_t)i * n + j] = right ? hT[(size_t)i * n + j] : hT[(size_t)j * m + i];
    std::vector<double> hv0((size_t)k * d);
    for (size_t i = 0; i < hv0.size(); i++) hv0[i] = gauss(seed * 131 + p + 31, i);
    float* A; double *v0, *U, *S, *V;
    if (hipMalloc(&A, (size_t)m * n * 4) || hipMalloc(&v0, hv0.size() * 8) || hipMalloc(&U, (size_t)m * k * 8) ||
        hipMalloc(&S, (size_t)k * 8) || hipMalloc(&V, (size_t)n * k * 8)) { fprintf(stderr, "device alloc\n"); return 1; }
    hipMemcpy(A, hA.data(), (size_t)m * n * 4, hipMemcpyHostToDevice);
    hipMemcpy(v0, hv0.data(), hv0.size() * 8, hipMemcpyHostToDevice);
    bufs.insert(bufs.end(), {(void*)A, (void*)v0, (void*)U, (void*)S, (void*)V});
    tsvd_problem& q = probs[p];
    q = tsvd_problem{};
    q.A = A; q.dtype = TSVD_F32; q.m = m; q.n = n; q.lda = n;
    tsvd_opts_default(&q.opts);
    q.opts.k = k; q.opts.eps = 5e-8; q.opts.gram = TSVD_GRAM_BF16X3; q.opts.v0 = v0;
    q.U = U; q.ldu = m; q.S = S; q.V = V; q.ldv = n;
  }
  tsvd_ctx* ctx;
  if (tsvd_ctx_create(0, &ctx) != TSVD_OK) { fprintf(stderr, "ctx\n"); return 1; }
  if (team_kib > 0) {
    tsvd_tuning tu = {};
    tu.team_kib = team_kib;
    if (tsvd_ctx_set_tuning(ctx, &tu) != TSVD_OK) { fprintf(stderr, "tuning\n"); return 2; }
  }
  std::vector<tsvd_info> infos(count);
  std::vector<std::vector<int>> its(count);
  for (int p = 0; p < count; p++) { its[p].resize(probs[p].opts.k); infos[p] = tsvd_info{}; infos[p].iters = its[p].data(); }
  std::vector<int32_t> sts(count);
  tsvd_status st = TSVD_OK;
  for (int w = 0; w < warmup; w++) st = tsvd_dense_batched(ctx, count, probs.data(), 0, infos.data(), sts.data(), nullptr);
  hipDeviceSynchronize();
  const auto t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < steps; i++) st = tsvd_dense_batched(ctx, count, probs.data(), 0, infos.data(), sts.data(), nullptr);
  hipDeviceSynchronize();
  const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  double err = 0;
  int ok = 0;
  long triplets = 0;
  for (int p = 0; p < count; p++) {
    const int k = probs[p].opts.k;
    triplets += k;
    if (sts[p] != TSVD_OK) continue;
    ok++;
    std::vector<double> hS(k);
    hipMemcpy(hS.data(), probs[p].S, (size_t)k * 8, hipMemcpyDeviceToHost);
    for (int l = 0; l < k; l++) err = fmax(err, fabs(hS[l] - sv[p][l]) / sv[p][l]);
  }
  printf("{\"status\": \"%s\", \"count\": %d, \"team_kib\": %d, \"ok\": %d, \"steps\": %d, \"ms_per_step\": %.3f, "
         "\"problems_per_s\": %.2f, \"triplets_per_s\": %.1f, \"gram_ms\": %.3f, \"power_ms\": %.3f, "
         "\"finish_ms\": %.3f, \"sigma_rel_err_max\": %.3e}\n",
         tsvd_status_string(st), count, team_kib, ok, steps, dt * 1e3 / steps, count * steps / dt, triplets * steps / dt,
         infos[0].t_gram_ms, infos[0].t_eig_ms, infos[0].t_final_ms, err);
  fflush(stdout);
  tsvd_ctx_destroy(ctx);
  for (void* b : bufs) hipFree(b);
  return ok == count ? 0 : 1;
}

int main(int argc, char** argv) {
  if (argc > 1 && argv[1][0] == 'm') return run_mfma();
  if (argc > 1 && argv[1][0] == 'e')
    return run_exchange(argc > 2 ? atoi(argv[2]) : 4096, argc > 3 ? atoi(argv[3]) : 4000);
  if (argc > 1 && argv[1][0] == 'b')
    return run_batch(argc > 2 ? atoi(argv[2]) : 64, argc > 3 ? atoi(argv[3]) : 3, argc > 4 ? atoi(argv[4]) : 1,
                     argc > 5 ? strtoull(argv[5], nullptr, 10) : 7, argc > 6 ? atoi(argv[6]) : 0);
  if (argc > 1 && argv[1][0] == 'g') return run_gather();
  if (argc > 1 && argv[1][0] == 'c')
    return run_copy(argc > 2 ? strtoull(argv[2], nullptr, 10) : ((size_t)1 << 30), argc > 3 ? atoi(argv[3]) : 5);
  const int64_t m = argc > 1 ? atoll(argv[1]) : 200000;
  const int64_t n = argc > 2 ? atoll(argv[2]) : 4096;
  const int k = argc > 3 ? atoi(argv[3]) : 64;
  const double eps = argc > 4 ? atof(argv[4]) : 5e-8;
  const int gram = argc > 5 ? atoi(argv[5]) : TSVD_GRAM_BF16X3;
  const int steps = argc > 6 ? atoi(argv[6]) : 3;
  const int warmup = argc > 7 ? atoi(argv[7]) : 1;
  const uint64_t seed = argc > 8 ? strtoull(argv[8], nullptr, 10) : 7;
  const size_t copy_bytes = argc > 9 ? strtoull(argv[9], nullptr, 10) : 0;
  if (copy_bytes > 0 && run_copy(copy_bytes, 1) != 0) return 1;
  if (m < n || k > n) { fprintf(stderr, "need m >= n >= k\n"); return 2; }

  std::vector<double> s(n);
  for (int64_t i = 0; i < n; i++) s[i] = pow(0.97, (double)i);
  float* hA = nullptr;
  if (hipHostMalloc((void**)&hA, (size_t)m * n * 4, hipHostMallocDefault) != hipSuccess) { fprintf(stderr, "host alloc\n"); return 1; }
  make_known(m, n, s, seed, hA);
  std::vector<double> hv0((size_t)k * n);
  for (size_t i = 0; i < hv0.size(); i++) hv0[i] = gauss(seed + 31, i);

  float* A; double *v0, *U, *S, *V;
  if (hipMalloc(&A, (size_t)m * n * 4) || hipMalloc(&v0, hv0.size() * 8) || hipMalloc(&U, (size_t)m * k * 8) ||
      hipMalloc(&S, (size_t)k * 8) || hipMalloc(&V, (size_t)n * k * 8)) { fprintf(stderr, "device alloc\n"); return 1; }
  hipMemcpy(A, hA, (size_t)m * n * 4, hipMemcpyHostToDevice);
  hipMemcpy(v0, hv0.data(), hv0.size() * 8, hipMemcpyHostToDevice);
  tsvd_ctx* ctx;
  if (tsvd_ctx_create(0, &ctx) != TSVD_OK) { fprintf(stderr, "ctx\n"); return 1; }
  tsvd_opts o;
  tsvd_opts_default(&o);
  o.k = k; o.eps = eps; o.gram = gram; o.v0 = v0;
  std::vector<int> iters(k);
  tsvd_info info = {};
  info.iters = iters.data();
  for (int w = 0; w < warmup; w++) tsvd_dense(ctx, A, TSVD_F32, TSVD_LOC_DEVICE, m, n, n, &o, U, m, S, V, n, &info, nullptr);
  hipDeviceSynchronize();
  double tg = 0, te = 0, tf = 0;
  const auto t0 = std::chrono::steady_clock::now();
  tsvd_status st = TSVD_OK;
  for (int i = 0; i < steps; i++) {
    st = tsvd_dense(ctx, A, TSVD_F32, TSVD_LOC_DEVICE, m, n, n, &o, U, m, S, V, n, &info, nullptr);
    tg += info.t_gram_ms; te += info.t_eig_ms; tf += info.t_final_ms;
  }
  hipDeviceSynchronize();
  const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  std::vector<double> hS(k);
  hipMemcpy(hS.data(), S, (size_t)k * 8, hipMemcpyDeviceToHost);
  double err = 0;
  for (int l = 0; l < k; l++) err = fmax(err, fabs(hS[l] - s[l]) / s[l]);
  long it_total = 0;
  for (int l = 0; l < k; l++) it_total += iters[l];
  printf("{\"status\": \"%s\", \"m\": %lld, \"n\": %lld, \"k\": %d, \"eps\": %g, \"gram\": %d, \"steps\": %d, "
         "\"ms_per_step\": %.3f, \"triplets_per_s\": %.2f, \"gram_ms\": %.3f, \"power_ms\": %.3f, \"finish_ms\": %.3f, "
         "\"iters_total\": %ld, \"sigma_rel_err_max\": %.3e}\n",
         tsvd_status_string(st), (long long)m, (long long)n, k, eps, gram, steps, dt * 1e3 / steps, k * steps / dt,
         tg / steps, te / steps, tf / steps, it_total, err);
  fflush(stdout);
  tsvd_ctx_destroy(ctx);
  hipFree(A); hipFree(v0); hipFree(U); hipFree(S); hipFree(V);
  hipHostFree(hA);
  return st == TSVD_OK ? 0 : 1;
}
