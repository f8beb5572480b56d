// Diagnostics of the method's analysis (not on the per-round path):
// eta = max_i ||M_i - M||_2 / ||M||_2 (Definition 2, local approximation), from
// the stacked Gram matrices of the local-Gram form (M_i' = A_i^T A_i, FP32).
// M = (1/n) sum_i M_i' is formed in FP64; each spectral norm is estimated by
// power iteration on the symmetric matrix with NB start vectors per matrix
// (x <- D x / ||D x||; ||D x|| for a unit x converges to ||D||_2 from below at
// the rate (lambda_2 / lambda_1)^2 per step, and the estimate is the largest over
// the start vectors).  D is never formed: the matvec reads M_i' and M.
#include "lp_internal.h"

namespace lp {
namespace {

constexpr int kNB = 4;   // start vectors per matrix

// M[e] = inv_n * sum_i Mi[i d^2 + e]
__global__ void __launch_bounds__(kBlock)
gram_mean_kernel(int m, int64_t dd, const float* __restrict__ Mi, double inv_n,
                 double* __restrict__ M) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= dd) return;
  double acc = 0.0;
  for (int i = 0; i < m; ++i) acc += (double)Mi[(int64_t)i * dd + e];
  M[e] = acc * inv_n;
}

// grid (ceil(d / 4), m + 1): one wave per row r of matrix b;
//   b <  m : Y_b = (inv_s[b] M_b' - M) X_b,   b == m : Y_m = M X_m.
// X, Y: (m + 1) x d x kNB, row-major per matrix.
__global__ void __launch_bounds__(kBlock)
eta_matvec_kernel(int64_t d, int m, const float* __restrict__ Mi, const double* __restrict__ inv_s,
                  const double* __restrict__ M, const double* __restrict__ X,
                  double* __restrict__ Y) {
  const int b = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= d) return;
  const int64_t dd = d * d;
  const double* xb = X + (int64_t)b * d * kNB;
  const double* Mr = M + r * d;
  const float* Mir = b < m ? Mi + (int64_t)b * dd + r * d : nullptr;
  const double sc = b < m ? inv_s[b] : 0.0;
  double acc[kNB];
#pragma unroll
  for (int j = 0; j < kNB; ++j) acc[j] = 0.0;
  for (int64_t c = lane; c < d; c += 64) {
    const double v = b < m ? fma(sc, (double)Mir[c], -Mr[c]) : Mr[c];
#pragma unroll
    for (int j = 0; j < kNB; ++j) acc[j] = fma(v, xb[c * kNB + j], acc[j]);
  }
#pragma unroll
  for (int j = 0; j < kNB; ++j) {
    double s = acc[j];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    acc[j] = s;
  }
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < kNB; ++j) Y[((int64_t)b * d + r) * kNB + j] = acc[j];
  }
}

// grid (m + 1): est[b][j] = ||Y_b[:, j]||; X_b[:, j] = Y_b[:, j] / est (kept when 0).
__global__ void __launch_bounds__(kBlock)
eta_normalize_kernel(int64_t d, const double* __restrict__ Y, double* __restrict__ X,
                     double* __restrict__ est) {
  __shared__ double red[kBlock / 64][kNB];
  __shared__ double nrm[kNB];
  const int b = blockIdx.x;
  const double* yb = Y + (int64_t)b * d * kNB;
  double* xb = X + (int64_t)b * d * kNB;
  double s[kNB];
#pragma unroll
  for (int j = 0; j < kNB; ++j) s[j] = 0.0;
  for (int64_t r = threadIdx.x; r < d; r += kBlock)
#pragma unroll
    for (int j = 0; j < kNB; ++j) s[j] = fma(yb[r * kNB + j], yb[r * kNB + j], s[j]);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < kNB; ++j) {
    double v = s[j];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[w][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < kNB) {
    double v = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) v += red[q][threadIdx.x];
    nrm[threadIdx.x] = sqrt(v);
    est[b * kNB + threadIdx.x] = sqrt(v);
  }
  __syncthreads();
  for (int64_t r = threadIdx.x; r < d; r += kBlock)
#pragma unroll
    for (int j = 0; j < kNB; ++j)
      if (nrm[j] > 0.0) xb[r * kNB + j] = yb[r * kNB + j] / nrm[j];
}

// deterministic start vectors: splitmix64 of the element index -> [-1, 1), then unit columns
// are produced by the first normalisation
__global__ void __launch_bounds__(kBlock)
eta_start_kernel(int64_t count, double* __restrict__ X) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= count) return;
  uint64_t z = (uint64_t)(e + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  X[e] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

inline int nblocks(int64_t n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

size_t eta_scratch_bytes(int64_t d, int m) {
  // M (d x d FP64), X and Y ((m + 1) x d x kNB), est ((m + 1) x kNB), inv_s (m)
  auto a = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t v = (size_t)(m + 1) * d * kNB * 8;
  return a((size_t)d * d * 8) + 2 * a(v) + a((size_t)(m + 1) * kNB * 8) + a((size_t)m * 8);
}

hipError_t launch_eta(int64_t d, int m, int64_t n, const float* Mi, const double* inv_s_host,
                      int iters, char* scratch, double* est_host, hipStream_t s) {
  auto a = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t v = (size_t)(m + 1) * d * kNB * 8;
  double* M = (double*)scratch;
  double* X = (double*)(scratch + a((size_t)d * d * 8));
  double* Y = (double*)((char*)X + a(v));
  double* est = (double*)((char*)Y + a(v));
  double* inv_s = (double*)((char*)est + a((size_t)(m + 1) * kNB * 8));
  hipError_t e;
  if ((e = hipMemcpyAsync(inv_s, inv_s_host, (size_t)m * 8, hipMemcpyHostToDevice, s)) != hipSuccess)
    return e;
  gram_mean_kernel<<<nblocks(d * d, kBlock), kBlock, 0, s>>>(m, d * d, Mi, 1.0 / (double)n, M);
  const int64_t count = (int64_t)(m + 1) * d * kNB;
  eta_start_kernel<<<nblocks(count, kBlock), kBlock, 0, s>>>(count, Y);
  eta_normalize_kernel<<<m + 1, kBlock, 0, s>>>(d, Y, X, est);
  const dim3 g(nblocks(d, 4), m + 1);
  for (int t = 0; t < iters; ++t) {
    eta_matvec_kernel<<<g, kBlock, 0, s>>>(d, m, Mi, inv_s, M, X, Y);
    eta_normalize_kernel<<<m + 1, kBlock, 0, s>>>(d, Y, X, est);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(est_host, est, (size_t)(m + 1) * kNB * 8, hipMemcpyDeviceToHost, s)) !=
      hipSuccess)
    return e;
  return hipStreamSynchronize(s);
}

int eta_start_vectors() { return kNB; }

}  // namespace lp
