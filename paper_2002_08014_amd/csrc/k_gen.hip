// The library's own random inputs, from Philox4x32-10 (philox.h):
//  * the Gaussian start Y0 of Algorithm 1 when the caller passes none;
//  * the exact-truth test matrix of the serving layer: A = W diag(sigma) V^T
//    with W (n x d) made of n / d row-permuted, sign-flipped Sylvester Hadamard
//    blocks (entries +-1, W^T W = n I) and V a permutation matrix, so that
//    A^T A = n V diag(sigma^2) V^T exactly, the top-k right singular vectors are
//    the columns of V for the k largest sigma, and every entry +-sigma_j is
//    exact in BF16 and FP32 (sigma rounded to BF16 beforehand).
#include "lp_internal.h"
#include "philox.h"

namespace lp {
namespace {

constexpr int kGenRows = 64;        // rows of A per workgroup of the matrix kernel
constexpr int kGenMaxD = 8192;      // columns the matrix kernel maps in LDS

__global__ void gaussian_kernel(int64_t count, uint64_t seed, double* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) Y[e] = normal_draw(seed, (uint64_t)e, kTagStart);
}

__device__ inline void store4(float* p, const float v[4]) {
  *(float4*)p = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ inline void store4(__hip_bfloat16* p, const float v[4]) {
  // the values are exact in BF16: keep the upper halves
  uint32_t u[4];
  for (int t = 0; t < 4; ++t) u[t] = __float_as_uint(v[t]) >> 16;
  *(uint2*)p = make_uint2(u[0] | (u[1] << 16), u[2] | (u[3] << 16));
}

// Stored element (R, c): generating row g = rowperm(R) (block b = g / d, row q =
// g % d of its Hadamard block), singular index j = colperm(c); the value is
// D1(g) D2(b, c) (-1)^popcount(q & j) sigma_j with D1(g) bit 0 of the row's
// Philox block and D2(b, c) bit c mod 128 of the block (c / 128, b).
template <typename T>
__global__ void __launch_bounds__(256)
truth_matrix_kernel(T* __restrict__ A, int64_t n, int64_t d, int64_t lda, int k, double gap,
                    double decay, uint64_t seed, int rbits, int cbits) {
  __shared__ int32_t jmap[kGenMaxD];
  __shared__ float sig[kGenMaxD];
  __shared__ int64_t grow[kGenRows];
  __shared__ float rsign[kGenRows];
  const int tid = threadIdx.x;
  const int64_t R0 = (int64_t)blockIdx.x * kGenRows;
  for (int64_t c = tid; c < d; c += 256) {
    const int64_t j = (int64_t)keyed_perm((uint64_t)c, (uint64_t)d, cbits, seed, kTagColPerm);
    jmap[c] = (int32_t)j;
    sig[c] = truth_sigma(j, k, gap, decay);
  }
  if (tid < kGenRows && R0 + tid < n) {
    const uint64_t g = keyed_perm((uint64_t)(R0 + tid), (uint64_t)n, rbits, seed, kTagRowPerm);
    grow[tid] = (int64_t)g;
    const U4 r = philox(seed, (uint32_t)g, (uint32_t)(g >> 32), 0u, kTagRowSign);
    rsign[tid] = (r.v[0] & 1u) ? -1.f : 1.f;
  }
  __syncthreads();
  const int64_t chunks = d / 4;
  const int rows = (int)min<int64_t>(kGenRows, n - R0);
  for (int r = 0; r < rows; ++r) {
    const int64_t g = grow[r];
    const uint64_t b = (uint64_t)(g / d);
    const uint32_t q = (uint32_t)(g % d);
    T* row = A + (R0 + r) * lda;
    for (int64_t ch = tid; ch < chunks; ch += 256) {
      const int64_t c0 = 4 * ch;
      const U4 cs = philox(seed, (uint32_t)(c0 >> 7), (uint32_t)b, (uint32_t)(b >> 32), kTagColSign);
      float v[4];
      for (int t = 0; t < 4; ++t) {
        const int64_t c = c0 + t;
        const uint32_t bit = (cs.v[(c & 127) >> 5] >> (c & 31)) & 1u;
        const uint32_t h = __popc(q & (uint32_t)jmap[c]) & 1u;
        const float s = (bit ^ h) ? -1.f : 1.f;
        v[t] = rsign[r] * s * sig[c];
      }
      store4(row + c0, v);
    }
  }
}

__global__ void truth_basis_kernel(int64_t d, int k, uint64_t seed, int cbits, double* __restrict__ U) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d) return;
  const int64_t j = (int64_t)keyed_perm((uint64_t)c, (uint64_t)d, cbits, seed, kTagColPerm);
  for (int jj = 0; jj < k; ++jj) U[c * k + jj] = (jj == j) ? 1.0 : 0.0;
}

}  // namespace

bool truth_shape_ok(int64_t n, int64_t d) {
  return d >= 16 && d <= kGenMaxD && (d & (d - 1)) == 0 && n >= d && n % d == 0;
}

hipError_t launch_gaussian(int64_t count, uint64_t seed, double* Y, hipStream_t s) {
  if (count < 1) return hipSuccess;
  gaussian_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(count, seed, Y);
  return hipGetLastError();
}

hipError_t launch_truth_matrix(void* A, lp_dtype dtype, int64_t n, int64_t d, int64_t lda, int k,
                               double gap, double decay, uint64_t seed, hipStream_t s) {
  const int rbits = perm_bits((uint64_t)n), cbits = perm_bits((uint64_t)d);
  const unsigned blocks = (unsigned)((n + kGenRows - 1) / kGenRows);
  if (dtype == LP_F32)
    truth_matrix_kernel<float><<<blocks, 256, 0, s>>>((float*)A, n, d, lda, k, gap, decay, seed,
                                                      rbits, cbits);
  else
    truth_matrix_kernel<__hip_bfloat16><<<blocks, 256, 0, s>>>((__hip_bfloat16*)A, n, d, lda, k, gap,
                                                               decay, seed, rbits, cbits);
  return hipGetLastError();
}

hipError_t launch_truth_basis(int64_t d, int k, uint64_t seed, double* U, hipStream_t s) {
  truth_basis_kernel<<<(unsigned)((d + 255) / 256), 256, 0, s>>>(d, k, seed, perm_bits((uint64_t)d), U);
  return hipGetLastError();
}

}  // namespace lp
