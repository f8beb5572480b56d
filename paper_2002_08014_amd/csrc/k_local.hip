// Local power iteration Y_i = A_i^T (A_i Z_i) for all partitions at once
// (the worker step of LocalPower, Eq. (power_yi), without the 1/s_i scale,
// which the aggregation applies as 1/n).
//
// Generic form (any dtype, d, k <= 64): two passes over each work item's rows,
//   pass 1: t = A_rows Z_i          (one wavefront per row, lanes stride d)
//   pass 2: part = A_rows^T t       (one thread per column of A, k accumulators)
// The per-item partial sums are reduced per partition in FP64, in item order.
#include "lp_internal.h"

namespace lp {
namespace {

template <typename T>
__device__ inline float to_f(T v);
template <>
__device__ inline float to_f<float>(float v) { return v; }
template <>
__device__ inline float to_f<__hip_bfloat16>(__hip_bfloat16 v) { return __bfloat162float(v); }

template <typename TA, typename TC>
__device__ inline TC load_a(const TA* p) {
  return (TC)to_f<TA>(*p);
}
template <>
__device__ inline double load_a<double, double>(const double* p) {
  return *p;
}

// pass 1: t[row][j] = sum_c A[row][c] Z_part[c][j]; grid (items, ceil(max_rows/4)), 256 threads
template <typename TA, typename TC, int KB>
__global__ void __launch_bounds__(256)
tpass_kernel(const TA* __restrict__ A, int64_t lda, int64_t d, int k, const TC* __restrict__ Zw,
             int64_t z_stride, const WorkItem* __restrict__ items, TC* __restrict__ t) {
  const WorkItem it = items[blockIdx.x];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t lr = (int64_t)blockIdx.y * 4 + wave;
  if (lr >= it.rows) return;
  const int64_t row = it.row0 + lr;
  const TA* a = A + row * lda;
  const TC* z = Zw + it.part * z_stride;
  TC acc[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) acc[j] = (TC)0;
  for (int64_t c = lane; c < d; c += 64) {
    const TC av = load_a<TA, TC>(a + c);
    const TC* zc = z + c * k;
#pragma unroll
    for (int j = 0; j < KB; ++j)
      if (j < k) acc[j] += av * zc[j];
  }
#pragma unroll
  for (int j = 0; j < KB; ++j) {
    TC v = acc[j];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    acc[j] = v;
  }
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < KB; ++j)
      if (j < k) t[row * k + j] = acc[j];
  }
}

// pass 2: part[slot][c][j] = sum_{rows of item} A[row][c] t[row][j]; grid (items, ceil(d/256))
template <typename TA, typename TC, int KB>
__global__ void __launch_bounds__(256)
ypass_kernel(const TA* __restrict__ A, int64_t lda, int64_t d, int k, const TC* __restrict__ t,
             const WorkItem* __restrict__ items, TC* __restrict__ part) {
  __shared__ TC ts[64 * KB];
  const WorkItem it = items[blockIdx.x];
  const int64_t c = (int64_t)blockIdx.y * 256 + threadIdx.x;
  TC acc[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) acc[j] = (TC)0;
  for (int64_t r0 = 0; r0 < it.rows; r0 += 64) {
    const int rows = (int)min<int64_t>(64, it.rows - r0);
    __syncthreads();
    for (int e = threadIdx.x; e < rows * k; e += 256) {
      const int rr = e / k, j = e - (e / k) * k;
      ts[rr * KB + j] = t[(it.row0 + r0) * k + e];
    }
    __syncthreads();
    if (c < d) {
      const TA* a = A + (it.row0 + r0) * lda + c;
      for (int rr = 0; rr < rows; ++rr) {
        const TC av = load_a<TA, TC>(a + rr * lda);
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] += av * ts[rr * KB + j];
      }
    }
  }
  if (c < d) {
    TC* o = part + (int64_t)it.slot * d * k + c * k;
#pragma unroll
    for (int j = 0; j < KB; ++j)
      if (j < k) o[j] = acc[j];
  }
}

// Y_i[e] = sum over the partition's slots (item order), FP64; grid (ceil(d*k/256), m)
template <typename TC>
__global__ void reduce_partials_kernel(int64_t dk, const TC* __restrict__ part,
                                       const int32_t* __restrict__ slot_off, double* __restrict__ Yi) {
  const int i = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= dk) return;
  const int s0 = slot_off[i], s1 = slot_off[i + 1];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int sl = s0;
  for (; sl + 3 < s1; sl += 4) {
    a0 += (double)part[(int64_t)sl * dk + e];
    a1 += (double)part[(int64_t)(sl + 1) * dk + e];
    a2 += (double)part[(int64_t)(sl + 2) * dk + e];
    a3 += (double)part[(int64_t)(sl + 3) * dk + e];
  }
  for (; sl < s1; ++sl) a0 += (double)part[(int64_t)sl * dk + e];
  Yi[(int64_t)i * dk + e] = (a0 + a1) + (a2 + a3);
}

template <typename TA, typename TC, int KB>
hipError_t two_pass(const Plan& P, const void* A, int64_t lda, int k, const void* Zw,
                    int64_t z_stride, void* tbuf, void* part, const WorkItem* items, int nitems,
                    hipStream_t s) {
  dim3 g1(nitems, (unsigned)((P.chunk_rows + 3) / 4));
  tpass_kernel<TA, TC, KB><<<g1, 256, 0, s>>>((const TA*)A, lda, P.d, k, (const TC*)Zw, z_stride,
                                              items, (TC*)tbuf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 g2(nitems, (unsigned)((P.d + 255) / 256));
  ypass_kernel<TA, TC, KB><<<g2, 256, 0, s>>>((const TA*)A, lda, P.d, k, (const TC*)tbuf, items,
                                              (TC*)part);
  return hipGetLastError();
}

template <typename TA, typename TC>
hipError_t two_pass_k(const Plan& P, const void* A, int64_t lda, int k, const void* Zw,
                      int64_t z_stride, void* tbuf, void* part, const WorkItem* items, int n,
                      hipStream_t s) {
  if (k <= 8) return two_pass<TA, TC, 8>(P, A, lda, k, Zw, z_stride, tbuf, part, items, n, s);
  if (k <= 16) return two_pass<TA, TC, 16>(P, A, lda, k, Zw, z_stride, tbuf, part, items, n, s);
  if (k <= 32) return two_pass<TA, TC, 32>(P, A, lda, k, Zw, z_stride, tbuf, part, items, n, s);
  return two_pass<TA, TC, 64>(P, A, lda, k, Zw, z_stride, tbuf, part, items, n, s);
}

}  // namespace

hipError_t launch_local_multiply_twopass(const Plan& P, const void* A, int64_t lda, int k,
                                         const void* Zw, int64_t z_stride, void* tbuf, void* part,
                                         const WorkItem* items, int nitems,
                                         hipStream_t s) {
  switch (P.dtype) {
    case LP_F64:
      return two_pass_k<double, double>(P, A, lda, k, Zw, z_stride, tbuf, part, items, nitems, s);
    case LP_F32:
      return two_pass_k<float, float>(P, A, lda, k, Zw, z_stride, tbuf, part, items, nitems, s);
    default:
      return two_pass_k<__hip_bfloat16, float>(P, A, lda, k, Zw, z_stride, tbuf, part, items,
                                               nitems, s);
  }
}

hipError_t launch_reduce_partials(const Plan& P, int k, const void* part, const int32_t* slot_off,
                                  double* Yi, hipStream_t s) {
  const int64_t dk = P.d * k;
  dim3 grid((unsigned)((dk + 255) / 256), P.m);
  if (P.acc_bytes == 8)
    reduce_partials_kernel<double><<<grid, 256, 0, s>>>(dk, (const double*)part, slot_off, Yi);
  else
    reduce_partials_kernel<float><<<grid, 256, 0, s>>>(dk, (const float*)part, slot_off, Yi);
  return hipGetLastError();
}

}  // namespace lp
