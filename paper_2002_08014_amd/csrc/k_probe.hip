// HBM stream-read probe: reads a buffer once with 128-bit loads so its duration
// gives the achievable read bandwidth (a measured roofline ceiling next to the
// published 8 TB/s) and a kernel of known traffic for calibrating counters.
#include "lp_internal.h"

namespace lp {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// Each workgroup streams one contiguous chunk with eight 128-bit nontemporal
// loads in flight per thread (the pattern that reaches the highest read rate).
__global__ void __launch_bounds__(256) stream_read_kernel(const f4* __restrict__ p, int64_t n4,
                                                          float* __restrict__ sink) {
  constexpr int U = 8;
  const int64_t per = (n4 + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = b0 + per < n4 ? b0 + per : n4;
  f4 acc = f4{0.f, 0.f, 0.f, 0.f};
  int64_t e = b0 + threadIdx.x;
  for (; e + (U - 1) * 256 < b1; e += U * 256) {
    f4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(p + e + u * 256);
#pragma unroll
    for (int u = 0; u < U; ++u) acc += v[u];
  }
  for (; e < b1; e += 256) acc += __builtin_nontemporal_load(p + e);
  const float v = acc[0] + acc[1] + acc[2] + acc[3];
  // keeps the loads alive; a sum of exactly this value essentially never occurs
  if (v == 1234.5678f) sink[blockIdx.x & 1023] = v;
}

// Copy with the same streaming pattern (known read and write traffic).
__global__ void __launch_bounds__(256) stream_copy_kernel(f4* __restrict__ dst,
                                                          const f4* __restrict__ src, int64_t n4) {
  constexpr int U = 8;
  const int64_t per = (n4 + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = b0 + per < n4 ? b0 + per : n4;
  int64_t e = b0 + threadIdx.x;
  for (; e + (U - 1) * 256 < b1; e += U * 256) {
    f4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + e + u * 256);
#pragma unroll
    for (int u = 0; u < U; ++u) dst[e + u * 256] = v[u];
  }
  for (; e < b1; e += 256) dst[e] = __builtin_nontemporal_load(src + e);
}

}  // namespace

__device__ float g_probe_sink[1024];

hipError_t launch_stream_read(const void* buf, size_t bytes, hipStream_t s) {
  float* sink = nullptr;
  hipError_t e = hipGetSymbolAddress((void**)&sink, HIP_SYMBOL(g_probe_sink));
  if (e != hipSuccess) return e;
  const int64_t n4 = (int64_t)(bytes / 16);
  stream_read_kernel<<<2048, 256, 0, s>>>((const f4*)buf, n4, sink);
  return hipGetLastError();
}

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  stream_copy_kernel<<<2048, 256, 0, s>>>((f4*)dst, (const f4*)src, (int64_t)(bytes / 16));
  return hipGetLastError();
}

}  // namespace lp
