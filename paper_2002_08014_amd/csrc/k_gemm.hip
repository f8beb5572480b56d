// Two-pass local multiply on FP32 matrix cores, for the shapes the fused
// kernels do not cover (large d, k up to 64, FP32 or BF16 A):
//   pass 1  t = A_rows Z_i              (per 128-row block of a work item)
//   pass 2  part = A_rows^T t           (per 256-column block of a work item)
// (Eq. (power_yi) without 1/s_i; the per-item partials are reduced per
// partition in FP64 afterwards.)  A is read twice; at k = 64 the two products
// cost 4 n d k flops against 2 n d b bytes, so FP32 matrix-core throughput,
// not HBM, bounds this path.
//
// Both kernels: 256 threads (4 waves), a 128 (pass 1) or 256 (pass 2) x (16 NT)
// output block per workgroup, K staged through LDS 16 at a time in two buffers (the next slice
// is fetched into registers while the current one is multiplied), operands
// read from LDS one element per lane in the v_mfma_f32_16x16x4f32 layouts
// (A: lane l holds [l%16][l/16]; B: [l/16][l%16]; D: rows 4(l/16)+r, col l%16).
// Products are exact in FP32; accumulation is FP32 (BF16 A is widened exactly).
#include "lp_internal.h"

namespace lp {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// output rows per workgroup of pass 1 and output columns per workgroup of pass 2
// (4 waves x 16-row or 16-column blocks; measured best at k = 64: 98 and 109
// TFLOP/s, against 95 with 256 rows in pass 1 and 104 with 128 columns in pass 2)
constexpr int kBM1 = 128;
constexpr int kBM2 = 256;
constexpr int kBK = 16;    // contraction slice staged per step (16 measured 11-12 % faster
                           // than 32 at k = 64: half the LDS, five waves per SIMD instead of two)

// LDS row strides (floats) of the staged operands.  A lane reads element
// [4 kk + l/16][16 nt + l%16] of a k-wide operand (or of the 128-wide A slice
// in pass 2): a stride of 16 modulo 64 words puts the 64 lanes on 64 distinct
// banks (16 (l/16) + l%16).  Pass 1 reads A as [16 mt + l%16][4 kk + l/16]:
// its stride 36 (16-byte aligned rows) gives 36 (l%16) + l/16, distinct
// modulo 64.
constexpr int pad16(int n) { return n <= 16 ? 16 : 80; }   // n <= 64

template <typename TA>
__device__ inline f4 load4(const TA* p);
template <>
__device__ inline f4 load4<float>(const float* p) {
  return *(const f4*)p;
}
template <>
__device__ inline f4 load4<__hip_bfloat16>(const __hip_bfloat16* p) {
  const uint2 v = *(const uint2*)p;
  return f4{__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xffff0000u),
            __uint_as_float(v.y << 16), __uint_as_float(v.y & 0xffff0000u)};
}

// pass 1: t[row][n] = sum_c A[row][c] Z[c][n]; grid (items, ceil(max item rows / 128));
// BK: contraction slice staged per step.  SPLIT > 1 (the local-Gram form, items of
// equal rows): grid (items x SPLIT, ...), workgroup column s of item it sums the
// contraction columns [s cs, (s + 1) cs) (cs = d / SPLIT rounded up to 4) into the
// partial t + ((it.slot SPLIT + s) it.rows + row) k
template <typename TA, int NT, int BK, int MT, int SPLIT = 1>
__global__ void __launch_bounds__(256)
tmm_kernel(const TA* __restrict__ A, int64_t lda, int64_t d, int k, const float* __restrict__ Zw,
           int64_t z_stride, const WorkItem* __restrict__ items, float* __restrict__ t,
           unsigned long long* __restrict__ stamps = nullptr) {
  constexpr int N = 16 * NT;
  constexpr int BM = 64 * MT;            // rows per workgroup (4 waves x MT 16-row blocks)
  constexpr int AP = BK + 4;             // padded A row (floats)
  constexpr int ZP = pad16(N);           // padded Z row
  constexpr int ZE = (BK * N) / 256;     // Z elements per thread per slice
  constexpr int AQ = BK / 4;             // 4-element groups per A row
  constexpr int AE = (BM * AQ) / 256;    // 4-element groups per thread per slice
  __shared__ float As[2][BM * AP];
  __shared__ float Zs[2][BK * ZP];
  const WorkItem it = items[blockIdx.x / SPLIT];
  const int64_t r0 = (int64_t)blockIdx.y * BM;
  const unsigned long long t_start = stamps != nullptr ? wall_clock64() : 0;
  const int64_t wg = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  if (r0 >= it.rows) {
    if (stamps != nullptr && threadIdx.x == 0) stamps[2 * wg] = stamps[2 * wg + 1] = t_start;
    return;
  }
  const int rows = (int)min<int64_t>(BM, it.rows - r0);
  const int sp = (int)(blockIdx.x % SPLIT);
  const int64_t cs = SPLIT == 1 ? d : ((d + 4 * SPLIT - 1) / (4 * SPLIT)) * 4;
  const int64_t cb = (int64_t)sp * cs;                   // first contraction column
  d = SPLIT == 1 ? d : min<int64_t>(cs, d - cb);          // contraction length of this block
  const TA* Ab = A + (it.row0 + r0) * lda + cb;
  const float* Z = Zw + (int64_t)it.part * z_stride + cb * k;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, i = lane & 15;

  // staging: A slice BM x BK as AE groups of 4 elements per thread (row (tid + 256 j) / AQ,
  // cols 4 (tid % AQ)..)
  f4 pa[AE];
  float pz[ZE];
  auto fetch = [&](int64_t c0) {
#pragma unroll
    for (int j = 0; j < AE; ++j) {
      const int r = (tid + 256 * j) / AQ;
      const int64_t c = c0 + 4 * (tid % AQ);
      pa[j] = (r < rows && c < d) ? load4<TA>(Ab + (int64_t)r * lda + c) : f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int j = 0; j < ZE; ++j) {
      const int e = tid + 256 * j;
      const int kk = e / N, n = e % N;
      const int64_t c = c0 + kk;
      pz[j] = (c < d && n < k) ? Z[c * k + n] : 0.f;
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int j = 0; j < AE; ++j) *(f4*)&As[b][((tid + 256 * j) / AQ) * AP + 4 * (tid % AQ)] = pa[j];
#pragma unroll
    for (int j = 0; j < ZE; ++j) {
      const int e = tid + 256 * j;
      Zs[b][(e / N) * ZP + e % N] = pz[j];
    }
  };

  f4 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};

  const int nsl = (int)((d + BK - 1) / BK);
  fetch(0);
  stash(0);
  __syncthreads();
  for (int s = 0; s < nsl; ++s) {
    const int b = s & 1;
    if (s + 1 < nsl) fetch((int64_t)(s + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      float a[MT], z[NT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) a[mt] = As[b][(16 * MT * w + 16 * mt + i) * AP + 4 * kk + g];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) z[nt] = Zs[b][(4 * kk + g) * ZP + 16 * nt + i];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt], z[nt], acc[mt][nt], 0, 0, 0);
    }
    if (s + 1 < nsl) stash(b ^ 1);
    __syncthreads();
  }
  float* tb = t + (SPLIT == 1 ? it.row0 + r0 : ((int64_t)it.slot * SPLIT + sp) * it.rows + r0) * k;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * MT * w + 16 * mt + 4 * g + r;
        const int n = 16 * nt + i;
        if (row < rows && n < k) tb[(int64_t)row * k + n] = acc[mt][nt][r];
      }
  if (stamps != nullptr) {
    __syncthreads();
    if (threadIdx.x == 0) {
      stamps[2 * wg] = t_start;
      stamps[2 * wg + 1] = wall_clock64();
    }
  }
}

// pass 2: part[slot][c][n] = sum_{rows of item} A[row][c] t[row][n]; grid (items, ceil(d / 128))
template <typename TA, int NT, int BK, int MT>
__global__ void __launch_bounds__(256)
ymm_kernel(const TA* __restrict__ A, int64_t lda, int64_t d, int k, const float* __restrict__ t,
           const WorkItem* __restrict__ items, float* __restrict__ part,
           unsigned long long* __restrict__ stamps = nullptr) {
  constexpr int N = 16 * NT;
  constexpr int BM = 64 * MT;            // columns per workgroup (4 waves x MT 16-column blocks)
  constexpr int AP = BM + 16;            // padded A slice row (floats)
  constexpr int AQ = BM / 4;             // 4-element groups per A slice row
  constexpr int TP = pad16(N);
  constexpr int TE = (BK * N) / 256;
  constexpr int AE = (BK * AQ) / 256;    // 4-element groups per thread per slice
  __shared__ float As[2][BK * AP];
  __shared__ float Ts[2][BK * TP];
  const WorkItem it = items[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.y * BM;
  const int rows = (int)it.rows;
  const TA* Ab = A + it.row0 * lda + c0;
  const float* tb = t + it.row0 * k;
  const unsigned long long t_start = stamps != nullptr ? wall_clock64() : 0;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, i = lane & 15;

  // staging: A slice BK rows x BM columns, thread -> row (tid + 256 j) / AQ, cols 4 (tid % AQ)..
  f4 pa[AE];
  float pt[TE];
  auto fetch = [&](int rs) {
#pragma unroll
    for (int j = 0; j < AE; ++j) {
      const int r = rs + (tid + 256 * j) / AQ;
      const int64_t c = c0 + 4 * (tid % AQ);
      pa[j] = (r < rows && c < d) ? load4<TA>(Ab + (int64_t)r * lda + 4 * (tid % AQ))
                                  : f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int j = 0; j < TE; ++j) {
      const int e = tid + 256 * j;
      const int rr = e / N, n = e % N;
      pt[j] = (rs + rr < rows && n < k) ? tb[(int64_t)(rs + rr) * k + n] : 0.f;
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int j = 0; j < AE; ++j) *(f4*)&As[b][((tid + 256 * j) / AQ) * AP + 4 * (tid % AQ)] = pa[j];
#pragma unroll
    for (int j = 0; j < TE; ++j) {
      const int e = tid + 256 * j;
      Ts[b][(e / N) * TP + e % N] = pt[j];
    }
  };

  f4 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};

  const int nsl = (rows + BK - 1) / BK;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int s = 0; s < nsl; ++s) {
    const int b = s & 1;
    if (s + 1 < nsl) fetch((s + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      float a[MT], y[NT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) a[mt] = As[b][(4 * kk + g) * AP + 16 * MT * w + 16 * mt + i];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) y[nt] = Ts[b][(4 * kk + g) * TP + 16 * nt + i];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt], y[nt], acc[mt][nt], 0, 0, 0);
    }
    if (s + 1 < nsl) stash(b ^ 1);
    __syncthreads();
  }
  float* o = part + (int64_t)it.slot * d * k;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t c = c0 + 16 * MT * w + 16 * mt + 4 * g + r;
        const int n = 16 * nt + i;
        if (c < d && n < k) o[c * k + n] = acc[mt][nt][r];
      }
  if (stamps != nullptr) {
    __syncthreads();
    if (threadIdx.x == 0) {
      const int64_t wg = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
      stamps[2 * wg] = t_start;
      stamps[2 * wg + 1] = wall_clock64();
    }
  }
}

// Gram products of the local-Gram form: M_i[c][n] = sum over the rows of
// partition i of A[row][c] A[row][n] (M_i' = A_i^T A_i, FP32 accumulation of
// exact products).  The same tiling as pass 2, with the second operand read
// from A itself: workgroup (i, cb, nb) owns columns [256 cb, 256 cb + 256) of
// rows [64 nb, 64 nb + 64) of M_i (M is symmetric, so rows and columns are
// interchangeable) and streams the partition's rows 16 at a time.
template <typename TA>
__global__ void __launch_bounds__(256)
gram_kernel(const TA* __restrict__ A, int64_t lda, int64_t d, const WorkItem* __restrict__ parts,
            float* __restrict__ M) {
  constexpr int NT = 4, N = 64, BK = kBK, MT = 4;
  constexpr int BM = 64 * MT;
  constexpr int AP = BM + 16;
  constexpr int AQ = BM / 4;
  constexpr int TP = pad16(N);
  constexpr int TE = (BK * N) / 256;
  constexpr int AE = (BK * AQ) / 256;
  __shared__ float As[2][BK * AP];
  __shared__ float Ts[2][BK * TP];
  const WorkItem it = parts[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.y * BM;
  const int64_t n0 = (int64_t)blockIdx.z * N;
  const int64_t rows = it.rows;
  const TA* Ab = A + it.row0 * lda;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, i = lane & 15;

  f4 pa[AE];
  float pt[TE];
  auto fetch = [&](int64_t rs) {
#pragma unroll
    for (int j = 0; j < AE; ++j) {
      const int64_t r = rs + (tid + 256 * j) / AQ;
      const int64_t c = c0 + 4 * (tid % AQ);
      pa[j] = (r < rows && c < d) ? load4<TA>(Ab + r * lda + c) : f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int j = 0; j < TE; ++j) {
      const int e = tid + 256 * j;
      const int64_t r = rs + e / N;
      const int64_t n = n0 + e % N;
      pt[j] = (r < rows && n < d) ? (float)Ab[r * lda + n] : 0.f;
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int j = 0; j < AE; ++j) *(f4*)&As[b][((tid + 256 * j) / AQ) * AP + 4 * (tid % AQ)] = pa[j];
#pragma unroll
    for (int j = 0; j < TE; ++j) {
      const int e = tid + 256 * j;
      Ts[b][(e / N) * TP + e % N] = pt[j];
    }
  };

  f4 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};

  const int64_t nsl = (rows + BK - 1) / BK;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int64_t s = 0; s < nsl; ++s) {
    const int b = (int)(s & 1);
    if (s + 1 < nsl) fetch((s + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      float a[MT], y[NT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) a[mt] = As[b][(4 * kk + g) * AP + 16 * MT * w + 16 * mt + i];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) y[nt] = Ts[b][(4 * kk + g) * TP + 16 * nt + i];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt], y[nt], acc[mt][nt], 0, 0, 0);
    }
    if (s + 1 < nsl) stash(b ^ 1);
    __syncthreads();
  }
  float* o = M + (int64_t)it.part * d * d;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t c = c0 + 16 * MT * w + 16 * mt + 4 * g + r;
        const int64_t n = n0 + 16 * nt + i;
        if (c < d && n < d) o[c * d + n] = acc[mt][nt][r];
      }
}

template <typename TA, int NT>
hipError_t gemm_pair(const Plan& P, const void* A, int64_t lda, int k, const void* Zw,
                     int64_t z_stride, void* tbuf, void* part, const WorkItem* items, int nitems,
                     hipStream_t s) {
  dim3 g1(nitems, (unsigned)((P.chunk_rows + kBM1 - 1) / kBM1));
  // profiled launch: pass 1's workgroups stamp first, pass 2's after them
  unsigned long long* st1 = P.stamps;
  unsigned long long* st2 = P.stamps != nullptr ? P.stamps + 2 * (int64_t)g1.x * g1.y : nullptr;
  tmm_kernel<TA, NT, kBK, kBM1 / 64><<<g1, 256, 0, s>>>((const TA*)A, lda, P.d, k, (const float*)Zw, z_stride, items,
                                        (float*)tbuf, st1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 g2(nitems, (unsigned)((P.d + kBM2 - 1) / kBM2));
  ymm_kernel<TA, NT, kBK, kBM2 / 64><<<g2, 256, 0, s>>>((const TA*)A, lda, P.d, k, (const float*)tbuf, items,
                                        (float*)part, st2);
  return hipGetLastError();
}

template <typename TA>
hipError_t gemm_k(const Plan& P, const void* A, int64_t lda, int k, const void* Zw, int64_t z_stride,
                  void* tbuf, void* part, const WorkItem* items, int nitems, hipStream_t s) {
  if (k <= 16) return gemm_pair<TA, 1>(P, A, lda, k, Zw, z_stride, tbuf, part, items, nitems, s);
  if (k <= 32) return gemm_pair<TA, 2>(P, A, lda, k, Zw, z_stride, tbuf, part, items, nitems, s);
  if (k <= 48) return gemm_pair<TA, 3>(P, A, lda, k, Zw, z_stride, tbuf, part, items, nitems, s);
  return gemm_pair<TA, 4>(P, A, lda, k, Zw, z_stride, tbuf, part, items, nitems, s);
}

}  // namespace

bool gemm_eligible(lp_dtype dtype, int64_t d, int64_t lda, const void* A) {
  const uintptr_t align = dtype == LP_F32 ? 16 : 8;
  return (dtype == LP_F32 || dtype == LP_BF16) && d % 4 == 0 && lda % 4 == 0 &&
         ((uintptr_t)A % align) == 0;
}

hipError_t launch_local_multiply_gemm(const Plan& P, const void* A, int64_t lda, int k,
                                      const void* Zw, int64_t z_stride, void* tbuf, void* part,
                                      const WorkItem* items, int nitems,
                                      hipStream_t s) {
  if (P.dtype == LP_F32)
    return gemm_k<float>(P, A, lda, k, Zw, z_stride, tbuf, part, items, nitems, s);
  return gemm_k<__hip_bfloat16>(P, A, lda, k, Zw, z_stride, tbuf, part, items, nitems, s);
}

hipError_t launch_gram_products(const Plan& P, const void* A, int64_t lda, const WorkItem* parts,
                                int m, float* M, hipStream_t s) {
  dim3 g(m, (unsigned)((P.d + 255) / 256), (unsigned)((P.d + 63) / 64));
  if (P.dtype == LP_F32)
    gram_kernel<float><<<g, 256, 0, s>>>((const float*)A, lda, P.d, parts, M);
  else
    gram_kernel<__hip_bfloat16><<<g, 256, 0, s>>>((const __hip_bfloat16*)A, lda, P.d, parts, M);
  return hipGetLastError();
}

hipError_t launch_gram_multiply(const Plan& P, const float* M, int k, const void* Zw,
                                int64_t z_stride, void* tbuf, const WorkItem* items, int m,
                                int split, hipStream_t s) {
  // pass 1 alone over the stacked d x d matrices: item i covers rows i d .. i d + d - 1
  dim3 g(m, (unsigned)((P.d + kBM1 - 1) / kBM1));
  const float* Z = (const float*)Zw;
  float* t = (float*)tbuf;
  constexpr int MT = kBM1 / 64;
  if (k <= 16) {
    // HBM-bound at k <= 16 (8 flop per byte of M): 64-row blocks (twice the
    // workgroups) and 32-deep slices (128-byte row segments per load) stream M at
    // 5.6 TB/s against 3.7 with the two-pass tiles (m = 32, d = 1024); splitting
    // the contraction in two halves (two partial Y_i per partition, summed by the
    // reduction) doubles the workgroups again: 6.3 TB/s (24.2 -> 21.5 us)
    if (split == 2) {
      dim3 g2(2 * m, (unsigned)((P.d + 63) / 64));
      tmm_kernel<float, 1, 32, 1, 2><<<g2, 256, 0, s>>>(M, P.d, P.d, k, Z, z_stride, items, t);
    } else {
      dim3 g1(m, (unsigned)((P.d + 63) / 64));
      tmm_kernel<float, 1, 32, 1><<<g1, 256, 0, s>>>(M, P.d, P.d, k, Z, z_stride, items, t);
    }
  } else if (k <= 32) tmm_kernel<float, 2, kBK, MT><<<g, 256, 0, s>>>(M, P.d, P.d, k, Z, z_stride, items, t);
  else if (k <= 48) tmm_kernel<float, 3, kBK, MT><<<g, 256, 0, s>>>(M, P.d, P.d, k, Z, z_stride, items, t);
  else tmm_kernel<float, 4, kBK, MT><<<g, 256, 0, s>>>(M, P.d, P.d, k, Z, z_stride, items, t);
  return hipGetLastError();
}

}  // namespace lp
