// Fused single-pass local multiply on the vector ALUs for small ranks
// (k <= 8, FP32 or BF16 A, d a power of two in [256, 4096]).
//
// Computes, for one work item (a contiguous row range of partition i),
//   part = A_rows^T (A_rows Z_i)            (Eq. (power_yi) without 1/s_i)
// reading every element of A once from HBM, in FP32 arithmetic (BF16 A is
// widened exactly).  At k < 16 the two products are too thin for the matrix
// cores, so both run as FP32 FMAs.
//
// Layout: 512 threads; each owns 8 columns of A (FP32: two 16-byte chunks at
// columns 4 t and 4 (t + TPR); BF16: one 16-byte chunk at columns 8 t) and
// keeps Z_i and the Y partial of those columns in registers.  TPR = d / 8
// threads cover a row; the 512 / TPR row groups take R = 4 rows each per step.
//   * product 1: each thread forms the partial t over its 8 columns for its
//     group's 4 rows (4 K values), written to LDS; the TPR partials of each of
//     the 4 K outputs are summed in two levels (blocks of 4 K consecutive
//     threads, then the blocks), in a fixed order;
//   * product 2: every thread of the group reads the group's t (broadcast) and
//     adds A_rows^T t to its Y columns.
// The next one or two steps' rows are loaded into registers (kept packed)
// while the current step computes.  At the end the row groups' Y partials are
// summed through LDS in a fixed order and written as the item's partial.  K is the rank padded to 1,
// 2, 4 or 8 (padding columns of Z are zero and are not written).
#include "lp_internal.h"

namespace lp {
namespace {

constexpr int kThreads = 512;
constexpr int kR = 4;        // rows per row group per step
constexpr int kCPT = 8;      // columns per thread

typedef float f4 __attribute__((ext_vector_type(4)));

typedef unsigned u4 __attribute__((ext_vector_type(4)));

// One row's eight columns as loaded (FP32: two 16-byte chunks; BF16: one), kept
// packed while in flight and widened to FP32 when their step computes.
template <typename TA>
struct Raw;
template <>
struct Raw<float> {
  f4 x, y;
};
template <>
struct Raw<__hip_bfloat16> {
  u4 v;
};

__device__ inline void load_raw(const float* row, int tl, int TPR, bool ok, Raw<float>& r) {
  if (ok) {
    r.x = __builtin_nontemporal_load((const f4*)(row + 4 * tl));
    r.y = __builtin_nontemporal_load((const f4*)(row + 4 * (tl + TPR)));
  } else {
    r.x = r.y = f4{0.f, 0.f, 0.f, 0.f};
  }
}
__device__ inline void load_raw(const __hip_bfloat16* row, int tl, int /*TPR*/, bool ok,
                                Raw<__hip_bfloat16>& r) {
  if (ok)
    r.v = __builtin_nontemporal_load((const u4*)(row + 8 * tl));
  else
    r.v = u4{0u, 0u, 0u, 0u};
}
__device__ inline void widen(const Raw<float>& r, float (&a)[kCPT]) {
  a[0] = r.x[0]; a[1] = r.x[1]; a[2] = r.x[2]; a[3] = r.x[3];
  a[4] = r.y[0]; a[5] = r.y[1]; a[6] = r.y[2]; a[7] = r.y[3];
}
__device__ inline void widen(const Raw<__hip_bfloat16>& r, float (&a)[kCPT]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    a[2 * q] = __uint_as_float(r.v[q] << 16);
    a[2 * q + 1] = __uint_as_float(r.v[q] & 0xffff0000u);
  }
}

// column of A held in slot c of thread tl
template <typename TA>
__device__ inline int col_of(int tl, int TPR, int c) {
  if constexpr (sizeof(TA) == 4)
    return c < 4 ? 4 * tl + c : 4 * (tl + TPR) + (c - 4);
  else
    return 8 * tl + c;
}

// PF: steps in flight ahead of the one computing (1 or 2; two where the
// registers allow: BF16 rows are half as wide while packed)
template <typename TA, int K, int PF>
__global__ void __launch_bounds__(kThreads, 1)
k1_valu(const TA* __restrict__ A, int64_t lda, int d, int k, const float* __restrict__ Zw,
        int64_t z_stride, const WorkItem* __restrict__ items, float* __restrict__ part) {
  constexpr int V = kR * K;            // t outputs per row group and step
  constexpr int PS = V + 4;            // padded LDS stride of one thread's partials
  // partials of one step; reused at the end for the row-group sum of Y
  // (two passes of half the columns: 512 threads x 4 columns x K <= 512 x PS)
  __shared__ __attribute__((aligned(16))) float pbuf[kThreads * PS];
  __shared__ float l1[kThreads];                      // level-1 sums
  __shared__ __attribute__((aligned(16))) float tsh[kThreads / 32 * V];   // t per row group
  const WorkItem it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const int TPR = d / kCPT;
  const int RG = kThreads / TPR;
  const int rg = tid / TPR, tl = tid % TPR;
  const int NB = TPR / V;              // level-1 blocks per row group
  const int rows = (int)it.rows;
  const TA* Ab = A + it.row0 * lda;

  float z[kCPT][K], y[kCPT][K];
  const float* Z = Zw + (int64_t)it.part * z_stride;
#pragma unroll
  for (int c = 0; c < kCPT; ++c) {
    const int col = col_of<TA>(tl, TPR, c);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      z[c][j] = j < k ? Z[(int64_t)col * k + j] : 0.f;
      y[c][j] = 0.f;
    }
  }

  const int step_rows = RG * kR;
  const int nsteps = (rows + step_rows - 1) / step_rows;
  Raw<TA> raw[PF][kR];
  auto load_step = [&](int st, Raw<TA> (&dst)[kR]) {
#pragma unroll
    for (int i = 0; i < kR; ++i) {
      const int r = st * step_rows + rg * kR + i;
      load_raw(Ab + (int64_t)min(r, rows - 1) * lda, tl, TPR, r < rows, dst[i]);
    }
  };
#pragma unroll
  for (int q = 0; q < PF; ++q)
    if (q < nsteps) load_step(q, raw[q]);
  for (int s0 = 0; s0 < nsteps; s0 += PF) {
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int s = s0 + q;
      if (s >= nsteps) break;
      float a[kR][kCPT];
#pragma unroll
      for (int i = 0; i < kR; ++i) widen(raw[q][i], a[i]);
      if (s + PF < nsteps) load_step(s + PF, raw[q]);
      // product 1: partial t over this thread's columns
      float p[V];
#pragma unroll
      for (int i = 0; i < kR; ++i)
#pragma unroll
        for (int j = 0; j < K; ++j) {
          float acc = 0.f;
#pragma unroll
          for (int c = 0; c < kCPT; ++c) acc = fmaf(a[i][c], z[c][j], acc);
          p[i * K + j] = acc;
        }
      float* mine = &pbuf[(rg * TPR + tl) * PS];
#pragma unroll
      for (int v = 0; v < V; v += 4) *(f4*)&mine[v] = f4{p[v], p[v + 1], p[v + 2], p[v + 3]};
      __syncthreads();
      // level 1: output v = tl % V over the V consecutive threads of block tl / V
      {
        const int v = tl % V, b = tl / V;
        const float* src = &pbuf[(rg * TPR + b * V) * PS + v];
        float acc = 0.f;
#pragma unroll
        for (int u = 0; u < V; ++u) acc += src[u * PS];
        if (NB == 1)
          tsh[rg * V + v] = acc;
        else
          l1[rg * TPR + b * V + v] = acc;
      }
      __syncthreads();
      if (NB > 1) {
        // level 2: the NB block sums of each output, in block order
        if (tl < V) {
          float acc = 0.f;
          for (int b = 0; b < NB; ++b) acc += l1[rg * TPR + b * V + tl];
          tsh[rg * V + tl] = acc;
        }
        __syncthreads();
      }
      // product 2: Y += A_rows^T t
      float t[V];
#pragma unroll
      for (int v = 0; v < V; v += 4) {
        const f4 qv = *(const f4*)&tsh[rg * V + v];
        t[v] = qv[0]; t[v + 1] = qv[1]; t[v + 2] = qv[2]; t[v + 3] = qv[3];
      }
#pragma unroll
      for (int c = 0; c < kCPT; ++c)
#pragma unroll
        for (int j = 0; j < K; ++j) {
          float acc = y[c][j];
#pragma unroll
          for (int i = 0; i < kR; ++i) acc = fmaf(a[i][c], t[i * K + j], acc);
          y[c][j] = acc;
        }
    }
  }

  // the item's partial: the row groups' Y summed in group order
  float* o = part + (int64_t)it.slot * d * k;
  if (RG == 1) {
#pragma unroll
    for (int c = 0; c < kCPT; ++c) {
      const int col = col_of<TA>(tl, TPR, c);
#pragma unroll
      for (int j = 0; j < K; ++j)
        if (j < k) o[(int64_t)col * k + j] = y[c][j];
    }
    return;
  }
  __syncthreads();   // every thread is past its last read of pbuf
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    // slots 4h .. 4h + 3 of every thread: pbuf[((rg TPR + tl) 4 + cc) K + j]
#pragma unroll
    for (int cc = 0; cc < 4; ++cc)
#pragma unroll
      for (int j = 0; j < K; ++j) pbuf[((rg * TPR + tl) * 4 + cc) * K + j] = y[4 * h + cc][j];
    __syncthreads();
    const int per_group = TPR * 4 * K;
    for (int e = tid; e < per_group; e += kThreads) {
      const int j = e % K, cc = (e / K) % 4, tt = e / (4 * K);
      float acc = 0.f;
      for (int g = 0; g < RG; ++g) acc += pbuf[((g * TPR + tt) * 4 + cc) * K + j];
      if (j < k) o[(int64_t)col_of<TA>(tt, TPR, 4 * h + cc) * k + j] = acc;
    }
    __syncthreads();
  }
}

template <typename TA, int K>
hipError_t launch_k(int64_t d, int k, const void* A, int64_t lda, const void* Zw, int64_t z_stride,
                    void* part, const WorkItem* items, int nitems, hipStream_t s) {
  // two steps in flight where the registers hold them without spilling (BF16
  // up to K = 4, FP32 up to K = 2), else one
  constexpr int PF = (sizeof(TA) == 2 ? K <= 4 : K <= 2) ? 2 : 1;
  k1_valu<TA, K, PF><<<nitems, kThreads, 0, s>>>((const TA*)A, lda, (int)d, k, (const float*)Zw,
                                                 z_stride, items, (float*)part);
  return hipGetLastError();
}

template <typename TA>
hipError_t launch_t(int64_t d, int k, const void* A, int64_t lda, const void* Zw, int64_t z_stride,
                    void* part, const WorkItem* items, int nitems, hipStream_t s) {
  if (k <= 1) return launch_k<TA, 1>(d, k, A, lda, Zw, z_stride, part, items, nitems, s);
  if (k <= 2) return launch_k<TA, 2>(d, k, A, lda, Zw, z_stride, part, items, nitems, s);
  if (k <= 4) return launch_k<TA, 4>(d, k, A, lda, Zw, z_stride, part, items, nitems, s);
  return launch_k<TA, 8>(d, k, A, lda, Zw, z_stride, part, items, nitems, s);
}

}  // namespace

bool valu_eligible(lp_dtype dtype, int64_t d, int64_t lda, int k, const void* A) {
  // TPR = d / 8 threads per row must divide 512 and hold at least 4 K of them
  // (one level-1 block): d a power of two in [256, 4096]
  const bool pow2 = d >= 256 && d <= 4096 && (d & (d - 1)) == 0;
  const uintptr_t align = 16;
  return (dtype == LP_F32 || dtype == LP_BF16) && pow2 && k >= 1 && k <= 8 &&
         (dtype == LP_F32 ? lda % 4 == 0 : lda % 8 == 0) && ((uintptr_t)A % align) == 0;
}

hipError_t launch_local_multiply_valu(const Plan& P, const void* A, int64_t lda, int k,
                                      const void* Zw, int64_t z_stride, void* part,
                                      const WorkItem* items, int nitems, hipStream_t s) {
  if (P.dtype == LP_F32)
    return launch_t<float>(P.d, k, A, lda, Zw, z_stride, part, items, nitems, s);
  return launch_t<__hip_bfloat16>(P.d, k, A, lda, Zw, z_stride, part, items, nitems, s);
}

}  // namespace lp
