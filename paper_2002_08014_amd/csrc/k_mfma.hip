// Fused single-pass local multiply on CDNA4 matrix cores (FP32 A, k = 16).
//
// Computes, for one work item (a contiguous row range of partition i),
//   part = A_rows^T (A_rows Z_i)            (Eq. (power_yi) without 1/s_i)
// reading every element of A once from HBM.  A 16-row tile is staged in LDS;
// t = A_tile Z (16 x 16) and Y += A_tile^T t both run on
// v_mfma_f32_16x16x4f32, so the intermediate t never leaves the chip.
//
// Layout (wave w of 4 owns the column slice [w*d/4, (w+1)*d/4), NQ = d/64):
//   * product 1, MFMA (q, c): K slot g = lane/16 <-> column 16q + 4g + c of the
//     slice, M index = tile row lane%16; Z_i lives in registers in the matching
//     B-operand layout (zr[q][c] = Z[16q + 4g + c][lane%16]);
//   * the four per-slice partial t's are summed through LDS; the result sits in
//     the accumulator layout t[4g + r][lane%16] (r = register);
//   * product 2, MFMA (h, s): K slot g <-> tile row 4g + s, so the B operand is
//     t register s as it stands; the M index i' <-> slice column NQ*i' + h, so
//     each lane reads NQ contiguous columns of one row (128-bit LDS reads).
//   * LDS rows are padded by 4 floats and 16-byte chunks are XOR-swizzled
//     (chunk c -> c ^ ((c >> 4) & 3)) so both read patterns are conflict-free.
#include "lp_internal.h"

namespace lp {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTileRows = 16;

__device__ inline int swz(int c4) { return c4 ^ ((c4 >> 4) & 3); }

// 128-bit load of A; nontemporal when A is streamed without reuse.
template <bool NT>
__device__ inline f4 ldA(const float* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load((const f4*)p);
  else
    return *(const f4*)p;
}

// NQ: 16-column groups per wave slice; W: waves per workgroup (d = 16*NQ*W).
template <int NQ, int W, int OCC, int PF, bool NTL>
__global__ void __launch_bounds__(64 * W, OCC)
k1_mfma_f32_k16(const float* __restrict__ A, int64_t lda, const float* __restrict__ Zw,
                int64_t z_stride, const WorkItem* __restrict__ items, float* __restrict__ part) {
  constexpr int NT = 64 * W;          // threads
  constexpr int D = 16 * NQ * W;      // columns of A
  constexpr int P = D + 4;            // padded LDS row (floats)
  constexpr int CPR = D / 4;          // 16-byte chunks per row
  constexpr int S = 16 * NQ;          // columns per wave slice
  constexpr int NL = (kTileRows * CPR) / NT;  // chunks per thread per tile (= NQ)
  __shared__ float tile[kTileRows * P];
  __shared__ f4 tpart[W][64];

  const WorkItem it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int lane = tid & 63;
  const int g = lane >> 4;
  const int i = lane & 15;
  const int slice0 = w * S;           // first column of this wave's slice
  const int c4s = slice0 / 4;         // first chunk of the slice

  // Z_i slice in B-operand layout
  const float* Z = Zw + (int64_t)it.part * z_stride;
  float zr[NQ][4];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int c = 0; c < 4; ++c) zr[q][c] = Z[(int64_t)(slice0 + 16 * q + 4 * g + c) * 16 + i];

  f4 acc[NQ];
#pragma unroll
  for (int h = 0; h < NQ; ++h) acc[h] = f4{0.f, 0.f, 0.f, 0.f};

  const float* Ab = A + it.row0 * lda;
  const int rows = (int)it.rows;
  // cooperative tile load: chunk e = j*NT + tid -> (row e / CPR, chunk e % CPR)
  auto load_tile = [&](f4 (&pre)[NL], int r0) {
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int e = j * NT + tid;
      const int r = e / CPR, c4 = e % CPR;
      if (r0 + r < rows)
        pre[j] = ldA<NTL>(Ab + (int64_t)(r0 + r) * lda + 4 * c4);
      else
        pre[j] = f4{0.f, 0.f, 0.f, 0.f};
    }
  };
  // One tile step: stage `pre` (the tile at rows r0..r0+15) in LDS, start the
  // load of the tile PF*16 rows ahead into `pre`, then run both products.
  auto step = [&](f4 (&pre)[NL], int r0) {
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int e = j * NT + tid;
      const int r = e / CPR, c4 = e % CPR;
      *(f4*)&tile[r * P + 4 * swz(c4)] = pre[j];
    }
    __syncthreads();
    if (r0 + PF * kTileRows < rows) load_tile(pre, r0 + PF * kTileRows);

    // all LDS operands of both products first, so the waits count down
    f4 a1[NQ], a2[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) a1[q] = *(const f4*)&tile[i * P + 4 * swz(c4s + 4 * q + g)];
#pragma unroll
    for (int st = 0; st < NQ; ++st) {
      const int s = st / (NQ / 4), cq = st % (NQ / 4);
      a2[st] = *(const f4*)&tile[(4 * g + s) * P + 4 * swz(c4s + (NQ / 4) * i + cq)];
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the whole read batch ahead of the MFMAs
    // product 1: partial t over this wave's slice (two independent chains)
    f4 tw0 = f4{0.f, 0.f, 0.f, 0.f}, tw1 = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      f4& tw = (q & 1) ? tw1 : tw0;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        tw = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[q][c], zr[q][c], tw, 0, 0, 0);
    }
    tpart[w][lane] = tw0 + tw1;
    __syncthreads();
    f4 t = tpart[0][lane];
#pragma unroll
    for (int v = 1; v < W; ++v) t += tpart[v][lane];

    // product 2: Y_slice += A_tile^T t
#pragma unroll
    for (int st = 0; st < NQ; ++st) {
      const int s = st / (NQ / 4), cq = st % (NQ / 4);
#pragma unroll
      for (int c = 0; c < 4; ++c)
        acc[4 * cq + c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[st][c], t[s], acc[4 * cq + c], 0, 0, 0);
    }
    __syncthreads();
  };

  if (PF == 1) {
    f4 pre0[NL];
    load_tile(pre0, 0);
    for (int r0 = 0; r0 < rows; r0 += kTileRows) step(pre0, r0);
  } else {
    f4 pre0[NL], pre1[NL];
    load_tile(pre0, 0);
    load_tile(pre1, kTileRows);
    for (int r0 = 0; r0 < rows; r0 += 2 * kTileRows) {
      step(pre0, r0);
      if (r0 + kTileRows < rows) step(pre1, r0 + kTileRows);
    }
  }
  // acc[h][r] = Y[slice0 + NQ*(4g + r) + h][i]
  float* o = part + (int64_t)it.slot * D * 16;
#pragma unroll
  for (int h = 0; h < NQ; ++h)
#pragma unroll
    for (int r = 0; r < 4; ++r) o[(int64_t)(slice0 + NQ * (4 * g + r) + h) * 16 + i] = acc[h][r];
}

// Software-pipelined form: two LDS tile buffers; in each step, product 2 of
// tile t and product 1 of tile t+1 are interleaved (independent matrix-core
// work from two tiles), with two barriers per tile.  One workgroup per CU.
template <int NQ, int W, bool NTL>
__global__ void __launch_bounds__(64 * W, 1)
k1_mfma_f32_k16_pipe(const float* __restrict__ A, int64_t lda, const float* __restrict__ Zw,
                     int64_t z_stride, const WorkItem* __restrict__ items,
                     float* __restrict__ part) {
  constexpr int NT = 64 * W;
  constexpr int D = 16 * NQ * W;
  constexpr int P = D + 4;
  constexpr int CPR = D / 4;
  constexpr int S = 16 * NQ;
  constexpr int NL = (kTileRows * CPR) / NT;
  __shared__ float tile[2][kTileRows * P];
  __shared__ f4 tpart[2][W][64];

  const WorkItem it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int lane = tid & 63;
  const int g = lane >> 4;
  const int i = lane & 15;
  const int slice0 = w * S;
  const int c4s = slice0 / 4;

  const float* Z = Zw + (int64_t)it.part * z_stride;
  float zr[NQ][4];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int c = 0; c < 4; ++c) zr[q][c] = Z[(int64_t)(slice0 + 16 * q + 4 * g + c) * 16 + i];
  f4 acc[NQ];
#pragma unroll
  for (int h = 0; h < NQ; ++h) acc[h] = f4{0.f, 0.f, 0.f, 0.f};

  const float* Ab = A + it.row0 * lda;
  const int rows = (int)it.rows;
  const int ntiles = (rows + kTileRows - 1) / kTileRows;
  f4 pre[NL];
  auto load_tile = [&](int tix) {
    const int r0 = tix * kTileRows;
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int e = j * NT + tid;
      const int r = e / CPR, c4 = e % CPR;
      if (r0 + r < rows)
        pre[j] = ldA<NTL>(Ab + (int64_t)(r0 + r) * lda + 4 * c4);
      else
        pre[j] = f4{0.f, 0.f, 0.f, 0.f};
    }
  };
  auto write_tile = [&](int b) {
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int e = j * NT + tid;
      const int r = e / CPR, c4 = e % CPR;
      *(f4*)&tile[b][r * P + 4 * swz(c4)] = pre[j];
    }
  };
  auto rd1 = [&](const float* tb, f4 (&a)[NQ]) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) a[q] = *(const f4*)&tb[i * P + 4 * swz(c4s + 4 * q + g)];
  };
  auto rd2 = [&](const float* tb, f4 (&a)[NQ]) {
#pragma unroll
    for (int st = 0; st < NQ; ++st) {
      const int s = st / (NQ / 4), cq = st % (NQ / 4);
      a[st] = *(const f4*)&tb[(4 * g + s) * P + 4 * swz(c4s + (NQ / 4) * i + cq)];
    }
  };
  auto p1 = [&](const f4 (&a)[NQ], int q, f4& tw) {
#pragma unroll
    for (int c = 0; c < 4; ++c) tw = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q][c], zr[q][c], tw, 0, 0, 0);
  };
  auto p2 = [&](const f4 (&a)[NQ], int st, const f4& t) {
    const int s = st / (NQ / 4), cq = st % (NQ / 4);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      acc[4 * cq + c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[st][c], t[s], acc[4 * cq + c], 0, 0, 0);
  };

  // prologue: tiles 0 and 1 staged, tile 2 in registers, product 1 of tile 0
  load_tile(0);
  write_tile(0);
  if (ntiles > 1) {
    load_tile(1);
    write_tile(1);
  }
  if (ntiles > 2) load_tile(2);
  __syncthreads();
  {
    f4 a1[NQ];
    rd1(tile[0], a1);
    f4 tw0 = f4{0.f, 0.f, 0.f, 0.f}, tw1 = tw0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) p1(a1, q, (q & 1) ? tw1 : tw0);
    tpart[0][w][lane] = tw0 + tw1;
  }
  for (int t = 0; t < ntiles; ++t) {
    __syncthreads();
    const float* cur = tile[t & 1];
    f4 a2[NQ];
    rd2(cur, a2);
    f4 tt = tpart[t & 1][0][lane];
#pragma unroll
    for (int v = 1; v < W; ++v) tt += tpart[t & 1][v][lane];
    if (t + 1 < ntiles) {
      f4 a1[NQ];
      rd1(tile[(t + 1) & 1], a1);
      __builtin_amdgcn_sched_barrier(0);  // keep the whole read batch ahead of the MFMAs
      f4 tw0 = f4{0.f, 0.f, 0.f, 0.f}, tw1 = tw0;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        p2(a2, q, tt);
        p1(a1, q, (q & 1) ? tw1 : tw0);
      }
      tpart[(t + 1) & 1][w][lane] = tw0 + tw1;
    } else {
#pragma unroll
      for (int q = 0; q < NQ; ++q) p2(a2, q, tt);
    }
    __syncthreads();
    if (t + 2 < ntiles) {
      write_tile(t & 1);
      if (t + 3 < ntiles) load_tile(t + 3);
    }
  }
  float* o = part + (int64_t)it.slot * D * 16;
#pragma unroll
  for (int h = 0; h < NQ; ++h)
#pragma unroll
    for (int r = 0; r < 4; ++r) o[(int64_t)(slice0 + NQ * (4 * g + r) + h) * 16 + i] = acc[h][r];
}

template <int NQ, int W, bool NT>
hipError_t launch_pipe_nq(int nitems, const float* a, int64_t lda, const float* z, int64_t z_stride,
                          const WorkItem* items, float* o, hipStream_t s) {
  if constexpr (16 * NQ * W <= 1024) {
    k1_mfma_f32_k16_pipe<NQ, W, NT><<<nitems, 64 * W, 0, s>>>(a, lda, z, z_stride, items, o);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int W, bool NT>
hipError_t launch_f32_pipe(int64_t d, int nitems, const float* a, int64_t lda, const float* z,
                           int64_t z_stride, const WorkItem* items, float* o, hipStream_t s) {
  switch (d / (16 * W)) {
    case 4: return launch_pipe_nq<4, W, NT>(nitems, a, lda, z, z_stride, items, o, s);
    case 8: return launch_pipe_nq<8, W, NT>(nitems, a, lda, z, z_stride, items, o, s);
    case 12: return launch_pipe_nq<12, W, NT>(nitems, a, lda, z, z_stride, items, o, s);
    case 16: return launch_pipe_nq<16, W, NT>(nitems, a, lda, z, z_stride, items, o, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace


template <int NQ, int W, int OCC, int PF, bool NT>
hipError_t launch_nq(int nitems, const float* a, int64_t lda, const float* z, int64_t z_stride,
                     const WorkItem* items, float* o, hipStream_t s) {
  if constexpr (16 * NQ * W <= 1024) {
    k1_mfma_f32_k16<NQ, W, OCC, PF, NT><<<nitems, 64 * W, 0, s>>>(a, lda, z, z_stride, items, o);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int W, int OCC, int PF, bool NT>
hipError_t launch_f32(int64_t d, int nitems, const float* a, int64_t lda, const float* z,
                      int64_t z_stride, const WorkItem* items, float* o, hipStream_t s) {
  switch (d / (16 * W)) {
    case 4: return launch_nq<4, W, OCC, PF, NT>(nitems, a, lda, z, z_stride, items, o, s);
    case 8: return launch_nq<8, W, OCC, PF, NT>(nitems, a, lda, z, z_stride, items, o, s);
    case 12: return launch_nq<12, W, OCC, PF, NT>(nitems, a, lda, z, z_stride, items, o, s);
    case 16: return launch_nq<16, W, OCC, PF, NT>(nitems, a, lda, z, z_stride, items, o, s);
    default: return hipErrorInvalidValue;
  }
}

bool mfma32_eligible(lp_dtype dtype, int64_t d, int64_t lda, int k) {
  return dtype == LP_F32 && k == 16 && (d == 256 || d == 512 || d == 768 || d == 1024) &&
         (lda % 4) == 0;
}

// Variants: 0: 4 waves, 1 WG/CU; 1: 8 waves, 1 WG/CU; 2: pipelined, 8 waves;
// 3: pipelined, 4 waves; 4: 8 waves with two tiles in flight.  The 8-wave forms need d in {512, 1024} (else 4 waves).
template <bool NT>
hipError_t dispatch_f32(const Plan& P, int nitems, const float* a, int64_t lda, const float* z,
                        int64_t z_stride, const WorkItem* items, float* o, hipStream_t s) {
  const bool w8 = P.d == 512 || P.d == 1024;
  switch (P.variant) {
    case 1:
      if (w8) return launch_f32<8, 1, 1, NT>(P.d, nitems, a, lda, z, z_stride, items, o, s);
      return launch_f32<4, 1, 1, NT>(P.d, nitems, a, lda, z, z_stride, items, o, s);
    case 2:
      if (w8) return launch_f32_pipe<8, NT>(P.d, nitems, a, lda, z, z_stride, items, o, s);
      return launch_f32_pipe<4, NT>(P.d, nitems, a, lda, z, z_stride, items, o, s);
    case 3: return launch_f32_pipe<4, NT>(P.d, nitems, a, lda, z, z_stride, items, o, s);
    case 4:
      if (w8) return launch_f32<8, 1, 2, NT>(P.d, nitems, a, lda, z, z_stride, items, o, s);
      return launch_f32<4, 1, 2, NT>(P.d, nitems, a, lda, z, z_stride, items, o, s);
    default: return launch_f32<4, 1, 1, NT>(P.d, nitems, a, lda, z, z_stride, items, o, s);
  }
}

hipError_t launch_local_multiply_mfma32(const Plan& P, const void* A, int64_t lda, int k,
                                        const void* Zw, int64_t z_stride, void* part,
                                        const WorkItem* items, hipStream_t s) {
  const int nitems = (int)P.items.size();
  const float* a = (const float*)A;
  const float* z = (const float*)Zw;
  float* o = (float*)part;
  if (P.nt_loads) return dispatch_f32<true>(P, nitems, a, lda, z, z_stride, items, o, s);
  return dispatch_f32<false>(P, nitems, a, lda, z, z_stride, items, o, s);
}

}  // namespace lp
