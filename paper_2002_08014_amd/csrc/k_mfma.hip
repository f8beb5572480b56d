// Fused single-pass local multiply on CDNA4 matrix cores (FP32 A, k <= 16: a
// rank below 16 runs the same 16-wide tiles with zero columns of Z_i, which
// are not stored).
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
                int64_t z_stride, const WorkItem* __restrict__ items, float* __restrict__ part, int kr) {
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
    for (int c = 0; c < 4; ++c) zr[q][c] = i < kr ? Z[(int64_t)(slice0 + 16 * q + 4 * g + c) * kr + i] : 0.f;

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
  float* o = part + (int64_t)it.slot * D * kr;
#pragma unroll
  for (int h = 0; h < NQ; ++h)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (i < kr) o[(int64_t)(slice0 + NQ * (4 * g + r) + h) * kr + i] = acc[h][r];
}

// Software-pipelined form: two LDS tile buffers; in each step, product 2 of
// tile t and product 1 of tile t+1 are interleaved (independent matrix-core
// work from two tiles), with two barriers per tile.  One workgroup per CU.
template <int NQ, int W, bool NTL>
__global__ void __launch_bounds__(64 * W, 1)
k1_mfma_f32_k16_pipe(const float* __restrict__ A, int64_t lda, const float* __restrict__ Zw,
                     int64_t z_stride, const WorkItem* __restrict__ items,
                     float* __restrict__ part, int kr) {
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
    for (int c = 0; c < 4; ++c) zr[q][c] = i < kr ? Z[(int64_t)(slice0 + 16 * q + 4 * g + c) * kr + i] : 0.f;
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
  float* o = part + (int64_t)it.slot * D * kr;
#pragma unroll
  for (int h = 0; h < NQ; ++h)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (i < kr) o[(int64_t)(slice0 + NQ * (4 * g + r) + h) * kr + i] = acc[h][r];
}

// Direct-to-LDS form: each wave copies its own column slice of every tile
// HBM -> LDS with global_load_lds_dwordx4 (no register staging, no barrier for
// the tile), two tile buffers per wave, explicit vmcnt waits.  Inside a wave
// row the 16-byte chunk c of tile row r sits at position
//   c ^ ((r ^ (c >> 4)) & 15)
// (the XOR stays inside the chunk's 256-byte group), which keeps the
// product-1 pattern (16 rows, one chunk) and the product-2 pattern (one row,
// chunks NQ/4 apart) free of bank conflicts.  Rows past the end of the item
// repeat the last row; their t is zeroed.  Operand layouts as in
// k1_mfma_f32_k16.  AUX: cache policy of the A loads (0, or 2 = nontemporal).
typedef __attribute__((address_space(3))) void lds_void;

__device__ inline int dpos(int r, int c) { return c ^ ((r ^ (c >> 4)) & 15); }

__device__ inline unsigned lds_addr(const void* p) {
  return (unsigned)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// Workgroup barrier for LDS data only: the LDS writes of this wave are complete
// (lgkmcnt), then s_barrier.  __syncthreads() would also wait for every
// outstanding global load, i.e. for the next tile's direct-to-LDS loads.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Four 128-bit LDS reads issued together and waited for inside the same asm
// block.  Reads of the tile buffers go through these so that the compiler,
// which cannot tell which buffer a pending direct-to-LDS load writes, does not
// wait for the next tile's loads before reading the current tile.
__device__ inline void lds_read4(f4& x0, f4& x1, f4& x2, f4& x3, unsigned a0, unsigned a1,
                                 unsigned a2, unsigned a3) {
  asm volatile(
      "ds_read_b128 %0, %4\n\t"
      "ds_read_b128 %1, %5\n\t"
      "ds_read_b128 %2, %6\n\t"
      "ds_read_b128 %3, %7\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(x0), "=&v"(x1), "=&v"(x2), "=&v"(x3)
      : "v"(a0), "v"(a1), "v"(a2), "v"(a3)
      : "memory");
}

// Wait for every outstanding global memory operation of this wave (the
// direct-to-LDS loads included); also a compiler barrier.
__device__ inline void wait_vm_all() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Wait until at most N global memory operations of this wave are outstanding
// (they complete in issue order).
template <int N>
__device__ inline void wait_vm_n() { asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory"); }

template <int NQ, int W, int AUX>
__global__ void __launch_bounds__(64 * W, 1)
k1_mfma_f32_dma(const float* __restrict__ A, int64_t lda, const float* __restrict__ Zw,
                int64_t z_stride, const WorkItem* __restrict__ items, float* __restrict__ part, int kr) {
  constexpr int D = 16 * NQ * W;
  constexpr int S = 16 * NQ;            // columns per wave slice
  constexpr int RB = 4 * S;             // bytes per slice row
  constexpr int TB = kTileRows * RB;    // bytes per wave tile
  constexpr int NI = TB / 1024;         // 1 KB direct-to-LDS loads per wave tile
  static_assert(NQ % 4 == 0 && TB % 1024 == 0, "slice rows must be whole 256-byte groups");
  __shared__ __attribute__((aligned(16))) unsigned char abuf[2][W][TB];
  __shared__ f4 tpart[W][64];

  const WorkItem it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int lane = tid & 63;
  const int g = lane >> 4;
  const int i = lane & 15;
  const int slice0 = w * S;
  const int rows = (int)it.rows;
  const int ntiles = (rows + kTileRows - 1) / kTileRows;
  const float* Ab = A + it.row0 * lda + slice0;

  // Per-lane element offsets of the NI 1 KB loads of a tile (tile row * lda +
  // column), fixed for the item; a full tile needs only the uniform tile base.
  int32_t loff[NI];
#pragma unroll
  for (int ii = 0; ii < NI; ++ii) {
    const int byte = ii * 1024 + 16 * lane;
    const int r = byte / RB;
    const int p = (byte % RB) / 16;
    loff[ii] = r * (int32_t)lda + 4 * (p ^ ((r ^ (p >> 4)) & 15));   // the chunk stored at position p
  }
  auto issue = [&](int r0, int b) {
    if (r0 + kTileRows <= rows) {
      const float* base = Ab + (int64_t)r0 * lda;
#pragma unroll
      for (int ii = 0; ii < NI; ++ii)
        __builtin_amdgcn_global_load_lds((const void*)(base + loff[ii]),
                                         (lds_void*)&abuf[b][w][ii * 1024], 16, 0, AUX);
    } else {
#pragma unroll
      for (int ii = 0; ii < NI; ++ii) {
        const int byte = ii * 1024 + 16 * lane;
        const int r = byte / RB;
        const int p = (byte % RB) / 16;
        const int row = min(r0 + r, rows - 1);
        const float* src = Ab + (int64_t)row * lda + 4 * (p ^ ((r ^ (p >> 4)) & 15));
        __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)&abuf[b][w][ii * 1024], 16, 0,
                                         AUX);
      }
    }
  };
  issue(0, 0);

  const float* Z = Zw + (int64_t)it.part * z_stride;
  float zr[NQ][4];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int c = 0; c < 4; ++c) zr[q][c] = i < kr ? Z[(int64_t)(slice0 + 16 * q + 4 * g + c) * kr + i] : 0.f;
  f4 acc[NQ];
#pragma unroll
  for (int h = 0; h < NQ; ++h) acc[h] = f4{0.f, 0.f, 0.f, 0.f};

  for (int j = 0; j < ntiles; ++j) {
    const int b = j & 1;
    // tile j was issued one iteration ago: wait for it (a full wait, so no other
    // memory operation the compiler placed in between can satisfy the count),
    // then start tile j + 1 into the other buffer; it lands while tile j computes
    wait_vm_all();
    if (j + 1 < ntiles) issue((j + 1) * kTileRows, b ^ 1);
    const unsigned tb = lds_addr(&abuf[b][w][0]);
    unsigned ad1[NQ], ad2[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) ad1[q] = tb + i * RB + 16 * dpos(i, 4 * q + g);
#pragma unroll
    for (int st = 0; st < NQ; ++st) {
      const int s = st / (NQ / 4), cq = st % (NQ / 4);
      const int r = 4 * g + s;
      ad2[st] = tb + r * RB + 16 * dpos(r, (NQ / 4) * i + cq);
    }
    f4 a1[NQ], a2[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q += 4)
      lds_read4(a1[q], a1[q + 1], a1[q + 2], a1[q + 3], ad1[q], ad1[q + 1], ad1[q + 2], ad1[q + 3]);
#pragma unroll
    for (int q = 0; q < NQ; q += 4)
      lds_read4(a2[q], a2[q + 1], a2[q + 2], a2[q + 3], ad2[q], ad2[q + 1], ad2[q + 2], ad2[q + 3]);
    f4 tw0 = f4{0.f, 0.f, 0.f, 0.f}, tw1 = tw0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      f4& tw = (q & 1) ? tw1 : tw0;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        tw = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[q][c], zr[q][c], tw, 0, 0, 0);
    }
    tpart[w][lane] = tw0 + tw1;
    lds_barrier();
    f4 t = tpart[0][lane];
#pragma unroll
    for (int v = 1; v < W; ++v) t += tpart[v][lane];
    const int valid = rows - j * kTileRows;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (4 * g + r >= valid) t[r] = 0.f;
#pragma unroll
    for (int st = 0; st < NQ; ++st) {
      const int s = st / (NQ / 4), cq = st % (NQ / 4);
#pragma unroll
      for (int c = 0; c < 4; ++c)
        acc[4 * cq + c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[st][c], t[s], acc[4 * cq + c], 0, 0, 0);
    }
    lds_barrier();   // every wave has read tpart before the next tile overwrites it
  }
  float* o = part + (int64_t)it.slot * D * kr;
#pragma unroll
  for (int h = 0; h < NQ; ++h)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (i < kr) o[(int64_t)(slice0 + NQ * (4 * g + r) + h) * kr + i] = acc[h][r];
}

// Software-pipelined direct-to-LDS form.  Per tile j: the operands of both
// products are read from the tile buffer while no tile load is in flight (plain
// LDS loads, waited for at first use), product 2 of tile j - 1 runs on the
// operands and t kept in registers from the previous step while those reads
// land, then the load of tile j + 1 starts and product 1 of tile j follows; the
// per-wave t partials go through a double-buffered LDS array, so one block
// barrier per tile suffices (a wave overwrites a t buffer only after the
// barrier that every wave reaches after reading it).
template <int NQ, int W, int AUX>
__global__ void __launch_bounds__(64 * W, 1)
k1_mfma_f32_dmap(const float* __restrict__ A, int64_t lda, const float* __restrict__ Zw,
                 int64_t z_stride, const WorkItem* __restrict__ items, float* __restrict__ part, int kr) {
  constexpr int D = 16 * NQ * W;
  constexpr int S = 16 * NQ;            // columns per wave slice
  constexpr int RB = 4 * S;             // bytes per slice row
  constexpr int TB = kTileRows * RB;    // bytes per wave tile
  constexpr int NI = TB / 1024;         // 1 KB direct-to-LDS loads per wave tile
  static_assert(NQ % 4 == 0 && TB % 1024 == 0, "slice rows must be whole 256-byte groups");
  __shared__ __attribute__((aligned(16))) unsigned char abuf[2][W][TB];
  __shared__ f4 tpart[2][W][64];

  const WorkItem it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int lane = tid & 63;
  const int g = lane >> 4;
  const int i = lane & 15;
  const int slice0 = w * S;
  const int rows = (int)it.rows;
  const int ntiles = (rows + kTileRows - 1) / kTileRows;
  const float* Ab = A + it.row0 * lda + slice0;

  int32_t loff[NI];
#pragma unroll
  for (int ii = 0; ii < NI; ++ii) {
    const int byte = ii * 1024 + 16 * lane;
    const int r = byte / RB;
    const int p = (byte % RB) / 16;
    loff[ii] = r * (int32_t)lda + 4 * (p ^ ((r ^ (p >> 4)) & 15));
  }
  auto issue = [&](int r0, int b) {
    if (r0 + kTileRows <= rows) {
      const float* base = Ab + (int64_t)r0 * lda;
#pragma unroll
      for (int ii = 0; ii < NI; ++ii)
        __builtin_amdgcn_global_load_lds((const void*)(base + loff[ii]),
                                         (lds_void*)&abuf[b][w][ii * 1024], 16, 0, AUX);
    } else {
#pragma unroll
      for (int ii = 0; ii < NI; ++ii) {
        const int byte = ii * 1024 + 16 * lane;
        const int r = byte / RB;
        const int p = (byte % RB) / 16;
        const int row = min(r0 + r, rows - 1);
        const float* src = Ab + (int64_t)row * lda + 4 * (p ^ ((r ^ (p >> 4)) & 15));
        __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)&abuf[b][w][ii * 1024], 16, 0,
                                         AUX);
      }
    }
  };
  issue(0, 0);

  const float* Z = Zw + (int64_t)it.part * z_stride;
  float zr[NQ][4];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int c = 0; c < 4; ++c) zr[q][c] = i < kr ? Z[(int64_t)(slice0 + 16 * q + 4 * g + c) * kr + i] : 0.f;
  f4 acc[NQ];
#pragma unroll
  for (int h = 0; h < NQ; ++h) acc[h] = f4{0.f, 0.f, 0.f, 0.f};

  // product 2 of a tile: acc += A_tile^T t (operands a2, t as in k1_mfma_f32_dma)
  auto product2 = [&](const f4 (&a2)[NQ], const f4& t, int st0, int st1) {
#pragma unroll
    for (int st = st0; st < st1; ++st) {
      const int s = st / (NQ / 4), cq = st % (NQ / 4);
#pragma unroll
      for (int c = 0; c < 4; ++c)
        acc[4 * cq + c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[st][c], t[s], acc[4 * cq + c], 0, 0, 0);
    }
  };

  f4 a2p[NQ];
  f4 tprev = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < NQ; ++q) a2p[q] = tprev;
  for (int j = 0; j < ntiles; ++j) {
    const int b = j & 1;
    wait_vm_all();   // tile j has landed; no tile load is in flight now
    const unsigned char* tbp = &abuf[b][w][0];
    f4 a1[NQ], a2[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) a1[q] = *(const f4*)(tbp + i * RB + 16 * dpos(i, 4 * q + g));
#pragma unroll
    for (int st = 0; st < NQ; ++st) {
      const int s = st / (NQ / 4), cq = st % (NQ / 4);
      const int r = 4 * g + s;
      a2[st] = *(const f4*)(tbp + r * RB + 16 * dpos(r, (NQ / 4) * i + cq));
    }
    __builtin_amdgcn_sched_barrier(0);
    // product 2 of the previous tile (zero operands at j = 0) while the reads land
    product2(a2p, tprev, 0, NQ / 2);
    __builtin_amdgcn_sched_barrier(0);
    if (j + 1 < ntiles) issue((j + 1) * kTileRows, b ^ 1);
    __builtin_amdgcn_sched_barrier(0);
    product2(a2p, tprev, NQ / 2, NQ);
    // product 1 of this tile: four accumulation chains
    f4 tw[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) tw[u] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        tw[(2 * q + (c >> 1)) & 3] =
            __builtin_amdgcn_mfma_f32_16x16x4f32(a1[q][c], zr[q][c], tw[(2 * q + (c >> 1)) & 3], 0, 0, 0);
    tpart[b][w][lane] = (tw[0] + tw[1]) + (tw[2] + tw[3]);
    lds_barrier();
    // the W partials (asm reads: the compiler would otherwise wait for the tile
    // load just issued before reading LDS)
    static_assert(W % 4 == 0, "t partials are read four at a time");
    f4 tv[W];
    const unsigned tp0 = lds_addr(&tpart[b][0][lane]);
#pragma unroll
    for (int v = 0; v < W; v += 4)
      lds_read4(tv[v], tv[v + 1], tv[v + 2], tv[v + 3], tp0 + 1024 * v, tp0 + 1024 * (v + 1),
                tp0 + 1024 * (v + 2), tp0 + 1024 * (v + 3));
    f4 t = tv[0];
#pragma unroll
    for (int v = 1; v < W; ++v) t += tv[v];
    const int valid = rows - j * kTileRows;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (4 * g + r >= valid) t[r] = 0.f;
#pragma unroll
    for (int q = 0; q < NQ; ++q) a2p[q] = a2[q];
    tprev = t;
  }
  product2(a2p, tprev, 0, NQ);
  float* o = part + (int64_t)it.slot * D * kr;
#pragma unroll
  for (int h = 0; h < NQ; ++h)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (i < kr) o[(int64_t)(slice0 + NQ * (4 * g + r) + h) * kr + i] = acc[h][r];
}

// Direct-to-LDS form with two tiles in flight per wave.  Once a tile's
// operands of both products are in registers (asm reads that wait inside),
// its buffer is refilled with the tile two ahead, so the other buffer's load
// and this one overlap: twice the bytes in flight of the other forms at the
// same LDS size.  Measured without any matrix-core work, the one-tile-ahead
// forms take as long as their loads' latency allows at 64 KB in flight per CU.
template <int NQ, int W, int AUX>
__global__ void __launch_bounds__(64 * W, 1)
k1_mfma_f32_dma2(const float* __restrict__ A, int64_t lda, const float* __restrict__ Zw,
                 int64_t z_stride, const WorkItem* __restrict__ items, float* __restrict__ part, int kr) {
  constexpr int D = 16 * NQ * W;
  constexpr int S = 16 * NQ;            // columns per wave slice
  constexpr int RB = 4 * S;             // bytes per slice row
  constexpr int TB = kTileRows * RB;    // bytes per wave tile
  constexpr int NI = TB / 1024;         // 1 KB direct-to-LDS loads per wave tile
  static_assert(NQ % 4 == 0 && TB % 1024 == 0, "slice rows must be whole 256-byte groups");
  __shared__ __attribute__((aligned(16))) unsigned char abuf[2][W][TB];
  __shared__ f4 tpart[2][W][64];

  const WorkItem it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int lane = tid & 63;
  const int g = lane >> 4;
  const int i = lane & 15;
  const int slice0 = w * S;
  const int rows = (int)it.rows;
  const int ntiles = (rows + kTileRows - 1) / kTileRows;
  const float* Ab = A + it.row0 * lda + slice0;

  int32_t loff[NI];
#pragma unroll
  for (int ii = 0; ii < NI; ++ii) {
    const int byte = ii * 1024 + 16 * lane;
    const int r = byte / RB;
    const int p = (byte % RB) / 16;
    loff[ii] = r * (int32_t)lda + 4 * (p ^ ((r ^ (p >> 4)) & 15));
  }
  auto issue = [&](int r0, int b) {
    if (r0 + kTileRows <= rows) {
      const float* base = Ab + (int64_t)r0 * lda;
#pragma unroll
      for (int ii = 0; ii < NI; ++ii)
        __builtin_amdgcn_global_load_lds((const void*)(base + loff[ii]),
                                         (lds_void*)&abuf[b][w][ii * 1024], 16, 0, AUX);
    } else {
#pragma unroll
      for (int ii = 0; ii < NI; ++ii) {
        const int byte = ii * 1024 + 16 * lane;
        const int r = byte / RB;
        const int p = (byte % RB) / 16;
        const int row = min(r0 + r, rows - 1);
        const float* src = Ab + (int64_t)row * lda + 4 * (p ^ ((r ^ (p >> 4)) & 15));
        __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)&abuf[b][w][ii * 1024], 16, 0,
                                         AUX);
      }
    }
  };

  const float* Z = Zw + (int64_t)it.part * z_stride;
  float zr[NQ][4];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int c = 0; c < 4; ++c) zr[q][c] = i < kr ? Z[(int64_t)(slice0 + 16 * q + 4 * g + c) * kr + i] : 0.f;
  f4 acc[NQ];
#pragma unroll
  for (int h = 0; h < NQ; ++h) acc[h] = f4{0.f, 0.f, 0.f, 0.f};
  // the Z loads were issued first, so the in-order count below covers them too
  issue(0, 0);
  if (ntiles > 1) issue(kTileRows, 1);

  for (int j = 0; j < ntiles; ++j) {
    const int b = j & 1;
    // tile j complete; tile j + 1 (issued after it) may still be in flight
    if (j + 1 < ntiles)
      wait_vm_n<NI>();
    else
      wait_vm_all();
    const unsigned tb = lds_addr(&abuf[b][w][0]);
    unsigned ad1[NQ], ad2[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) ad1[q] = tb + i * RB + 16 * dpos(i, 4 * q + g);
#pragma unroll
    for (int st = 0; st < NQ; ++st) {
      const int s = st / (NQ / 4), cq = st % (NQ / 4);
      const int r = 4 * g + s;
      ad2[st] = tb + r * RB + 16 * dpos(r, (NQ / 4) * i + cq);
    }
    f4 a1[NQ], a2[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q += 4)
      lds_read4(a1[q], a1[q + 1], a1[q + 2], a1[q + 3], ad1[q], ad1[q + 1], ad1[q + 2], ad1[q + 3]);
#pragma unroll
    for (int q = 0; q < NQ; q += 4)
      lds_read4(a2[q], a2[q + 1], a2[q + 2], a2[q + 3], ad2[q], ad2[q + 1], ad2[q + 2], ad2[q + 3]);
    // this wave's part of buffer b is in registers: refill it with tile j + 2
    if (j + 2 < ntiles) issue((j + 2) * kTileRows, b);
    f4 tw[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) tw[u] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        tw[(2 * q + (c >> 1)) & 3] =
            __builtin_amdgcn_mfma_f32_16x16x4f32(a1[q][c], zr[q][c], tw[(2 * q + (c >> 1)) & 3], 0, 0, 0);
    tpart[b][w][lane] = (tw[0] + tw[1]) + (tw[2] + tw[3]);
    lds_barrier();
    static_assert(W % 4 == 0, "t partials are read four at a time");
    f4 tv[W];
    const unsigned tp0 = lds_addr(&tpart[b][0][lane]);
#pragma unroll
    for (int v = 0; v < W; v += 4)
      lds_read4(tv[v], tv[v + 1], tv[v + 2], tv[v + 3], tp0 + 1024 * v, tp0 + 1024 * (v + 1),
                tp0 + 1024 * (v + 2), tp0 + 1024 * (v + 3));
    f4 t = tv[0];
#pragma unroll
    for (int v = 1; v < W; ++v) t += tv[v];
    const int valid = rows - j * kTileRows;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (4 * g + r >= valid) t[r] = 0.f;
#pragma unroll
    for (int st = 0; st < NQ; ++st) {
      const int s = st / (NQ / 4), cq = st % (NQ / 4);
#pragma unroll
      for (int c = 0; c < 4; ++c)
        acc[4 * cq + c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[st][c], t[s], acc[4 * cq + c], 0, 0, 0);
    }
  }
  float* o = part + (int64_t)it.slot * D * kr;
#pragma unroll
  for (int h = 0; h < NQ; ++h)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (i < kr) o[(int64_t)(slice0 + NQ * (4 * g + r) + h) * kr + i] = acc[h][r];
}

template <int NQ, int W, int AUX>
hipError_t launch_dma2_nq(int nitems, const float* a, int64_t lda, const float* z, int64_t z_stride,
                          const WorkItem* items, float* o, int kr, hipStream_t s) {
  if constexpr (16 * NQ * W <= 1024 && NQ % 4 == 0) {
    k1_mfma_f32_dma2<NQ, W, AUX><<<nitems, 64 * W, 0, s>>>(a, lda, z, z_stride, items, o, kr);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int W, int AUX>
hipError_t launch_f32_dma2(int64_t d, int nitems, const float* a, int64_t lda, const float* z,
                           int64_t z_stride, const WorkItem* items, float* o, int kr, hipStream_t s) {
  switch (d / (16 * W)) {
    case 4: return launch_dma2_nq<4, W, AUX>(nitems, a, lda, z, z_stride, items, o, kr, s);
    case 8: return launch_dma2_nq<8, W, AUX>(nitems, a, lda, z, z_stride, items, o, kr, s);
    case 12: return launch_dma2_nq<12, W, AUX>(nitems, a, lda, z, z_stride, items, o, kr, s);
    case 16: return launch_dma2_nq<16, W, AUX>(nitems, a, lda, z, z_stride, items, o, kr, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NQ, int W, int AUX>
hipError_t launch_dmap_nq(int nitems, const float* a, int64_t lda, const float* z, int64_t z_stride,
                          const WorkItem* items, float* o, int kr, hipStream_t s) {
  if constexpr (16 * NQ * W <= 1024 && NQ % 4 == 0 && NQ <= 8) {
    k1_mfma_f32_dmap<NQ, W, AUX><<<nitems, 64 * W, 0, s>>>(a, lda, z, z_stride, items, o, kr);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int W, int AUX>
hipError_t launch_f32_dmap(int64_t d, int nitems, const float* a, int64_t lda, const float* z,
                           int64_t z_stride, const WorkItem* items, float* o, int kr, hipStream_t s) {
  switch (d / (16 * W)) {
    case 4: return launch_dmap_nq<4, W, AUX>(nitems, a, lda, z, z_stride, items, o, kr, s);
    case 8: return launch_dmap_nq<8, W, AUX>(nitems, a, lda, z, z_stride, items, o, kr, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NQ, int W, int AUX>
hipError_t launch_dma_nq(int nitems, const float* a, int64_t lda, const float* z, int64_t z_stride,
                         const WorkItem* items, float* o, int kr, hipStream_t s) {
  if constexpr (16 * NQ * W <= 1024 && NQ % 4 == 0) {
    k1_mfma_f32_dma<NQ, W, AUX><<<nitems, 64 * W, 0, s>>>(a, lda, z, z_stride, items, o, kr);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int W, int AUX>
hipError_t launch_f32_dma(int64_t d, int nitems, const float* a, int64_t lda, const float* z,
                          int64_t z_stride, const WorkItem* items, float* o, int kr, hipStream_t s) {
  switch (d / (16 * W)) {
    case 4: return launch_dma_nq<4, W, AUX>(nitems, a, lda, z, z_stride, items, o, kr, s);
    case 8: return launch_dma_nq<8, W, AUX>(nitems, a, lda, z, z_stride, items, o, kr, s);
    case 12: return launch_dma_nq<12, W, AUX>(nitems, a, lda, z, z_stride, items, o, kr, s);
    case 16: return launch_dma_nq<16, W, AUX>(nitems, a, lda, z, z_stride, items, o, kr, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NQ, int W, bool NT>
hipError_t launch_pipe_nq(int nitems, const float* a, int64_t lda, const float* z, int64_t z_stride,
                          const WorkItem* items, float* o, int kr, hipStream_t s) {
  if constexpr (16 * NQ * W <= 1024) {
    k1_mfma_f32_k16_pipe<NQ, W, NT><<<nitems, 64 * W, 0, s>>>(a, lda, z, z_stride, items, o, kr);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int W, bool NT>
hipError_t launch_f32_pipe(int64_t d, int nitems, const float* a, int64_t lda, const float* z,
                           int64_t z_stride, const WorkItem* items, float* o, int kr, hipStream_t s) {
  switch (d / (16 * W)) {
    case 4: return launch_pipe_nq<4, W, NT>(nitems, a, lda, z, z_stride, items, o, kr, s);
    case 8: return launch_pipe_nq<8, W, NT>(nitems, a, lda, z, z_stride, items, o, kr, s);
    case 12: return launch_pipe_nq<12, W, NT>(nitems, a, lda, z, z_stride, items, o, kr, s);
    case 16: return launch_pipe_nq<16, W, NT>(nitems, a, lda, z, z_stride, items, o, kr, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace


template <int NQ, int W, int OCC, int PF, bool NT>
hipError_t launch_nq(int nitems, const float* a, int64_t lda, const float* z, int64_t z_stride,
                     const WorkItem* items, float* o, int kr, hipStream_t s) {
  if constexpr (16 * NQ * W <= 1024) {
    k1_mfma_f32_k16<NQ, W, OCC, PF, NT><<<nitems, 64 * W, 0, s>>>(a, lda, z, z_stride, items, o, kr);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int W, int OCC, int PF, bool NT>
hipError_t launch_f32(int64_t d, int nitems, const float* a, int64_t lda, const float* z,
                      int64_t z_stride, const WorkItem* items, float* o, int kr, hipStream_t s) {
  switch (d / (16 * W)) {
    case 4: return launch_nq<4, W, OCC, PF, NT>(nitems, a, lda, z, z_stride, items, o, kr, s);
    case 8: return launch_nq<8, W, OCC, PF, NT>(nitems, a, lda, z, z_stride, items, o, kr, s);
    case 12: return launch_nq<12, W, OCC, PF, NT>(nitems, a, lda, z, z_stride, items, o, kr, s);
    case 16: return launch_nq<16, W, OCC, PF, NT>(nitems, a, lda, z, z_stride, items, o, kr, s);
    default: return hipErrorInvalidValue;
  }
}

bool mfma32_eligible(lp_dtype dtype, int64_t d, int64_t lda, int k) {
  // ranks below 16 run the k = 16 tiles with zero columns of Z (not stored)
  return dtype == LP_F32 && k >= 1 && k <= 16 && (d == 256 || d == 512 || d == 768 || d == 1024) &&
         (lda % 4) == 0 && lda <= (int64_t(1) << 26);   // 32-bit in-tile load offsets
}

// Variants: 0: 4 waves, 1 WG/CU; 1: 8 waves, 1 WG/CU; 2: pipelined, 8 waves;
// 3: pipelined, 4 waves; 4: 8 waves with two tiles in flight; 5: direct-to-LDS tile
// loads (8 waves at d = 1024, else 4); 6: direct-to-LDS, 4 waves; 7: direct-to-LDS,
// software-pipelined (8 waves at d = 1024, else 4); 8: direct-to-LDS with two tiles in
// flight per wave (8 waves at d = 1024, else 4).  The 8-wave forms need d in {512, 1024} (else 4 waves).
template <bool NT>
hipError_t dispatch_f32(const Plan& P, int nitems, const float* a, int64_t lda, const float* z,
                        int64_t z_stride, const WorkItem* items, float* o, int kr, hipStream_t s) {
  const bool w8 = P.d == 512 || P.d == 1024;
  switch (P.variant) {
    case 1:
      if (w8) return launch_f32<8, 1, 1, NT>(P.d, nitems, a, lda, z, z_stride, items, o, kr, s);
      return launch_f32<4, 1, 1, NT>(P.d, nitems, a, lda, z, z_stride, items, o, kr, s);
    case 2:
      if (w8) return launch_f32_pipe<8, NT>(P.d, nitems, a, lda, z, z_stride, items, o, kr, s);
      return launch_f32_pipe<4, NT>(P.d, nitems, a, lda, z, z_stride, items, o, kr, s);
    case 3: return launch_f32_pipe<4, NT>(P.d, nitems, a, lda, z, z_stride, items, o, kr, s);
    case 4:
      if (w8) return launch_f32<8, 1, 2, NT>(P.d, nitems, a, lda, z, z_stride, items, o, kr, s);
      return launch_f32<4, 1, 2, NT>(P.d, nitems, a, lda, z, z_stride, items, o, kr, s);
    case 5: {
      // direct-to-LDS form: 8 waves when the slice is a whole number of 256-byte
      // groups (d = 512 gives 64-column slices: 4 waves), else 4 waves
      constexpr int AUX = NT ? 2 : 0;
      if (P.d == 1024) return launch_f32_dma<8, AUX>(P.d, nitems, a, lda, z, z_stride, items, o, kr, s);
      return launch_f32_dma<4, AUX>(P.d, nitems, a, lda, z, z_stride, items, o, kr, s);
    }
    case 6: {
      // direct-to-LDS form with four waves (one per SIMD, 512 registers each)
      constexpr int AUX = NT ? 2 : 0;
      return launch_f32_dma<4, AUX>(P.d, nitems, a, lda, z, z_stride, items, o, kr, s);
    }
    case 7: {
      // software-pipelined direct-to-LDS form with 64- or 128-column slices (eight
      // waves at d = 1024, four at d = 256 and 512); the plain form at d = 768
      constexpr int AUX = NT ? 2 : 0;
      if (P.d == 1024) return launch_f32_dmap<8, AUX>(P.d, nitems, a, lda, z, z_stride, items, o, kr, s);
      if (P.d == 256 || P.d == 512)
        return launch_f32_dmap<4, AUX>(P.d, nitems, a, lda, z, z_stride, items, o, kr, s);
      return launch_f32_dma<4, AUX>(P.d, nitems, a, lda, z, z_stride, items, o, kr, s);
    }
    case 8: {
      // direct-to-LDS with two tiles in flight per wave (8 waves at d = 1024, else 4)
      constexpr int AUX = NT ? 2 : 0;
      if (P.d == 1024) return launch_f32_dma2<8, AUX>(P.d, nitems, a, lda, z, z_stride, items, o, kr, s);
      return launch_f32_dma2<4, AUX>(P.d, nitems, a, lda, z, z_stride, items, o, kr, s);
    }
    default: return launch_f32<4, 1, 1, NT>(P.d, nitems, a, lda, z, z_stride, items, o, kr, s);
  }
}

hipError_t launch_local_multiply_mfma32(const Plan& P, const void* A, int64_t lda, int k,
                                        const void* Zw, int64_t z_stride, void* part,
                                        const WorkItem* items, int nitems,
                                        hipStream_t s) {
  const float* a = (const float*)A;
  const float* z = (const float*)Zw;
  float* o = (float*)part;
  if (P.nt_loads) return dispatch_f32<true>(P, nitems, a, lda, z, z_stride, items, o, k, s);
  return dispatch_f32<false>(P, nitems, a, lda, z, z_stride, items, o, k, s);
}

}  // namespace lp
