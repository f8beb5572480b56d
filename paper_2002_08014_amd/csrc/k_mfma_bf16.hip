// Fused single-pass local multiply on CDNA4 matrix cores for BF16 A
// (k <= 32, d in {512, 1024, 1536, 2048}; a rank below 16, or between 16 and
// 32, runs the 16- or 32-wide tiles with zero columns of Z_i, not stored).
//
// Computes, for one work item (a contiguous row range of partition i),
//   part = A_rows^T bf16(A_rows bf16(Z_i))      (Eq. (power_yi) without 1/s_i)
// reading every element of A once from HBM.  Both products run on BF16
// matrix-core instructions with FP32 accumulation; Z_i and the intermediate
// t = A_rows Z_i are rounded to BF16 (round to nearest even) as operands.
// With SPLIT each operand is a pair hi = bf16(x), lo = bf16(x - hi) and every
// product is taken twice (A hi + A lo; A is exact in BF16), so the operands
// carry about 16 significant bits instead of 8: twice the matrix-core work for
// FP32-class results (the single rounding leaves a sin theta floor near 1e-3).
//
// Layout: W waves (4 or 8), wave w owns the column slice [w*d/W, (w+1)*d/W) of
// every 16-row tile; NC = d/(32 W) 32-column chunks per slice.
//   * A tiles are copied HBM -> LDS by direct-to-LDS loads (no registers), two
//     tile buffers per wave; each wave reads only its own slice, so the only
//     cross-wave traffic is the t reduction.  LDS row r of a wave tile holds
//     the slice's 16-byte chunks XOR-swizzled by s(r) = (2r + r/8) mod 16,
//     which keeps both read patterns below free of bank conflicts.
//   * product 1 (v_mfma_f32_16x16x32_bf16, per chunk c and 16-wide k block):
//     M = tile row (lane%16), K = 8 consecutive columns 32c + 8(lane/16) + e,
//     read as one 128-bit LDS load per lane; Z_i sits in registers in the
//     matching B-operand layout for the whole work item.
//   * the W per-slice partial t's (FP32) are summed through LDS in a fixed
//     order, rounded to BF16 and stored as t^T (k-major), so each lane's
//     product-2 B operand is one 64-bit LDS load.
//   * product 2 (v_mfma_f32_16x16x16_bf16, per 16-column block): the A operand
//     is the transposed tile block, read with ds_read_b64_tr_b16 (lane
//     16g + 4f + q loads 4 columns of row 4g + f; the transpose hands lane
//     16g + i column i of rows 4g..4g+3), K = tile rows; the Y partial for
//     the slice lives in accumulators for the whole work item.
#include "lp_internal.h"

namespace lp {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

constexpr int kRows = 16;   // tile rows

__device__ inline int bswz(int r) { return (2 * r + (r >> 3)) & 15; }

__device__ inline uint16_t bf16_bits(float x) {
  __bf16 h = (__bf16)x;   // round to nearest even
  return __builtin_bit_cast(uint16_t, h);
}

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ inline unsigned lds_addr(const void* p) {
  return (unsigned)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// Workgroup barrier for LDS data only: the LDS writes of this wave are complete
// (lgkmcnt), then s_barrier.  __syncthreads() would also wait for every
// outstanding global load, i.e. for the next tile's direct-to-LDS loads.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Tile-buffer reads, issued together and waited for inside the same asm block:
// the compiler cannot tell which buffer a pending direct-to-LDS load writes and
// would otherwise wait for the next tile's loads before reading this one.
__device__ inline void lds_read4_b128(bf8& x0, bf8& x1, bf8& x2, bf8& x3, unsigned a0, unsigned a1,
                                      unsigned a2, unsigned a3) {
  f4v y0, y1, y2, y3;
  asm volatile(
      "ds_read_b128 %0, %4\n\t"
      "ds_read_b128 %1, %5\n\t"
      "ds_read_b128 %2, %6\n\t"
      "ds_read_b128 %3, %7\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(y0), "=&v"(y1), "=&v"(y2), "=&v"(y3)
      : "v"(a0), "v"(a1), "v"(a2), "v"(a3)
      : "memory");
  x0 = __builtin_bit_cast(bf8, y0);
  x1 = __builtin_bit_cast(bf8, y1);
  x2 = __builtin_bit_cast(bf8, y2);
  x3 = __builtin_bit_cast(bf8, y3);
}

// Four transposing 64-bit reads (ds_read_b64_tr_b16, semantics in the header).
__device__ inline void lds_read4_tr(s4& x0, s4& x1, s4& x2, s4& x3, unsigned a0, unsigned a1,
                                    unsigned a2, unsigned a3) {
  asm volatile(
      "ds_read_b64_tr_b16 %0, %4\n\t"
      "ds_read_b64_tr_b16 %1, %5\n\t"
      "ds_read_b64_tr_b16 %2, %6\n\t"
      "ds_read_b64_tr_b16 %3, %7\n\t"
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

// W: waves; NC: 32-column chunks per wave slice (d = 32 NC W); KT: 16-wide k
// blocks (k = 16 KT); AUX: cache policy of the A loads (0 default, 2 nontemporal);
// AHEAD: two tiles in flight per wave (a buffer is refilled with the tile two
// ahead as soon as this wave's last read of it is done) instead of one.
template <int W, int NC, int KT, int AUX, bool AHEAD, bool SPLIT, bool FULL>
__global__ void __launch_bounds__(64 * W, 1)
k1_mfma_bf16(const uint16_t* __restrict__ A, int64_t lda, const float* __restrict__ Zw,
             int64_t z_stride, const WorkItem* __restrict__ items, float* __restrict__ part, int kr_in) {
  constexpr int K = 16 * KT;
  // FULL: the rank is the tile width (a compile-time stride and no column tests:
  // at d = 2048, k = 32 the register file is full and a run-time rank spills)
  const int kr = FULL ? K : kr_in;
  constexpr int CW = 32 * NC;        // columns per wave slice
  constexpr int RB = 2 * CW;         // bytes of one slice row
  constexpr int TB = kRows * RB;     // bytes of one wave tile
  constexpr int NI = TB / 1024;      // direct-to-LDS loads (1 KB each) per wave tile
  constexpr int NCT = 2 * NC;        // 16-column blocks per slice
  constexpr int D = W * CW;
  static_assert(NC % 4 == 0 && TB % 1024 == 0, "slice must be a whole number of 256-byte groups");
  __shared__ __attribute__((aligned(16))) unsigned char abuf[2][W][TB];
  __shared__ f4 tpart[W][KT][64];
  __shared__ __attribute__((aligned(16))) uint16_t tbf[SPLIT ? 2 : 1][K * kRows];   // t^T, k-major

  const WorkItem it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int lane = tid & 63;
  const int g = lane >> 4;
  const int i = lane & 15;
  const int slice0 = w * CW;
  const int rows = (int)it.rows;
  const int ntiles = (rows + kRows - 1) / kRows;
  const uint16_t* Ab = A + it.row0 * lda + slice0;

  // Rows past the end of the item repeat the last row (their t is zeroed).
  auto issue = [&](int r0, int b) {
#pragma unroll
    for (int ii = 0; ii < NI; ++ii) {
      const int byte = ii * 1024 + 16 * lane;
      const int r = byte / RB;
      const int p = (byte % RB) / 16;
      const int row = min(r0 + r, rows - 1);
      const uint16_t* src = Ab + (int64_t)row * lda + 8 * (p ^ bswz(r));
      __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)&abuf[b][w][ii * 1024], 16, 0, AUX);
    }
  };
  issue(0, 0);
  if constexpr (AHEAD) {
    if (ntiles > 1) issue(kRows, 1);
  }

  // Z_i slice in B-operand layout: zb[c][kt][e] = Z[slice0 + 32c + 8g + e][16kt + i]
  const float* Z = Zw + (int64_t)it.part * z_stride;
  bf8 zb[NC][KT];
  bf8 zl[SPLIT ? NC : 1][KT];   // the low parts (SPLIT)
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float z = (FULL || 16 * kt + i < kr) ? Z[(int64_t)(slice0 + 32 * c + 8 * g + e) * kr + 16 * kt + i] : 0.f;
        zb[c][kt][e] = (__bf16)z;
        if constexpr (SPLIT) zl[c][kt][e] = (__bf16)(z - (float)zb[c][kt][e]);
      }

  f4 yacc[NCT][KT];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) yacc[ct][kt] = f4{0.f, 0.f, 0.f, 0.f};

  // per-lane LDS byte offsets inside a wave tile
  int off1[4];   // product 1, chunk c: 256 (c / 4) + off1[c % 4]
#pragma unroll
  for (int c = 0; c < 4; ++c) off1[c] = i * RB + 16 * ((4 * c + g) ^ bswz(i));
  const int f = (lane >> 2) & 3, q = lane & 3;
  const int tr_row = 4 * g + f;
  int off2[8];   // product 2, block ct: 256 (ct / 8) + off2[ct % 8]
#pragma unroll
  for (int c = 0; c < 8; ++c)
    off2[c] = tr_row * RB + 16 * ((2 * c + (q >> 1)) ^ bswz(tr_row)) + 8 * (q & 1);

  for (int j = 0; j < ntiles; ++j) {
    const int b = j & 1;
    // tile j was issued one iteration ago: wait for it (a full wait, so no other
    // memory operation the compiler placed in between can satisfy the count),
    // then start tile j + 1 into the other buffer; it lands while tile j computes
    if constexpr (AHEAD) {
      // tile j complete; tile j + 1 (issued after it) may still be in flight
      if (j + 1 < ntiles)
        wait_vm_n<NI>();
      else
        wait_vm_all();
    } else {
      wait_vm_all();
      if (j + 1 < ntiles) issue((j + 1) * kRows, b ^ 1);
    }
    const unsigned tb = lds_addr(&abuf[b][w][0]);

    // product 1: partial t over this wave's slice (two chains per k block)
    f4 tacc[KT][2];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) tacc[kt][0] = tacc[kt][1] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c0 = 0; c0 < NC; c0 += 4) {
      bf8 a1[4];
      const unsigned base1 = tb + 256 * (c0 / 4);
      lds_read4_b128(a1[0], a1[1], a1[2], a1[3], base1 + off1[0], base1 + off1[1], base1 + off1[2],
                     base1 + off1[3]);
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
          if constexpr (SPLIT) {
            tacc[kt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[c], zb[c0 + c][kt], tacc[kt][0], 0, 0, 0);
            tacc[kt][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[c], zl[c0 + c][kt], tacc[kt][1], 0, 0, 0);
          } else {
            tacc[kt][c & 1] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[c], zb[c0 + c][kt], tacc[kt][c & 1], 0, 0, 0);
          }
        }
    }
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) tpart[w][kt][lane] = tacc[kt][0] + tacc[kt][1];
    lds_barrier();

    // sum the W slice partials (fixed order), round to BF16, store t^T;
    // rows past the end of the item get t = 0
    const int valid = min(kRows, rows - j * kRows);
    // (k block, register) combination cb = kt*4 + r goes to wave cb % W
#pragma unroll
    for (int cb = w; cb < 4 * KT; cb += W) {
      const int kt = cb >> 2, r = cb & 3;
      float s = tpart[0][kt][lane][r];
#pragma unroll
      for (int v = 1; v < W; ++v) s += tpart[v][kt][lane][r];
      const int row = 4 * g + r;
      const float tv = row < valid ? s : 0.f;
      const uint16_t hb = bf16_bits(tv);
      tbf[0][(i + 16 * kt) * kRows + row] = hb;
      if constexpr (SPLIT) {
        const float hi = __uint_as_float((uint32_t)hb << 16);
        tbf[SPLIT ? 1 : 0][(i + 16 * kt) * kRows + row] = bf16_bits(tv - hi);
      }
    }
    lds_barrier();

    // product 2: Y_slice += A_tile^T t
    s4 tb_op[KT], tl_op[SPLIT ? KT : 1];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      tb_op[kt] = *(const s4*)&tbf[0][(i + 16 * kt) * kRows + 4 * g];
      if constexpr (SPLIT) tl_op[kt] = *(const s4*)&tbf[SPLIT ? 1 : 0][(i + 16 * kt) * kRows + 4 * g];
    }
#pragma unroll
    for (int c0 = 0; c0 < NCT; c0 += 8) {
      s4 a2[8];
      const unsigned base2 = tb + 256 * (c0 / 8);
      lds_read4_tr(a2[0], a2[1], a2[2], a2[3], base2 + off2[0], base2 + off2[1], base2 + off2[2],
                   base2 + off2[3]);
      lds_read4_tr(a2[4], a2[5], a2[6], a2[7], base2 + off2[4], base2 + off2[5], base2 + off2[6],
                   base2 + off2[7]);
#pragma unroll
      for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
          yacc[c0 + c][kt] =
              __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2[c], tb_op[kt], yacc[c0 + c][kt], 0, 0, 0);
          if constexpr (SPLIT)
            yacc[c0 + c][kt] =
                __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2[c], tl_op[kt], yacc[c0 + c][kt], 0, 0, 0);
        }
    }
    if constexpr (AHEAD) {
      // this wave's reads of buffer b are done (the asm reads wait inside)
      if (j + 2 < ntiles) issue((j + 2) * kRows, b);
    }
  }
  // yacc[ct][kt][r] = Y[slice0 + 16ct + 4g + r][16kt + i]
  float* o = part + (int64_t)it.slot * D * kr;
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (FULL || 16 * kt + i < kr) o[(int64_t)(slice0 + 16 * ct + 4 * g + r) * kr + 16 * kt + i] = yacc[ct][kt][r];
}

template <int W, int NC, int KT, bool AHEAD, bool SPLIT>
hipError_t launch_nc(int nitems, bool nt, const uint16_t* a, int64_t lda, const float* z,
                     int64_t z_stride, const WorkItem* items, float* o, int kr, hipStream_t s) {
  const bool full = kr == 16 * KT;
  if (nt && full)
    k1_mfma_bf16<W, NC, KT, 2, AHEAD, SPLIT, true><<<nitems, 64 * W, 0, s>>>(a, lda, z, z_stride, items, o, kr);
  else if (nt)
    k1_mfma_bf16<W, NC, KT, 2, AHEAD, SPLIT, false><<<nitems, 64 * W, 0, s>>>(a, lda, z, z_stride, items, o, kr);
  else if (full)
    k1_mfma_bf16<W, NC, KT, 0, AHEAD, SPLIT, true><<<nitems, 64 * W, 0, s>>>(a, lda, z, z_stride, items, o, kr);
  else
    k1_mfma_bf16<W, NC, KT, 0, AHEAD, SPLIT, false><<<nitems, 64 * W, 0, s>>>(a, lda, z, z_stride, items, o, kr);
  return hipGetLastError();
}

template <int KT, bool AHEAD, bool SPLIT>
hipError_t launch_kt_ahead(int64_t d, bool w8, int nitems, bool nt, const uint16_t* a, int64_t lda,
                           const float* z, int64_t z_stride, const WorkItem* items, float* o, int kr,
                           hipStream_t s) {
  if (w8 && d == 1024) return launch_nc<8, 4, KT, AHEAD, SPLIT>(nitems, nt, a, lda, z, z_stride, items, o, kr, s);
  if constexpr (!(SPLIT && KT == 2)) {
    if (w8 && d == 2048) return launch_nc<8, 8, KT, AHEAD, SPLIT>(nitems, nt, a, lda, z, z_stride, items, o, kr, s);
  }
  switch (d) {
    case 512: return launch_nc<4, 4, KT, AHEAD, SPLIT>(nitems, nt, a, lda, z, z_stride, items, o, kr, s);
    case 1024: return launch_nc<4, 8, KT, AHEAD, SPLIT>(nitems, nt, a, lda, z, z_stride, items, o, kr, s);
    case 1536: return launch_nc<4, 12, KT, AHEAD, SPLIT>(nitems, nt, a, lda, z, z_stride, items, o, kr, s);
    case 2048:
      // split operands at k = 32 need 2 (Z) + 1 (Y) x 256 registers per lane over the
      // slice of a 2048-wide row: more than one CU holds (the launcher's caller
      // routes that case to the two-pass kernel)
      if constexpr (SPLIT && KT == 2) return hipErrorInvalidValue;
      else return launch_nc<4, 16, KT, AHEAD, SPLIT>(nitems, nt, a, lda, z, z_stride, items, o, kr, s);
    default: return hipErrorInvalidValue;
  }
}

// variant 0: four waves (any eligible d); 1: eight waves (d = 1024 or 2048);
// 2, 3: the same with two tiles in flight per wave
template <int KT, bool SPLIT>
hipError_t launch_kt(int64_t d, int variant, int nitems, bool nt, const uint16_t* a, int64_t lda,
                     const float* z, int64_t z_stride, const WorkItem* items, float* o, int kr,
                     hipStream_t s) {
  const bool w8 = variant == 1 || variant == 3;
  if (variant >= 2)
    return launch_kt_ahead<KT, true, SPLIT>(d, w8, nitems, nt, a, lda, z, z_stride, items, o, kr, s);
  return launch_kt_ahead<KT, false, SPLIT>(d, w8, nitems, nt, a, lda, z, z_stride, items, o, kr, s);
}

}  // namespace

bool mfma16_eligible(lp_dtype dtype, int64_t d, int64_t lda, int k, const void* A, bool split) {
  return dtype == LP_BF16 && k >= 1 && k <= 32 &&
         (d == 512 || d == 1024 || d == 1536 || d == 2048) && (lda % 8) == 0 &&
         ((uintptr_t)A % 16) == 0 && !(split && k > 16 && d == 2048);
}

hipError_t launch_local_multiply_mfma16(const Plan& P, const void* A, int64_t lda, int k,
                                        const void* Zw, int64_t z_stride, void* part,
                                        const WorkItem* items, int nitems,
                                        hipStream_t s) {
  const uint16_t* a = (const uint16_t*)A;
  const float* z = (const float*)Zw;
  float* o = (float*)part;
  // ranks below 16 (or between 16 and 32) run the 16- (32-) wide tiles with zero
  // columns of Z_i, which are not stored
  if (P.split_operands) {
    if (k > 16) return launch_kt<2, true>(P.d, P.variant, nitems, P.nt_loads, a, lda, z, z_stride, items, o, k, s);
    return launch_kt<1, true>(P.d, P.variant, nitems, P.nt_loads, a, lda, z, z_stride, items, o, k, s);
  }
  if (k > 16) return launch_kt<2, false>(P.d, P.variant, nitems, P.nt_loads, a, lda, z, z_stride, items, o, k, s);
  return launch_kt<1, false>(P.d, P.variant, nitems, P.nt_loads, a, lda, z, z_stride, items, o, k, s);
}

}  // namespace lp
