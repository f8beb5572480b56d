// Two-pass local multiply with FP32-class products on BF16 matrix cores, for
// the shapes the fused kernels do not cover (large d, k up to 64, FP32 or BF16 A):
//   pass 1  t = A_rows Z_i              (per 128-row block of a work item)
//   pass 2  part = A_rows^T t           (per 256-column block of a work item)
// (Eq. (power_yi) without 1/s_i; the per-item partials are reduced per
// partition in FP64 afterwards.)  The same two products as the FP32 two-pass
// kernel, on v_mfma_f32_16x16x32_bf16 instead of v_mfma_f32_16x16x4f32: at
// k = 64 the FP32 matrix cores bound that kernel, while the BF16 ones have
// sixteen times their rate.
//
// Exact operand splitting.  Every FP32 operand x is written as three BF16
// numbers x = x0 + x1 + x2 with x0 = bf16(x), x1 = bf16(x - x0), x2 = x - x0 - x1
// (round to nearest even; both differences are exact in FP32, and x2 has at
// most 8 significant bits, so it is a BF16 number: the split is exact for every
// FP32 x whose pieces stay normal).  With |x1| <= 2^-8 |x| and |x2| <= 2^-16 |x|,
// a product x y is the sum of the six terms x_a y_b with a + b <= 2, up to the
// three dropped terms, at most 2^-23 |x y| together: each product carries an
// error below two FP32 roundings, and the six partial products are exact in
// the FP32 accumulators.  BF16 A is its own first piece (three terms per
// product).  The intermediate t is kept in FP32 between the passes.
//
// MFMA operand layout (16x16x32): lane l = 16 g + i holds 8 K-elements of row
// (A operand) or column (B operand) i.  Here element e of lane group g is K
// index krow(g, e) = 16 (e / 4) + 4 g + e % 4 of a 32-deep slice, the same in
// both operands, so that
//   * pass 1 reads A straight from HBM into registers, two 16-byte loads per
//     16-row block (columns 4g..4g+3 and 16+4g..16+4g+3 of the slice);
//   * pass 2 reads the transposed A slice from LDS with ds_read_b64_tr_b16
//     (rows 4g..4g+3 of each 16-row half);
//   * the staged B operand (Z_i slice in pass 1, t slice in pass 2) sits in
//     LDS column-major with its K positions permuted to match, one 16-byte
//     read per lane and piece.
#include <type_traits>

#include "lp_internal.h"

namespace lp {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s4 lds_s4;

constexpr int kBK = 32;     // contraction slice: one 16x16x32 step
constexpr int kZR = 40;     // BF16 per row of a staged B-operand piece (32 + 8: 80-byte rows,
                            // so the 16 lanes of a 16-byte read cover all 64 banks)
constexpr int kBM1 = 128;   // rows per workgroup of pass 1
constexpr int kWC = 64;     // columns per wave of pass 2 (256 per workgroup)
constexpr int kPF1 = 1;     // A slices in registers ahead of the one multiplied, pass 1
constexpr int kPF2 = 1;     // the same, pass 2 (two would cost occupancy)

// K index of element e of lane group g inside a 32-deep slice, and the slot a
// K index takes in the staged B operand (slot 8 g + e)
__device__ inline int krow(int g, int e) { return 16 * (e >> 2) + 4 * g + (e & 3); }

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

typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 b2 __attribute__((ext_vector_type(2)));

// two FP32 values rounded to BF16 (nearest even), packed (first in the low half)
__device__ inline uint32_t cvt2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2{a, b}, b2));
}

// Pieces of a pair: x = x0 + x1 + x2 (exact), each piece a packed BF16 pair;
// NP = 1 keeps x0 only (BF16 data, exact already)
template <int NP>
__device__ inline void split2(float a, float b, uint32_t* o) {
  const uint32_t h = cvt2(a, b);
  o[0] = h;
  if constexpr (NP > 1) {
    const float ra = a - __uint_as_float(h << 16), rb = b - __uint_as_float(h & 0xffff0000u);
    const uint32_t m = cvt2(ra, rb);
    o[1] = m;
    o[2] = cvt2(ra - __uint_as_float(m << 16), rb - __uint_as_float(m & 0xffff0000u));
  }
}

template <int NP>
__device__ inline void split8(const float (&x)[8], bf8 (&o)[NP]) {
  uint32_t u[4][3];
#pragma unroll
  for (int e = 0; e < 4; ++e) split2<NP>(x[2 * e], x[2 * e + 1], u[e]);
#pragma unroll
  for (int q = 0; q < NP; ++q) o[q] = __builtin_bit_cast(bf8, uint4{u[0][q], u[1][q], u[2][q], u[3][q]});
}

template <int NP>
__device__ inline void split4(f4 x, bf4 (&o)[NP]) {
  uint32_t u[2][3];
  split2<NP>(x[0], x[1], u[0]);
  split2<NP>(x[2], x[3], u[1]);
#pragma unroll
  for (int q = 0; q < NP; ++q) o[q] = __builtin_bit_cast(bf4, uint2{u[0][q], u[1][q]});
}

// acc += x y over the kept terms x_a y_b, a + b <= 2 (x has PA pieces, y three).
// YT = 2 (BF16 x only: operand pairs) drops x_0 y_2 as well: y is then carried by
// its first two pieces, within 2^-16 of itself.
template <int PA, int YT>
__device__ inline f4 mfma_terms(const bf8 (&x)[PA], const bf8 (&y)[3], f4 acc) {
  static_assert(YT == 3 || (YT == 2 && PA == 1), "operand pairs only with BF16 A");
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0], y[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0], y[1], acc, 0, 0, 0);
  if constexpr (PA > 1) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[1], y[0], acc, 0, 0, 0);
  if constexpr (YT == 3) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0], y[2], acc, 0, 0, 0);
  if constexpr (PA > 1) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[1], y[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[2], y[0], acc, 0, 0, 0);
  }
  return acc;
}

// pass 1: t[row][n] = sum_c A[row][c] Z[c][n]; grid (items, ceil(max item rows / 128)),
// 4 waves, wave w owns rows 32 w .. 32 w + 31 of the block (MT = 2 16-row blocks).
// A goes from HBM straight into registers, PF slices ahead; the Z_i slice is
// split into its three pieces once per workgroup and staged in LDS (two buffers).
template <typename TA, int NT, int PF, int YT>
__global__ void __launch_bounds__(256)
tmm3_kernel(const TA* __restrict__ A, int64_t lda, int64_t d, int k, const float* __restrict__ Zw,
            int64_t z_stride, const WorkItem* __restrict__ items, float* __restrict__ t,
            unsigned long long* __restrict__ stamps) {
  constexpr int PA = std::is_same<TA, float>::value ? 3 : 1;
  constexpr int N = 16 * NT;
  constexpr int MT = kBM1 / 64;
  __shared__ __attribute__((aligned(16))) __bf16 Zs[2][3][N * kZR];
  const WorkItem it = items[blockIdx.x];
  const int64_t r0 = (int64_t)blockIdx.y * kBM1;
  const unsigned long long t_start = stamps != nullptr ? wall_clock64() : 0;
  const int64_t wg = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  if (r0 >= it.rows) {
    if (stamps != nullptr && threadIdx.x == 0) stamps[2 * wg] = stamps[2 * wg + 1] = t_start;
    return;
  }
  const int rows = (int)min<int64_t>(kBM1, it.rows - r0);
  const TA* Ab = A + (it.row0 + r0) * lda;
  const float* Z = Zw + (int64_t)it.part * z_stride;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, i = lane & 15;
  const int zn = tid & 63, zg = tid >> 6;   // staging: column zn of Z, slots 8 zg .. 8 zg + 7
  const int dd = (int)d;
  const int nsl = (dd + kBK - 1) / kBK;

  // clamped row pointers: every load is issued (no branches around the loads),
  // and the values outside the item or the matrix are zeroed where they are used
  const TA* arow[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) arow[mt] = Ab + (int64_t)min(16 * MT * w + 16 * mt + i, rows - 1) * lda;
  const float* zcol = Z + min(zn, k - 1);
  const bool rows_whole = 16 * MT * (w + 1) <= rows;   // wave-uniform
  const bool k_whole = k >= N;
  int zoff[8];      // offsets of this thread's Z slots inside a slice
#pragma unroll
  for (int e = 0; e < 8; ++e) zoff[e] = krow(zg, e) * k;

  typedef f4 ASlice[MT][2];   // A operand of one slice: columns 4g.. and 16 + 4g.. of rows 16 mt + i
  ASlice ra[PF];
  float rz[8];                // Z values of this thread's slots (next slice)
  auto fetch_a = [&](int c0, ASlice& dst) {
    if (c0 + kBK <= dd) {   // whole slice (uniform): plain offsets
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int h = 0; h < 2; ++h) dst[mt][h] = load4<TA>(arow[mt] + c0 + 16 * h + 4 * g);
    } else {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int h = 0; h < 2; ++h) dst[mt][h] = load4<TA>(arow[mt] + min(c0 + 16 * h + 4 * g, dd - 4));
    }
  };
  auto fetch_z = [&](int c0) {
    if (c0 + kBK <= dd) {
      const float* zs = zcol + (int64_t)c0 * k;
#pragma unroll
      for (int e = 0; e < 8; ++e) rz[e] = zs[zoff[e]];
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) rz[e] = zcol[min(c0 + krow(zg, e), dd - 1) * k];
    }
  };
  auto stash_z = [&](int b, int c0) {
    if (zn < N) {
      if (c0 + kBK > dd || !k_whole) {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (c0 + krow(zg, e) >= dd || zn >= k) rz[e] = 0.f;
      }
      bf8 zp[3];
      split8<3>(rz, zp);
#pragma unroll
      for (int p = 0; p < 3; ++p) *(bf8*)&Zs[b][p][zn * kZR + 8 * zg] = zp[p];
    }
  };

  f4 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};

  // slice s: split the A registers, refill them with slice s + PF, fetch the next
  // Z slice, multiply, stage the next Z slice
  auto step = [&](int s, ASlice& cur) {
    const int b = s & 1;
    const int c0 = s * kBK;
    if (c0 + kBK > dd || !rows_whole) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (16 * MT * w + 16 * mt + i >= rows || c0 + 16 * h + 4 * g >= dd) cur[mt][h] = f4{0.f, 0.f, 0.f, 0.f};
    }
    bf8 ap[MT][PA];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const float x[8] = {cur[mt][0][0], cur[mt][0][1], cur[mt][0][2], cur[mt][0][3],
                          cur[mt][1][0], cur[mt][1][1], cur[mt][1][2], cur[mt][1][3]};
      split8<PA>(x, ap[mt]);
    }
    if (s + PF < nsl) fetch_a(c0 + PF * kBK, cur);
    if (s + 1 < nsl) fetch_z(c0 + kBK);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      bf8 zp[3];
#pragma unroll
      for (int p = 0; p < 3; ++p) zp[p] = *(const bf8*)&Zs[b][p][(16 * nt + i) * kZR + 8 * g];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma_terms<PA, YT>(ap[mt], zp, acc[mt][nt]);
    }
    if (s + 1 < nsl) stash_z(b ^ 1, c0 + kBK);
    __syncthreads();
  };

#pragma unroll
  for (int q = 0; q < PF; ++q)
    if (q < nsl) fetch_a(q * kBK, ra[q]);
  fetch_z(0);
  stash_z(0, 0);
  __syncthreads();
  for (int s = 0; s < nsl; s += PF) {
    step(s, ra[0]);
    if constexpr (PF > 1) {
      if (s + 1 < nsl) step(s + 1, ra[1]);
    }
  }
  float* tb = t + (it.row0 + r0) * k;
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

// LDS byte offset of the 8-byte unit u (columns 4u..4u+3) of row r in a wave's
// A piece (64 columns = 128-byte rows): 16-byte chunks XOR-swizzled by
// 2 ((r / 2) mod 4), so the transposing reads of 8 consecutive rows (a
// half-wave) and the staging writes each touch all 64 banks once
__device__ inline int aoff(int r, int u) {
  return r * (2 * kWC) + 16 * ((u >> 1) ^ (((r >> 1) & 3) << 1)) + 8 * (u & 1);
}

// pass 2: part[slot][c][n] = sum_{rows of item} A[row][c] t[row][n]; grid (items, ceil(d / 256)),
// 4 waves, wave w owns columns 64 w .. 64 w + 63 of the block (four 16-column blocks).
// A slices come into registers PF slices ahead, each wave splits its own 32 x 64
// block into LDS (no other wave reads it); the t slice is split once per
// workgroup into two LDS buffers.
template <typename TA, int NT, int PF, int YT>
__global__ void __launch_bounds__(256)
ymm3_kernel(const TA* __restrict__ A, int64_t lda, int64_t d, int k, const float* __restrict__ t,
            const WorkItem* __restrict__ items, float* __restrict__ part,
            unsigned long long* __restrict__ stamps) {
  constexpr int PA = std::is_same<TA, float>::value ? 3 : 1;
  constexpr int N = 16 * NT;
  constexpr int MT = kWC / 16;
  constexpr int PB = kBK * 2 * kWC;          // bytes of one wave's A piece (32 rows)
  constexpr int LPR = kWC / 4;               // lanes per A row when staging (16)
  constexpr int RPI = 64 / LPR;              // rows per staging load (4)
  constexpr int NLD = kBK / RPI;             // staging loads per lane and slice (8)
  __shared__ __attribute__((aligned(16))) unsigned char As[4][PA][PB];
  __shared__ __attribute__((aligned(16))) __bf16 Ts[2][3][N * kZR];
  const WorkItem it = items[blockIdx.x];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, i = lane & 15;
  const int64_t cw = (int64_t)blockIdx.y * 4 * kWC + kWC * w;   // first column of this wave
  const int rows = (int)it.rows;
  const TA* Ab = A + it.row0 * lda + cw;
  const float* tb = t + it.row0 * k;
  const unsigned long long t_start = stamps != nullptr ? wall_clock64() : 0;
  const int tn = tid & 63, tg = tid >> 6;   // staging: column tn of t, slots 8 tg .. 8 tg + 7
  const int su = lane % LPR, sr = lane / LPR;
  const int nsl = (rows + kBK - 1) / kBK;

  // clamped loads (no branches around them); values outside the item or the
  // matrix are zeroed when staged
  const TA* acol = Ab + min<int64_t>(4 * su, d - 4 - cw);
  const float* tcol = tb + min(tn, k - 1);
  const bool cols_whole = cw + kWC <= d;   // wave-uniform
  const bool k_whole = k >= N;
  int toffs[8];     // offsets of this thread's t slots inside a slice
#pragma unroll
  for (int e = 0; e < 8; ++e) toffs[e] = krow(tg, e) * k;
  const int64_t lda_r = (int64_t)RPI * lda;

  struct Slice {
    f4 a[NLD];
    float t[8];
  };
  Slice rs_[PF];
  auto fetch = [&](int rs, Slice& dst) {
    if (rs + kBK <= rows) {   // whole slice (uniform): plain strides
      const TA* p = acol + (int64_t)(rs + sr) * lda;
#pragma unroll
      for (int j = 0; j < NLD; ++j) dst.a[j] = load4<TA>(p + j * lda_r);
      const float* ts = tcol + (int64_t)rs * k;
#pragma unroll
      for (int e = 0; e < 8; ++e) dst.t[e] = ts[toffs[e]];
    } else {
#pragma unroll
      for (int j = 0; j < NLD; ++j) dst.a[j] = load4<TA>(acol + (int64_t)min(rs + RPI * j + sr, rows - 1) * lda);
#pragma unroll
      for (int e = 0; e < 8; ++e) dst.t[e] = tcol[min(rs + krow(tg, e), rows - 1) * k];
    }
  };
  auto stash = [&](int b, int rs, Slice& src) {
    const bool rows_whole = rs + kBK <= rows;
    if (!rows_whole || !cols_whole) {
#pragma unroll
      for (int j = 0; j < NLD; ++j)
        if (rs + RPI * j + sr >= rows || cw + 4 * su >= d) src.a[j] = f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      bf4 ap[PA];
      split4<PA>(src.a[j], ap);
#pragma unroll
      for (int p = 0; p < PA; ++p) *(bf4*)&As[w][p][aoff(RPI * j + sr, su)] = ap[p];
    }
    if (tn < N) {
      if (!rows_whole || !k_whole) {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (rs + krow(tg, e) >= rows || tn >= k) src.t[e] = 0.f;
      }
      bf8 tp[3];
      split8<3>(src.t, tp);
#pragma unroll
      for (int p = 0; p < 3; ++p) *(bf8*)&Ts[b][p][tn * kZR + 8 * tg] = tp[p];
    }
  };

  f4 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};

  // transposing reads: lane 16 g + 4 f + q reads columns 16 mt + 4 q.. of row 16 h + 4 g + f
  const int f = (lane >> 2) & 3, q = lane & 3;
  int toff[2][MT];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) toff[h][mt] = aoff(16 * h + 4 * g + f, 4 * mt + q);

  // slice s: stage it from registers, refill the registers with slice s + PF, multiply
  auto step = [&](int s, Slice& cur) {
    const int b = s & 1;
    stash(b, s * kBK, cur);
    __syncthreads();
    if (s + PF < nsl) fetch((s + PF) * kBK, cur);
    bf8 tp[NT][3];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int p = 0; p < 3; ++p) tp[nt][p] = *(const bf8*)&Ts[b][p][(16 * nt + i) * kZR + 8 * g];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      bf8 ap[PA];
#pragma unroll
      for (int p = 0; p < PA; ++p) {
        const s4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s4*)&As[w][p][toff[0][mt]]);
        const s4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s4*)&As[w][p][toff[1][mt]]);
        ap[p] = __builtin_bit_cast(bf8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma_terms<PA, YT>(ap, tp[nt], acc[mt][nt]);
    }
  };

#pragma unroll
  for (int p = 0; p < PF; ++p)
    if (p < nsl) fetch(p * kBK, rs_[p]);
  for (int s = 0; s < nsl; s += PF) {
    step(s, rs_[0]);
    if constexpr (PF > 1) {
      if (s + 1 < nsl) step(s + 1, rs_[1]);
    }
  }
  // acc[mt][nt][r] = part[cw + 16 mt + 4 g + r][16 nt + i]
  float* o = part + (int64_t)it.slot * d * k;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t c = cw + 16 * mt + 4 * g + r;
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

template <typename TA, int NT, int YT>
hipError_t pair3(const Plan& P, const void* A, int64_t lda, int k, const void* Zw, int64_t z_stride,
                 void* tbuf, void* part, const WorkItem* items, int nitems, hipStream_t s) {
  dim3 g1(nitems, (unsigned)((P.chunk_rows + kBM1 - 1) / kBM1));
  unsigned long long* st1 = P.stamps;
  unsigned long long* st2 = P.stamps != nullptr ? P.stamps + 2 * (int64_t)g1.x * g1.y : nullptr;
  tmm3_kernel<TA, NT, kPF1, YT><<<g1, 256, 0, s>>>((const TA*)A, lda, P.d, k, (const float*)Zw, z_stride,
                                         items, (float*)tbuf, st1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 g2(nitems, (unsigned)((P.d + 4 * kWC - 1) / (4 * kWC)));
  ymm3_kernel<TA, NT, kPF2, YT><<<g2, 256, 0, s>>>((const TA*)A, lda, P.d, k, (const float*)tbuf, items,
                                         (float*)part, st2);
  return hipGetLastError();
}

template <typename TA, int YT>
hipError_t pair3_k(const Plan& P, const void* A, int64_t lda, int k, const void* Zw,
                   int64_t z_stride, void* tbuf, void* part, const WorkItem* items, int nitems,
                   hipStream_t s) {
  if (k <= 16) return pair3<TA, 1, YT>(P, A, lda, k, Zw, z_stride, tbuf, part, items, nitems, s);
  if (k <= 32) return pair3<TA, 2, YT>(P, A, lda, k, Zw, z_stride, tbuf, part, items, nitems, s);
  if (k <= 48) return pair3<TA, 3, YT>(P, A, lda, k, Zw, z_stride, tbuf, part, items, nitems, s);
  return pair3<TA, 4, YT>(P, A, lda, k, Zw, z_stride, tbuf, part, items, nitems, s);
}

}  // namespace

hipError_t launch_local_multiply_gemm3(const Plan& P, const void* A, int64_t lda, int k,
                                       const void* Zw, int64_t z_stride, void* tbuf, void* part,
                                       const WorkItem* items, int nitems, hipStream_t s) {
  if (P.dtype == LP_F32)
    return pair3_k<float, 3>(P, A, lda, k, Zw, z_stride, tbuf, part, items, nitems, s);
  // BF16 A with operand pairs asked for (split_operands) and no kernel named: Z_i and
  // t carried by two BF16 pieces each, the precision of the fused kernel's pairs,
  // for two products instead of three
  if (P.split_operands && P.two_pass_auto && !P.split_products)
    return pair3_k<__hip_bfloat16, 2>(P, A, lda, k, Zw, z_stride, tbuf, part, items, nitems, s);
  return pair3_k<__hip_bfloat16, 3>(P, A, lda, k, Zw, z_stride, tbuf, part, items, nitems, s);
}

void two_pass_geometry(const Plan& P, int64_t* rows_per_wg1, int64_t* cols_per_wg2) {
  (void)P;   // both forms of the two-pass kernel use the same blocks
  *rows_per_wg1 = kBM1;
  *cols_per_wg2 = 4 * kWC;
}

}  // namespace lp
