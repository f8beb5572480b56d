// Small FP64 kernels of LocalPower: Gram matrices, Cholesky + triangular
// inverse (CholeskyQR2), right multiplication by k x k matrices, sign-fixing
// and orthogonal-Procrustes alignment, aggregation, Jacobi eigen/SVD and the
// sin-theta distance.  All of them work on d x k (k <= 64) FP64 row-major
// matrices, batched over the m partitions where the method batches them.
#include "lp_internal.h"

#include <cmath>

namespace lp {
namespace {

// Cross-Gram partial out[i][j] = sum_r Xs[r][i] Ws[r][j] over `rows` rows of the
// LDS blocks Xs, Ws (row stride k <= 16 KC); thread (ty, tx) = (tid / 16, tid % 16)
// owns the entries (ty + 16a, tx + 16c), a, c < KC.  Needs kBlock threads.
template <int KC>
__device__ void gram_tile(const double* Xs, const double* Ws, int rows, int k, double* out) {
  if constexpr (KC == 1) {
    // k <= 16: FP64 matrix cores.  v_mfma_f64_16x16x4f64 with A[i][q] = X[r + q][i] and
    // B[q][j] = W[r + q][j] (lane l supplies row r + l/16, column l%16 of each, zero
    // past k and past `rows`); wave w sums rows 4s (s = w, w + 4, ...), and the four
    // wave sums are added in a fixed order through LDS.
    __shared__ double gsum[4][256];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = lane & 15, q = lane >> 4;
    typedef double d4 __attribute__((ext_vector_type(4)));
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int r = 4 * w; r < rows; r += 16) {
      const int rr = r + q;
      const bool ok = rr < rows && c < k;
      const double a = ok ? Xs[rr * k + c] : 0.0;
      const double b = ok ? Ws[rr * k + c] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    // the FP64 16x16x4 result interleaves rows: lane l holds entries (4t + l/16, l%16), t < 4
    // (measured on gfx950; the FP32 16x16x4 form holds rows 4(l/16) + t instead)
#pragma unroll
    for (int t = 0; t < 4; ++t) gsum[w][(4 * t + q) * 16 + c] = acc[t];
    __syncthreads();
    for (int e = threadIdx.x; e < k * k; e += kBlock) {
      const int i = e / k, j = e - (e / k) * k;
      out[e] = ((gsum[0][i * 16 + j] + gsum[1][i * 16 + j]) + gsum[2][i * 16 + j]) + gsum[3][i * 16 + j];
    }
    return;
  }
  // k > 16: FP64 matrix cores, one 16 x 16 output block (bi, bj) at a time per
  // wave (blocks bi * KC + bj = w, w + 4, ...), K = rows in steps of 4:
  // A[i][q] = X[r + q][16 bi + i], B[q][j] = W[r + q][16 bj + j]
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = lane & 15, q = lane >> 4;
  for (int blk = w; blk < KC * KC; blk += 4) {
    const int bi = blk / KC, bj = blk - (blk / KC) * KC;
    const int ci = 16 * bi + c, cj = 16 * bj + c;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int r = 0; r < rows; r += 4) {
      const int rr = r + q;
      const double a = (rr < rows && ci < k) ? Xs[rr * k + ci] : 0.0;
      const double b = (rr < rows && cj < k) ? Ws[rr * k + cj] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    // lane l holds entries (16 bi + 4t + l/16, 16 bj + l%16)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = 16 * bi + 4 * t + q, j = cj;
      if (i < k && j < k) out[i * k + j] = acc[t];
    }
  }
}

// 16-column blocks needed for k columns
constexpr int kc_of(int km) { return (km + 15) / 16; }

// dst[e] = src[e] for e < count (global -> LDS), at most EPT elements per
// thread.  All loads are issued (clamped index) before the first store: a store
// right after each load waits for it, one round trip per element.
template <int EPT>
__device__ inline void load_tile(const double* __restrict__ src, int count, double* dst) {
  double v[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) v[u] = src[min((int)threadIdx.x + u * kBlock, count - 1)];
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = threadIdx.x + u * kBlock;
    if (e < count) dst[e] = v[u];
  }
}

// ---------------------------------------------------------------------------
// G_b(chunk) = X_b[rows]^T W_b[rows]  (k x k partial, chunk of kGramRows rows)
// grid: (nchunks, batch), block kBlock
// ---------------------------------------------------------------------------
template <int KC>
__global__ void __launch_bounds__(kBlock)
cross_gram_kernel(int64_t d, int k, const double* __restrict__ X, int64_t x_stride,
                  const double* __restrict__ W, int64_t w_stride, double* __restrict__ out) {
  __shared__ double xs[kGramRows * kMaxK];
  __shared__ double ws[kGramRows * kMaxK];
  const int b = blockIdx.y;
  const int c = blockIdx.x;
  const int nchunks = gridDim.x;
  const int64_t r0 = (int64_t)c * kGramRows;
  const int rows = (int)min<int64_t>(kGramRows, d - r0);
  const double* Xb = X + b * x_stride + r0 * k;
  const double* Wb = W + b * w_stride + r0 * k;
  load_tile<4 * KC>(Xb, rows * k, xs);
  load_tile<4 * KC>(Wb, rows * k, ws);
  __syncthreads();
  gram_tile<KC>(xs, ws, rows, k, out + ((int64_t)b * nchunks + c) * k * k);
}

// sum_{q < n} p[q * stride] with eight interleaved accumulators combined in a
// fixed order (deterministic, and eight loads in flight instead of one).
template <typename T>
__device__ inline double sum_strided(const T* __restrict__ p, int64_t stride, int n) {
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int q = 0;
  for (; q + 7 < n; q += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += (double)p[(int64_t)(q + u) * stride];
  }
  for (; q < n; ++q) a[q & 7] += (double)p[(int64_t)q * stride];
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// acc[u] = sum over q < n of p[q * stride + e_u] for this thread's elements
// e_u = threadIdx.x + u * kBlock (0 where e_u >= count), added in increasing q.
// The loads of QU consecutive q for all EPT elements (32 in all) are issued
// together, instead of one element's at a time.
template <int EPT, typename T>
__device__ inline void sum_rows(const T* __restrict__ p, int64_t stride, int n, int count,
                                double (&acc)[EPT]) {
  constexpr int QU = EPT >= 16 ? 2 : 32 / EPT;
#pragma unroll
  for (int u = 0; u < EPT; ++u) acc[u] = 0.0;
  int q = 0;
  for (; q + QU <= n; q += QU) {
    double v[QU][EPT];
    // unconditional loads (clamped index, then zeroed): a load under a branch is
    // waited for inside its branch, which would serialise all of them
#pragma unroll
    for (int j = 0; j < QU; ++j)
#pragma unroll
      for (int u = 0; u < EPT; ++u) {
        const int e = threadIdx.x + u * kBlock;
        v[j][u] = (double)p[(int64_t)(q + j) * stride + min(e, count - 1)];
      }
#pragma unroll
    for (int j = 0; j < QU; ++j)
#pragma unroll
      for (int u = 0; u < EPT; ++u) acc[u] += (threadIdx.x + u * kBlock < count) ? v[j][u] : 0.0;
  }
  for (; q < n; ++q) {
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + u * kBlock;
      const double x = (double)p[(int64_t)q * stride + min(e, count - 1)];
      acc[u] += e < count ? x : 0.0;
    }
  }
}

// Sum of the gram partials of batch b into an LDS k x k array (fixed order).
__device__ void sum_partials(const double* __restrict__ part, int b, int nchunks, int k,
                             double* G) {
  const int kk = k * k;
  for (int e = threadIdx.x; e < kk; e += blockDim.x)
    G[e] = sum_strided(part + (int64_t)b * nchunks * kk + e, kk, nchunks);
}

// grid (ceil(kk / kBlock), batch): out[b][e] = sum of the nch partials of entry e
// of matrix b (fixed order), one thread per entry.
__global__ void __launch_bounds__(kBlock)
sum_gram_kernel(int nch, int kk, const double* __restrict__ part, double* __restrict__ out) {
  const int b = blockIdx.y;
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= kk) return;
  out[(int64_t)b * kk + e] = sum_strided(part + (int64_t)b * nch * kk + e, kk, nch);
}

__device__ inline double rdlane(double v, int l) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// 1 / sqrt(x) for finite x > 0: the hardware estimate refined by two Newton
// steps y <- y + y (1 - x y^2) / 2 (each at least doubles the correct bits; the
// result is within a few ulp, and sqrt(x) is taken as x / sqrt(x)).
__device__ inline double rsqrt_pos(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double r = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, r, y);
  }
  return y;
}

// Cholesky G = R^T R (upper R, positive diagonal) of the k x k LDS matrix G and
// R^{-1} into the LDS matrix Ri (row stride k, zero below the diagonal), by the
// first wavefront of the block (k <= KM <= 32): lane c holds column c of G in
// registers and rows are broadcast with readlane.  G is padded to KM x KM with
// the identity, whose factor and inverse are blockdiag(R, I) and
// blockdiag(R^{-1}, I), so no step branches on k or on the lane.  On breakdown
// (non-positive or non-finite pivot) *bad is set and Ri is the identity.  Call
// from all threads; returns after a block barrier with Ri ready.
template <int KM>
__device__ __forceinline__ void chol_inv_wave(const double* G, double* Ri, int k, int* bad) {
  static_assert(KM <= 32, "register-resident factorization for k <= 32");
  if (threadIdx.x < 64) {
    const int c = threadIdx.x;
    const int cc = c < KM ? c : KM - 1;    // lanes past KM shadow the last column
    double g[KM], r[KM], rd[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) {
      const double v = G[min(i, k - 1) * k + min(cc, k - 1)];
      g[i] = (i < k && cc < k) ? v : (i == cc ? 1.0 : 0.0);
    }
    // G = I + E with max |E| < 1e-8 (the second pass of CholeskyQR2 on an
    // already orthonormal block): R = I + F + O(E^2) with F = the strict upper
    // triangle of E plus half its diagonal, so R^{-1} = I - F + O(E^2), exact to
    // rounding at this size of E; no pivots, square roots or substitution
    // (a NaN entry fails the comparison and takes the full factorization, which
    // flags it)
    bool near = true;
#pragma unroll
    for (int i = 0; i < KM; ++i) near = near && fabs(g[i] - (i == cc ? 1.0 : 0.0)) < 1e-8;
    if (__all(near)) {
      if (c < k) {
#pragma unroll
        for (int i = 0; i < KM; ++i)
          if (i < k) Ri[i * k + c] = i < c ? -g[i] : (i == c ? 1.5 - 0.5 * g[i] : 0.0);
      }
    } else {
    bool badw = false;
    // column-oriented elimination: step j makes row j of R (lane c: R[j][c]) and
    // updates the trailing rows; entries below the diagonal are never read
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      double djj = rdlane(g[j], j);
      const bool ok = djj > 0.0 && isfinite(djj);
      badw = badw || !ok;
      djj = ok ? djj : 1.0;
      const double inv = rsqrt_pos(djj);
      const double rjj = djj * inv;
      rd[j] = inv;
      const double rjc = (c == j) ? rjj : (c > j ? g[j] * inv : 0.0);
      r[j] = rjc;
#pragma unroll
      for (int i = j + 1; i < KM; ++i) g[i] = fma(-rdlane(rjc, i), rjc, g[i]);
    }
    // back substitution R x = e_c (R[i][l] is lane l's r[i]); x overwrites g
#pragma unroll
    for (int i = KM - 1; i >= 0; --i) {
      double acc = (i == c) ? 1.0 : 0.0;
#pragma unroll
      for (int l = i + 1; l < KM; ++l) acc = fma(-rdlane(r[i], l), g[l], acc);
      g[i] = acc * rd[i];
    }
    if (c < k) {
#pragma unroll
      for (int i = 0; i < KM; ++i)
        if (i < k) Ri[i * k + c] = badw ? (i == c ? 1.0 : 0.0) : g[i];
    }
    if (c == 0 && badw) *bad = 1;
    }
  }
  __syncthreads();
}

// Cholesky S = R^T R of the 16 x 16 LDS block S (row stride ld) and X = R^{-1},
// by the first wavefront (the column-per-lane form above without padding; lanes
// 16..63 repeat lanes 0..15).  R and X are written with row stride ld, zero
// below the diagonal.  A non-positive or non-finite pivot sets *bad and is taken
// as 1.  No barrier inside.
__device__ __forceinline__ void chol16_wave(const double* S, double* R, double* X, int ld, int* bad) {
  if (threadIdx.x < 64) {
    const int c = threadIdx.x & 15;
    double g[16], r[16], rd[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) g[i] = S[i * ld + c];
    bool badw = false;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      double djj = rdlane(g[j], j);
      const bool ok = djj > 0.0 && isfinite(djj);
      badw = badw || !ok;
      djj = ok ? djj : 1.0;
      const double inv = rsqrt_pos(djj);
      rd[j] = inv;
      const double rjc = (c == j) ? djj * inv : (c > j ? g[j] * inv : 0.0);
      r[j] = rjc;
#pragma unroll
      for (int i = j + 1; i < 16; ++i) g[i] = fma(-rdlane(rjc, i), rjc, g[i]);
    }
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      double acc = (i == c) ? 1.0 : 0.0;
#pragma unroll
      for (int l = i + 1; l < 16; ++l) acc = fma(-rdlane(r[i], l), g[l], acc);
      g[i] = acc * rd[i];
    }
    if (threadIdx.x < 16) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        R[i * ld + c] = r[i];
        X[i * ld + c] = g[i];
      }
    }
    if (threadIdx.x == 0 && badw) *bad = 1;
  }
}

// grid (batch), block kBlock: R^{-1} of chol(sum of the Gram partials) for
// matrix b, k <= 16 NB, by 16 x 16 blocks.  G (padded to 16 NB with the identity)
// goes through right-looking block elimination: the diagonal block J of the
// Schur complement is factored by chol16_wave (R_JJ and R_JJ^{-1}), then
// R_JI = R_JJ^{-T} S_JI for I > J and S_IK -= R_JI^T R_JK for J < I <= K, each a
// 16 x 16 product with one entry per thread.  The inverse is upper block
// triangular: X_JJ = R_JJ^{-1} and X_IJ = -(sum_{L=I}^{J-1} X_IL R_LJ) X_JJ for
// I < J.  On breakdown flags[b] is set and R^{-1} is the identity.
template <int NB>
__global__ void __launch_bounds__(kBlock)
chol_inv_blocked_kernel(int nch, int k, const double* __restrict__ gin, double* __restrict__ rinv,
                        int32_t* __restrict__ flags) {
  constexpr int KM = 16 * NB;
  __shared__ double S[KM * KM];
  __shared__ double R[KM * KM];
  __shared__ double X[KM * KM];
  __shared__ int bad;
  const int b = blockIdx.x, t = threadIdx.x;
  const int rr = t >> 4, cc = t & 15;   // one entry of a 16 x 16 block per thread
  const int kk = k * k;
  if (t == 0) bad = 0;
  for (int e = t; e < KM * KM; e += kBlock) {
    const int i = e / KM, j = e - (e / KM) * KM;
    S[e] = (i < k && j < k) ? sum_strided(gin + (int64_t)b * nch * kk + i * k + j, kk, nch)
                            : (i == j ? 1.0 : 0.0);
    R[e] = 0.0;
    X[e] = 0.0;
  }
  // G = I + E with every |E_ij| < 1e-8 (the second pass of CholeskyQR2): the
  // first-order inverse factor I - F (F = strict upper triangle of E plus half its
  // diagonal) is exact to FP64 rounding; a NaN entry fails the test
  int near = 1;
  for (int e = t; e < KM * KM; e += kBlock) {
    const int i = e / KM, j = e - (e / KM) * KM;
    near = near && fabs(S[e] - (i == j ? 1.0 : 0.0)) < 1e-8;
  }
  if (__syncthreads_and(near)) {
    for (int e = t; e < kk; e += kBlock) {
      const int i = e / k, j = e - (e / k) * k;
      const double g = S[i * KM + j];
      rinv[(int64_t)b * kk + e] = i < j ? -g : (i == j ? 1.5 - 0.5 * g : 0.0);
    }
    return;
  }
  for (int J = 0; J < NB; ++J) {
    const int dj = 16 * J * KM + 16 * J;
    chol16_wave(&S[dj], &R[dj], &X[dj], KM, &bad);
    __syncthreads();
    for (int I = J + 1; I < NB; ++I) {
      double v = 0.0;
#pragma unroll
      for (int l = 0; l < 16; ++l)
        v = fma(X[(16 * J + l) * KM + 16 * J + rr], S[(16 * J + l) * KM + 16 * I + cc], v);
      R[(16 * J + rr) * KM + 16 * I + cc] = v;
    }
    __syncthreads();
    for (int I = J + 1; I < NB; ++I)
      for (int K = I; K < NB; ++K) {
        double v = S[(16 * I + rr) * KM + 16 * K + cc];
#pragma unroll
        for (int l = 0; l < 16; ++l)
          v = fma(-R[(16 * J + l) * KM + 16 * I + rr], R[(16 * J + l) * KM + 16 * K + cc], v);
        S[(16 * I + rr) * KM + 16 * K + cc] = v;
      }
    __syncthreads();
  }
  // off-diagonal blocks of the inverse, column block by column block; the
  // products P_IJ go to the (no longer needed) blocks S_IJ
  for (int J = 1; J < NB; ++J) {
    for (int I = 0; I < J; ++I) {
      double v = 0.0;
      for (int L = I; L < J; ++L)
#pragma unroll
        for (int l = 0; l < 16; ++l)
          v = fma(X[(16 * I + rr) * KM + 16 * L + l], R[(16 * L + l) * KM + 16 * J + cc], v);
      S[(16 * I + rr) * KM + 16 * J + cc] = v;
    }
    __syncthreads();
    for (int I = 0; I < J; ++I) {
      double v = 0.0;
#pragma unroll
      for (int l = 0; l < 16; ++l)
        v = fma(-S[(16 * I + rr) * KM + 16 * J + l], X[(16 * J + l) * KM + 16 * J + cc], v);
      X[(16 * I + rr) * KM + 16 * J + cc] = v;
    }
    __syncthreads();
  }
  const bool fail = bad != 0;
  for (int e = t; e < kk; e += kBlock) {
    const int i = e / k, j = e - (e / k) * k;
    rinv[(int64_t)b * kk + e] = fail ? (i == j ? 1.0 : 0.0) : X[i * KM + j];
  }
  if (t == 0 && fail && flags != nullptr) flags[b] = 1;
}

// grid (nch, nb): Y_i rows of chunk c = sum of the partition's partial slots, and
// their Gram, for partition i = b0 + blockIdx.y.
template <typename TC, int KM>
__global__ void __launch_bounds__(kBlock)
reduce_gram_kernel(int64_t d, int k, int b0, const TC* __restrict__ part,
                   const int32_t* __restrict__ slot_off, double* __restrict__ Yi,
                   double* __restrict__ gram) {
  __shared__ double ys[kGramRows * KM];
  const int b = b0 + (int)blockIdx.y, c = blockIdx.x, nch = gridDim.x;
  const int64_t r0 = (int64_t)c * kGramRows;
  const int rows = (int)min<int64_t>(kGramRows, d - r0);
  const int64_t dk = d * k;
  const int s0 = slot_off[b], s1 = slot_off[b + 1];
  constexpr int EPT = kGramRows * KM / kBlock;
  double acc[EPT];
  sum_rows<EPT>(part + (int64_t)s0 * dk + r0 * k, dk, s1 - s0, rows * k, acc);
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = threadIdx.x + u * kBlock;
    if (e < rows * k) {
      Yi[(int64_t)b * dk + r0 * k + e] = acc[u];
      ys[e] = acc[u];
    }
  }
  __syncthreads();
  gram_tile<kc_of(KM)>(ys, ys, rows, k, gram + ((int64_t)b * nch + c) * k * k);
}

// grid (nch): Y rows = scale * sum_i Yi rows, and their Gram.
template <int KM>
__global__ void __launch_bounds__(kBlock)
aggregate_gram_kernel(int m, int64_t d, int k, const double* __restrict__ Yi, double scale,
                      double* __restrict__ Y, double* __restrict__ gram) {
  __shared__ double ys[kGramRows * KM];
  const int c = blockIdx.x;
  const int64_t r0 = (int64_t)c * kGramRows;
  const int rows = (int)min<int64_t>(kGramRows, d - r0);
  const int64_t dk = d * k;
  constexpr int EPT = kGramRows * KM / kBlock;
  double acc[EPT];
  sum_rows<EPT>(Yi + r0 * k, dk, m, rows * k, acc);
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = threadIdx.x + u * kBlock;
    if (e < rows * k) {
      const double v = scale * acc[u];
      Y[r0 * k + e] = v;
      ys[e] = v;
    }
  }
  __syncthreads();
  gram_tile<kc_of(KM)>(ys, ys, rows, k, gram + (int64_t)c * k * k);
}




// Rows [0, rows) of Xs (row stride k) times the k x k matrix S (LDS, row stride
// k) on FP64 matrix cores, for a tile of at most 64 rows: wave w owns rows
// 16w..16w+15 and all KC 16-column blocks; K = k in steps of 4 with
// A[i][q] = X[16w + i][l + q], B[q][j] = S[l + q][16 bj + j] (S zero below the
// diagonal when `upper`).  Returns the accumulators: lane l, block bj, t holds
// the entry (16w + 4t + l/16, 16 bj + l%16).
template <int KC>
__device__ inline void tile_times_s(const double* Xs, const double* S, int rows, int k, bool upper,
                                    double (&res)[KC][4]) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = lane & 15, q = lane >> 4;
  const int row = 16 * w + c;
  d4 acc[KC];
#pragma unroll
  for (int bj = 0; bj < KC; ++bj) acc[bj] = d4{0.0, 0.0, 0.0, 0.0};
  for (int l = 0; l < k; l += 4) {
    const int lq = l + q;
    const double a = (row < rows && lq < k) ? Xs[row * k + lq] : 0.0;
#pragma unroll
    for (int bj = 0; bj < KC; ++bj) {
      const int j = 16 * bj + c;
      const double b = (lq < k && j < k && (!upper || lq <= j)) ? S[lq * k + j] : 0.0;
      acc[bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[bj], 0, 0, 0);
    }
  }
#pragma unroll
  for (int bj = 0; bj < KC; ++bj)
#pragma unroll
    for (int t = 0; t < 4; ++t) res[bj][t] = acc[bj][t];
}

// grid (ceil(d / 64), batch): Q = X R^{-1} for the 64-row chunk c of matrix b
// (R^{-1} upper triangular), the optional working copy, and the optional Gram
// partial of the chunk's rows of Q (partial index b * gridDim.x + c).  With
// FACTOR (k <= 16) every workgroup sums the nch_in Gram partials in `rin` and
// factors and inverts them itself (a few microseconds of one wavefront, cheaper
// than a separate launch at this k; breakdown sets flags[b] and takes R = I);
// otherwise `rin` holds R^{-1} of every matrix.  The chunk of X is loaded into
// LDS before the factorization so that the loads overlap it.
template <typename TW, int KC, bool FACTOR>
__global__ void __launch_bounds__(kBlock)
apply_gram_kernel(int64_t d, int k, int nch_in, const double* __restrict__ X,
                  const double* __restrict__ rin, double* __restrict__ Q, TW* __restrict__ zw,
                  double* __restrict__ gout, int32_t* __restrict__ flags) {
  constexpr int KM = 16 * KC;
  __shared__ double Ri[KM * KM];
  __shared__ double Xs[kGramRows * KM];
  const int b = blockIdx.y, c = blockIdx.x, nch = gridDim.x;
  const int64_t r0 = (int64_t)c * kGramRows;
  const int rows = (int)min<int64_t>(kGramRows, d - r0);
  const int64_t base = (int64_t)b * d * k + r0 * k;
  load_tile<4 * KC>(X + base, rows * k, Xs);
  if constexpr (FACTOR) {
    static_assert(KC == 1, "in-kernel factorization only for k <= 16");
    __shared__ double G[KM * KM];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    sum_partials(rin, b, nch_in, k, G);
    __syncthreads();
    chol_inv_wave<KM>(G, Ri, k, &bad);
    if (threadIdx.x == 0 && c == 0 && bad && flags != nullptr) flags[b] = 1;
  } else {
    load_tile<KC * KC>(rin + (int64_t)b * k * k, k * k, Ri);
    __syncthreads();
  }
  double res[KC][4];
  tile_times_s<KC>(Xs, Ri, rows, k, true, res);
  __syncthreads();   // every wave has read Xs; it now holds the chunk of Q
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int bj = 0; bj < KC; ++bj)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int r = 16 * w + 4 * t + (lane >> 4), j = 16 * bj + (lane & 15);
      if (r < rows && j < k) {
        const double v = res[bj][t];
        Q[base + (int64_t)r * k + j] = v;
        if (zw != nullptr) zw[base + (int64_t)r * k + j] = (TW)v;
        Xs[r * k + j] = v;
      }
    }
  if (gout != nullptr) {
    __syncthreads();
    gram_tile<KC>(Xs, Xs, rows, k, gout + ((int64_t)b * nch + c) * k * k);
  }
}


// grid (nch, batch): partial column dots of chunk c: part[(b*nch + c)*k + j].
__global__ void __launch_bounds__(kBlock)
diag_dot_kernel(int64_t d, int k, const double* __restrict__ Zi, const double* __restrict__ Zb,
                double* __restrict__ part) {
  __shared__ double red[kBlock];
  const int b = blockIdx.y, c = blockIdx.x, nch = gridDim.x;
  const int64_t r0 = (int64_t)c * kGramRows;
  const int rows = (int)min<int64_t>(kGramRows, d - r0);
  // thread t: column j = t % k, rows t / k, t / k + (kBlock / k), ...
  const int per = kBlock / k;             // threads per column (k <= 64)
  const int j = threadIdx.x % k, r = threadIdx.x / k;
  double s = 0.0;
  if (r < per)
    for (int rr = r; rr < rows; rr += per)
      s = fma(Zi[(int64_t)b * d * k + (r0 + rr) * k + j], Zb[(r0 + rr) * k + j], s);
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < k) {
    double t = 0.0;
    for (int q = 0; q < per; ++q) t += red[q * k + threadIdx.x];
    part[((int64_t)b * nch + c) * k + threadIdx.x] = t;
  }
}

// grid (nch, batch): sign of the summed dots, applied to chunk c of Zi (and zw).
template <typename TW>
__global__ void __launch_bounds__(kBlock)
sign_apply_kernel(int64_t d, int k, const double* __restrict__ part, double* __restrict__ Zi,
                  TW* __restrict__ zw, int8_t* __restrict__ sgn) {
  __shared__ double sg[kMaxK];
  const int b = blockIdx.y, c = blockIdx.x, nch = gridDim.x;
  if (threadIdx.x < k) {
    double t = 0.0;
    for (int q = 0; q < nch; ++q) t += part[((int64_t)b * nch + q) * k + threadIdx.x];
    const double v = (t >= 0.0) ? 1.0 : -1.0;
    sg[threadIdx.x] = v;
    if (c == 0 && sgn != nullptr) sgn[b * k + threadIdx.x] = (v > 0.0) ? (int8_t)1 : (int8_t)-1;
  }
  __syncthreads();
  const int64_t r0 = (int64_t)c * kGramRows;
  const int rows = (int)min<int64_t>(kGramRows, d - r0);
  const int64_t base = (int64_t)b * d * k + r0 * k;
  for (int e = threadIdx.x; e < rows * k; e += kBlock) {
    const double v = Zi[base + e] * sg[e % k];
    Zi[base + e] = v;
    if (zw != nullptr) zw[base + e] = (TW)v;
  }
}

// ---------------------------------------------------------------------------
// Q_b = X_b S_b (S upper triangular when `upper`); grid (ceil(d / 64), batch)
// ---------------------------------------------------------------------------
template <typename TW, int KC>
__global__ void __launch_bounds__(kBlock)
right_mult_kernel(int64_t d, int k, const double* __restrict__ X, const double* __restrict__ S,
                  int64_t s_stride, int upper, double* __restrict__ Q, TW* __restrict__ zw) {
  // 64-row tile of X and S staged in LDS, the product on FP64 matrix cores
  constexpr int TR = 64;
  __shared__ double Ss[kMaxK * kMaxK];
  __shared__ double Xs[TR * kMaxK];
  const int b = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * TR;
  const int rows = (int)min<int64_t>(TR, d - r0);
  const double* Sb = S + b * s_stride;
  const double* Xb = X + (int64_t)b * d * k + r0 * k;
  load_tile<KC * KC>(Sb, k * k, Ss);
  load_tile<4 * KC>(Xb, rows * k, Xs);
  __syncthreads();
  double res[KC][4];
  tile_times_s<KC>(Xs, Ss, rows, k, upper != 0, res);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int bj = 0; bj < KC; ++bj)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int r = 16 * w + 4 * t + (lane >> 4), j = 16 * bj + (lane & 15);
      if (r < rows && j < k) {
        const int64_t o = (int64_t)b * d * k + (r0 + r) * k + j;
        if (Q != nullptr) Q[o] = res[bj][t];
        if (zw != nullptr) zw[o] = (TW)res[bj][t];
      }
    }
}

template <typename TW>
__global__ void to_working_kernel(int64_t count, const double* __restrict__ X, TW* __restrict__ zw) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) zw[e] = (TW)X[e];
}

// ---------------------------------------------------------------------------
// sign-fixing: sgn[b][j] = sign(<Zi[:,j], Zb[:,j]>), sgn(0) = +1
// ---------------------------------------------------------------------------
__global__ void sign_from_gram_kernel(int batch, int nchunks, int k, const double* __restrict__ part,
                                      int8_t* __restrict__ sgn) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= batch * k) return;
  const int b = t / k, j = t - (t / k) * k;
  const int kk = k * k;
  double s = 0.0;
  const double* p = part + (int64_t)b * nchunks * kk + j * k + j;
  for (int c = 0; c < nchunks; ++c) s += p[(int64_t)c * kk];
  sgn[t] = (s >= 0.0) ? (int8_t)1 : (int8_t)-1;
}


// ---------------------------------------------------------------------------
// Jacobi helpers (one workgroup, matrices in LDS)
// ---------------------------------------------------------------------------

// Round-robin ("circle") pairing: step s of kk-1, pair i of kk/2 -> (p, q), p < q.
__device__ inline void rr_pair(int kk, int s, int i, int* p, int* q) {
  int a, b;
  if (i == 0) {
    a = kk - 1;
    b = s;
  } else {
    a = (s + i) % (kk - 1);
    b = (s - i + (kk - 1)) % (kk - 1);
  }
  *p = min(a, b);
  *q = max(a, b);
}

// Rotation (c, s) that annihilates the (p,q) entry of the symmetric 2x2 block
// [[app, apq], [apq, aqq]] (Golub & Van Loan, symmetric Schur decomposition).
__device__ inline void sym_schur2(double app, double aqq, double apq, double* c, double* s) {
  if (apq == 0.0) {
    *c = 1.0;
    *s = 0.0;
    return;
  }
  const double tau = (aqq - app) / (2.0 * apq);
  const double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                 : -1.0 / (-tau + sqrt(1.0 + tau * tau));
  *c = 1.0 / sqrt(1.0 + t * t);
  *s = t * (*c);
}

// Largest eigenvalue of the symmetric positive semidefinite k x k matrix G in
// the LDS array A (overwritten; B is LDS scratch of the same size), by repeated
// squaring: A_0 = G / s_0 and A_i = A_{i-1}^2 / s_i, with s_i the trace that
// gives A_i trace one.  Then tr(G^(2^j)) = prod_{i <= j} s_i^(2^(j-i)), and
//   lambda_max <= (tr G^(2^j))^(2^-j) = s_0 s_1^(1/2) ... s_j^(2^-j)
//              <= mult^(2^-j) lambda_max,
// mult being the number of eigenvalues that survive the squarings next to
// lambda_max (at most k = 64).  48 squarings bound the overestimate by
// 64^(2^-48) - 1 < 1.5e-14; the squaring stops early once a trace is one to
// rounding (A is then a rank-one projector and every later s_i is one).  The
// product is evaluated as s_0 sqrt(s_1 sqrt(s_2 ...)) from the innermost
// factor.  Each rounding error enters with weight 2^-i, so the relative error
// stays a few ulps.  A zero trace gives 0 and a NaN trace NaN.  Every thread
// gets the value.  A^2 = A^T A is the Gram tile of A with itself (A symmetric).
constexpr int kSquarings = 48;

template <int KC>
__device__ double lam_max_psd(double* A, double* B, int k) {
  __shared__ double sv[kSquarings + 1];
  const int kk = k * k;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int j = 0; j < k; ++j) t += A[j * k + j];
    sv[0] = t;
  }
  __syncthreads();
  const double s0 = sv[0];
  if (s0 != s0) return s0;
  if (!(s0 > 0.0)) return 0.0;
  for (int e = threadIdx.x; e < kk; e += kBlock) A[e] /= s0;
  __syncthreads();
  double* cur = A;
  double* nxt = B;
  int last = 0;
  for (int i = 1; i <= kSquarings; ++i) {
    gram_tile<KC>(cur, cur, k, k, nxt);
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int j = 0; j < k; ++j) t += nxt[j * k + j];
      sv[i] = t;
    }
    __syncthreads();
    const double s = sv[i];
    for (int e = threadIdx.x; e < kk; e += kBlock) nxt[e] /= s;
    __syncthreads();
    double* sw = cur;
    cur = nxt;
    nxt = sw;
    last = i;
    if (fabs(s - 1.0) <= 4.0 * 2.220446049250313e-16) break;
  }
  double t = sv[last];
  for (int q = last - 1; q >= 1; --q) t = sv[q] * sqrt(t);
  return last >= 1 ? s0 * sqrt(t) : s0;
}

// Parallel cyclic Jacobi on the symmetric k x k LDS matrix S; V (k x k, LDS,
// may be NULL) accumulates the rotations.  On exit diag(S) holds eigenvalues.
__device__ void jacobi_sym_lds(double* S, double* V, int k, double* cs, double* sn, int* flag) {
  const int kk = k + (k & 1);
  const int npairs = kk / 2;
  if (V != nullptr)
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) V[e] = (e / k == e % k) ? 1.0 : 0.0;
  __shared__ double roff[kBlock], rtot[kBlock];
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    // convergence test on the off-diagonal mass (per-thread sums, then a tree
    // in a fixed order; the launch has kBlock threads)
    {
      double off = 0.0, tot = 0.0;
      for (int e = threadIdx.x; e < k * k; e += kBlock) {
        const double v = S[e] * S[e];
        tot += v;
        if (e / k != e % k) off += v;
      }
      roff[threadIdx.x] = off;
      rtot[threadIdx.x] = tot;
      __syncthreads();
      for (int h = kBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
          roff[threadIdx.x] += roff[threadIdx.x + h];
          rtot[threadIdx.x] += rtot[threadIdx.x + h];
        }
        __syncthreads();
      }
      if (threadIdx.x == 0) *flag = (roff[0] <= 1e-30 * rtot[0]) ? 1 : 0;
    }
    __syncthreads();
    if (*flag) break;
    __syncthreads();
    for (int st = 0; st < kk - 1; ++st) {
      for (int i = threadIdx.x; i < npairs; i += blockDim.x) {
        int p, q;
        rr_pair(kk, st, i, &p, &q);
        double c = 1.0, s = 0.0;
        if (q < k) sym_schur2(S[p * k + p], S[q * k + q], S[p * k + q], &c, &s);
        cs[i] = c;
        sn[i] = s;
      }
      __syncthreads();
      // columns: S <- S J, V <- V J
      for (int t = threadIdx.x; t < npairs * k; t += blockDim.x) {
        const int i = t / k, r = t - (t / k) * k;
        int p, q;
        rr_pair(kk, st, i, &p, &q);
        if (q >= k) continue;
        const double c = cs[i], s = sn[i];
        const double sp = S[r * k + p], sq = S[r * k + q];
        S[r * k + p] = c * sp - s * sq;
        S[r * k + q] = s * sp + c * sq;
        if (V != nullptr) {
          const double vp = V[r * k + p], vq = V[r * k + q];
          V[r * k + p] = c * vp - s * vq;
          V[r * k + q] = s * vp + c * vq;
        }
      }
      __syncthreads();
      // rows: S <- J^T S
      for (int t = threadIdx.x; t < npairs * k; t += blockDim.x) {
        const int i = t / k, r = t - (t / k) * k;
        int p, q;
        rr_pair(kk, st, i, &p, &q);
        if (q >= k) continue;
        const double c = cs[i], s = sn[i];
        const double sp = S[p * k + r], sq = S[q * k + r];
        S[p * k + r] = c * sp - s * sq;
        S[q * k + r] = s * sp + c * sq;
      }
      __syncthreads();
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Orthogonal Procrustes factor O_b = W1 W2^T of C_b = Z_b_i^T Z_base (Eq. (opt:o)),
// i.e. the orthogonal polar factor C (C^T C)^{-1/2}: one workgroup per matrix,
// Newton-Schulz iteration X <- X (3I - X^T X) / 2 from X_0 = C / s, s =
// sqrt(max row sum of |C^T C|) >= sigma_max(C), which converges (quadratically
// at the end) for every nonsingular C; it stops one iteration after
// max|X^T X - I| <= 1e-13.  A C that does not converge within the cap (singular
// or nearly so, where O is not unique) adds one to *flags.  grid (batch)
// ---------------------------------------------------------------------------
template <int KC>
__global__ void __launch_bounds__(kBlock)
polar_kernel(int nchunks, int k, const double* part, double* O, int32_t* flags) {
  __shared__ double X[kMaxK * kMaxK];
  __shared__ double A[kMaxK * kMaxK];
  __shared__ double red[kMaxK];
  __shared__ int off;
  const int b = blockIdx.x;
  const int kk = k * k;
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  sum_partials(part, b, nchunks, k, X);
  __syncthreads();
  // scale: s^2 = max_i sum_j |(C^T C)_ij|
  gram_tile<KC>(X, X, k, k, A);
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += kBlock) {
    double rs = 0.0;
    for (int j = 0; j < k; ++j) rs += fabs(A[i * k + j]);
    red[i] = rs;
  }
  __syncthreads();
  double s2 = 0.0;
  for (int i = 0; i < k; ++i) s2 = fmax(s2, red[i]);
  const double inv_s = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
  __syncthreads();
  for (int e = threadIdx.x; e < kk; e += kBlock) X[e] *= inv_s;
  __syncthreads();
  bool converged = false;
  int extra = -1;   // iterations still to run after convergence
  for (int it = 0; it < 120; ++it) {
    gram_tile<KC>(X, X, k, k, A);     // A = X^T X
    if (threadIdx.x == 0) off = 0;
    __syncthreads();
    if (extra < 0) {
      for (int e = threadIdx.x; e < kk; e += kBlock) {
        const double dv = A[e] - ((e / k == e % k) ? 1.0 : 0.0);
        if (!(fabs(dv) <= 1e-13)) off = 1;   // benign race: every writer stores 1
      }
      __syncthreads();
      if (off == 0) extra = 1;
    }
    if (extra == 0) {
      converged = true;
      break;
    }
    if (extra > 0) --extra;
    // X <- 1.5 X - 0.5 X A
    double acc[KC][KC];
#pragma unroll
    for (int a = 0; a < KC; ++a)
#pragma unroll
      for (int c = 0; c < KC; ++c) acc[a][c] = 0.0;
    for (int l = 0; l < k; ++l) {
      double xv[KC], av[KC];
#pragma unroll
      for (int a = 0; a < KC; ++a) xv[a] = (ty + 16 * a < k) ? X[(ty + 16 * a) * k + l] : 0.0;
#pragma unroll
      for (int c = 0; c < KC; ++c) av[c] = (tx + 16 * c < k) ? A[l * k + tx + 16 * c] : 0.0;
#pragma unroll
      for (int a = 0; a < KC; ++a)
#pragma unroll
        for (int c = 0; c < KC; ++c) acc[a][c] = fma(xv[a], av[c], acc[a][c]);
    }
    __syncthreads();   // every thread has read X
#pragma unroll
    for (int a = 0; a < KC; ++a)
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        const int i = ty + 16 * a, j = tx + 16 * c;
        if (i < k && j < k) X[i * k + j] = 1.5 * X[i * k + j] - 0.5 * acc[a][c];
      }
    __syncthreads();
  }
  if (threadIdx.x == 0 && flags != nullptr && (!converged || s2 == 0.0)) atomicAdd(flags, 1);
  double* Ob = O + (int64_t)b * kk;
  for (int e = threadIdx.x; e < kk; e += kBlock) Ob[e] = X[e];
}

// ---------------------------------------------------------------------------
// aggregation Y = scale * sum_i Yi
// ---------------------------------------------------------------------------
__global__ void aggregate_kernel(int m, int64_t dk, const double* __restrict__ Yi, double scale,
                                 double* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= dk) return;
  double s = 0.0;
  for (int i = 0; i < m; ++i) s += Yi[(int64_t)i * dk + e];
  Y[e] = scale * s;
}

// ---------------------------------------------------------------------------
// symmetric eigen-decomposition of H (sum of partials), sorted descending
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
sym_eig_kernel(int nchunks, int k, const double* __restrict__ part, double* __restrict__ lam,
               double* __restrict__ Vout) {
  __shared__ double S[kMaxK * kMaxK];
  __shared__ double V[kMaxK * kMaxK];
  __shared__ double cs[kMaxK / 2 + 1], sn[kMaxK / 2 + 1];
  __shared__ int flag;
  __shared__ int order[kMaxK];
  sum_partials(part, 0, nchunks, k, S);
  __syncthreads();
  // symmetrise: H = (H + H^T)/2
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int i = e / k, j = e - (e / k) * k;
    if (i < j) {
      const double v = 0.5 * (S[i * k + j] + S[j * k + i]);
      S[i * k + j] = v;
      S[j * k + i] = v;
    }
  }
  __syncthreads();
  jacobi_sym_lds(S, V, k, cs, sn, &flag);
  if (threadIdx.x == 0) {
    // selection order by descending eigenvalue, ties to the lower index
    bool used[kMaxK];
    for (int j = 0; j < k; ++j) used[j] = false;
    for (int o = 0; o < k; ++o) {
      int best = -1;
      for (int j = 0; j < k; ++j)
        if (!used[j] && (best < 0 || S[j * k + j] > S[best * k + best])) best = j;
      used[best] = true;
      order[o] = best;
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += blockDim.x) lam[j] = S[order[j] * k + order[j]];
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int r = e / k, j = e - (e / k) * k;
    Vout[e] = V[r * k + order[j]];
  }
}

// ---------------------------------------------------------------------------
// sin theta_k(Z, U) = sqrt(lambda_max(W^T W)), W = U - Z (Z^T U); one workgroup
// per Z (Z + blockIdx.x z_stride, result out[blockIdx.x]).  Z is d x r (the
// iterate, r >= k columns), U is d x k (the reference).  With diff (r == k) the
// kernel returns ||Z - U||_2 instead (W = Z - U).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
sin_theta_kernel(int64_t d, int r, int k, const double* __restrict__ Zs, int64_t z_stride,
                 int diff, const double* __restrict__ U, double* __restrict__ out,
                 double* __restrict__ hist, int32_t* __restrict__ ctr) {
  const double* Z = Zs + (int64_t)blockIdx.x * z_stride;
  __shared__ double C[kMaxK * kMaxK];
  __shared__ double G[kMaxK * kMaxK];
  __shared__ double Wt[16 * kMaxK];
  const int kk = k * k;
  // C = Z^T U (r x k)
  for (int e = threadIdx.x; e < (diff ? 0 : r * k); e += blockDim.x) {
    const int i = e / k, j = e - (e / k) * k;
    double s = 0.0;
    for (int64_t q = 0; q < d; ++q) s = fma(Z[q * r + i], U[q * k + j], s);
    C[e] = s;
  }
  double g[(kMaxK * kMaxK) / kBlock];
#pragma unroll
  for (int q = 0; q < (kMaxK * kMaxK) / kBlock; ++q) g[q] = 0.0;
  __syncthreads();
  for (int64_t r0 = 0; r0 < d; r0 += 16) {
    const int rows = (int)min<int64_t>(16, d - r0);
    for (int e = threadIdx.x; e < rows * k; e += blockDim.x) {
      const int rr = e / k, j = e - (e / k) * k;
      const double* zr = Z + (r0 + rr) * r;
      double s = U[(r0 + rr) * k + j];
      if (diff) {
        s = zr[j] - s;
      } else {
        for (int l = 0; l < r; ++l) s = fma(-zr[l], C[l * k + j], s);
      }
      Wt[e] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (kMaxK * kMaxK) / kBlock; ++q) {
      const int e = threadIdx.x + q * kBlock;
      if (e < kk) {
        const int i = e / k, j = e - (e / k) * k;
        double s = g[q];
        for (int rr = 0; rr < rows; ++rr) s = fma(Wt[rr * k + i], Wt[rr * k + j], s);
        g[q] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < (kMaxK * kMaxK) / kBlock; ++q) {
    const int e = threadIdx.x + q * kBlock;
    if (e < kk) G[e] = g[q];
  }
  __syncthreads();
  const double lam = lam_max_psd<kMaxK / 16>(G, C, k);   // C is free again
  if (threadIdx.x == 0) {
    const double v = sqrt(fmax(lam, 0.0));
    if (out != nullptr) out[blockIdx.x] = v;
    if (hist != nullptr) {
      hist[*ctr] = v;
      *ctr = *ctr + 1;
    }
  }
}

// ---------------------------------------------------------------------------
// The same sin theta_k(Z, U) over many workgroups (the per-round form): the
// O(d r k) products run per 64-row chunk and only the k x k eigenvalue problem
// runs in one workgroup.
//   1. partial C_c = Z_c^T U_c per chunk            (sin_cross_kernel)
//   2. C = sum_c C_c                                  (sum_gram_kernel)
//   3. W_c = U_c - Z_c C, partial G_c = W_c^T W_c     (sin_resid_kernel)
//   4. G = sum_c G_c                                  (sum_gram_kernel)
//   5. sqrt(lambda_max(G))                            (sin_eig_kernel)
// ---------------------------------------------------------------------------

// out[i][j] = sum_{q < rows} Xs[q][i] Ws[q][j] (i < rx, j < kw; row strides rx
// and kw <= 16 KC) on FP64 matrix cores: wave w owns the 16 x 16 output blocks
// w, w + 4, ...; K = rows in steps of 4 with A[i][q] = X[r + q][16 bi + i] and
// B[q][j] = W[r + q][16 bj + j].
template <int KC>
__device__ void cross_tile(const double* Xs, int rx, const double* Ws, int kw, int rows,
                           double* out) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = lane & 15, q = lane >> 4;
  const int bx = (rx + 15) / 16, bw = (kw + 15) / 16;
  for (int blk = w; blk < bx * bw; blk += 4) {
    const int bi = blk / bw, bj = blk - (blk / bw) * bw;
    const int ci = 16 * bi + c, cj = 16 * bj + c;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int r = 0; r < rows; r += 4) {
      const int rr = r + q;
      const double a = (rr < rows && ci < rx) ? Xs[rr * rx + ci] : 0.0;
      const double b = (rr < rows && cj < kw) ? Ws[rr * kw + cj] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    // lane l holds entries (16 bi + 4t + l/16, 16 bj + l%16)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = 16 * bi + 4 * t + q, j = cj;
      if (i < rx && j < kw) out[i * kw + j] = acc[t];
    }
  }
}

// grid (ceil(d / 64)): part[c] = Z_c^T U_c (r x k) of the 64-row chunk c.
template <int KC>
__global__ void __launch_bounds__(kBlock)
sin_cross_kernel(int64_t d, int r, int k, const double* __restrict__ Z,
                 const double* __restrict__ U, double* __restrict__ part) {
  __shared__ double zs[kGramRows * kMaxK];
  __shared__ double us[kGramRows * kMaxK];
  const int c = blockIdx.x;
  const int64_t r0 = (int64_t)c * kGramRows;
  const int rows = (int)min<int64_t>(kGramRows, d - r0);
  load_tile<4 * KC>(Z + r0 * r, rows * r, zs);
  load_tile<4 * KC>(U + r0 * k, rows * k, us);
  __syncthreads();
  cross_tile<KC>(zs, r, us, k, rows, part + (int64_t)c * r * k);
}

// grid (ceil(d / 64)): W_c = U_c - Z_c C for the 64-row chunk c and its Gram
// partial gpart[c] = W_c^T W_c (k x k).  The product runs on FP64 matrix cores
// with the accumulators started at U_c: wave w owns rows 16w..16w+15, lane l,
// block bj, t holds W entry (16w + 4t + l/16, 16 bj + l%16).
template <int KC>
__global__ void __launch_bounds__(kBlock)
sin_resid_kernel(int64_t d, int r, int k, const double* __restrict__ Z,
                 const double* __restrict__ U, const double* __restrict__ C,
                 double* __restrict__ gpart) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  __shared__ double cm[kMaxK * kMaxK];
  __shared__ double zs[kGramRows * kMaxK];
  __shared__ double ws[kGramRows * kMaxK];
  const int c = blockIdx.x;
  const int64_t r0 = (int64_t)c * kGramRows;
  const int rows = (int)min<int64_t>(kGramRows, d - r0);
  load_tile<KC * KC>(C, r * k, cm);
  load_tile<4 * KC>(Z + r0 * r, rows * r, zs);
  load_tile<4 * KC>(U + r0 * k, rows * k, ws);
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int cl = lane & 15, q = lane >> 4;
  const int row = 16 * w + cl;
  d4 acc[KC];
#pragma unroll
  for (int bj = 0; bj < KC; ++bj)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int rr = 16 * w + 4 * t + q, j = 16 * bj + cl;
      acc[bj][t] = (rr < rows && j < k) ? ws[rr * k + j] : 0.0;
    }
  for (int l = 0; l < r; l += 4) {
    const int lq = l + q;
    const double a = (row < rows && lq < r) ? -zs[row * r + lq] : 0.0;
#pragma unroll
    for (int bj = 0; bj < KC; ++bj) {
      const int j = 16 * bj + cl;
      const double b = (lq < r && j < k) ? cm[lq * k + j] : 0.0;
      acc[bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[bj], 0, 0, 0);
    }
  }
  // each W entry is read (above) and written (here) by the lane that owns it
#pragma unroll
  for (int bj = 0; bj < KC; ++bj)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int rr = 16 * w + 4 * t + q, j = 16 * bj + cl;
      if (rr < rows && j < k) ws[rr * k + j] = acc[bj][t];
    }
  __syncthreads();
  gram_tile<KC>(ws, ws, rows, k, gpart + (int64_t)c * k * k);
}

// one workgroup: out = sqrt(lambda_max(G)) of the symmetric positive
// semidefinite k x k G (repeated squaring); if hist != NULL also
// hist[*ctr] = out, then ++*ctr.
template <int KC>
__global__ void __launch_bounds__(kBlock)
sin_eig_kernel(int k, const double* __restrict__ Gin, double* __restrict__ out,
               double* __restrict__ hist, int32_t* __restrict__ ctr) {
  __shared__ double G[kMaxK * kMaxK];
  __shared__ double B[kMaxK * kMaxK];
  for (int e = threadIdx.x; e < k * k; e += kBlock) G[e] = Gin[e];
  __syncthreads();
  const double lam = lam_max_psd<KC>(G, B, k);
  if (threadIdx.x == 0) {
    const double v = sqrt(fmax(lam, 0.0));
    if (out != nullptr) out[0] = v;
    if (hist != nullptr) {
      hist[*ctr] = v;
      *ctr = *ctr + 1;
    }
  }
}

__global__ void fill_i32_kernel(int32_t* p, int count, int32_t v) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = v;
}

inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

// Result cells of lp_sin_theta: one per call in flight (each GPU holds its own
// copy of the array; a call takes a free cell under a host lock and hands it
// back after it has synchronised, so concurrent callers never share a cell).
__device__ double g_sin_slots[kSinSlots];

hipError_t sin_slot_address(double** p) {
  return hipGetSymbolAddress((void**)p, HIP_SYMBOL(g_sin_slots));
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_cross_gram(int batch, int64_t d, int k, const double* X, int64_t x_stride,
                             const double* W, int64_t w_stride, double* gram_part, hipStream_t s) {
  dim3 grid(nblk(d, kGramRows), batch);
  if (k <= 16)
    cross_gram_kernel<1><<<grid, kBlock, 0, s>>>(d, k, X, x_stride, W, w_stride, gram_part);
  else if (k <= 32)
    cross_gram_kernel<2><<<grid, kBlock, 0, s>>>(d, k, X, x_stride, W, w_stride, gram_part);
  else
    cross_gram_kernel<4><<<grid, kBlock, 0, s>>>(d, k, X, x_stride, W, w_stride, gram_part);
  return hipGetLastError();
}


hipError_t launch_right_mult(int batch, int64_t d, int k, const double* X, const double* S,
                             int64_t s_stride, bool upper, double* Q, void* zw, size_t zw_bytes,
                             hipStream_t s) {
  dim3 grid(nblk(d, 64), batch);
  const int up = upper ? 1 : 0;
  if (zw == nullptr || zw_bytes == 8) {
    if (k <= 16) right_mult_kernel<double, 1><<<grid, kBlock, 0, s>>>(d, k, X, S, s_stride, up, Q, (double*)zw);
    else if (k <= 32) right_mult_kernel<double, 2><<<grid, kBlock, 0, s>>>(d, k, X, S, s_stride, up, Q, (double*)zw);
    else right_mult_kernel<double, 4><<<grid, kBlock, 0, s>>>(d, k, X, S, s_stride, up, Q, (double*)zw);
  } else {
    if (k <= 16) right_mult_kernel<float, 1><<<grid, kBlock, 0, s>>>(d, k, X, S, s_stride, up, Q, (float*)zw);
    else if (k <= 32) right_mult_kernel<float, 2><<<grid, kBlock, 0, s>>>(d, k, X, S, s_stride, up, Q, (float*)zw);
    else right_mult_kernel<float, 4><<<grid, kBlock, 0, s>>>(d, k, X, S, s_stride, up, Q, (float*)zw);
  }
  return hipGetLastError();
}

hipError_t launch_to_working(const Plan& P, int batch, int64_t d, int k, const double* X, void* Zw,
                             hipStream_t s) {
  const int64_t count = (int64_t)batch * d * k;
  if (P.zw_bytes == 8)
    to_working_kernel<double><<<nblk(count, kBlock), kBlock, 0, s>>>(count, X, (double*)Zw);
  else
    to_working_kernel<float><<<nblk(count, kBlock), kBlock, 0, s>>>(count, X, (float*)Zw);
  return hipGetLastError();
}

hipError_t launch_sign_from_gram(int batch, int nchunks, int k, const double* gram_part,
                                 int8_t* sgn, hipStream_t s) {
  sign_from_gram_kernel<<<nblk((int64_t)batch * k, kBlock), kBlock, 0, s>>>(batch, nchunks, k,
                                                                           gram_part, sgn);
  return hipGetLastError();
}


hipError_t launch_procrustes(int batch, int nchunks, int k, const double* gram_part, double* O,
                             int32_t* flags, hipStream_t s) {
  const double* src = gram_part;
  int nch = nchunks;
  if (k > 16 && nchunks > 1) {
    // sum the partials with a wide launch into O (the kernel reads O[b] in full
    // before it writes O[b])
    sum_gram_kernel<<<dim3(nblk((int64_t)k * k, kBlock), batch), kBlock, 0, s>>>(nchunks, k * k,
                                                                               gram_part, O);
    src = O;
    nch = 1;
  }
  if (k <= 16)
    polar_kernel<1><<<batch, kBlock, 0, s>>>(nch, k, src, O, flags);
  else if (k <= 32)
    polar_kernel<2><<<batch, kBlock, 0, s>>>(nch, k, src, O, flags);
  else
    polar_kernel<4><<<batch, kBlock, 0, s>>>(nch, k, src, O, flags);
  return hipGetLastError();
}

hipError_t launch_aggregate(int m, int64_t d, int k, const double* Yi, double scale, double* Y,
                            hipStream_t s) {
  const int64_t dk = d * k;
  aggregate_kernel<<<nblk(dk, kBlock), kBlock, 0, s>>>(m, dk, Yi, scale, Y);
  return hipGetLastError();
}

hipError_t launch_sym_eig(int nchunks, int k, const double* gram_part, double* lam, double* V,
                          hipStream_t s) {
  sym_eig_kernel<<<1, kBlock, 0, s>>>(nchunks, k, gram_part, lam, V);
  return hipGetLastError();
}

hipError_t launch_sin_theta(int64_t d, int r, int k, const double* Z, const double* U,
                            double* out, double* hist, int32_t* ctr, hipStream_t s) {
  sin_theta_kernel<<<1, kBlock, 0, s>>>(d, r, k, Z, 0, 0, U, out, hist, ctr);
  return hipGetLastError();
}

template <int KC>
static void sin_theta_chunked_kc(int64_t d, int r, int k, const double* Z, const double* U,
                                 double* scratch, double* out, double* hist, int32_t* ctr,
                                 hipStream_t s) {
  const int nch = nblk(d, kGramRows);
  const int rk = r * k, kk = k * k;
  double* cpart = scratch;
  double* C = cpart + (int64_t)nch * rk;
  double* gpart = C + rk;
  double* G = gpart + (int64_t)nch * kk;
  sin_cross_kernel<KC><<<nch, kBlock, 0, s>>>(d, r, k, Z, U, cpart);
  sum_gram_kernel<<<dim3(nblk(rk, kBlock), 1), kBlock, 0, s>>>(nch, rk, cpart, C);
  sin_resid_kernel<KC><<<nch, kBlock, 0, s>>>(d, r, k, Z, U, C, gpart);
  sum_gram_kernel<<<dim3(nblk(kk, kBlock), 1), kBlock, 0, s>>>(nch, kk, gpart, G);
  sin_eig_kernel<KC><<<1, kBlock, 0, s>>>(k, G, out, hist, ctr);
}

size_t sin_theta_scratch_doubles(int64_t d, int r, int k) {
  const int64_t nch = (d + kGramRows - 1) / kGramRows;
  return (size_t)((nch + 1) * ((int64_t)r * k + (int64_t)k * k));
}

hipError_t launch_sin_theta_chunked(int64_t d, int r, int k, const double* Z, const double* U,
                                    double* scratch, double* out, double* hist, int32_t* ctr,
                                    hipStream_t s) {
  if (r <= 16) sin_theta_chunked_kc<1>(d, r, k, Z, U, scratch, out, hist, ctr, s);
  else if (r <= 32) sin_theta_chunked_kc<2>(d, r, k, Z, U, scratch, out, hist, ctr, s);
  else if (r <= 48) sin_theta_chunked_kc<3>(d, r, k, Z, U, scratch, out, hist, ctr, s);
  else sin_theta_chunked_kc<4>(d, r, k, Z, U, scratch, out, hist, ctr, s);
  return hipGetLastError();
}

// rho (Definition 3) of the m local iterates Zi (m x d x k) against partition 0's:
// per partition ||Z_i - Z_1||_2, or with OPT sin theta_max(Z_i, Z_1) turned into
// min_O ||Z_i O - Z_1||_2 = 2 sin(theta_max / 2); the maximum is appended to
// hist[*ctr].  m == 0 appends 0 (rounds of one local step).
__global__ void rho_finish_kernel(int m, int opt, const double* __restrict__ part,
                                  double* __restrict__ hist, int32_t* __restrict__ ctr) {
  if (threadIdx.x != 0) return;
  double v = 0.0;
  for (int i = 0; i < m; ++i) v = fmax(v, part[i]);
  if (opt) {
    const double sn = fmin(v, 1.0);
    v = sn * sqrt(2.0 / (1.0 + sqrt(fmax(0.0, 1.0 - sn * sn))));
  }
  hist[*ctr] = v;
  *ctr = *ctr + 1;
}

hipError_t launch_rho(int m, int64_t d, int k, bool opt, const double* Zi, double* part,
                      double* hist, int32_t* ctr, hipStream_t s) {
  if (m > 0)
    sin_theta_kernel<<<m, kBlock, 0, s>>>(d, k, k, Zi, d * k, opt ? 0 : 1, Zi, part, nullptr,
                                          nullptr);
  rho_finish_kernel<<<1, 64, 0, s>>>(m, opt ? 1 : 0, part, hist, ctr);
  return hipGetLastError();
}



hipError_t launch_reduce_gram(const Plan& P, int k, const void* part, const int32_t* slot_off,
                              double* Yi, double* gram, int b0, int nb, hipStream_t s) {
  if (nb < 1) return hipSuccess;
  dim3 grid(nblk(P.d, kGramRows), nb);
  if (P.acc_bytes == 8) {
    const double* pp = (const double*)part;
    if (k <= 16) reduce_gram_kernel<double, 16><<<grid, kBlock, 0, s>>>(P.d, k, b0, pp, slot_off, Yi, gram);
    else if (k <= 32) reduce_gram_kernel<double, 32><<<grid, kBlock, 0, s>>>(P.d, k, b0, pp, slot_off, Yi, gram);
    else reduce_gram_kernel<double, kMaxK><<<grid, kBlock, 0, s>>>(P.d, k, b0, pp, slot_off, Yi, gram);
  } else {
    const float* pp = (const float*)part;
    if (k <= 16) reduce_gram_kernel<float, 16><<<grid, kBlock, 0, s>>>(P.d, k, b0, pp, slot_off, Yi, gram);
    else if (k <= 32) reduce_gram_kernel<float, 32><<<grid, kBlock, 0, s>>>(P.d, k, b0, pp, slot_off, Yi, gram);
    else reduce_gram_kernel<float, kMaxK><<<grid, kBlock, 0, s>>>(P.d, k, b0, pp, slot_off, Yi, gram);
  }
  return hipGetLastError();
}

hipError_t launch_aggregate_gram(int m, int64_t d, int k, const double* Yi, double scale, double* Y,
                                 double* gram, hipStream_t s) {
  dim3 grid(nblk(d, kGramRows));
  if (k <= 16) aggregate_gram_kernel<16><<<grid, kBlock, 0, s>>>(m, d, k, Yi, scale, Y, gram);
  else if (k <= 32) aggregate_gram_kernel<32><<<grid, kBlock, 0, s>>>(m, d, k, Yi, scale, Y, gram);
  else aggregate_gram_kernel<kMaxK><<<grid, kBlock, 0, s>>>(m, d, k, Yi, scale, Y, gram);
  return hipGetLastError();
}







template <typename TW, int KM>
static hipError_t chol_solve_km(int batch, int64_t d, int k, int nch_in, const double* X,
                                const double* gin, double* rfac, double* Q, TW* zw, double* gout,
                                int32_t* flags, hipStream_t s) {
  const dim3 grid(nblk(d, kGramRows), batch);
  if constexpr (KM <= 16) {
    apply_gram_kernel<TW, 1, true><<<grid, kBlock, 0, s>>>(d, k, nch_in, X, gin, Q, zw, gout, flags);
  } else {
    // larger k: factor and invert once per matrix, then multiply the 64-row chunks
    // the Gram partials are summed by a wide launch first (one sum per entry,
    // all of them in parallel), then factored and inverted once per matrix
    double* gsum = rfac + (int64_t)batch * k * k;
    sum_gram_kernel<<<dim3(nblk((int64_t)k * k, kBlock), batch), kBlock, 0, s>>>(nch_in, k * k, gin, gsum);
    chol_inv_blocked_kernel<KM / 16><<<batch, kBlock, 0, s>>>(1, k, gsum, rfac, flags);
    apply_gram_kernel<TW, kc_of(KM), false><<<grid, kBlock, 0, s>>>(d, k, 0, X, rfac, Q, zw, gout,
                                                                     nullptr);
  }
  return hipGetLastError();
}

template <typename TW>
static hipError_t chol_solve_t(int batch, int64_t d, int k, int nch_in, const double* X,
                               const double* gin, double* rfac, double* Q, TW* zw, double* gout,
                               int32_t* flags, hipStream_t s) {
  if (k <= 16) return chol_solve_km<TW, 16>(batch, d, k, nch_in, X, gin, rfac, Q, zw, gout, flags, s);
  if (k <= 32) return chol_solve_km<TW, 32>(batch, d, k, nch_in, X, gin, rfac, Q, zw, gout, flags, s);
  return chol_solve_km<TW, kMaxK>(batch, d, k, nch_in, X, gin, rfac, Q, zw, gout, flags, s);
}

int chol_solve_chunks(int64_t d, int /*k*/) { return nblk(d, kGramRows); }

hipError_t launch_chol_solve(int batch, int64_t d, int k, int nch_in, const double* X,
                             const double* gram_in, double* rfac, double* Q, void* zw,
                             size_t zw_bytes, double* gram_out, int32_t* flags, hipStream_t s) {
  if (zw == nullptr || zw_bytes == 8)
    return chol_solve_t<double>(batch, d, k, nch_in, X, gram_in, rfac, Q, (double*)zw, gram_out,
                                flags, s);
  return chol_solve_t<float>(batch, d, k, nch_in, X, gram_in, rfac, Q, (float*)zw, gram_out, flags,
                             s);
}

hipError_t launch_diag_dot(int batch, int64_t d, int k, const double* Zi, const double* Zb,
                           double* part, hipStream_t s) {
  dim3 grid(nblk(d, kGramRows), batch);
  diag_dot_kernel<<<grid, kBlock, 0, s>>>(d, k, Zi, Zb, part);
  return hipGetLastError();
}

hipError_t launch_sign_apply(int batch, int64_t d, int k, const double* part, double* Zi, void* zw,
                             size_t zw_bytes, int8_t* sgn, hipStream_t s) {
  dim3 grid(nblk(d, kGramRows), batch);
  if (zw == nullptr || zw_bytes == 8)
    sign_apply_kernel<double><<<grid, kBlock, 0, s>>>(d, k, part, Zi, (double*)zw, sgn);
  else
    sign_apply_kernel<float><<<grid, kBlock, 0, s>>>(d, k, part, Zi, (float*)zw, sgn);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int count, int32_t v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  fill_i32_kernel<<<nblk(count, kBlock), kBlock, 0, s>>>(p, count, v);
  return hipGetLastError();
}

}  // namespace lp
