// Small FP64 kernels of LocalPower: Gram matrices, Cholesky + triangular
// inverse (CholeskyQR2), right multiplication by k x k matrices, sign-fixing
// and orthogonal-Procrustes alignment, aggregation, Jacobi eigen/SVD and the
// sin-theta distance.  All of them work on d x k (k <= 64) FP64 row-major
// matrices, batched over the m partitions where the method batches them.
#include "lp_internal.h"

#include <cmath>

namespace lp {
namespace {

constexpr int kTile = 64;  // rows staged in LDS per step of the Gram kernel

// ---------------------------------------------------------------------------
// G_b(chunk) = X_b[rows]^T W_b[rows]  (k x k partial, chunk of kGramRows rows)
// grid: (nchunks, batch), block kBlock
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
cross_gram_kernel(int64_t d, int k, const double* __restrict__ X, int64_t x_stride,
                  const double* __restrict__ W, int64_t w_stride, double* __restrict__ out) {
  __shared__ double xs[kTile * kMaxK];
  __shared__ double ws[kTile * kMaxK];
  const int b = blockIdx.y;
  const int c = blockIdx.x;
  const int nchunks = gridDim.x;
  const int64_t r_begin = (int64_t)c * kGramRows;
  const int64_t r_end = min(d, r_begin + kGramRows);
  const double* Xb = X + b * x_stride;
  const double* Wb = W + b * w_stride;
  const int kk = k * k;
  double acc[(kMaxK * kMaxK) / kBlock];
#pragma unroll
  for (int e = 0; e < (kMaxK * kMaxK) / kBlock; ++e) acc[e] = 0.0;
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kTile) {
    const int rows = (int)min<int64_t>(kTile, r_end - r0);
    __syncthreads();
    for (int e = threadIdx.x; e < rows * k; e += kBlock) {
      xs[e] = Xb[r0 * k + e];
      ws[e] = Wb[r0 * k + e];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (kMaxK * kMaxK) / kBlock; ++q) {
      const int e = threadIdx.x + q * kBlock;
      if (e < kk) {
        const int i = e / k, j = e - (e / k) * k;
        double s = acc[q];
        for (int r = 0; r < rows; ++r) s = fma(xs[r * k + i], ws[r * k + j], s);
        acc[q] = s;
      }
    }
  }
  double* o = out + ((int64_t)b * nchunks + c) * kk;
#pragma unroll
  for (int q = 0; q < (kMaxK * kMaxK) / kBlock; ++q) {
    const int e = threadIdx.x + q * kBlock;
    if (e < kk) o[e] = acc[q];
  }
}

// Sum of the gram partials of batch b into an LDS k x k array (fixed order).
__device__ void sum_partials(const double* __restrict__ part, int b, int nchunks, int k,
                             double* G) {
  const int kk = k * k;
  for (int e = threadIdx.x; e < kk; e += blockDim.x) {
    double s = 0.0;
    const double* p = part + (int64_t)b * nchunks * kk + e;
    for (int c = 0; c < nchunks; ++c) s += p[(int64_t)c * kk];
    G[e] = s;
  }
}

// ---------------------------------------------------------------------------
// Cholesky G = R^T R (R upper, positive diagonal) and R^{-1}; grid (batch)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
chol_inv_kernel(int nchunks, int k, const double* __restrict__ part, double* __restrict__ rinv,
                int32_t* __restrict__ flags) {
  __shared__ double R[kMaxK * kMaxK];
  __shared__ double X[kMaxK * kMaxK];
  __shared__ int bad;
  const int b = blockIdx.x;
  if (threadIdx.x == 0) bad = 0;
  sum_partials(part, b, nchunks, k, R);
  __syncthreads();
  // left-looking Cholesky, row j of R at step j
  for (int j = 0; j < k; ++j) {
    if (threadIdx.x == 0) {
      double djj = R[j * k + j];
      for (int l = 0; l < j; ++l) djj -= R[l * k + j] * R[l * k + j];
      if (!(djj > 0.0) || !isfinite(djj)) {
        bad = 1;
        djj = 1.0;
      }
      R[j * k + j] = sqrt(djj);
    }
    __syncthreads();
    const double rjj = R[j * k + j];
    for (int c = j + 1 + threadIdx.x; c < k; c += blockDim.x) {
      double v = R[j * k + c];
      for (int l = 0; l < j; ++l) v -= R[l * k + j] * R[l * k + c];
      R[j * k + c] = v / rjj;
    }
    __syncthreads();
  }
  // inverse of the upper triangular R, one column per thread (back substitution)
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    X[c * k + c] = 1.0 / R[c * k + c];
    for (int i = c - 1; i >= 0; --i) {
      double s = 0.0;
      for (int l = i + 1; l <= c; ++l) s += R[i * k + l] * X[l * k + c];
      X[i * k + c] = -s / R[i * k + i];
    }
  }
  __syncthreads();
  double* out = rinv + (int64_t)b * k * k;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int i = e / k, c = e - (e / k) * k;
    double v = (i <= c) ? X[e] : 0.0;
    if (bad) v = (i == c) ? 1.0 : 0.0;
    out[e] = v;
  }
  if (threadIdx.x == 0 && flags != nullptr && bad) flags[b] = 1;
}

// ---------------------------------------------------------------------------
// Q_b = X_b S_b; grid (ceil(d*k / kBlock), batch)
// ---------------------------------------------------------------------------
template <typename TW>
__global__ void __launch_bounds__(kBlock)
right_mult_kernel(int64_t d, int k, const double* __restrict__ X, const double* __restrict__ S,
                  int64_t s_stride, int upper, double* __restrict__ Q, TW* __restrict__ zw) {
  __shared__ double Ss[kMaxK * kMaxK];
  const int b = blockIdx.y;
  const double* Sb = S + b * s_stride;
  for (int e = threadIdx.x; e < k * k; e += kBlock) Ss[e] = Sb[e];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= d * k) return;
  const int64_t r = e / k;
  const int j = (int)(e - r * k);
  const double* xr = X + (int64_t)b * d * k + r * k;
  const int lend = upper ? j + 1 : k;
  double s = 0.0;
  for (int l = 0; l < lend; ++l) s = fma(xr[l], Ss[l * k + j], s);
  if (Q != nullptr) Q[(int64_t)b * d * k + e] = s;
  if (zw != nullptr) zw[(int64_t)b * d * k + e] = (TW)s;
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

template <typename TW>
__global__ void apply_signs_kernel(int batch, int64_t d, int k, double* __restrict__ X,
                                   const int8_t* __restrict__ sgn, TW* __restrict__ zw) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)batch * d * k) return;
  const int64_t b = e / (d * k);
  const int j = (int)(e % k);
  const double v = X[e] * (double)sgn[b * k + j];
  X[e] = v;
  if (zw != nullptr) zw[e] = (TW)v;
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

// Parallel cyclic Jacobi on the symmetric k x k LDS matrix S; V (k x k, LDS,
// may be NULL) accumulates the rotations.  On exit diag(S) holds eigenvalues.
__device__ void jacobi_sym_lds(double* S, double* V, int k, double* cs, double* sn, int* flag) {
  const int kk = k + (k & 1);
  const int npairs = kk / 2;
  if (V != nullptr)
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) V[e] = (e / k == e % k) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    // convergence test on the off-diagonal mass
    if (threadIdx.x == 0) {
      double off = 0.0, tot = 0.0;
      for (int e = 0; e < k * k; ++e) {
        const double v = S[e] * S[e];
        tot += v;
        if (e / k != e % k) off += v;
      }
      *flag = (off <= 1e-30 * tot) ? 1 : 0;
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
// Orthogonal Procrustes O = W1 W2^T of C = W1 S W2^T (one-sided Jacobi); grid (batch)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
procrustes_kernel(int nchunks, int k, const double* __restrict__ part, double* __restrict__ O,
                  int32_t* __restrict__ flags) {
  __shared__ double X[kMaxK * kMaxK];
  __shared__ double V[kMaxK * kMaxK];
  __shared__ double nrm[kMaxK];
  __shared__ int rotated;
  const int b = blockIdx.x;
  sum_partials(part, b, nchunks, k, X);
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) V[e] = (e / k == e % k) ? 1.0 : 0.0;
  const int kk = k + (k & 1);
  const int npairs = kk / 2;
  // threads per pair: a power of two within one wavefront
  int g = 64;
  while (g > 1 && g * npairs > kBlock) g >>= 1;
  const int pair = threadIdx.x / g;
  const int lane = threadIdx.x % g;
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int st = 0; st < kk - 1; ++st) {
      if (pair < npairs) {
        int p, q;
        rr_pair(kk, st, pair, &p, &q);
        if (q < k) {
          double al = 0.0, be = 0.0, ga = 0.0;
          for (int r = lane; r < k; r += g) {
            const double xp = X[r * k + p], xq = X[r * k + q];
            al += xp * xp;
            be += xq * xq;
            ga += xp * xq;
          }
          for (int o = g / 2; o > 0; o >>= 1) {
            al += __shfl_xor(al, o, g);
            be += __shfl_xor(be, o, g);
            ga += __shfl_xor(ga, o, g);
          }
          if (fabs(ga) > 1e-15 * sqrt(al * be) && ga != 0.0) {
            double c, s;
            sym_schur2(al, be, ga, &c, &s);
            for (int r = lane; r < k; r += g) {
              const double xp = X[r * k + p], xq = X[r * k + q];
              X[r * k + p] = c * xp - s * xq;
              X[r * k + q] = s * xp + c * xq;
              const double vp = V[r * k + p], vq = V[r * k + q];
              V[r * k + p] = c * vp - s * vq;
              V[r * k + q] = s * vp + c * vq;
            }
            if (lane == 0) rotated = 1;
          }
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  // singular values = column norms; W1 = X diag(1/sigma); O = W1 V^T
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < k; ++r) s += X[r * k + j] * X[r * k + j];
    nrm[j] = sqrt(s);
  }
  __syncthreads();
  if (threadIdx.x == 0 && flags != nullptr) {
    double mx = 0.0, mn = 1e300;
    for (int j = 0; j < k; ++j) {
      mx = fmax(mx, nrm[j]);
      mn = fmin(mn, nrm[j]);
    }
    if (!(mn > 1e-12 * mx)) flags[b] = 1;
  }
  double* Ob = O + (int64_t)b * k * k;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int i = e / k, j = e - (e / k) * k;
    double s = 0.0;
    for (int l = 0; l < k; ++l) {
      const double u = (nrm[l] > 0.0) ? X[i * k + l] / nrm[l] : 0.0;
      s += u * V[j * k + l];
    }
    Ob[e] = s;
  }
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
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
sin_theta_kernel(int64_t d, int k, const double* __restrict__ Z, const double* __restrict__ U,
                 double* __restrict__ out, double* __restrict__ hist, int32_t* __restrict__ ctr) {
  __shared__ double C[kMaxK * kMaxK];
  __shared__ double G[kMaxK * kMaxK];
  __shared__ double Wt[16 * kMaxK];
  __shared__ double cs[kMaxK / 2 + 1], sn[kMaxK / 2 + 1];
  __shared__ int flag;
  const int kk = k * k;
  // C = Z^T U
  for (int e = threadIdx.x; e < kk; e += blockDim.x) {
    const int i = e / k, j = e - (e / k) * k;
    double s = 0.0;
    for (int64_t r = 0; r < d; ++r) s = fma(Z[r * k + i], U[r * k + j], s);
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
      const double* zr = Z + (r0 + rr) * k;
      double s = U[(r0 + rr) * k + j];
      for (int l = 0; l < k; ++l) s = fma(-zr[l], C[l * k + j], s);
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
  jacobi_sym_lds(G, nullptr, k, cs, sn, &flag);
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int j = 0; j < k; ++j) mx = fmax(mx, G[j * k + j]);
    const double v = sqrt(fmax(mx, 0.0));
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

// One-double result slot of lp_sin_theta (per device; concurrent calls race).
__device__ double g_sin_slot[1];

hipError_t sin_slot_address(double** p) {
  return hipGetSymbolAddress((void**)p, HIP_SYMBOL(g_sin_slot));
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_cross_gram(int batch, int64_t d, int k, const double* X, int64_t x_stride,
                             const double* W, int64_t w_stride, double* gram_part, hipStream_t s) {
  dim3 grid(nblk(d, kGramRows), batch);
  cross_gram_kernel<<<grid, kBlock, 0, s>>>(d, k, X, x_stride, W, w_stride, gram_part);
  return hipGetLastError();
}

hipError_t launch_chol_inv(int batch, int nchunks, int k, const double* gram_part, double* rinv,
                           int32_t* flags, hipStream_t s) {
  chol_inv_kernel<<<batch, kBlock, 0, s>>>(nchunks, k, gram_part, rinv, flags);
  return hipGetLastError();
}

hipError_t launch_right_mult(int batch, int64_t d, int k, const double* X, const double* S,
                             int64_t s_stride, bool upper, double* Q, void* zw, size_t zw_bytes,
                             hipStream_t s) {
  dim3 grid(nblk(d * k, kBlock), batch);
  if (zw == nullptr || zw_bytes == 8)
    right_mult_kernel<double><<<grid, kBlock, 0, s>>>(d, k, X, S, s_stride, upper ? 1 : 0, Q,
                                                       (double*)zw);
  else
    right_mult_kernel<float><<<grid, kBlock, 0, s>>>(d, k, X, S, s_stride, upper ? 1 : 0, Q,
                                                      (float*)zw);
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

hipError_t launch_apply_signs(int batch, int64_t d, int k, double* X, const int8_t* sgn, void* zw,
                              size_t zw_bytes, hipStream_t s) {
  const int64_t count = (int64_t)batch * d * k;
  if (zw == nullptr || zw_bytes == 8)
    apply_signs_kernel<double><<<nblk(count, kBlock), kBlock, 0, s>>>(batch, d, k, X, sgn,
                                                                     (double*)zw);
  else
    apply_signs_kernel<float><<<nblk(count, kBlock), kBlock, 0, s>>>(batch, d, k, X, sgn,
                                                                    (float*)zw);
  return hipGetLastError();
}

hipError_t launch_procrustes(int batch, int nchunks, int k, const double* gram_part, double* O,
                             int32_t* flags, hipStream_t s) {
  procrustes_kernel<<<batch, kBlock, 0, s>>>(nchunks, k, gram_part, O, flags);
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

hipError_t launch_sin_theta(int64_t d, int k, const double* Z, const double* U, double* out,
                            double* hist, int32_t* ctr, hipStream_t s) {
  sin_theta_kernel<<<1, kBlock, 0, s>>>(d, k, Z, U, out, hist, ctr);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int count, int32_t v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  fill_i32_kernel<<<nblk(count, kBlock), kBlock, 0, s>>>(p, count, v);
  return hipGetLastError();
}

}  // namespace lp
