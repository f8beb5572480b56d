// Counter-based random numbers for the library's own draws: Philox4x32-10
// (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2,
// 3", SC 2011).  Ten rounds of the Philox S-box on a 128-bit counter under a
// 64-bit key, the key advanced by the Weyl constants between rounds.  Usable
// on the host and the device; integer arithmetic only, so both give the same
// bits.  The draws built on it (a uniform in (0, 1], a Box-Muller normal, a
// keyed permutation of [0, N)) are defined here once.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

namespace lp {

// Stream tags: the fourth counter word, so that different draws from one seed
// never share a counter.
enum : uint32_t {
  kTagStart = 0x5a300001u,     // Gaussian start Y0
  kTagRowSign = 0x5a300002u,   // exact-truth matrix: row signs
  kTagColSign = 0x5a300003u,   // exact-truth matrix: per-block column signs
  kTagRowPerm = 0x5a300004u,   // exact-truth matrix: row permutation keys
  kTagColPerm = 0x5a300005u,   // exact-truth matrix: column permutation keys
};

struct U4 {
  uint32_t v[4];
};

__host__ __device__ inline void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  const uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo32(0xD2511F53u, c.v[0], &hi0, &lo0);
    mulhilo32(0xCD9E8D57u, c.v[2], &hi1, &lo1);
    U4 o;
    o.v[0] = hi1 ^ c.v[1] ^ k0;
    o.v[1] = lo1;
    o.v[2] = hi0 ^ c.v[3] ^ k1;
    o.v[3] = lo0;
    c = o;
  }
  return c;
}

__host__ __device__ inline U4 philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                                     uint32_t tag) {
  U4 c;
  c.v[0] = c0;
  c.v[1] = c1;
  c.v[2] = c2;
  c.v[3] = tag;
  return philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// A double in (0, 1] from two words: 53 random bits, offset by one unit.
__host__ __device__ inline double unit_open0(uint32_t a, uint32_t b) {
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 1.0) * (1.0 / 9007199254740992.0);
}

// Standard normal number e of stream `tag`: Box-Muller on the two uniforms of
// one Philox block (the cosine branch).
__host__ __device__ inline double normal_draw(uint64_t seed, uint64_t e, uint32_t tag) {
  const U4 r = philox(seed, (uint32_t)e, (uint32_t)(e >> 32), 0u, tag);
  const double u1 = unit_open0(r.v[0], r.v[1]);
  const double u2 = unit_open0(r.v[2], r.v[3]);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Even bit count with 2^bits >= N (at least 2), the domain of the Feistel permutation.
__host__ __device__ inline int perm_bits(uint64_t N) {
  int b = 2;
  while (b < 62 && ((uint64_t)1 << b) < N) b += 2;
  return b;
}

// A keyed permutation of [0, N): a four-round balanced Feistel network on
// `bits` bits (round function: the first Philox word of (right half, round),
// masked to the half width), walked until the value falls back inside [0, N)
// (cycle walking; the walk stays on x's cycle, which contains x < N, so it ends).
__host__ __device__ inline uint64_t keyed_perm(uint64_t x, uint64_t N, int bits, uint64_t seed,
                                               uint32_t tag) {
  const int h = bits / 2;
  const uint64_t mask = ((uint64_t)1 << h) - 1;
  do {
    uint64_t L = x >> h, R = x & mask;
    for (uint32_t r = 0; r < 4; ++r) {
      const U4 f = philox(seed, (uint32_t)R, (uint32_t)(R >> 32), r, tag);
      const uint64_t F = ((uint64_t)f.v[1] << 32 | f.v[0]) & mask;
      const uint64_t t = R;
      R = L ^ F;
      L = t;
    }
    x = (L << h) | R;
  } while (x >= N);
  return x;
}

// sigma_j of the exact-truth matrix: 1/(j + 1) for j < k, sigma_{k-1} / gap at
// j = k, then times decay per index (the power by repeated squaring, so host
// and device round identically), rounded to FP32 and then to BF16 (nearest,
// ties to even) so that every entry +-sigma_j is exact in both storage types.
__host__ __device__ inline float truth_sigma(int64_t j, int k, double gap, double decay) {
  double s;
  if (j < k) {
    s = 1.0 / (double)(j + 1);
  } else {
    double pw = 1.0, base = decay;
    for (int64_t e = j - k; e > 0; e >>= 1) {
      if (e & 1) pw = pw * base;
      base = base * base;
    }
    s = (1.0 / (double)k) / gap;
    s = s * pw;
  }
  const float f = (float)s;
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
  float out;
  __builtin_memcpy(&out, &u, 4);
  return out;
}

}  // namespace lp
