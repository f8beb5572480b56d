"""Philox4x32-10 and the draws built on it, for inputs the library can also
draw by itself (seeded input generator; holds none of the method's arithmetic).

Philox4x32-10 is the counter-based generator of Salmon, Moraes, Dror and Shaw
("Parallel random numbers: as easy as 1, 2, 3", SC 2011): ten rounds of the
Philox S-box on a 128-bit counter (four 32-bit words) under a 64-bit key, the
key advanced by the Weyl constants before every round after the first.  On it:

* ``unit_open0``: a double in (0, 1] from two words (53 random bits plus one unit);
* ``gaussian_start``: the standard normal start Y0 (d x k, element e = i k + j
  from the counter (e, 0, tag)), Box-Muller's cosine branch;
* ``keyed_perm``: a permutation of [0, N), a four-round balanced Feistel network
  on an even number of bits with cycle walking;
* ``truth_matrix`` / ``truth_basis``: the exact-truth matrix A = W diag(sigma) V^T
  (W stacked row-permuted, sign-flipped Sylvester Hadamard blocks with entries
  +-1, V a permutation matrix, sigma rounded to BF16) and its top-k right
  singular vectors, so that A^T A = n V diag(sigma^2) V^T exactly.

Plain Python integers (exact); the matrix generator is meant for small shapes.
"""

from __future__ import annotations

import math

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK32 = 0xFFFFFFFF

TAG_START = 0x5A300001
TAG_ROW_SIGN = 0x5A300002
TAG_COL_SIGN = 0x5A300003
TAG_ROW_PERM = 0x5A300004
TAG_COL_PERM = 0x5A300005


def philox4x32_10(ctr, key):
    """Ten Philox rounds: (c0, c1, c2, c3), (k0, k1) -> four 32-bit words."""
    c0, c1, c2, c3 = (int(x) & MASK32 for x in ctr)
    k0, k1 = (int(x) & MASK32 for x in key)
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK32
        hi1, lo1 = p1 >> 32, p1 & MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def philox(seed: int, c0: int, c1: int, c2: int, tag: int):
    return philox4x32_10((c0, c1, c2, tag), (seed & MASK32, (seed >> 32) & MASK32))


def unit_open0(a: int, b: int) -> float:
    return ((a >> 5) * 67108864.0 + (b >> 6) + 1.0) * (1.0 / 9007199254740992.0)


def normal_draw(seed: int, e: int, tag: int) -> float:
    r = philox(seed, e & MASK32, (e >> 32) & MASK32, 0, tag)
    u1 = unit_open0(r[0], r[1])
    u2 = unit_open0(r[2], r[3])
    return math.sqrt(-2.0 * math.log(u1)) * math.cos(6.283185307179586 * u2)


def gaussian_start(d: int, k: int, seed: int) -> np.ndarray:
    """Y0 (d x k float64) as the library draws it when no start is passed."""
    out = np.empty(d * k, dtype=np.float64)
    for e in range(d * k):
        out[e] = normal_draw(seed, e, TAG_START)
    return out.reshape(d, k)


def perm_bits(N: int) -> int:
    b = 2
    while b < 62 and (1 << b) < N:
        b += 2
    return b


def keyed_perm(x: int, N: int, bits: int, seed: int, tag: int) -> int:
    h = bits // 2
    mask = (1 << h) - 1
    while True:
        L, R = x >> h, x & mask
        for r in range(4):
            f = philox(seed, R & MASK32, (R >> 32) & MASK32, r, tag)
            F = ((f[1] << 32) | f[0]) & mask
            L, R = R, L ^ F
        x = (L << h) | R
        if x < N:
            return x


def truth_sigma(j: int, k: int, gap: float, decay: float) -> float:
    """sigma_j: 1/(j+1) for j < k, (1/k)/gap times decay^(j-k) after (the power
    by repeated squaring), rounded to FP32 and then to BF16 (ties to even)."""
    if j < k:
        s = 1.0 / float(j + 1)
    else:
        pw, base, e = 1.0, float(decay), j - k
        while e > 0:
            if e & 1:
                pw = pw * base
            base = base * base
            e >>= 1
        s = (1.0 / float(k)) / gap
        s = s * pw
    u = int(np.array([s], dtype=np.float32).view(np.uint32)[0])
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return float(np.array([u], dtype=np.uint32).view(np.float32)[0])


def truth_matrix(n: int, d: int, k: int, gap: float, decay: float, seed: int) -> np.ndarray:
    """The exact-truth matrix (float32 values, all exact in BF16): stored element
    (R, c) = D1(g) D2(b, c) (-1)^popcount(q & j) sigma_j with g = rowperm(R),
    b = g // d, q = g % d, j = colperm(c); D1(g) bit 0 of the row block, D2(b, c)
    bit c mod 128 of the block (c // 128, b)."""
    assert d >= 16 and d & (d - 1) == 0 and n % d == 0
    rb, cb = perm_bits(n), perm_bits(d)
    jmap = [keyed_perm(c, d, cb, seed, TAG_COL_PERM) for c in range(d)]
    sig = [truth_sigma(j, k, gap, decay) for j in jmap]
    A = np.empty((n, d), dtype=np.float32)
    for R in range(n):
        g = keyed_perm(R, n, rb, seed, TAG_ROW_PERM)
        b, q = g // d, g % d
        d1 = -1.0 if philox(seed, g & MASK32, g >> 32, 0, TAG_ROW_SIGN)[0] & 1 else 1.0
        for c0 in range(0, d, 128):
            cs = philox(seed, c0 >> 7, b & MASK32, b >> 32, TAG_COL_SIGN)
            for c in range(c0, min(d, c0 + 128)):
                bit = (cs[(c & 127) >> 5] >> (c & 31)) & 1
                h = bin(q & jmap[c]).count("1") & 1
                A[R, c] = d1 * (-1.0 if bit ^ h else 1.0) * sig[c]
    return A


def truth_basis(d: int, k: int, seed: int) -> np.ndarray:
    """Top-k right singular vectors of truth_matrix: U[c, j] = 1 where colperm(c) = j."""
    cb = perm_bits(d)
    U = np.zeros((d, k), dtype=np.float64)
    for c in range(d):
        j = keyed_perm(c, d, cb, seed, TAG_COL_PERM)
        if j < k:
            U[c, j] = 1.0
    return U
