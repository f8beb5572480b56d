"""Seeded generators for the synthetic LocalPower workloads.

Every workload is a row-partitioned n x d matrix A (rows = samples, Section 2:
the data matrix is split by rows over m workers), a start matrix Y0 (the
Gaussian initialisation of Algorithm 1), a communication schedule (the set
I_T written as local steps per round) and an alignment mode.

The paper's experiments use LIBSVM datasets that are not available here; the
matrices below stand in for them, with spectra chosen so that the gap, the
noise floor and the per-node sample counts are controlled:

* low-rank-plus-noise:   A = sqrt(n) * U diag(sigma) V^T + noise * G,
  U (n x d) and V (d x d) Haar-orthonormal, G standard Gaussian, so that
  M = A^T A / n ~ V diag(sigma^2) V^T + noise^2 I;
* Gaussian rows:          a_r = V diag(lambda^{1/2}) g_r, V Haar (d x d).

All random numbers come from torch generators seeded explicitly; the draw order
is part of the recipe and is stated next to each function.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
import torch

# Row block used when drawing large matrices; part of the recipe (the Philox
# stream is consumed block after block), so changing it changes the data.
GEN_BLOCK_ROWS = 65536
# above this many elements the low-rank generator orthonormalises U block by block
LARGE_ELEMENTS = 1 << 30


@dataclasses.dataclass
class Workload:
    """A LocalPower problem instance (inputs only)."""

    name: str
    A: torch.Tensor            # n x d, row-major, stored dtype
    offsets: np.ndarray        # int64 [m+1], offsets[0]=0, offsets[m]=n
    k: int
    p_sched: List[int]         # local steps per communication round
    mode: str                  # "vanilla" | "sign" | "opt"
    Y0: np.ndarray             # d x k float64 Gaussian start (host)
    sigma: Optional[np.ndarray] = None   # generating spectrum (context only)
    seed: int = 0

    @property
    def n(self) -> int:
        return int(self.A.shape[0])

    @property
    def d(self) -> int:
        return int(self.A.shape[1])

    @property
    def m(self) -> int:
        return int(len(self.offsets) - 1)


# --------------------------------------------------------------------------
# spectra
# --------------------------------------------------------------------------

def spectrum_c1(d: int, k: int = 5) -> np.ndarray:
    """sigma_j = 1/j for j <= k, then 0.5/j (a factor-2 drop after the head)."""
    j = np.arange(1, d + 1, dtype=np.float64)
    return np.where(j <= k, 1.0 / j, 0.5 / j)


def spectrum_gap(d: int, k: int, gap: float = 1.2, decay: float = 0.97) -> np.ndarray:
    """sigma_j = 1/j for j <= k, sigma_{k+1} = sigma_k/gap, then geometric decay."""
    s = np.empty(d, dtype=np.float64)
    head = np.arange(1, k + 1, dtype=np.float64)
    s[:k] = 1.0 / head
    if d > k:
        s[k] = s[k - 1] / gap
        tail = np.arange(1, d - k, dtype=np.float64)
        s[k + 1:] = s[k] * decay ** tail
    return s


def power_law_cov(d: int, alpha: float = 1.5) -> np.ndarray:
    """Covariance eigenvalues lambda_j = j^-alpha."""
    return np.arange(1, d + 1, dtype=np.float64) ** (-alpha)


# --------------------------------------------------------------------------
# random matrices
# --------------------------------------------------------------------------

def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def haar(rows: int, cols: int, gen: torch.Generator, device) -> torch.Tensor:
    """Haar-distributed orthonormal rows x cols matrix (float64).

    Q factor of a standard Gaussian matrix, with column signs chosen so that
    the triangular factor has a positive diagonal (this makes Q Haar).
    """
    g = torch.randn(rows, cols, generator=gen, dtype=torch.float64, device=device)
    q, r = torch.linalg.qr(g, mode="reduced")
    s = torch.sign(torch.diagonal(r))
    s[s == 0] = 1.0
    return q * s


def _cast(x64: torch.Tensor, dtype: torch.dtype) -> torch.Tensor:
    # torch's float64 -> float32/bfloat16 conversions round to nearest even.
    return x64.to(dtype)


def lowrank_plus_noise(n: int, d: int, sigma: np.ndarray, noise: float, seed: int,
                       device="cpu", dtype=torch.float64) -> torch.Tensor:
    """A = sqrt(n) * U diag(sigma) V^T + noise * G.

    Draw order from one generator seeded with `seed`: V (d x d Gaussian, then
    Haar), U (n x d Gaussian, then Haar), then G in blocks of GEN_BLOCK_ROWS rows.
    The product is formed in float64 and rounded once to `dtype`.  Needs n >= d.
    """
    if n < d:
        raise ValueError("low-rank-plus-noise needs n >= d (U is n x d orthonormal)")
    if n * d > LARGE_ELEMENTS:
        return _lowrank_plus_noise_blocked(n, d, sigma, noise, seed, device, dtype)
    gen = _gen(seed, device)
    V = haar(d, d, gen, device)
    U = haar(n, d, gen, device)
    W = (torch.as_tensor(sigma, dtype=torch.float64, device=device)[:, None] * V.T) * math.sqrt(n)
    out = torch.empty(n, d, dtype=dtype, device=device)
    for r0 in range(0, n, GEN_BLOCK_ROWS):
        r1 = min(n, r0 + GEN_BLOCK_ROWS)
        blk = U[r0:r1] @ W
        if noise != 0.0:
            blk += noise * torch.randn(r1 - r0, d, generator=gen, dtype=torch.float64, device=device)
        out[r0:r1] = _cast(blk, dtype)
    del U
    return out


def _lowrank_plus_noise_blocked(n: int, d: int, sigma: np.ndarray, noise: float, seed: int,
                                device, dtype) -> torch.Tensor:
    """The same construction for matrices too large to orthonormalise whole.

    U = X R^{-1} with X an n x d standard Gaussian and R the Cholesky factor
    of X^T X (the Q factor of X with a positive-diagonal R, i.e. Haar), formed
    block by block: one pass accumulates X^T X, a second pass re-draws each X
    block from the saved generator state.  Streams: V from a generator seeded
    with `seed`, X from `seed + 1_000_003`, the noise from `seed + 2_000_006`.
    """
    gen = _gen(seed, device)
    V = haar(d, d, gen, device)
    gx = _gen(seed + 1_000_003, device)
    gn = _gen(seed + 2_000_006, device)
    state = gx.get_state()
    G = torch.zeros(d, d, dtype=torch.float64, device=device)
    for r0 in range(0, n, GEN_BLOCK_ROWS):
        r1 = min(n, r0 + GEN_BLOCK_ROWS)
        X = torch.randn(r1 - r0, d, generator=gx, dtype=torch.float64, device=device)
        G += X.T @ X
    R = torch.linalg.cholesky(G, upper=True)
    Rinv = torch.linalg.solve_triangular(R, torch.eye(d, dtype=torch.float64, device=device), upper=True)
    W = (torch.as_tensor(sigma, dtype=torch.float64, device=device)[:, None] * V.T) * math.sqrt(n)
    M = Rinv @ W
    gx.set_state(state)
    out = torch.empty(n, d, dtype=dtype, device=device)
    for r0 in range(0, n, GEN_BLOCK_ROWS):
        r1 = min(n, r0 + GEN_BLOCK_ROWS)
        X = torch.randn(r1 - r0, d, generator=gx, dtype=torch.float64, device=device)
        blk = X @ M
        if noise != 0.0:
            blk += noise * torch.randn(r1 - r0, d, generator=gn, dtype=torch.float64, device=device)
        out[r0:r1] = _cast(blk, dtype)
    return out


def gaussian_rows(n: int, d: int, lam: np.ndarray, seed: int, device="cpu",
                  dtype=torch.float64) -> torch.Tensor:
    """Rows a_r = V diag(lam^{1/2}) g_r with V Haar (d x d), g_r standard Gaussian.

    Draw order: V first, then G in blocks of GEN_BLOCK_ROWS rows; each block is
    formed in float64 and rounded once to `dtype`.
    """
    gen = _gen(seed, device)
    V = haar(d, d, gen, device)
    W = torch.as_tensor(np.sqrt(lam), dtype=torch.float64, device=device)[:, None] * V.T
    out = torch.empty(n, d, dtype=dtype, device=device)
    for r0 in range(0, n, GEN_BLOCK_ROWS):
        r1 = min(n, r0 + GEN_BLOCK_ROWS)
        g = torch.randn(r1 - r0, d, generator=gen, dtype=torch.float64, device=device)
        out[r0:r1] = _cast(g @ W, dtype)
    return out


# --------------------------------------------------------------------------
# partitions, start matrix, schedules (integer / host inputs)
# --------------------------------------------------------------------------

def equal_offsets(n: int, m: int) -> np.ndarray:
    """m contiguous row ranges; the n mod m leftover rows go to the first ranges."""
    if m < 1 or n < m:
        raise ValueError("need 1 <= m <= n")
    base, rem = divmod(n, m)
    sizes = np.full(m, base, dtype=np.int64)
    sizes[:rem] += 1
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def lognormal_offsets(n: int, m: int, mu: float, sigma: float, k: int, seed: int) -> np.ndarray:
    """Uneven partition sizes drawn lognormal and integerised to sum to n.

    x_i = exp(mu + sigma * g_i) (numpy PCG64 seeded with `seed`);
    s_i = floor(x_i * n / sum x); the leftover rows go one each to the largest
    fractional parts (ties to the lower index); then every s_i < k is raised to
    k by taking rows from the currently largest partition (lowest index on ties).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.exp(mu + sigma * rng.standard_normal(m))
    share = x * n / x.sum()
    s = np.floor(share).astype(np.int64)
    frac = share - s
    left = int(n - s.sum())
    order = sorted(range(m), key=lambda i: (-frac[i], i))
    for i in order[:left]:
        s[i] += 1
    for i in range(m):
        while s[i] < k:
            j = int(np.argmax(s))
            s[j] -= 1
            s[i] += 1
    assert int(s.sum()) == n and int(s.min()) >= k
    return np.concatenate([[0], np.cumsum(s)]).astype(np.int64)


def gaussian_start(d: int, k: int, seed: int) -> np.ndarray:
    """Y0: d x k standard Gaussian (numpy PCG64 seeded with seed + 7919)."""
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    return rng.standard_normal((d, k))


def fixed_schedule(p: int, rounds: int) -> List[int]:
    return [int(p)] * int(rounds)


def decay_schedule(stages: Sequence[int], rounds_per_stage: int) -> List[int]:
    """e.g. stages (8, 4, 2, 1), 10 rounds each -> 8 x10, 4 x10, 2 x10, 1 x10."""
    out: List[int] = []
    for p in stages:
        out += [int(p)] * int(rounds_per_stage)
    return out


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def make_fp64_2000x100(device="cpu", seed: int = 0, mode: str = "sign", p: int = 4, rounds: int = 30) -> Workload:
    """Plain FP64: A 2000 x 100 low-rank-plus-noise, k=5, m=4 x 500 rows."""
    n, d, k, m = 2000, 100, 5, 4
    sig = spectrum_c1(d, k)
    A = lowrank_plus_noise(n, d, sig, 0.01, seed, device, torch.float64)
    return Workload("plain-fp64-2000x100-k5-m4", A, equal_offsets(n, m), k,
                    fixed_schedule(p, rounds), mode, gaussian_start(d, k, seed), sig, seed)


def make_fp32_262144x1024(device="cuda", seed: int = 1, mode: str = "sign", p: int = 4, rounds: int = 50,
            n: int = 262144, d: int = 1024, k: int = 16, m: int = 32) -> Workload:
    """FP32 fused path: A 262144 x 1024 FP32, gap sigma_16/sigma_17 = 1.2, k=16, m=32."""
    sig = spectrum_gap(d, k, 1.2, 0.97)
    A = lowrank_plus_noise(n, d, sig, 0.01, seed, device, torch.float32)
    return Workload(f"fp32-{n}x{d}-k{k}-m{m}", A, equal_offsets(n, m), k,
                    fixed_schedule(p, rounds), mode, gaussian_start(d, k, seed), sig, seed)


def make_bf16_1048576x2048(device="cuda", seed: int = 2, mode: str = "opt", dtype=torch.bfloat16,
            n: int = 1048576, d: int = 2048, k: int = 32, m: int = 64) -> Workload:
    """Precision form: Gaussian rows with covariance spectrum j^-1.5, stored BF16."""
    lam = power_law_cov(d, 1.5)
    A = gaussian_rows(n, d, lam, seed, device, dtype)
    tag = "bf16" if dtype == torch.bfloat16 else "fp32"
    return Workload(f"{tag}-{n}x{d}-k{k}-m{m}", A, equal_offsets(n, m), k,
                    decay_schedule((8, 4, 2, 1), 10), mode, gaussian_start(d, k, seed),
                    np.sqrt(lam), seed)


def make_fp32_uneven_500000x4096(device="cuda", seed: int = 3, mode: str = "opt", rounds: int = 30,
            n: int = 500000, d: int = 4096, k: int = 64, m: int = 100) -> Workload:
    """Uneven partitions: A 500000 x 4096 FP32, m=100 lognormal row counts, k=64."""
    sig = spectrum_gap(d, k, 1.2, 0.97)
    A = lowrank_plus_noise(n, d, sig, 0.01, seed, device, torch.float32)
    offs = lognormal_offsets(n, m, math.log(5000.0), 0.8, k, seed)
    return Workload(f"fp32-uneven-{n}x{d}-k{k}-m{m}", A, offs, k,
                    fixed_schedule(4, rounds), mode, gaussian_start(d, k, seed), sig, seed)


def make_small(n: int, d: int, k: int, m: int, seed: int = 0, dtype=torch.float64,
               device="cpu", mode: str = "sign", p_sched: Optional[List[int]] = None,
               gap: float = 1.5, noise: float = 0.01, uneven: bool = False) -> Workload:
    """A small low-rank-plus-noise instance for parity tests and pins."""
    sig = spectrum_gap(d, k, gap, 0.9)
    A = lowrank_plus_noise(n, d, sig, noise, seed, device, dtype)
    if uneven:
        offs = lognormal_offsets(n, m, math.log(max(n / m, 1.0)), 0.8, k, seed)
    else:
        offs = equal_offsets(n, m)
    return Workload(f"small-{n}x{d}-k{k}-m{m}", A, offs, k,
                    p_sched if p_sched is not None else fixed_schedule(4, 10), mode,
                    gaussian_start(d, k, seed), sig, seed)


def spectrum_cluster(d: int, k: int, r: int, spread: float = 0.985, drop: float = 0.45,
                     decay: float = 0.8) -> np.ndarray:
    """A small gap after the target rank and a large one after the iteration rank:
    sigma_j = 1/j for j <= k, sigma_{j+1} = spread * sigma_j for k <= j < r,
    sigma_{r+1} = drop * sigma_r, then geometric decay."""
    s = np.empty(d, dtype=np.float64)
    s[:k] = 1.0 / np.arange(1, k + 1, dtype=np.float64)
    for j in range(k, min(r, d)):
        s[j] = s[j - 1] * spread
    if d > r:
        s[r] = s[r - 1] * drop
        for j in range(r + 1, d):
            s[j] = s[j - 1] * decay
    return s
