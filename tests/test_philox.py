"""The counter-based generator the library and the host share (Philox4x32-10),
the draws built on it and the exact-truth matrix, pinned on the CPU:

* Philox4x32-10 against the known-answer vectors published with the
  generator (Random123's kat_vectors, the three 10-round philox4x32 cases);
* the Gaussian start: mean, variance and a normality check (Box-Muller);
* the keyed permutation is a bijection for domains that need cycle walking;
* the exact-truth matrix: A^T A = n diag(sigma^2) in the permuted basis exactly,
  every entry exact in BF16, the top-k eigenvectors of the FP64 Gram equal
  truth_basis, sigma as documented.
"""

import os

import numpy as np
import pytest
import torch

from synth import philox as ph

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2002_08014_amd",
                   "liblp.so")

KAT = [
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff, 0xffffffff, 0xffffffff, 0xffffffff), (0xffffffff, 0xffffffff),
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


@pytest.mark.parametrize("ctr,key,expect", KAT)
def test_philox_known_answers(ctr, key, expect):
    assert ph.philox4x32_10(ctr, key) == expect


def test_unit_open0_range():
    assert ph.unit_open0(0, 0) == 2.0 ** -53
    assert ph.unit_open0(0xFFFFFFFF, 0xFFFFFFFF) == 1.0


def test_gaussian_start_statistics():
    Y = ph.gaussian_start(200, 50, 12345)
    x = Y.ravel()
    assert abs(x.mean()) < 4 / np.sqrt(x.size)
    assert abs(x.var() - 1.0) < 6 * np.sqrt(2.0 / x.size)
    # fraction within one standard deviation (0.6827 for a normal)
    assert abs(np.mean(np.abs(x) < 1.0) - 0.6827) < 0.02
    assert not np.array_equal(Y, ph.gaussian_start(200, 50, 12346))
    assert np.array_equal(Y[:3, :4].ravel()[:4], ph.gaussian_start(200, 50, 12345)[:3, :4].ravel()[:4])


@pytest.mark.parametrize("N", [1, 2, 5, 17, 1000, 4096, 6000])
def test_keyed_perm_is_a_bijection(N):
    b = ph.perm_bits(N)
    img = [ph.keyed_perm(x, N, b, 99, ph.TAG_ROW_PERM) for x in range(N)]
    assert sorted(img) == list(range(N))
    if N >= 1000:
        assert sum(1 for x in range(N) if img[x] == x) < 20      # not close to the identity


@pytest.mark.parametrize("n,d,k", [(64, 16, 4), (96, 32, 5), (128, 64, 16)])
def test_truth_matrix_exact_gram_and_basis(n, d, k):
    A = ph.truth_matrix(n, d, k, 1.2, 0.97, 7 + d)
    A64 = A.astype(np.float64)
    # every entry is exact in BF16
    assert np.array_equal(torch.from_numpy(A).to(torch.bfloat16).to(torch.float32).numpy(), A)
    G = A64.T @ A64
    U = ph.truth_basis(d, k, 7 + d)
    cb = ph.perm_bits(d)
    jmap = [ph.keyed_perm(c, d, cb, 7 + d, ph.TAG_COL_PERM) for c in range(d)]
    sig = np.array([ph.truth_sigma(j, k, 1.2, 0.97) for j in jmap])
    # A^T A = n diag(sigma^2) exactly (entries +-sigma_j with orthogonal sign patterns)
    assert np.array_equal(G, np.diag(n * sig * sig))
    lam, V = np.linalg.eigh(G)
    top = V[:, np.argsort(lam)[::-1][:k]]
    assert np.abs(np.abs(top.T @ U) - np.eye(k)).max() < 1e-12
    # rows are not all alike: the partitions of a LocalPower job differ
    assert len({tuple(np.sign(r)) for r in A}) == n


def test_truth_sigma_spectrum():
    k, gap, decay = 8, 1.2, 0.97
    s = [ph.truth_sigma(j, k, gap, decay) for j in range(40)]
    exact = [1.0 / (j + 1) if j < k else (1.0 / k) / gap * decay ** (j - k) for j in range(40)]
    assert all(abs(a - b) <= 2 ** -8 * b for a, b in zip(s, exact))
    assert all(s[j] > s[j + 1] for j in range(39))


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblp.so not built")
def test_generate_host_validation():
    from paper_2002_08014_amd import _lib
    # nothing to write
    assert _lib.load().lp_generate(None, 1, 128, 16, 16, 4, 1.2, 0.97, 1, None, None) == _lib.LP_EINVAL
    for n, d, k in ((1000, 100, 4), (100, 64, 4), (64, 32, 0), (64, 32, 33)):
        st = _lib.load().lp_generate(None, 1, n, d, d, k, 1.2, 0.97, 1, 8, None)
        assert st == _lib.LP_EINVAL, (n, d, k)
