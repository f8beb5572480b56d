"""The seeded input generators (inputs only, no method arithmetic): the
low-rank-plus-noise construction has exactly the prescribed singular values
when the noise is off, in both its direct and its block-by-block form; the
partition offsets are valid integer splits; Gaussian starts are reproducible."""

import numpy as np
import pytest
import torch

import synth
from synth import workloads as W


@pytest.mark.parametrize("blocked", [False, True])
def test_lowrank_has_the_prescribed_spectrum(monkeypatch, blocked):
    if blocked:
        monkeypatch.setattr(W, "LARGE_ELEMENTS", 1000)
        monkeypatch.setattr(W, "GEN_BLOCK_ROWS", 700)
    n, d = 3000, 64
    sig = W.spectrum_gap(d, 8, 1.2, 0.97)
    A = W.lowrank_plus_noise(n, d, sig, 0.0, seed=5)
    s = np.linalg.svd(A.numpy(), compute_uv=False)
    assert np.allclose(s / np.sqrt(n), np.sort(sig)[::-1], rtol=0, atol=1e-13)


def test_blocked_generator_is_seeded_and_noise_enters():
    old = W.LARGE_ELEMENTS
    try:
        W.LARGE_ELEMENTS = 1000
        a = W.lowrank_plus_noise(2000, 32, W.spectrum_gap(32, 4, 1.5, 0.9), 0.01, seed=3)
        b = W.lowrank_plus_noise(2000, 32, W.spectrum_gap(32, 4, 1.5, 0.9), 0.01, seed=3)
        c = W.lowrank_plus_noise(2000, 32, W.spectrum_gap(32, 4, 1.5, 0.9), 0.0, seed=3)
    finally:
        W.LARGE_ELEMENTS = old
    assert torch.equal(a, b)
    noise = (a - c).numpy() / 0.01
    assert abs(noise.std() - 1.0) < 0.02 and abs(noise.mean()) < 0.02


@pytest.mark.parametrize("n,m,k", [(500000, 100, 64), (10007, 7, 5), (4096, 4, 16)])
def test_lognormal_offsets_are_a_valid_split(n, m, k):
    o = W.lognormal_offsets(n, m, np.log(max(n / m, 1.0)), 0.8, k, seed=1)
    assert o.dtype == np.int64 and o[0] == 0 and o[-1] == n and len(o) == m + 1
    assert np.all(np.diff(o) >= k)
    assert np.array_equal(o, W.lognormal_offsets(n, m, np.log(max(n / m, 1.0)), 0.8, k, seed=1))


def test_equal_offsets_and_start():
    assert list(W.equal_offsets(10, 3)) == [0, 4, 7, 10]       # leftovers to the first ranges
    assert list(W.equal_offsets(262144, 32)) == list(range(0, 262145, 8192))
    y1, y2 = W.gaussian_start(50, 4, 9), W.gaussian_start(50, 4, 9)
    assert y1.shape == (50, 4) and np.array_equal(y1, y2)
