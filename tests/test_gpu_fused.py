"""Parity of the fused matrix-core local multiply (FP32 A, k <= 16) against the
FP64 oracle, for every kernel variant, at small shapes with ragged tiles, at
ranks below the tile width, and at the full 262144 x 1024 benchmark shape
(sampled partitions)."""

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import host, sin_theta_np, upcast

pytestmark = pytest.mark.gpu

VARIANTS = (1, 2, 3, 4, 5, 6, 7, 8, 9, 10)   # two-pass, then the fused forms (see lp_tuning)


@pytest.fixture(scope="module")
def lp(gpu_lib):
    import paper_2002_08014_amd as lp
    return lp


def _check_partitions(Y, A, offsets, Zw, parts):
    u = 2.0 ** -24
    for i in parts:
        Ai = A[offsets[i]:offsets[i + 1]]
        ref = Ai.T @ (Ai @ Zw)
        bound = np.abs(Ai).T @ (np.abs(Ai) @ np.abs(Zw))
        gamma = (Ai.shape[1] + Ai.shape[0]) * u
        err = np.abs(Y[i] - ref)
        assert np.all(err <= gamma * bound), (i, float(err.max()), float((gamma * bound).min()))


@pytest.mark.parametrize("cached", [False, True])
@pytest.mark.parametrize("d", [256, 512, 768, 1024])
@pytest.mark.parametrize("variant", VARIANTS)
def test_fused_small(lp, d, variant, cached):
    print(f"fused small d={d} variant={variant} cached={cached}", flush=True)
    n, m = 3 * d + 37, 3
    w = synth.make_small(n, d, 16, m, seed=d, dtype=torch.float32, uneven=True)
    A_dev = w.A.to("cuda:0")
    A = upcast(A_dev)
    P = lp.lp_create(A_dev, w.offsets, 16)
    lp.lp_set_tuning(P, variant, 0, cached)
    t = lp.lp_get_tuning(P)
    assert t["local_kernel"] == variant and t["cached_loads"] == cached
    Z = oracle.orth(np.random.default_rng(d).standard_normal((d, 16)))
    Y = host(lp.lp_local_multiply(P, 16, torch.as_tensor(Z)))
    _check_partitions(Y, A, w.offsets, Z.astype(np.float32).astype(np.float64), range(m))


@pytest.mark.parametrize("variant", [0, 2, 7, 9])
@pytest.mark.parametrize("k", [1, 5, 8, 12, 15])
@pytest.mark.parametrize("d", [256, 768])
def test_fused_lower_ranks(lp, d, k, variant):
    """Ranks below 16 run the k = 16 tiles with zero columns of Z, which are not
    stored (local_kernel 0: the vector-ALU kernel where it applies, k <= 8 and d a
    power of two, else the fused kernel); the same FP32 bound holds."""
    print(f"fused lower rank d={d} k={k} variant={variant}", flush=True)
    n, m = 3 * d + 37, 3
    w = synth.make_small(n, d, k, m, seed=d + k, dtype=torch.float32, uneven=True)
    A_dev = w.A.to("cuda:0")
    P = lp.lp_create(A_dev, w.offsets, 16)
    lp.lp_set_tuning(P, variant, 0)
    Z = oracle.orth(np.random.default_rng(d + k).standard_normal((d, k)))
    Y = host(lp.lp_local_multiply(P, k, torch.as_tensor(Z)))
    assert Y.shape == (m, d, k)
    _check_partitions(Y, upcast(A_dev), w.offsets, Z.astype(np.float32).astype(np.float64), range(m))


def test_fused_rank12_run_parity(lp):
    """Rounds of p = 4 at k = 12 through the fused kernel (zero-padded tiles):
    within 1e-5 of the oracle, sign decisions equal."""
    print("fused run k=12", flush=True)
    w = synth.make_small(16384, 512, 12, 4, seed=31, dtype=torch.float32, gap=1.3, p_sched=[4] * 6,
                         device="cuda:0")
    P = lp.lp_create(w.A, w.offsets, 12)
    lp.lp_set_tuning(P, 9, 0)
    r = lp.lp_run(P, 12, w.p_sched, "sign", w.Y0, record_signs=True)
    ro = oracle.localpower(upcast(w.A), w.offsets, 12, w.p_sched, "sign", w.Y0)
    assert sin_theta_np(host(r["Z"]), ro["Z"]) < 1e-5
    assert ro["ambiguous"] == 0
    assert np.array_equal(r["signs"], np.stack(ro["signs"]))


@pytest.fixture(scope="module")
def fp32_dense(lp):
    print("generating the 262144 x 1024 FP32 workload", flush=True)
    w = synth.make_fp32_262144x1024(device="cuda:0", rounds=3)
    return w


@pytest.mark.parametrize("variant", VARIANTS)
def test_fused_full_size_sampled(lp, fp32_dense, variant):
    """Bench shape, the launch configuration the benchmark times: sampled partitions."""
    print(f"full-size local multiply variant={variant}", flush=True)
    w = fp32_dense
    P = lp.lp_create(w.A, w.offsets, 16)
    lp.lp_set_tuning(P, variant, 0)
    Z = oracle.orth(np.random.default_rng(5).standard_normal((w.d, 16)))
    Y = host(lp.lp_local_multiply(P, 16, torch.as_tensor(Z)))
    parts = (0, 13, 31)
    A = {}
    for i in parts:
        A[i] = w.A[w.offsets[i]:w.offsets[i + 1]].to("cpu").to(torch.float64).numpy()
    Zw = Z.astype(np.float32).astype(np.float64)
    u = 2.0 ** -24
    for i in parts:
        ref = A[i].T @ (A[i] @ Zw)
        bound = np.abs(A[i]).T @ (np.abs(A[i]) @ np.abs(Zw))
        assert np.all(np.abs(Y[i] - ref) <= (w.d + A[i].shape[0]) * u * bound)


def test_full_size_run_parity(lp, fp32_dense):
    """Three rounds of p = 4 sign-fixing at the bench shape against the oracle on
    the same FP32 values: subspace within 1e-5, sign decisions bit-exact."""
    print("full-size run vs oracle", flush=True)
    w = fp32_dense
    P = lp.lp_create(w.A, w.offsets, 16)
    r = lp.lp_run(P, 16, w.p_sched, "sign", w.Y0, record_signs=True)
    A = w.A.to("cpu").to(torch.float64).numpy()
    ro = oracle.localpower(A, w.offsets, 16, w.p_sched, "sign", w.Y0)
    assert sin_theta_np(host(r["Z"]), ro["Z"]) < 1e-5
    assert ro["ambiguous"] == 0
    assert np.array_equal(r["signs"], np.stack(ro["signs"]))


def test_autotune_applies_a_valid_choice(lp, tmp_path):
    """The autotuner picks one of the candidates, caches it, and the result of
    the chosen kernel still meets the parity bound."""
    print("autotune", flush=True)
    w = synth.make_small(4096, 512, 16, 4, seed=3, dtype=torch.float32)
    A_dev = w.A.to("cuda:0")
    P = lp.lp_create(A_dev, w.offsets, 16)
    cache = str(tmp_path / "tune.txt")
    t = lp.lp_autotune(P, 16, cache)
    assert 2 <= t["local_kernel"] <= 10 and t["chunk_rows"] % 16 == 0
    assert lp.lp_get_tuning(P)["local_kernel"] == t["local_kernel"]
    assert open(cache).read().count("=") == 1
    P2 = lp.lp_create(A_dev, w.offsets, 16)
    assert lp.lp_autotune(P2, 16, cache) == t          # served from the cache
    Z = oracle.orth(np.random.default_rng(4).standard_normal((512, 16)))
    Y = host(lp.lp_local_multiply(P, 16, torch.as_tensor(Z)))
    _check_partitions(Y, upcast(A_dev), w.offsets, Z.astype(np.float32).astype(np.float64), range(4))
