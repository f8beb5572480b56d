"""Parity of the fused vector-ALU local multiply (k <= 8, FP32 or BF16 A, A read
once, no matrix cores) against the FP64 oracle: every width it takes and ranks
1..8 at small shapes with uneven partitions and ragged row tiles, sampled
partitions of a 262144 x 1024 matrix, and whole runs.

BF16 values are widened exactly and all arithmetic is FP32, so every entry of
Y = A^T (A Z) obeys the inner-product bound
  |Y - A^T A Z| <= (d + s) u_32 |A|^T (|A| |Z|),  u_32 = 2^-24."""

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import host, sin_theta_np, upcast

pytestmark = pytest.mark.gpu

U_32 = 2.0 ** -24


@pytest.fixture(scope="module")
def lp(gpu_lib):
    import paper_2002_08014_amd as lp
    return lp


def _check(Y, A, offsets, Zw, parts):
    for i in parts:
        Ai = A[offsets[i]:offsets[i + 1]]
        ref = Ai.T @ (Ai @ Zw)
        bound = np.abs(Ai).T @ (np.abs(Ai) @ np.abs(Zw))
        err = np.abs(Y[i] - ref)
        fac = (Ai.shape[1] + Ai.shape[0]) * U_32
        assert np.all(err <= fac * bound), (i, float((err / np.maximum(bound, 1e-300)).max()), fac)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8])
@pytest.mark.parametrize("d", [256, 512, 1024, 2048, 4096])
def test_valu_small(lp, d, k, dtype):
    print(f"valu small d={d} k={k} {dtype}", flush=True)
    n, m = 2 * d + 61, 3
    w = synth.make_small(n, d, k, m, seed=d + k, dtype=dtype, uneven=True)
    A_dev = w.A.to("cuda:0")
    P = lp.lp_create(A_dev, w.offsets, 8)
    Z = oracle.orth(np.random.default_rng(d + 3 * k).standard_normal((d, k)))
    Y = host(lp.lp_local_multiply(P, k, torch.as_tensor(Z)))
    _check(Y, upcast(A_dev), w.offsets, Z.astype(np.float32).astype(np.float64), range(m))


def test_valu_many_work_items(lp):
    """More rows than one work item per partition: the per-item partials of a
    partition are summed by the reduction (several items, ragged last item)."""
    w = synth.make_small(40000, 512, 8, 3, seed=3, dtype=torch.float32, uneven=True)
    A_dev = w.A.to("cuda:0")
    P = lp.lp_create(A_dev, w.offsets, 8)          # 80-row items: about 167 per partition
    lp.lp_set_tuning(P, 0, 160)
    Z = oracle.orth(np.random.default_rng(9).standard_normal((512, 8)))
    Y = host(lp.lp_local_multiply(P, 8, torch.as_tensor(Z)))
    _check(Y, upcast(A_dev), w.offsets, Z.astype(np.float32).astype(np.float64), range(3))


def test_valu_full_size_sampled(lp):
    """The 262144 x 1024 FP32 matrix at k = 8 (32 partitions): sampled partitions."""
    print("valu full-size 262144x1024 k=8", flush=True)
    w = synth.make_fp32_262144x1024(device="cuda:0", rounds=2)
    P = lp.lp_create(w.A, w.offsets, 16)
    Z = oracle.orth(np.random.default_rng(5).standard_normal((w.d, 8)))
    Y = host(lp.lp_local_multiply(P, 8, torch.as_tensor(Z)))
    Zw = Z.astype(np.float32).astype(np.float64)
    for i in (0, 17, 31):
        Ai = w.A[w.offsets[i]:w.offsets[i + 1]].to("cpu").to(torch.float64).numpy()
        ref = Ai.T @ (Ai @ Zw)
        bound = np.abs(Ai).T @ (np.abs(Ai) @ np.abs(Zw))
        assert np.all(np.abs(Y[i] - ref) <= (w.d + Ai.shape[0]) * U_32 * bound)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("mode", ["sign", "opt"])
def test_valu_run_parity(lp, dtype, mode):
    """Whole runs at k = 8 (decaying p) against the oracle on the same stored
    values: subspace within 1e-5, sign decisions bit-exact."""
    print(f"valu run {dtype} {mode}", flush=True)
    sched = synth.decay_schedule((4, 2, 1), 4)
    w = synth.make_small(24576, 1024, 8, 6, seed=31, dtype=dtype, gap=1.3, p_sched=sched)
    A_dev = w.A.to("cuda:0")
    P = lp.lp_create(A_dev, w.offsets, 8)
    r = lp.lp_run(P, 8, sched, mode, w.Y0, record_signs=True)
    ro = oracle.localpower(upcast(A_dev), w.offsets, 8, sched, mode, w.Y0)
    assert sin_theta_np(host(r["Z"]), ro["Z"]) < 1e-5
    if mode == "sign":
        assert ro["ambiguous"] == 0
        aligned = [t for t, sv in enumerate(ro["signs"]) if sv is not None]
        assert np.array_equal(r["signs"][aligned], np.stack([ro["signs"][t] for t in aligned]))


def test_valu_off_runs_two_pass(lp):
    """local_kernel = 1 turns the vector-ALU kernel off (two-pass kernel); both
    meet the bound and agree to FP32 rounding."""
    w = synth.make_small(8192, 1024, 4, 4, seed=2, dtype=torch.float32)
    A_dev = w.A.to("cuda:0")
    P = lp.lp_create(A_dev, w.offsets, 4)
    Z = torch.as_tensor(oracle.orth(np.random.default_rng(1).standard_normal((1024, 4))))
    Y1 = host(lp.lp_local_multiply(P, 4, Z))
    lp.lp_set_tuning(P, 1)
    Y2 = host(lp.lp_local_multiply(P, 4, Z))
    Zw = Z.numpy().astype(np.float32).astype(np.float64)
    for Y in (Y1, Y2):
        _check(Y, upcast(A_dev), w.offsets, Zw, range(4))
    assert np.abs(Y1 - Y2).max() <= 1e-4 * np.abs(Y1).max()
