"""Parity of the fused BF16 matrix-core local multiply (BF16 A, k <= 32)
against the FP64 oracle: small shapes with ragged tiles for every width, k and
variant, the full 1048576 x 2048 precision-form shape on sampled partitions,
and whole runs.

The kernel rounds Z and t = A Z to BF16 (round to nearest even) and
accumulates in FP32, so every entry of Y = A^T (A Z) obeys
  |Y - A^T A Z| <= (2 u_b + (d + s) u_32) (1 + 4 u_b) |A|^T (|A| |Z|)
with u_b = 2^-8, u_32 = 2^-24 (two operand roundings plus the inner-product
bounds of the two FP32-accumulated products)."""

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import host, sin_theta_np, upcast

pytestmark = pytest.mark.gpu

U_B = 2.0 ** -8
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
        fac = (2 * U_B + (Ai.shape[1] + Ai.shape[0]) * U_32) * (1 + 4 * U_B)
        err = np.abs(Y[i] - ref)
        assert np.all(err <= fac * bound), (i, float((err / np.maximum(bound, 1e-300)).max()), fac)
        # and the result is not trivially loose: BF16 operands keep about 2-3 digits
        assert float(np.abs(Y[i] - ref).max()) <= 0.05 * float(np.abs(ref).max())


@pytest.mark.parametrize("cached", [False, True])
@pytest.mark.parametrize("variant", [2, 3, 4, 5])
@pytest.mark.parametrize("k", [16, 32])
@pytest.mark.parametrize("d", [512, 1024, 1536, 2048])
def test_bf16_fused_small(lp, d, k, variant, cached):
    print(f"bf16 fused small d={d} k={k} variant={variant} cached={cached}", flush=True)
    n, m = 3 * d + 37, 3
    w = synth.make_small(n, d, k, m, seed=d + k, dtype=torch.bfloat16, uneven=True)
    A_dev = w.A.to("cuda:0")
    P = lp.lp_create(A_dev, w.offsets, k)
    lp.lp_set_tuning(P, variant, 0, cached)
    t = lp.lp_get_tuning(P)
    w8 = d in (1024, 2048)
    assert t["local_kernel"] == (variant if (variant in (2, 4) or w8) else variant - 1)
    assert t["cached_loads"] == cached
    Z = oracle.orth(np.random.default_rng(d + k).standard_normal((d, k)))
    Y = host(lp.lp_local_multiply(P, k, torch.as_tensor(Z)))
    _check(Y, upcast(A_dev), w.offsets, Z.astype(np.float32).astype(np.float64), range(m))


def test_bf16_fused_rejects_extra_variants(lp):
    w = synth.make_small(2048, 512, 16, 2, seed=1, dtype=torch.bfloat16)
    P = lp.lp_create(w.A.to("cuda:0"), w.offsets, 16)
    with pytest.raises(RuntimeError):
        lp.lp_set_tuning(P, 6, 0)


@pytest.mark.parametrize("variant", [2, 5])
@pytest.mark.parametrize("k", [3, 8, 12, 20, 31])
@pytest.mark.parametrize("d", [512, 1536])
def test_bf16_fused_other_ranks(lp, d, k, variant):
    """Ranks below 16, or between 16 and 32, run the 16- or 32-wide tiles with
    zero columns of Z (not stored); the BF16-operand bound holds."""
    print(f"bf16 fused rank d={d} k={k} variant={variant}", flush=True)
    n, m = 3 * d + 37, 3
    w = synth.make_small(n, d, k, m, seed=d + k + 5, dtype=torch.bfloat16, uneven=True)
    A_dev = w.A.to("cuda:0")
    P = lp.lp_create(A_dev, w.offsets, 32)
    lp.lp_set_tuning(P, variant, 0)
    Z = oracle.orth(np.random.default_rng(d + k + 5).standard_normal((d, k)))
    Y = host(lp.lp_local_multiply(P, k, torch.as_tensor(Z)))
    assert Y.shape == (m, d, k)
    _check(Y, upcast(A_dev), w.offsets, Z.astype(np.float32).astype(np.float64), range(m))


@pytest.fixture(scope="module")
def bf16_wide(lp):
    print("generating the 1048576 x 2048 BF16 workload", flush=True)
    return synth.make_bf16_1048576x2048(device="cuda:0")


@pytest.mark.parametrize("variant", [2, 3, 4, 5])
def test_bf16_fused_full_size_sampled(lp, bf16_wide, variant):
    """Precision-form shape (64 partitions of 16384 x 2048, k = 32), the launch
    configuration the benchmark times: three sampled partitions."""
    print(f"bf16 full-size local multiply variant={variant}", flush=True)
    w = bf16_wide
    P = lp.lp_create(w.A, w.offsets, w.k)
    lp.lp_set_tuning(P, variant, 0)
    Z = oracle.orth(np.random.default_rng(7).standard_normal((w.d, w.k)))
    Y = host(lp.lp_local_multiply(P, w.k, torch.as_tensor(Z)))
    parts = (0, 37, 63)
    Zw = Z.astype(np.float32).astype(np.float64)
    for i in parts:
        Ai = w.A[w.offsets[i]:w.offsets[i + 1]].to("cpu").to(torch.float64).numpy()
        ref = Ai.T @ (Ai @ Zw)
        bound = np.abs(Ai).T @ (np.abs(Ai) @ np.abs(Zw))
        fac = (2 * U_B + (w.d + Ai.shape[0]) * U_32) * (1 + 4 * U_B)
        assert np.all(np.abs(Y[i] - ref) <= fac * bound)


@pytest.mark.parametrize("mode", ["sign", "opt"])
def test_bf16_fused_run_parity(lp, mode):
    """A whole run on the fused BF16 kernel (d = 1024, k = 32, decaying p)
    against the oracle on the same BF16 values and on the original FP64 A:
    subspace within 2e-2 of both, sign decisions bit-exact."""
    print(f"bf16 fused run {mode}", flush=True)
    sched = synth.decay_schedule((4, 2, 1), 4)
    w64 = synth.make_small(32768, 1024, 32, 4, seed=21, dtype=torch.float64, gap=1.3,
                           p_sched=sched)
    A_dev = w64.A.to(torch.bfloat16).to("cuda:0")
    P = lp.lp_create(A_dev, w64.offsets, 32)
    assert lp.lp_get_tuning(P)["local_kernel"] == 2
    r = lp.lp_run(P, 32, sched, mode, w64.Y0, record_signs=True)
    Zg = host(r["Z"])
    ro = oracle.localpower(upcast(A_dev), w64.offsets, 32, sched, mode, w64.Y0)
    r64 = oracle.localpower(w64.A.numpy(), w64.offsets, 32, sched, mode, w64.Y0)
    assert sin_theta_np(Zg, ro["Z"]) < 2e-2
    assert sin_theta_np(Zg, r64["Z"]) < 2e-2
    if mode == "sign":
        assert ro["ambiguous"] == 0
        aligned = [t for t, sv in enumerate(ro["signs"]) if sv is not None]   # rounds with p >= 2
        assert aligned
        assert np.array_equal(r["signs"][aligned], np.stack([ro["signs"][t] for t in aligned]))


# ---------------------------------------------------------------- split operand pairs

def _check_split(Y, A, offsets, Zw, parts):
    """Operand pairs hi + lo leave |x - hi - lo| <= 2^-17 |x| (x - hi is exact in
    FP32, lo rounds it once), so each entry obeys
      |Y - A^T A Z| <= (2^-16 + (d + s) u_32) (1 + 4 u_b) |A|^T (|A| |Z|)."""
    for i in parts:
        Ai = A[offsets[i]:offsets[i + 1]]
        ref = Ai.T @ (Ai @ Zw)
        bound = np.abs(Ai).T @ (np.abs(Ai) @ np.abs(Zw))
        fac = (2.0 ** -16 + (Ai.shape[1] + Ai.shape[0]) * U_32) * (1 + 4 * U_B)
        err = np.abs(Y[i] - ref)
        assert np.all(err <= fac * bound), (i, float((err / np.maximum(bound, 1e-300)).max()), fac)


@pytest.mark.parametrize("variant", [2, 3, 4, 5])
@pytest.mark.parametrize("k", [5, 16, 24, 32])
@pytest.mark.parametrize("d", [512, 1024, 1536, 2048])
def test_bf16_split_operands_small(lp, d, k, variant):
    print(f"bf16 split operands d={d} k={k} variant={variant}", flush=True)
    n, m = 3 * d + 37, 3
    w = synth.make_small(n, d, k, m, seed=d + k + 1, dtype=torch.bfloat16, uneven=True)
    A_dev = w.A.to("cuda:0")
    P = lp.lp_create(A_dev, w.offsets, k)
    lp.lp_set_tuning(P, variant, 0, False, True)
    assert lp.lp_get_tuning(P)["split_operands"]
    Z = oracle.orth(np.random.default_rng(d + k + 1).standard_normal((d, k)))
    Y = host(lp.lp_local_multiply(P, k, torch.as_tensor(Z)))
    Zw = Z.astype(np.float32).astype(np.float64)
    if k > 16 and d == 2048:
        # the pairs do not fit: the two-pass kernel with FP32 operands runs
        for i in range(m):
            Ai = upcast(A_dev)[w.offsets[i]:w.offsets[i + 1]]
            bound = np.abs(Ai).T @ (np.abs(Ai) @ np.abs(Zw))
            assert np.all(np.abs(Y[i] - Ai.T @ (Ai @ Zw)) <= (d + Ai.shape[0]) * U_32 * bound)
    else:
        _check_split(Y, upcast(A_dev), w.offsets, Zw, range(m))


@pytest.mark.parametrize("d,k", [(256, 16), (2048, 24), (4096, 64)])
def test_bf16_pairs_on_the_two_pass_kernel(lp, d, k):
    """Operand pairs with no kernel named, on shapes no fused kernel takes: the
    two-pass kernel on BF16 matrix cores carries Z_i and t as hi/lo BF16 pairs (two
    products per FP32 product).  A pair leaves |x - hi - lo| <= u_b^2 |x| (two
    round-to-nearest steps to 8 bits), so each entry obeys
      |Y - A^T A Z| <= (2 u_b^2 + (d + s + 4) u_32)(1 + 4 u_b) |A|^T (|A| |Z|)."""
    print(f"bf16 pairs two-pass d={d} k={k}", flush=True)
    n, m = 3 * d + 37, 3
    w = synth.make_small(n, d, k, m, seed=d + k + 3, dtype=torch.bfloat16, uneven=True)
    A_dev = w.A.to("cuda:0")
    P = lp.lp_create(A_dev, w.offsets, k)
    lp.lp_set_tuning(P, 0, 0, False, True)
    Z = oracle.orth(np.random.default_rng(d + k + 3).standard_normal((d, k)))
    Y = host(lp.lp_local_multiply(P, k, torch.as_tensor(Z)))
    Zw = Z.astype(np.float32).astype(np.float64)
    A = upcast(A_dev)
    for i in range(m):
        Ai = A[w.offsets[i]:w.offsets[i + 1]]
        bound = np.abs(Ai).T @ (np.abs(Ai) @ np.abs(Zw))
        gamma = (2 * U_B ** 2 + (d + Ai.shape[0] + 4) * U_32) * (1 + 4 * U_B)
        assert np.all(np.abs(Y[i] - Ai.T @ (Ai @ Zw)) <= gamma * bound)


def test_bf16_split_operands_run_parity(lp):
    """A whole run with operand pairs (d = 1024, k = 16) is FP32-class: within
    1e-5 of the oracle on the same BF16 values (single roundings sit near 1e-3)."""
    print("bf16 split operands run", flush=True)
    sched = synth.decay_schedule((4, 2, 1), 5)
    w64 = synth.make_small(32768, 1024, 16, 4, seed=22, dtype=torch.float64, gap=1.3, p_sched=sched)
    A_dev = w64.A.to(torch.bfloat16).to("cuda:0")
    P = lp.lp_create(A_dev, w64.offsets, 16)
    ro = oracle.localpower(upcast(A_dev), w64.offsets, 16, sched, "opt", w64.Y0)
    single = host(lp.lp_run(P, 16, sched, "opt", w64.Y0)["Z"])
    lp.lp_set_tuning(P, 0, 0, False, True)
    split = host(lp.lp_run(P, 16, sched, "opt", w64.Y0)["Z"])
    s_single, s_split = sin_theta_np(single, ro["Z"]), sin_theta_np(split, ro["Z"])
    print(f"single BF16 {s_single:.2e}, pairs {s_split:.2e}", flush=True)
    assert s_split < 1e-5 and s_split < s_single / 10
