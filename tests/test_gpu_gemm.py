"""Parity of the two-pass matrix-core local multiply (FP32 or BF16 A, any k up
to 64, large d) against the FP64 oracle: small uneven shapes with ragged row
and column blocks, the full 500000 x 4096 uneven-partition shape on sampled
partitions, and a whole run at k = 64.

Two forms of the kernel (tuning local_kernel 1 and 11):
* FP32 matrix cores: both products are exact in FP32 and accumulate in FP32
  (BF16 A is widened exactly), so every entry obeys the inner-product bound
    |Y - A^T A Z_w| <= (d + s) u_32 |A|^T (|A| |Z_w|),   u_32 = 2^-24,
  with Z_w the FP32 working copy of Z;
* BF16 matrix cores on exactly split operands (x = x0 + x1 + x2 in BF16, the six
  partial products x_a y_b with a + b <= 2 kept): each product is off by at most
  2^-23 of itself (the three dropped terms), two more roundings per product on
  top of the same FP32 accumulation, so the bound carries (d + s + 4) u_32."""

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


def _slack(lk):
    """Roundings per product beyond the FP32 inner-product bound."""
    return 4 if lk == 11 else 0


def _check(Y, A, offsets, Zw, parts, lk=1):
    for i in parts:
        Ai = A[offsets[i]:offsets[i + 1]]
        ref = Ai.T @ (Ai @ Zw)
        bound = np.abs(Ai).T @ (np.abs(Ai) @ np.abs(Zw))
        err = np.abs(Y[i] - ref)
        assert np.all(err <= (Ai.shape[1] + Ai.shape[0] + _slack(lk)) * U_32 * bound), \
            (i, float((err / np.maximum(bound, 1e-300)).max()))


CASES = [(260, k) for k in (1, 5, 33, 64)] + [(1100, k) for k in (5, 16, 64)] + \
        [(4096, k) for k in (16, 64)]


@pytest.mark.parametrize("lk", [1, 11])
@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("d,k", CASES)
def test_gemm_small(lp, d, k, dtype, lk):
    print(f"two-pass matrix-core d={d} k={k} {dtype} local_kernel {lk}", flush=True)
    n, m = 2 * d + 77, 3
    w = synth.make_small(n, d, k, m, seed=d + k, dtype=dtype, uneven=True, device="cuda:0")
    A_dev = w.A
    P = lp.lp_create(A_dev, w.offsets, k)
    assert lp.lp_get_tuning(P)["local_kernel"] in (1, 2, 9)    # untuned defaults
    lp.lp_set_tuning(P, lk, 0)         # the two-pass kernel, whatever the fused options
    assert lp.lp_get_tuning(P)["local_kernel"] == lk
    Z = oracle.orth(np.random.default_rng(d * k).standard_normal((d, k)))
    Y = host(lp.lp_local_multiply(P, k, torch.as_tensor(Z)))
    _check(Y, upcast(A_dev), w.offsets, Z.astype(np.float32).astype(np.float64), range(m), lk)


@pytest.fixture(scope="module")
def fp32_uneven(lp):
    print("generating the 500000 x 4096 uneven-partition workload", flush=True)
    return synth.make_fp32_uneven_500000x4096(device="cuda:0")


@pytest.mark.parametrize("lk", [1, 11])
def test_gemm_full_size_sampled(lp, fp32_uneven, lk):
    """500000 x 4096 FP32, k = 64, 100 lognormal partitions (the launch
    configuration the uneven-partition benchmark times): the smallest, the
    largest and a middle partition."""
    print(f"two-pass full size, local_kernel {lk}", flush=True)
    w = fp32_uneven
    P = lp.lp_create(w.A, w.offsets, w.k)
    lp.lp_set_tuning(P, lk, 0)
    Z = oracle.orth(np.random.default_rng(11).standard_normal((w.d, w.k)))
    Y = host(lp.lp_local_multiply(P, w.k, torch.as_tensor(Z)))
    sizes = np.diff(w.offsets)
    parts = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 50})
    Zw = Z.astype(np.float32).astype(np.float64)
    for i in parts:
        Ai = w.A[w.offsets[i]:w.offsets[i + 1]].to("cpu").to(torch.float64).numpy()
        ref = Ai.T @ (Ai @ Zw)
        bound = np.abs(Ai).T @ (np.abs(Ai) @ np.abs(Zw))
        assert np.all(np.abs(Y[i] - ref) <= (w.d + Ai.shape[0] + _slack(lk)) * U_32 * bound)


@pytest.mark.parametrize("lk", [1, 11])
def test_gemm_run_parity_k64(lp, lk):
    """Rounds of p = 4 OPT alignment at k = 64 on uneven partitions through the
    two-pass kernel: subspace within 1e-5 of the oracle on the same FP32 values."""
    print(f"two-pass run k=64, local_kernel {lk}", flush=True)
    w = synth.make_small(24576, 512, 64, 6, seed=5, dtype=torch.float32, uneven=True,
                         gap=1.3, p_sched=[4] * 6, device="cuda:0")
    P = lp.lp_create(w.A, w.offsets, 64)
    lp.lp_set_tuning(P, lk, 0)
    r = lp.lp_run(P, 64, w.p_sched, "opt", w.Y0)
    ro = oracle.localpower(upcast(w.A), w.offsets, 64, w.p_sched, "opt", w.Y0)
    assert sin_theta_np(host(r["Z"]), ro["Z"]) < 1e-5


def test_profiled_local_multiply_stamps(lp):
    """Workgroup stamps of one two-pass local multiply over uneven partitions: one
    row per workgroup of both passes, ends after starts, items in range, and the
    launch's partials still give the right product."""
    w = synth.make_small(20000, 512, 40, 6, seed=8, dtype=torch.float32, uneven=True)
    A_dev = w.A.to("cuda:0")
    P = lp.lp_create(A_dev, w.offsets, 40)
    Z = oracle.orth(np.random.default_rng(2).standard_normal((512, 40)))
    st = lp.lp_profile_local_multiply(P, 40, Z)
    cr = lp.lp_get_tuning(P)["chunk_rows"]
    nitems = sum(-(-int(s) // cr) for s in np.diff(w.offsets))
    g1, g2 = nitems * -(-cr // 128), nitems * -(-512 // 256)
    assert st.shape == (g1 + g2, 4)
    assert np.all(st[:g1, 0] == 1) and np.all(st[g1:, 0] == 2)
    assert np.all((st[:, 1] >= 0) & (st[:, 1] < nitems))
    assert np.all(st[:, 3] >= st[:, 2]) and st[:, 2].min() == 0.0
    assert st[g1:, 2].min() >= st[:g1, 2].min()
    Y = host(lp.lp_local_multiply(P, 40, torch.as_tensor(Z)))
    A = upcast(A_dev)
    Zw = Z.astype(np.float32).astype(np.float64)
    for i in range(w.m):
        Ai = A[w.offsets[i]:w.offsets[i + 1]]
        bound = np.abs(Ai).T @ (np.abs(Ai) @ np.abs(Zw))
        assert np.all(np.abs(Y[i] - Ai.T @ (Ai @ Zw)) <= (512 + Ai.shape[0]) * 2.0 ** -24 * bound)
