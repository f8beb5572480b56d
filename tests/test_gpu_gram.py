"""Parity of the local-Gram form (lp_gram_enable: M_i = A_i^T A_i formed once in
FP32, then Y_i = M_i Z_i on the FP32 matrix cores) against the FP64 oracle.

M_i is an FP32 GEMM over s_i rows and M_i Z_w an FP32 inner product over d
terms, so every entry obeys
  |Y - A^T A Z_w| <= (s + d) u_32 (1 + s u_32) |A|^T (|A| |Z_w|),  u_32 = 2^-24,
with Z_w the FP32 working copy of Z (BF16 A is widened exactly)."""

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
        s, d = Ai.shape
        ref = Ai.T @ (Ai @ Zw)
        bound = np.abs(Ai).T @ (np.abs(Ai) @ np.abs(Zw))
        err = np.abs(Y[i] - ref)
        assert np.all(err <= (s + d) * U_32 * (1 + s * U_32) * bound), \
            (i, float((err / np.maximum(bound, 1e-300)).max()))


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("d,k,rows", [(96, 5, 3), (260, 16, 3), (260, 16, 1), (260, 33, 3),
                                      (1100, 64, 3)])
def test_gram_local_multiply(lp, d, k, rows, dtype):
    """rows = n / (m d): 3 lets the k <= 16 multiply split its contraction in two
    (2 m d <= n), 1 keeps it whole."""
    print(f"gram form d={d} k={k} n/(m d)={rows} {dtype}", flush=True)
    m = 5
    n = rows * m * d + 77
    w = synth.make_small(n, d, k, m, seed=d + k, dtype=dtype, uneven=True, device="cuda:0")
    P = lp.lp_create(w.A, w.offsets, k)
    lp.lp_gram_enable(P)
    Z = oracle.orth(np.random.default_rng(d * k).standard_normal((d, k)))
    Y = host(lp.lp_local_multiply(P, k, torch.as_tensor(Z)))
    _check(Y, upcast(w.A), w.offsets, Z.astype(np.float32).astype(np.float64), range(m))


@pytest.mark.parametrize("mode", ["sign", "opt"])
def test_gram_run_parity(lp, mode):
    """Rounds of p = 4 on uneven FP32 partitions in the Gram form: the subspace
    within 1e-5 of the oracle on the same values; disabling the form gives back
    the A form's bits (its captured rounds were dropped and recaptured)."""
    print(f"gram form run {mode}", flush=True)
    w = synth.make_small(20000, 128, 12, 6, seed=7, dtype=torch.float32, uneven=True,
                         p_sched=[4] * 8, device="cuda:0")
    P = lp.lp_create(w.A, w.offsets, 12)
    r_a = lp.lp_run(P, 12, w.p_sched, mode, w.Y0, record_signs=True)
    lp.lp_gram_enable(P)
    r_g = lp.lp_run(P, 12, w.p_sched, mode, w.Y0, ritz=True)
    r_g2 = lp.lp_run(P, 12, w.p_sched, mode, w.Y0, ritz=True, use_graph=False)
    assert torch.equal(r_g["Z"], r_g2["Z"])
    assert r_g["stats"]["split_rounds"] == 0
    lp.lp_gram_disable(P)
    r_a2 = lp.lp_run(P, 12, w.p_sched, mode, w.Y0, record_signs=True)
    assert torch.equal(r_a["Z"], r_a2["Z"])
    ro = oracle.localpower(upcast(w.A), w.offsets, 12, w.p_sched, mode, w.Y0)
    lam_o, Zr_o, _ = oracle.ritz(upcast(w.A), ro["Z"])
    assert sin_theta_np(host(r_g["Z"]), ro["Z"]) < 1e-5
    assert sin_theta_np(host(r_a["Z"]), ro["Z"]) < 1e-5
    assert np.abs(host(r_g["ritz"]) - lam_o).max() < 1e-5 * lam_o[0]


def test_gram_solve(lp):
    print("gram form lp_solve", flush=True)
    w = synth.make_small(16000, 64, 6, 4, seed=9, dtype=torch.float32, device="cuda:0")
    P = lp.lp_create(w.A, w.offsets, 6)
    lp.lp_gram_enable(P)
    g = lp.lp_solve(P, 6, "opt", w.Y0, 4, 1e-5, 200)
    assert g["status"] == lp.LP_OK and g["p_used"][-1] == 1
    U, _ = oracle.top_k(upcast(w.A), 6)
    assert sin_theta_np(host(g["Z"]), U) < 1e-4


@pytest.fixture(scope="module")
def fp32_default(lp):
    print("generating the 262144 x 1024 workload", flush=True)
    return synth.make_fp32_262144x1024(device="cuda:0")


def test_gram_full_size_sampled(lp, fp32_default):
    """262144 x 1024 FP32, k = 16, 32 partitions of 8192 rows (the benchmark
    workload) in the Gram form: the first, a middle and the last partition."""
    print("gram form full size", flush=True)
    w = fp32_default
    P = lp.lp_create(w.A, w.offsets, w.k)
    lp.lp_gram_enable(P)
    Z = oracle.orth(np.random.default_rng(12).standard_normal((w.d, w.k)))
    Y = host(lp.lp_local_multiply(P, w.k, torch.as_tensor(Z)))
    Zw = Z.astype(np.float32).astype(np.float64)
    for i in (0, 17, w.m - 1):
        Ai = w.A[w.offsets[i]:w.offsets[i + 1]].to("cpu").to(torch.float64).numpy()
        ref = Ai.T @ (Ai @ Zw)
        bound = np.abs(Ai).T @ (np.abs(Ai) @ np.abs(Zw))
        s = Ai.shape[0]
        assert np.all(np.abs(Y[i] - ref) <= (s + w.d) * U_32 * (1 + s * U_32) * bound)


def test_gram_refusals(lp):
    print("gram form refusals", flush=True)
    w64 = synth.make_small(2000, 64, 4, 4, seed=1, device="cuda:0")
    P = lp.lp_create(w64.A, w64.offsets, 4)
    with pytest.raises(lp.LPError):
        lp.lp_gram_enable(P)                       # FP64 A
    w = synth.make_small(600, 100, 4, 8, seed=1, dtype=torch.float32, device="cuda:0")
    P = lp.lp_create(w.A, w.offsets, 4)
    with pytest.raises(lp.LPError):
        lp.lp_gram_enable(P)                       # m d = 800 > n = 600
    w = synth.make_small(4000, 98, 4, 4, seed=1, dtype=torch.float32, device="cuda:0")
    P = lp.lp_create(w.A, w.offsets, 4)
    with pytest.raises(lp.LPError):
        lp.lp_gram_enable(P)                       # d % 4 != 0


@pytest.mark.parametrize("m", [4, 16])
def test_eta_against_oracle(lp, m):
    """eta (Definition 2) from the Gram form's matrices against the oracle's
    dense spectral norms on the same stored FP32 values."""
    print(f"eta m={m}", flush=True)
    w = synth.make_small(8192, 64, 4, m, seed=m, dtype=torch.float32, noise=0.05, device="cuda:0")
    P = lp.lp_create(w.A, w.offsets, 4)
    with pytest.raises(lp.LPError):
        lp.lp_eta(P)                               # needs the Gram form
    lp.lp_gram_enable(P)
    eta, per = lp.lp_eta(P, 400)
    A = upcast(w.A)
    n = A.shape[0]
    Mm = A.T @ A / n
    nm = np.linalg.norm(Mm, 2)
    per_o = [np.linalg.norm(A[w.offsets[i]:w.offsets[i + 1]].T @ A[w.offsets[i]:w.offsets[i + 1]]
                            / (w.offsets[i + 1] - w.offsets[i]) - Mm, 2) / nm for i in range(m)]
    assert abs(eta - oracle.eta(A, w.offsets)) < 1e-3 * eta
    assert np.abs(per - np.array(per_o)).max() < 1e-3 * max(per_o)


@pytest.mark.parametrize("which", ["bf16-1048576x2048", "fp32-uneven-500000x4096"])
def test_gram_full_size_sampled_large(lp, which):
    """The other two benchmark shapes in the Gram form (the launch configuration of
    `bench.py --gram`): BF16 1048576 x 2048 with k = 32 over 64 partitions, and FP32
    500000 x 4096 with k = 64 over 100 lognormal partitions; the smallest, the
    largest and one middle partition against the FP32 bound."""
    print(f"gram form full size {which}", flush=True)
    w = (synth.make_bf16_1048576x2048 if which.startswith("bf16") else
         synth.make_fp32_uneven_500000x4096)(device="cuda:0")
    P = lp.lp_create(w.A, w.offsets, w.k)
    lp.lp_gram_enable(P)
    Z = oracle.orth(np.random.default_rng(13).standard_normal((w.d, w.k)))
    Y = host(lp.lp_local_multiply(P, w.k, torch.as_tensor(Z)))
    Zw = Z.astype(np.float32).astype(np.float64)
    sizes = np.diff(w.offsets)
    for i in sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), w.m // 2}):
        Ai = w.A[w.offsets[i]:w.offsets[i + 1]].to("cpu").to(torch.float64).numpy()
        ref = Ai.T @ (Ai @ Zw)
        bound = np.abs(Ai).T @ (np.abs(Ai) @ np.abs(Zw))
        s = Ai.shape[0]
        assert np.all(np.abs(Y[i] - ref) <= (s + w.d) * U_32 * (1 + s * U_32) * bound), i
    del P, w
    torch.cuda.empty_cache()
