"""Boundary behaviour through the C ABI:

* lp_sin_theta from two threads on two streams at once: each call has its own
  result cell, and both match the oracle (Definition 1);
* lp_generate writes the exact-truth matrix and basis bit for bit as the host
  generator (same Philox4x32-10 draws), FP32 and BF16;
* lp_run / lp_solve without a start matrix draw the Gaussian start from the seed
  exactly as the host does, and match the oracle run from that start (1e-10);
* a served job whose A and start are generated at admission reaches the exact
  subspace, and equals (bitwise) the same job run alone through lp_solve;
* a served job waits for the work its caller queued on its stream before
  submitting (A still being written there).
"""

import threading

import numpy as np
import pytest
import torch

import oracle
import synth
from synth import philox as ph
from tests._util import host, sin_theta_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lp(gpu_lib):
    import paper_2002_08014_amd as lp
    return lp


def test_sin_theta_two_threads_two_streams(lp):
    print("sin theta: two threads, two streams", flush=True)
    rng = np.random.default_rng(5)
    cases = []
    for t in range(2):
        d, k = 300 + 37 * t, 6 + 3 * t
        Z = oracle.orth(rng.standard_normal((d, k)))
        U = oracle.orth(Z + 0.05 * (t + 1) * rng.standard_normal((d, k)))
        cases.append((torch.as_tensor(Z, device="cuda:0"), torch.as_tensor(U, device="cuda:0"),
                      oracle.sin_theta(Z, U)))
    torch.cuda.synchronize()
    results = [[], []]
    errors = []

    def worker(t):
        try:
            s = torch.cuda.Stream()
            Zd, Ud, _ = cases[t]
            for _ in range(300):
                results[t].append(lp.lp_sin_theta(Zd, Ud, stream=s))
        except Exception as e:     # reported below, in the test's thread
            errors.append(e)

    th = [threading.Thread(target=worker, args=(t,)) for t in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert not errors, errors
    for t in range(2):
        ref = cases[t][2]
        assert len(results[t]) == 300
        assert max(abs(v - ref) for v in results[t]) <= 1e-12 * max(ref, 1e-300), (t, ref)
    assert abs(cases[0][2] - cases[1][2]) > 1e-3        # the two answers differ


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("n,d,k", [(256, 32, 5), (1024, 64, 16), (128, 128, 3)])
def test_generate_matches_host(lp, dtype, n, d, k):
    print(f"generate {n}x{d} k={k} {dtype}", flush=True)
    seed = 1000 + n + d
    A, U = lp.lp_generate(n, d, k, 1.2, 0.97, seed, dtype=dtype)
    ref = ph.truth_matrix(n, d, k, 1.2, 0.97, seed)
    got = A.to(torch.float32).cpu().numpy()
    assert np.array_equal(got, ref)
    assert np.array_equal(host(U), ph.truth_basis(d, k, seed))


def test_generate_into_strided_rows(lp):
    """A with a leading dimension above d: only the first d entries of each row are written."""
    L = lp.load()
    n, d, k, lda, seed = 256, 32, 4, 40, 77
    A = torch.full((n, lda), 7.0, dtype=torch.float32, device="cuda:0")
    from paper_2002_08014_amd import _lib
    st = L.lp_generate(_lib._ptr(A), 1, n, d, lda, k, 1.2, 0.97, seed, None, None)
    assert st == 0
    torch.cuda.synchronize()
    got = A.cpu().numpy()
    assert np.array_equal(got[:, :d], ph.truth_matrix(n, d, k, 1.2, 0.97, seed))
    assert np.all(got[:, d:] == 7.0)


def test_run_draws_the_seeded_start(lp):
    print("lp_run without Y0", flush=True)
    w = synth.make_small(3000, 64, 5, 4, seed=8, p_sched=[4] * 8)
    A = w.A.numpy()
    P = lp.lp_create(w.A.to("cuda:0"), w.offsets, w.k)
    for seed in (0, 12345678901234):
        Y0 = ph.gaussian_start(w.d, w.k, seed)
        for mode in ("sign", "opt"):
            r = lp.lp_run(P, w.k, w.p_sched, mode, None, seed=seed)
            ro = oracle.localpower(A, w.offsets, w.k, w.p_sched, mode, Y0)
            assert np.abs(host(r["Z"]) - ro["Z"]).max() < 1e-10
        # the same start passed explicitly gives the same answer
        r2 = lp.lp_run(P, w.k, w.p_sched, "opt", Y0)
        assert np.abs(host(r2["Z"]) - host(r["Z"])).max() < 1e-13


def test_solve_draws_the_seeded_start(lp):
    w = synth.make_small(3000, 64, 5, 4, seed=9)
    P = lp.lp_create(w.A.to("cuda:0"), w.offsets, w.k)
    a = lp.lp_solve(P, w.k, "sign", None, 4, 1e-8, 100, seed=31)
    b = lp.lp_solve(P, w.k, "sign", ph.gaussian_start(w.d, w.k, 31), 4, 1e-8, 100)
    assert a["status"] == 0 and list(a["p_used"]) == list(b["p_used"])
    assert np.abs(host(a["Z"]) - host(b["Z"])).max() < 1e-12


@pytest.mark.parametrize("dtype,d,k,m", [(torch.float32, 512, 8, 4), (torch.bfloat16, 512, 16, 4),
                                         (torch.float32, 256, 16, 16)])
def test_served_generated_job(lp, dtype, d, k, m):
    print(f"served generated job {dtype} d={d} k={k}", flush=True)
    n, seed = 32 * d, 4000 + d + k
    offs = synth.equal_offsets(n, m)
    S = lp.Server(hbm_budget_bytes=4 << 30, max_active=2)
    jid = S.submit(None, offs, k, None, p0=4, mode="sign", target=1e-5, max_rounds=300,
                   gen=(n, d, dtype, seed, 1.2, 0.97))
    assert S.wait(1, timeout_s=120)
    r = S.poll()[0]
    S.close()
    assert r["id"] == jid and r["status"] == 0, r
    _, U = lp.lp_generate(n, d, k, 1.2, 0.97, seed, dtype=None)
    assert sin_theta_np(host(r["Z"]), host(U)) < 1e-4
    # the same job alone through lp_solve on the same generated matrix and start
    A, _ = lp.lp_generate(n, d, k, 1.2, 0.97, seed, dtype=dtype, basis=False)
    P = lp.lp_create(A, offs, k)
    # the server's kernel choice: BF16 jobs use operand pairs; ranks up to 8 run the
    # fused matrix-core kernel where one takes the shape (FP32 from k = 5)
    if dtype == torch.bfloat16:
        fused_bf16 = k <= 8 and d in (512, 1024, 1536, 2048)
        lp.lp_set_tuning(P, 2 if fused_bf16 else 0, 0, False, True)
    elif 5 <= k <= 8 and d in (256, 512, 768, 1024):
        lp.lp_set_tuning(P, 9, 0)
    alone = lp.lp_solve(P, k, "sign", None, 4, 1e-5, 300, seed=seed)
    assert alone["stats"]["rounds"] == r["rounds"]
    assert torch.equal(alone["Z"], r["Z"])


def test_served_job_waits_for_the_callers_stream(lp):
    """A is written on a side stream after a long kernel there, and the job is
    submitted right away with that stream: the job must see the finished A."""
    print("served job ordered after the caller's stream", flush=True)
    w = synth.make_small(16384, 512, 8, 4, seed=12, dtype=torch.float32, device="cuda:0")
    ref_S = lp.Server(hbm_budget_bytes=4 << 30, max_active=1)
    ref_S.submit(w.A, w.offsets, w.k, w.Y0, mode="sign", target=1e-5)
    assert ref_S.wait(1, timeout_s=60)
    ref = ref_S.poll()[0]
    ref_S.close()
    side = torch.cuda.Stream()
    A = torch.zeros_like(w.A)
    big = torch.randn(4096, 4096, device="cuda:0")
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        for _ in range(20):
            big = big @ big * (1.0 / 64.0)       # keeps the side stream busy for a while
        A.copy_(w.A)
    S = lp.Server(hbm_budget_bytes=4 << 30, max_active=1)
    S.submit(A, w.offsets, w.k, w.Y0, mode="sign", target=1e-5, stream=side)
    assert S.wait(1, timeout_s=60)
    got = S.poll()[0]
    S.close()
    torch.cuda.synchronize()
    assert got["status"] == 0 and torch.equal(got["Z"], ref["Z"])
