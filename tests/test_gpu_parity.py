"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 A 1e-10 on Z and sin theta; FP32 (and BF16-stored, FP32
accumulated) A 1e-5 on sin theta(Z_gpu, Z_oracle), the oracle running in FP64
on the same stored values; integer outputs (sign decisions) bit-exact.
"""

import math

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import host, rule_schedule, sign_normalise, sin_theta_np, to_device, upcast

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


def _problem(lib, A_dev, offsets, k_max):
    return lib.lp_create(A_dev, offsets, k_max)


@pytest.fixture(scope="module")
def lib(gpu_lib):
    import paper_2002_08014_amd as lp
    return lp


@pytest.fixture(scope="module")
def fp64_small():
    w = synth.make_fp64_2000x100()
    A = w.A.numpy()
    U, lam = oracle.top_k(A, w.k)
    return w, A, U, lam


# --------------------------------------------------------------------- FP64 2000 x 100

@pytest.mark.parametrize("mode", ["sign", "opt", "vanilla"])
def test_fp64_small_full_run(lib, fp64_small, mode):
    w, A, U, lam = fp64_small
    _flush(f"fp64_small mode={mode}")
    P = _problem(lib, to_device(w), w.offsets, w.k)
    r = lib.lp_run(P, w.k, w.p_sched, mode, w.Y0, U_ref=torch.as_tensor(U), record_signs=True)
    ro = oracle.localpower(A, w.offsets, w.k, w.p_sched, mode, w.Y0, U_ref=U)
    Zg = host(r["Z"])
    assert np.abs(Zg - ro["Z"]).max() < 1e-10
    assert sin_theta_np(Zg, ro["Z"]) < 1e-10
    assert np.abs(r["sin_hist"] - np.array(ro["sin_hist"])).max() < 1e-10
    if mode == "sign":
        assert ro["ambiguous"] == 0
        exp = np.stack([s for s in ro["signs"]])
        assert np.array_equal(r["signs"], exp)
    st = r["stats"]
    assert st["rounds"] == 30 and st["local_iters"] == 120 and st["breakdowns"] == 0


def test_fp64_small_p1_is_dpi(lib, fp64_small):
    w, A, U, lam = fp64_small
    _flush("fp64_small p=1")
    P = _problem(lib, to_device(w), w.offsets, w.k)
    r = lib.lp_run(P, w.k, [1] * 30, "sign", w.Y0)
    Zd, _ = oracle.dpi(A, w.Y0, 30)
    assert np.abs(host(r["Z"]) - Zd).max() < 1e-10
    assert sin_theta_np(host(r["Z"]), U) < 1e-12


def test_fp64_small_decay_and_ritz(lib, fp64_small):
    w, A, U, lam = fp64_small
    _flush("fp64_small decay+ritz")
    sched = synth.decay_schedule((8, 4, 2, 1), 10)
    P = _problem(lib, to_device(w), w.offsets, w.k)
    r = lib.lp_run(P, w.k, sched, "opt", w.Y0, ritz=True)
    ro = oracle.localpower(A, w.offsets, w.k, sched, "opt", w.Y0)
    lam_o, Zr_o, _ = oracle.ritz(A, ro["Z"])
    rz = host(r["ritz"])
    assert np.abs(rz - lam_o).max() < 1e-10 * lam_o[0]
    assert np.abs(rz - lam[:w.k]).max() < 1e-9 * lam[0]
    Zg = sign_normalise(host(r["Z"]))
    assert np.abs(Zg - sign_normalise(Zr_o)).max() < 1e-8
    assert sin_theta_np(Zg, U) < 1e-10


def test_uneven_partitions_fp64(lib):
    w = synth.make_small(3001, 77, 6, 5, seed=4, uneven=True, p_sched=[3] * 12)
    _flush("uneven fp64")
    A = w.A.numpy()
    assert len(set(np.diff(w.offsets))) > 1
    P = _problem(lib, to_device(w), w.offsets, w.k)
    for mode in ("sign", "opt"):
        r = lib.lp_run(P, w.k, w.p_sched, mode, w.Y0, record_signs=True)
        ro = oracle.localpower(A, w.offsets, w.k, w.p_sched, mode, w.Y0)
        assert np.abs(host(r["Z"]) - ro["Z"]).max() < 1e-10
        if mode == "sign":
            assert np.array_equal(r["signs"], np.stack(ro["signs"]))


# --------------------------------------------------------------------- kernel-level

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("k", [1, 5, 16, 33])
def test_local_multiply(lib, dtype, k):
    """Y_i = A_i^T (A_i Z) for every partition; ragged rows/columns, uneven partitions."""
    _flush(f"local multiply {dtype} k={k}")
    n, d, m = 5000, 301, 4
    w = synth.make_small(n, d, min(k, 8), m, seed=7, uneven=True)
    A_dev = to_device(w, dtype)
    A = upcast(A_dev)
    P = _problem(lib, A_dev, w.offsets, k)
    Z = oracle.orth(np.random.default_rng(1).standard_normal((d, k)))
    Y = host(lib.lp_local_multiply(P, k, torch.as_tensor(Z)))
    Zw = Z if dtype == torch.float64 else Z.astype(np.float32).astype(np.float64)
    u = 2.0 ** -53 if dtype == torch.float64 else 2.0 ** -24
    for i in range(m):
        Ai = A[w.offsets[i]:w.offsets[i + 1]]
        ref = Ai.T @ (Ai @ Zw)
        bound = np.abs(Ai).T @ (np.abs(Ai) @ np.abs(Zw))
        gamma = (d + Ai.shape[0]) * u
        assert np.all(np.abs(Y[i] - ref) <= gamma * bound + 1e-300), (i, np.abs(Y[i] - ref).max())


@pytest.mark.parametrize("k", [9, 16, 32, 40, 64])
def test_orth_batched(lib, k):
    """CholeskyQR2 of a batch: k <= 16 factors in every row-chunk workgroup,
    17..32 in one wavefront per matrix, larger k block-wide per matrix."""
    _flush(f"orth k={k}")
    rng = np.random.default_rng(3 + k)
    d, b = 333, 3
    w = synth.make_small(400, d, 4, 4, seed=1)
    P = _problem(lib, to_device(w), w.offsets, k)
    Y = rng.standard_normal((b, d, k)) @ np.diag(np.logspace(0, -4, k))
    Q, flags = lib.lp_orth(P, torch.as_tensor(Y, device="cuda:0"))
    Q = host(Q)
    assert int(flags.sum()) == 0
    for i in range(b):
        assert np.abs(Q[i] - oracle.orth(Y[i])).max() < 1e-12
        assert np.abs(Q[i].T @ Q[i] - np.eye(k)).max() < 1e-14


@pytest.mark.parametrize("k", [4, 24, 40])
def test_orth_breakdown_flag(lib, k):
    """A rank-deficient iterate is reported (host-forced: a zero column), on
    each of the three factorization paths; the other matrix of the batch is not."""
    _flush(f"orth breakdown k={k}")
    w = synth.make_small(200, 50, 4, 4, seed=1)
    P = _problem(lib, to_device(w), w.offsets, k)
    Y = np.random.default_rng(0).standard_normal((2, 50, k))
    Y[0, :, 2] = 0.0
    Q, flags = lib.lp_orth(P, torch.as_tensor(Y, device="cuda:0"))
    assert int(flags[0]) == 1 and int(flags[1]) == 0
    assert np.abs(host(Q)[1] - oracle.orth(Y[1])).max() < 1e-12


def test_align(lib):
    _flush("align")
    rng = np.random.default_rng(8)
    d, k, b = 257, 12, 5
    w = synth.make_small(400, d, 4, 5, seed=1)
    P = _problem(lib, to_device(w), w.offsets, k)
    Zb = oracle.orth(rng.standard_normal((d, k)))
    Zi = np.stack([oracle.orth(Zb @ oracle.orth(rng.standard_normal((k, k))) * 1.0
                               + 0.05 * rng.standard_normal((d, k))) for _ in range(b)])
    sg = host(lib.lp_align(P, "sign", torch.as_tensor(Zi, device="cuda:0"),
                           torch.as_tensor(Zb, device="cuda:0")))
    O = host(lib.lp_align(P, "opt", torch.as_tensor(Zi, device="cuda:0"),
                          torch.as_tensor(Zb, device="cuda:0")))
    for i in range(b):
        assert np.array_equal(sg[i], oracle.sign_fix(Zi[i], Zb).astype(np.int8))
        assert np.abs(O[i] - oracle.opt_matrix(Zi[i], Zb)).max() < 1e-12


def test_sin_theta(lib):
    _flush("sin theta")
    rng = np.random.default_rng(2)
    for d, k in ((100, 5), (1024, 16), (4096, 64)):
        U = oracle.orth(rng.standard_normal((d, k)))
        Z = oracle.orth(U + 1e-3 * rng.standard_normal((d, k)))
        g = lib.lp_sin_theta(torch.as_tensor(Z, device="cuda:0"), torch.as_tensor(U, device="cuda:0"))
        o = oracle.sin_theta(Z, U)
        assert abs(g - o) < 1e-12 * max(1.0, o) + 1e-6 * o


# --------------------------------------------------------------------- FP32 / BF16 runs

@pytest.mark.parametrize("mode", ["sign", "opt"])
def test_fp32_run_parity(lib, mode):
    _flush(f"fp32 run {mode}")
    w = synth.make_small(32768, 256, 16, 8, seed=12, dtype=torch.float32, gap=1.3,
                         p_sched=[4] * 20)
    A_dev = to_device(w)
    A = upcast(A_dev)
    U, _ = oracle.top_k(A, 16)
    P = _problem(lib, A_dev, w.offsets, 16)
    r = lib.lp_run(P, 16, w.p_sched, mode, w.Y0, record_signs=(mode == "sign"))
    ro = oracle.localpower(A, w.offsets, 16, w.p_sched, mode, w.Y0)
    Zg = host(r["Z"])
    assert sin_theta_np(Zg, ro["Z"]) < 1e-5
    assert abs(sin_theta_np(Zg, U) - sin_theta_np(ro["Z"], U)) < 1e-5
    if mode == "sign":
        assert ro["ambiguous"] == 0
        assert np.array_equal(r["signs"], np.stack(ro["signs"]))


def test_bf16_run_parity(lib):
    _flush("bf16 run")
    w = synth.make_small(32768, 256, 16, 8, seed=13, dtype=torch.bfloat16, gap=1.3,
                         p_sched=synth.decay_schedule((4, 2, 1), 6))
    A_dev = to_device(w)
    A = upcast(A_dev)
    P = _problem(lib, A_dev, w.offsets, 16)
    r = lib.lp_run(P, 16, w.p_sched, "opt", w.Y0)
    ro = oracle.localpower(A, w.offsets, 16, w.p_sched, "opt", w.Y0)
    assert sin_theta_np(host(r["Z"]), ro["Z"]) < 1e-5


# --------------------------------------------------------------------- runtime properties

def test_graph_plain_and_repeat_bitwise(lib, fp64_small):
    w, A, U, lam = fp64_small
    _flush("graph vs plain")
    P = _problem(lib, to_device(w), w.offsets, w.k)
    r1 = lib.lp_run(P, w.k, w.p_sched, "opt", w.Y0, use_graph=True)
    r2 = lib.lp_run(P, w.k, w.p_sched, "opt", w.Y0, use_graph=False)
    r3 = lib.lp_run(P, w.k, w.p_sched, "opt", w.Y0, use_graph=True)
    assert torch.equal(r1["Z"], r2["Z"]) and torch.equal(r1["Z"], r3["Z"])


def test_resume_bitwise(lib, fp64_small):
    """State at a round boundary is Z alone: resuming from the saved Z gives the
    uninterrupted result bit for bit."""
    w, A, U, lam = fp64_small
    _flush("resume")
    P = _problem(lib, to_device(w), w.offsets, w.k)
    full = lib.lp_run(P, w.k, [4] * 12, "sign", w.Y0)
    half = lib.lp_run(P, w.k, [4] * 5, "sign", w.Y0)
    rest = lib.lp_run(P, w.k, [4] * 7, "sign", half["Z"], z0_orthonormal=True)
    assert torch.equal(full["Z"], rest["Z"])


def test_invalid_arguments(lib, fp64_small):
    w, A, U, lam = fp64_small
    _flush("invalid args")
    P = _problem(lib, to_device(w), w.offsets, w.k)
    with pytest.raises(lib.LPError):
        lib.lp_run(P, w.k + 1, [4], "sign", w.Y0)            # k > k_max
    with pytest.raises(lib.LPError):
        lib.lp_run(P, w.k, [4, 0], "sign", w.Y0)             # p = 0
    P2 = lib.lp_create(to_device(w), [0, 3, 2000], 5)
    with pytest.raises(lib.LPError):
        lib.lp_run(P2, 5, [1], "sign", w.Y0)                 # s_0 = 3 < k
    with pytest.raises(lib.LPError):
        lib.lp_create(to_device(w), [0, 3, 3, 2000], 5)      # empty partition
    Zt = torch.zeros(100, 4, dtype=torch.float64, device="cuda:0")
    with pytest.raises(lib.LPError):
        lib.lp_sin_theta(Zt, torch.zeros(100, 5, dtype=torch.float64, device="cuda:0"))  # k > r


def test_create_right_after_queued_work(lib):
    """Regression: the workspace may reuse memory that kernels still queued on
    the caller's stream write; lp_create and lp_set_tuning must wait for that
    stream before their first write to it."""
    _flush("create after queued work")
    w = synth.make_small(20000, 256, 16, 8, seed=21, dtype=torch.float32, p_sched=[4] * 4)
    A_dev = w.A.to("cuda:0")
    for _ in range(3):
        x = torch.randn(4096, 4096, device="cuda:0")
        y = x @ x
        del x, y
        P = lib.lp_create(A_dev, w.offsets, 16)
        lib.lp_set_tuning(P, 0, 0)
        r = lib.lp_run(P, 16, w.p_sched, "sign", w.Y0)
    ro = oracle.localpower(upcast(A_dev), w.offsets, 16, w.p_sched, "sign", w.Y0)
    assert sin_theta_np(host(r["Z"]), ro["Z"]) < 1e-5


def test_timed_graph_rounds(lib, fp64_small):
    """Timing the local multiply inside replayed graphs changes nothing in the
    result, times every launch, and keeps the rounds on graphs."""
    w, A, U, lam = fp64_small
    _flush("timed graphs")
    sched = synth.decay_schedule((8, 4, 2, 1), 5)
    P = _problem(lib, to_device(w), w.offsets, w.k)
    r0 = lib.lp_run(P, w.k, sched, "sign", w.Y0, use_graph=False)
    r1 = lib.lp_run(P, w.k, sched, "sign", w.Y0, time_local=True)
    r2 = lib.lp_run(P, w.k, sched, "sign", w.Y0, time_local=True, use_graph=False)
    assert torch.equal(r0["Z"], r1["Z"]) and torch.equal(r0["Z"], r2["Z"])
    for r in (r1, r2):
        st = r["stats"]
        assert st["local_launches"] == sum(sched) and st["ms_local"] > 0
    assert r1["stats"]["graph_rounds"] == len(sched)
    assert r2["stats"]["graph_rounds"] == 0
    # sampled timing: only the first local multiply of every round, same result
    r3 = lib.lp_run(P, w.k, sched, "sign", w.Y0, time_local=2)
    r4 = lib.lp_run(P, w.k, sched, "sign", w.Y0, time_local=2, use_graph=False)
    for r in (r3, r4):
        assert torch.equal(r0["Z"], r["Z"])
        assert r["stats"]["local_launches"] == len(sched) and r["stats"]["ms_local"] > 0
    assert r3["stats"]["graph_rounds"] == len(sched)
    with pytest.raises(lib.LPError):
        lib.lp_run(P, w.k, sched, "sign", w.Y0, time_local=3)


# --------------------------------------------------------------------- split rounds

@pytest.mark.parametrize("mode", ["sign", "opt", "vanilla"])
@pytest.mark.parametrize("dtype,k", [(torch.float64, 8), (torch.float32, 16), (torch.float32, 40)])
def test_split_rounds_match_one_stream(lib, mode, dtype, k):
    """Rounds split into two halves on two streams give the same bits as the
    one-stream rounds (every partition's arithmetic is unchanged; only the order
    across partitions differs), graph-replayed and plain, and agree with the
    oracle.  Uneven partitions, so the largest (base) partition can sit in
    either half; p = 1 rounds included."""
    _flush(f"split rounds {mode} {dtype} k={k}")
    sched = [4, 3, 1, 2, 4]
    w = synth.make_small(6000, 96, k, 7, seed=k + 3, uneven=True, p_sched=sched)
    A_dev = to_device(w, dtype)
    P = _problem(lib, A_dev, w.offsets, k)
    r1 = lib.lp_run(P, k, sched, mode, w.Y0, split_rounds=False, record_signs=True)
    r2 = lib.lp_run(P, k, sched, mode, w.Y0, split_rounds=True, record_signs=True)
    r3 = lib.lp_run(P, k, sched, mode, w.Y0, split_rounds=True, use_graph=False,
                    record_signs=True)
    r4 = lib.lp_run(P, k, sched, mode, w.Y0, split_rounds=True, time_local=1)
    r5 = lib.lp_run(P, k, sched, mode, w.Y0)      # the library's choice
    for r in (r2, r3, r4, r5):
        assert torch.equal(r1["Z"], r["Z"])
    assert np.array_equal(r1["signs"], r2["signs"]) and np.array_equal(r1["signs"], r3["signs"])
    assert r4["stats"]["local_launches"] == sum(sched)
    assert r1["stats"]["split_rounds"] == 0 and r2["stats"]["split_rounds"] == 1
    ro = oracle.localpower(upcast(A_dev), w.offsets, k, sched, mode, w.Y0)
    tol = 1e-10 if dtype == torch.float64 else 1e-5
    assert sin_theta_np(host(r2["Z"]), ro["Z"]) < tol


def test_split_rounds_base_in_second_half(lib):
    """The largest partition last: the half that holds it runs first."""
    _flush("split rounds, base last")
    n, d, k = 4000, 64, 6
    offsets = np.array([0, 500, 1000, 1500, 4000], dtype=np.int64)
    w = synth.make_small(n, d, k, 4, seed=2, p_sched=[3, 3, 3])
    P = _problem(lib, to_device(w), offsets, k)
    for mode in ("sign", "opt"):
        r1 = lib.lp_run(P, k, w.p_sched, mode, w.Y0, split_rounds=False)
        r2 = lib.lp_run(P, k, w.p_sched, mode, w.Y0, split_rounds=True)
        assert torch.equal(r1["Z"], r2["Z"])
        ro = oracle.localpower(w.A.numpy(), offsets, k, w.p_sched, mode, w.Y0)
        assert sin_theta_np(host(r2["Z"]), ro["Z"]) < 1e-10


# --------------------------------------------------------------------- iteration rank r > k

@pytest.mark.parametrize("mode,p", [("sign", 4), ("opt", 4), ("sign", 1)])
def test_oversampled_run(lib, mode, p):
    """Iteration rank r = 8 above the target rank k = 4 (Algorithm 1's r >= k):
    sin theta_k of the rank-r iterate per round, Z and the top-k Ritz pairs
    against the oracle.  The data put sigma_k close to sigma_{k+1} and a wide gap
    after sigma_r."""
    n, d, k, r, m = 2400, 60, 4, 8, 4
    _flush(f"oversampled {mode} p={p}")
    sig = synth.spectrum_cluster(d, k, r)
    A = synth.lowrank_plus_noise(n, d, sig, 0.0, 5)
    offs = synth.equal_offsets(n, m)
    Y0 = synth.gaussian_start(d, r, 5)
    U, _ = oracle.top_k(A.numpy(), k)
    P = _problem(lib, A.to("cuda:0"), offs, r)
    sched = [p] * 12
    g = lib.lp_run(P, r, sched, mode, Y0, ritz=True, U_ref=torch.as_tensor(U))
    ro = oracle.localpower(A.numpy(), offs, r, sched, mode, Y0, U_ref=U)
    assert ro["ambiguous"] == 0
    assert np.abs(g["sin_hist"] - np.array(ro["sin_hist"])).max() < 1e-10
    lam_o, Zr_o, _ = oracle.ritz(A.numpy(), ro["Z"])
    assert np.abs(host(g["ritz"]) - lam_o).max() < 1e-10 * lam_o[0]
    Zg = host(g["Z"])
    assert sin_theta_np(Zg[:, :k], Zr_o[:, :k]) < 1e-9
    assert abs(lib.lp_sin_theta(g["Z"], torch.as_tensor(U, device="cuda:0"))
               - oracle.sin_theta(Zr_o, U)) < 1e-10
    # the same problem and rank with the full-width reference (another history width)
    U8, _ = oracle.top_k(A.numpy(), r)
    g8 = lib.lp_run(P, r, sched, mode, Y0, U_ref=torch.as_tensor(U8))
    ro8 = oracle.localpower(A.numpy(), offs, r, sched, mode, Y0, U_ref=U8)
    assert np.abs(g8["sin_hist"] - np.array(ro8["sin_hist"])).max() < 1e-10
    with pytest.raises(ValueError):
        lib.lp_run(P, k, sched, mode, Y0[:, :k], U_ref=torch.as_tensor(U8))   # k_ref > k


def test_sin_theta_wider_iterate(lib):
    _flush("sin theta, r > k")
    rng = np.random.default_rng(3)
    for d, r, k in ((100, 8, 5), (1031, 64, 1), (4096, 40, 33), (77, 16, 16)):
        U = oracle.orth(rng.standard_normal((d, k)))
        Z = oracle.orth(np.hstack([U, rng.standard_normal((d, r - k))])
                        + 1e-3 * rng.standard_normal((d, r)))
        g = lib.lp_sin_theta(torch.as_tensor(Z, device="cuda:0"), torch.as_tensor(U, device="cuda:0"))
        o = oracle.sin_theta(Z, U)
        assert abs(g - o) < 1e-12 * max(1.0, o) + 1e-6 * o


# --------------------------------------------------------------------- truth-free stop, decaying p

@pytest.mark.parametrize("mode", ["sign", "opt"])
def test_solve_against_oracle(lib, fp64_small, mode):
    """lp_solve: every round's change sin theta(Z_r, Z_{r-1}) against the oracle
    run round by round on the schedule the library chose, that schedule against
    the stated rule applied to the oracle's changes, the final Z and Ritz pairs
    against the oracle, and the final distance to the true subspace."""
    w, A, U, lam = fp64_small
    _flush(f"lp_solve {mode}")
    target = 1e-8
    P = _problem(lib, to_device(w), w.offsets, w.k)
    g = lib.lp_solve(P, w.k, mode, w.Y0, 4, target, 200, ritz=True)
    assert g["status"] == lib.LP_OK
    ps = [int(x) for x in g["p_used"]]
    assert ps[0] == 4 and ps[-1] == 1 and all(a >= b for a, b in zip(ps, ps[1:]))
    Z = oracle.orth(w.Y0)
    ch = []
    for p in ps:
        Zn = oracle.localpower(A, w.offsets, w.k, [p], mode, w.Y0, Z_init=Z)["Z"]
        ch.append(oracle.sin_theta(Zn, Z))
        Z = Zn
    assert np.abs(np.array(ch) - g["changes"]).max() < 1e-10
    ps_rule, done = rule_schedule(ch, 4, target)
    assert done and ps_rule == ps
    lam_o, Zr_o, _ = oracle.ritz(A, Z)
    assert np.abs(host(g["ritz"]) - lam_o).max() < 1e-10 * lam_o[0]
    assert sin_theta_np(host(g["Z"]), Zr_o) < 1e-10
    assert sin_theta_np(host(g["Z"]), U) < target
    st = g["stats"]
    assert st["rounds"] == len(ps) and st["local_iters"] == sum(ps) and st["p_final"] == 1
    assert st["breakdowns"] == 0 and abs(st["change"] - ch[-1]) < 1e-10


def test_solve_round_limit_and_arguments(lib, fp64_small):
    w, A, U, lam = fp64_small
    _flush("lp_solve limits")
    P = _problem(lib, to_device(w), w.offsets, w.k)
    g = lib.lp_solve(P, w.k, "opt", w.Y0, 4, 1e-12, 3)
    assert g["status"] == lib.LP_ENOTCONV and g["stats"]["rounds"] == 3 and g["p_used"][0] == 4
    ro = oracle.localpower(A, w.offsets, w.k, [int(x) for x in g["p_used"]], "opt", w.Y0)
    assert np.abs(host(g["Z"]) - ro["Z"]).max() < 1e-10
    for p0, target, rounds in ((0, 1e-6, 10), (4, 0.0, 10), (4, 1e-6, 0)):
        with pytest.raises(lib.LPError):
            lib.lp_solve(P, w.k, "opt", w.Y0, p0, target, rounds)


# --------------------------------------------------------------------- residual error (Definition 3)

@pytest.mark.parametrize("mode", ["sign", "opt", "vanilla"])
def test_rho_against_oracle(lib, fp64_small, mode):
    """rho at every round's last local step (0 for p = 1 rounds), graph-replayed
    and plain, against the oracle; the iterates are unchanged by measuring it."""
    w, A, U, lam = fp64_small
    _flush(f"rho {mode}")
    sched = [4, 1, 3, 2, 4, 4]
    P = _problem(lib, to_device(w), w.offsets, w.k)
    r0 = lib.lp_run(P, w.k, sched, mode, w.Y0)
    r = lib.lp_run(P, w.k, sched, mode, w.Y0, record_rho=True, split_rounds=True)
    r2 = lib.lp_run(P, w.k, sched, mode, w.Y0, record_rho=True, use_graph=False)
    assert torch.equal(r0["Z"], r["Z"]) and np.array_equal(r["rho"], r2["rho"])
    assert r["stats"]["split_rounds"] == 0
    ro = oracle.localpower(A, w.offsets, w.k, sched, mode, w.Y0)
    assert np.abs(r["rho"] - np.array(ro["rho"])).max() < 1e-10
    assert r["rho"][1] == 0.0 and r["rho"][0] > 0.0
