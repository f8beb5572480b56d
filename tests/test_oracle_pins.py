"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: an
independent formulation (DPI on the whole matrix, single-node power
iteration), a closed form (the Procrustes lemma), brute force (all 2^k sign
matrices, textbook Jacobi), or a trend the paper reports.
"""

import itertools
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.localpower import sign_ambiguous


def _c1():
    w = synth.make_fp64_2000x100()
    A = w.A.numpy()
    U, lam = oracle.top_k(A, w.k)
    return w, A, U, lam


def _rand_orth(rng, d, k):
    q, r = np.linalg.qr(rng.standard_normal((d, k)))
    return q * np.sign(np.diag(r))


# ---------------------------------------------------------------- partitions

def test_partition_setup_integers():
    s, w, b = oracle.partition_setup([0, 3, 10, 17, 20])
    assert list(s) == [3, 7, 7, 3] and b == 1            # argmax, first on ties
    assert abs(w.sum() - 1.0) < 1e-15
    with pytest.raises(ValueError):
        oracle.partition_setup([0, 5, 5, 9])
    with pytest.raises(ValueError):
        oracle.partition_setup([1, 5])


def test_equal_and_lognormal_offsets():
    o = synth.equal_offsets(2003, 4)
    assert list(np.diff(o)) == [501, 501, 501, 500]
    o = synth.lognormal_offsets(500000, 100, math.log(5000), 0.8, 64, 3)
    s = np.diff(o)
    assert o[0] == 0 and o[-1] == 500000 and len(s) == 100 and s.min() >= 64
    # deterministic
    assert np.array_equal(o, synth.lognormal_offsets(500000, 100, math.log(5000), 0.8, 64, 3))


# ---------------------------------------------------------------- T1: p=1 is DPI

@pytest.mark.parametrize("mode", ["vanilla", "sign", "opt"])
def test_p1_equals_dpi_uneven(mode):
    """LocalPower with p = 1 is DPI (Section 3: the standard distributed power
    iteration is the special case p = 1); checked on uneven partitions so the
    weights p_i = s_i/n and the 1/s_i of M_i both matter."""
    w = synth.make_small(1200, 40, 4, 6, seed=11, uneven=True)
    A = w.A.numpy()
    assert len(set(np.diff(w.offsets))) > 1
    r = oracle.localpower(A, w.offsets, w.k, [1] * 25, mode, w.Y0)
    Zd, _ = oracle.dpi(A, w.Y0, 25)
    assert np.abs(r["Z"] - Zd).max() < 1e-12


def test_wrong_weights_break_t1():
    """The pin has teeth: uniform weights instead of p_i move the result."""
    w = synth.make_small(1200, 40, 4, 6, seed=11, uneven=True)
    A = w.A.numpy()
    blocks = [A[w.offsets[i]:w.offsets[i + 1]] for i in range(w.m)]
    Z = oracle.orth(w.Y0)
    for _ in range(25):
        Z = oracle.orth(sum(oracle.local_multiply(B, Z) for B in blocks) / w.m)
    Zd, _ = oracle.dpi(A, w.Y0, 25)
    assert oracle.sin_theta(Z, Zd) > 1e-6


# ---------------------------------------------------------------- T2: eta = 0

@pytest.mark.parametrize("mode", ["vanilla", "sign", "opt"])
@pytest.mark.parametrize("p", [2, 3, 5])
def test_identical_partitions_reduce_to_power_iteration(mode, p):
    """With identical partitions every M_i = M (eta = 0, Definition 2) and all
    local iterates coincide, so R rounds of p local steps are R*p steps of
    single-node power iteration (the update rule: D = I after a sync)."""
    rng = np.random.default_rng(3)
    B = rng.standard_normal((60, 12)) @ np.diag(np.linspace(2, 0.2, 12))
    m, k, R = 4, 3, 6
    A = np.vstack([B] * m)
    offs = synth.equal_offsets(A.shape[0], m)
    Y0 = rng.standard_normal((12, k))
    r = oracle.localpower(A, offs, k, [p] * R, mode, Y0)
    Z1 = oracle.power_iteration(B.T @ B / B.shape[0], Y0, R * p)
    tol = 1e-12 if mode != "opt" else 1e-11
    assert np.abs(r["Z"] - Z1).max() < tol
    assert oracle.eta(A, offs) < 1e-14


# ---------------------------------------------------------------- T3: k = 1

def test_k1_opt_equals_sign():
    """For k = 1, OPT and sign-fixing coincide (remark after Eq. (opt:d))."""
    w = synth.make_small(800, 30, 1, 4, seed=5)
    A = w.A.numpy()
    ro = oracle.localpower(A, w.offsets, 1, [4] * 12, "opt", w.Y0)
    rs = oracle.localpower(A, w.offsets, 1, [4] * 12, "sign", w.Y0)
    assert np.abs(ro["Z"] - rs["Z"]).max() < 1e-13


# ---------------------------------------------------------------- T4: injected bases

def _identical_problem():
    rng = np.random.default_rng(9)
    B = rng.standard_normal((80, 15)) @ np.diag(np.linspace(3, 0.3, 15))
    m, k = 5, 4
    A = np.vstack([B] * m)
    return A, B, synth.equal_offsets(A.shape[0], m), rng.standard_normal((15, k)), k


def test_opt_undoes_injected_rotations():
    """Local bases that differ by arbitrary rotations: OPT (Eq. (opt:o)) maps
    each Z_i back onto the base node, so the subspace equals single-node power
    iteration.  A transposed W1 W2^T or an alignment taken from the wrong
    iterate fails here."""
    A, B, offs, Y0, k = _identical_problem()
    rng = np.random.default_rng(21)

    def rot(Y):
        return oracle.orth(Y) @ _rand_orth(rng, k, k)

    R, p = 5, 3
    M = B.T @ B / B.shape[0]
    r = oracle.localpower(A, offs, k, [p] * R, "opt", Y0, local_orth=rot)
    Z1 = oracle.power_iteration(M, Y0, R * p)
    assert oracle.sin_theta(r["Z"], Z1) < 1e-12
    # The aggregate itself: with every Z_i O_i equal to the base's input, Y is
    # M times an orthonormal basis, so its singular values are those of
    # M Z_prev (basis-invariant).  Averaging unaligned rotations shrinks them.
    sv_ref = np.linalg.svd(M @ oracle.power_iteration(M, Y0, R * p - 1), compute_uv=False)
    sv = np.linalg.svd(r["Y"], compute_uv=False)
    assert np.abs(sv - sv_ref).max() < 1e-12 * sv_ref[0]
    rv = oracle.localpower(A, offs, k, [p] * R, "vanilla", Y0, local_orth=rot)
    sv_v = np.linalg.svd(rv["Y"], compute_uv=False)
    assert np.abs(sv_v - sv_ref).max() > 1e-3 * sv_ref[0]      # teeth


def test_sign_undoes_injected_sign_flips():
    """Local bases that differ by column signs: sign-fixing and OPT both
    restore single-node power iteration, elementwise up to column signs."""
    A, B, offs, Y0, k = _identical_problem()
    rng = np.random.default_rng(22)

    def flip(Y):
        return oracle.orth(Y) * rng.choice([-1.0, 1.0], Y.shape[1])

    R, p = 5, 3
    Z1 = oracle.power_iteration(B.T @ B / B.shape[0], Y0, R * p)
    for mode in ("sign", "opt"):
        r = oracle.localpower(A, offs, k, [p] * R, mode, Y0, local_orth=flip)
        Z = r["Z"] * np.sign(np.sum(r["Z"] * Z1, axis=0))
        assert np.abs(Z - Z1).max() < 1e-11


# ---------------------------------------------------------------- T5: sign brute force

@pytest.mark.parametrize("k", [1, 3, 6, 8])
def test_sign_fix_is_brute_force_minimum(k):
    """Eq. (opt:d): the column formula minimises ||Z_i D - Z_b||_F over all
    2^k diagonal sign matrices."""
    rng = np.random.default_rng(k)
    Zi, Zb = _rand_orth(rng, 20, k), _rand_orth(rng, 20, k)
    best, arg = np.inf, None
    for sv in itertools.product([-1.0, 1.0], repeat=k):
        v = np.linalg.norm(Zi * np.array(sv) - Zb)
        if v < best - 1e-14:
            best, arg = v, np.array(sv)
    assert np.array_equal(oracle.sign_fix(Zi, Zb), arg)


def test_sign_zero_is_plus():
    Zi = np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]])
    Zb = np.array([[0.0, 0.0], [0.0, -1.0], [1.0, 0.0]])
    assert list(oracle.sign_fix(Zi, Zb)) == [1.0, -1.0]
    assert list(sign_ambiguous(Zi, Zb)) == [True, False]


# ---------------------------------------------------------------- T6: Procrustes lemma

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_opt_closed_form(seed):
    """Procrustes lemma (appendix): O* = W1 W2^T is orthogonal,
    O*^T (Ut^T U) is symmetric positive semi-definite, and
    ||U - Ut O*||_2 = sqrt(2 - 2 sqrt(1 - dist^2)) = 2 sin(theta_k / 2)."""
    rng = np.random.default_rng(seed)
    d, k = 30, 5
    U = _rand_orth(rng, d, k)
    Ut = oracle.orth(U @ _rand_orth(rng, k, k) + 0.3 * rng.standard_normal((d, k)))
    O = oracle.opt_matrix(Ut, U)
    assert np.abs(O.T @ O - np.eye(k)).max() < 1e-14
    S = O.T @ (Ut.T @ U)
    assert np.abs(S - S.T).max() < 1e-14 and np.linalg.eigvalsh(S).min() > -1e-14
    dist = oracle.projection_distance(U, Ut)
    lhs = np.linalg.norm(U - Ut @ O, 2)
    assert abs(lhs - math.sqrt(2 - 2 * math.sqrt(1 - dist ** 2))) < 1e-13
    assert abs(lhs - 2 * math.sin(math.asin(dist) / 2)) < 1e-13
    # O* beats every rotation nearby and random orthogonal matrices
    f0 = np.linalg.norm(Ut @ O - U)
    for _ in range(200):
        K = rng.standard_normal((k, k))
        K = 0.05 * (K - K.T)
        Q = O @ (np.eye(k) + K) @ np.linalg.inv(np.eye(k) - K)    # Cayley: orthogonal
        assert np.linalg.norm(Ut @ Q - U) >= f0 - 1e-13
        assert np.linalg.norm(Ut @ _rand_orth(rng, k, k) - U) >= f0 - 1e-13


def test_opt_k2_grid():
    """k = 2: brute force over the whole orthogonal group O(2) on a fine grid."""
    rng = np.random.default_rng(7)
    U, Ut = _rand_orth(rng, 12, 2), _rand_orth(rng, 12, 2)
    O = oracle.opt_matrix(Ut, U)
    f0 = np.linalg.norm(Ut @ O - U)
    for a in np.linspace(0, 2 * np.pi, 3601):
        c, s = math.cos(a), math.sin(a)
        for Q in (np.array([[c, -s], [s, c]]), np.array([[c, s], [s, -c]])):
            assert np.linalg.norm(Ut @ Q - U) >= f0 - 1e-12


# ---------------------------------------------------------------- T7: tiny d, Jacobi truth

def test_jacobi_matches_lapack_and_dpi_converges():
    rng = np.random.default_rng(4)
    d, k = 8, 3
    A = rng.standard_normal((400, d)) @ np.diag([3, 2.5, 2, 1, 0.8, 0.6, 0.4, 0.2])
    M = A.T @ A / A.shape[0]
    lam_j, V_j = oracle.jacobi_eig(M)
    lam_l = np.sort(np.linalg.eigvalsh(M))[::-1]
    assert np.abs(lam_j - lam_l).max() < 1e-13 * lam_l[0]
    assert np.abs(V_j.T @ V_j - np.eye(d)).max() < 1e-13
    assert np.abs(V_j @ np.diag(lam_j) @ V_j.T - M).max() < 1e-13 * lam_l[0]
    Uk = V_j[:, :k]
    U_l, _ = oracle.top_k(A, k)
    assert oracle.sin_theta(U_l, Uk) < 1e-12
    Y0 = rng.standard_normal((d, k))
    Zd, hist = oracle.dpi(A, Y0, 200, Uk)
    assert hist[-1] < 1e-12
    offs = synth.equal_offsets(400, 4)
    r = oracle.localpower(A, offs, k, synth.decay_schedule((4, 2, 1), 25), "sign", Y0, U_ref=Uk)
    assert r["sin_hist"][-1] < 1e-12


# ---------------------------------------------------------------- T8: sign invariance

def test_sign_fix_invariant_to_local_sign_choice():
    """Sign-fixing makes the run independent of the local QR's column signs:
    a random-sign orth gives the positive-diagonal result up to global signs."""
    w, A, U, lam = _c1()
    rng = np.random.default_rng(5)

    def flip(Y):
        return oracle.orth(Y) * rng.choice([-1.0, 1.0], Y.shape[1])

    sched = [4] * 8
    r0 = oracle.localpower(A, w.offsets, w.k, sched, "sign", w.Y0)
    r1 = oracle.localpower(A, w.offsets, w.k, sched, "sign", w.Y0, local_orth=flip)
    Z1 = r1["Z"] * np.sign(np.sum(r1["Z"] * r0["Z"], axis=0))
    assert np.abs(Z1 - r0["Z"]).max() < 1e-12


# ---------------------------------------------------------------- T9: DPI rate

def test_dpi_contraction_rate():
    """Lemma 1 / Eq. (power): tan theta_k shrinks by lambda_{k+1}/lambda_k per
    round once the tail is clean."""
    w, A, U, lam = _c1()
    _, h = oracle.dpi(A, w.Y0, 16, U)
    tan = [x / math.sqrt(1 - x * x) for x in h]
    q = lam[w.k] / lam[w.k - 1]
    for t in range(8, 14):
        assert abs(tan[t + 1] / tan[t] / q - 1) < 0.05


# ---------------------------------------------------------------- T10: orthonormality

def test_orthonormal_iterates():
    w, A, U, lam = _c1()
    worst = [0.0]

    def checked(Y):
        Q = oracle.orth(Y)
        worst[0] = max(worst[0], np.abs(Q.T @ Q - np.eye(Q.shape[1])).max())
        return Q

    r = oracle.localpower(A, w.offsets, w.k, [4] * 10, "opt", w.Y0, local_orth=checked)
    Z = r["Z"]
    assert worst[0] < 1e-14 and np.abs(Z.T @ Z - np.eye(w.k)).max() < 1e-14


def _gram_schmidt(Y):
    """Thin QR by modified Gram-Schmidt in plain loops: each column is the
    remainder of y_j after removing its components along q_1..q_{j-1},
    divided by its (positive) norm, so R_jj > 0 by construction."""
    d, k = Y.shape
    Q = [[float(Y[i, j]) for j in range(k)] for i in range(d)]
    for j in range(k):
        for i in range(j):
            c = sum(Q[r][i] * Q[r][j] for r in range(d))
            for r in range(d):
                Q[r][j] -= c * Q[r][i]
        nrm = math.sqrt(sum(Q[r][j] ** 2 for r in range(d)))
        for r in range(d):
            Q[r][j] /= nrm
    return np.array(Q)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_orth_is_the_positive_diagonal_qr(seed):
    """orth(Y) is the thin QR factor whose R has a positive diagonal (the
    reading of the paper's unspecified QR sign convention): Q^T Q = I,
    R = Q^T Y upper triangular with R_jj > 0, Q R = Y, and Q equals plain
    Gram-Schmidt.  The inputs are chosen so that LAPACK's own Householder R
    has negative diagonal entries, which orth must flip."""
    rng = np.random.default_rng(100 + seed)
    d, k = 40, 7
    for _ in range(50):
        Y = rng.standard_normal((d, k)) * rng.uniform(0.5, 2.0, k)[None, :]
        if np.any(np.diag(np.linalg.qr(Y)[1]) < 0):
            break
    else:
        pytest.fail("no input with a negative Householder diagonal")
    Q = oracle.orth(Y)
    R = Q.T @ Y
    scale = np.abs(Y).max()
    assert np.abs(Q.T @ Q - np.eye(k)).max() < 1e-14
    assert np.abs(np.tril(R, -1)).max() < 1e-14 * scale
    assert np.all(np.diag(R) > 0)
    assert np.abs(Q @ np.triu(R) - Y).max() < 1e-14 * scale
    assert np.abs(Q - _gram_schmidt(Y)).max() < 1e-12


# ---------------------------------------------------------------- T14: initial angle

def _tan_theta(U, Z):
    """tan theta_k(U, Z) = ||(U_perp^T Z)(U^T Z)^+||_2 (the appendix's list of
    facts on principal angles), U d x k orthonormal, Z d x r (r >= k)."""
    d, k = U.shape
    full, _ = np.linalg.qr(np.hstack([U, np.eye(d)]))
    Uperp = full[:, k:d]
    return float(np.linalg.norm((Uperp.T @ Z) @ np.linalg.pinv(U.T @ Z), 2))


@pytest.mark.parametrize("r", [5, 6, 8, 16])
def test_initial_angle_bound(r):
    """T14, Lemma "initial" (Hardt and Price's Lemma 2.4): for a random
    orthonormal start Z_0 (orth of the Gaussian start, as every run starts),
    tan theta_k(U, Z_0) <= tau sqrt(d) / (sqrt(r) - sqrt(k - 1)) except with
    probability tau^-Omega(r + 1 - k) + e^-Omega(d); tau = 10 over 200 draws.
    With r = k the failure probability is only tau^-Omega(1): a k x k Gaussian
    block has sigma_min below eps / sqrt(k) with probability about eps, which
    puts the rate near 1 / (2 tau) = 5 %; with r > k no draw may fail.
    Statistical; a degenerate start orthogonal to U violates it (tan =
    infinity), and for r = k the tangent agrees with the principal-angle form
    sin/cos of sigma_min(U^T Z)."""
    d, k, tau = 200, 5, 10.0
    rng = np.random.default_rng(r)
    U = _rand_orth(rng, d, k)
    bound = tau * math.sqrt(d) / (math.sqrt(r) - math.sqrt(k - 1))
    tans = []
    for t in range(200):
        Z0 = oracle.orth(synth.gaussian_start(d, r, 1000 * r + t))
        tans.append(_tan_theta(U, Z0))
        if r == k and t < 20:
            c = np.linalg.svd(U.T @ Z0, compute_uv=False).min()
            assert abs(tans[-1] - math.sqrt(1 - c * c) / c) < 1e-9 * max(1.0, tans[-1])
    fails = float(np.mean(np.array(tans) > bound))
    if r == k:
        assert fails <= 0.12
    else:
        assert fails == 0.0
    # more columns than the target rank shrink the angle (the r in the bound)
    assert np.median(tans) < bound / 5
    # a start orthogonal to U has no component to amplify: the bound fails
    basis, _ = np.linalg.qr(np.hstack([U, rng.standard_normal((d, r))]))
    assert not (_tan_theta(U, basis[:, k:k + r]) <= bound)


# ---------------------------------------------------------------- T11-T13: trends

def test_floor_grows_with_p_and_decay_reaches_dpi():
    """Fixed p > 1 leaves a floor that grows with p; decaying p to 1 reaches
    DPI precision (Section 3 'Decaying p', Corollary 1)."""
    w, A, U, lam = _c1()
    floors = [oracle.localpower(A, w.offsets, w.k, [p] * 30, "sign", w.Y0, U_ref=U)["sin_hist"][-1]
              for p in (2, 4, 8)]
    assert 1e-4 < floors[0] < floors[1] < floors[2]
    r = oracle.localpower(A, w.offsets, w.k, synth.decay_schedule((8, 4, 2, 1), 10), "sign",
                          w.Y0, U_ref=U)
    assert r["sin_hist"][-1] < 1e-10


def test_opt_floor_below_sign_floor():
    """OPT is the more accurate alignment (Table 1 trend)."""
    w, A, U, lam = _c1()
    fs = oracle.localpower(A, w.offsets, w.k, w.p_sched, "sign", w.Y0, U_ref=U)["sin_hist"][-1]
    fo = oracle.localpower(A, w.offsets, w.k, w.p_sched, "opt", w.Y0, U_ref=U)["sin_hist"][-1]
    assert fo < fs


def test_vanilla_unstable_under_sign_flips():
    """Without alignment, local sign flips spoil the average (stability
    paragraph); sign-fixing and OPT do not care."""
    w, A, U, lam = _c1()
    rng = np.random.default_rng(5)

    def flip(Y):
        return oracle.orth(Y) * rng.choice([-1.0, 1.0], Y.shape[1])

    fv = oracle.localpower(A, w.offsets, w.k, w.p_sched, "vanilla", w.Y0, U_ref=U,
                           local_orth=flip)["sin_hist"][-1]
    fs = oracle.localpower(A, w.offsets, w.k, w.p_sched, "sign", w.Y0, U_ref=U,
                           local_orth=flip)["sin_hist"][-1]
    assert fv > 0.05 and fs < 1e-2


# ---------------------------------------------------------------- distance, Ritz, init

def test_sin_theta_prescribed_angles():
    """Z = [diag(cos t); diag(sin t); 0] against U = [I; 0; 0] has principal
    angles t, so sin theta_k = max sin t -- also for tiny angles where the
    cosine form would lose everything."""
    k = 4
    for th in ([0.3, 0.1, 0.2, 0.05], [1e-12, 3e-12, 2e-12, 1e-13]):
        th = np.array(th)
        d = 3 * k
        U = np.zeros((d, k)); U[:k] = np.eye(k)
        Z = np.zeros((d, k)); Z[:k] = np.diag(np.cos(th)); Z[k:2 * k] = np.diag(np.sin(th))
        assert abs(oracle.sin_theta(Z, U) - np.sin(th).max()) < 1e-3 * np.sin(th).max()
    rng = np.random.default_rng(1)
    U, Z = _rand_orth(rng, 15, 3), _rand_orth(rng, 15, 3)
    assert abs(oracle.sin_theta(Z, U) - oracle.projection_distance(Z, U)) < 1e-13


def test_ritz_values_at_convergence():
    w, A, U, lam = _c1()
    Zd, _ = oracle.dpi(A, w.Y0, 40)
    rl, Zr, sg = oracle.ritz(A, Zd)
    assert np.abs(rl - lam[:w.k]).max() < 1e-12 * lam[0]
    assert np.abs(sg - np.sqrt(A.shape[0] * lam[:w.k])).max() < 1e-9
    assert oracle.sin_theta(Zr, U) < 1e-12


def test_generator_spectrum_c1():
    """The stand-in for the paper's data has the intended eigen-gap."""
    w, A, U, lam = _c1()
    assert A.shape == (2000, 100) and w.A.dtype == torch.float64
    assert 4.0 < lam[4] / lam[5] < 8.0


# ---------------------------------------------------------------- iteration rank r > k

def _cluster(n=2400, d=60, k=4, r=8, seed=5):
    """sigma_k close to sigma_{k+1}, a wide gap after sigma_r, noise-free, so
    M = A^T A / n has eigenvalues sigma_j^2 exactly."""
    sig = synth.spectrum_cluster(d, k, r)
    A = synth.lowrank_plus_noise(n, d, sig, 0.0, seed).numpy()
    lam, V = np.linalg.eigh(A.T @ A / n)
    lam, V = lam[::-1], V[:, ::-1]
    return A, lam, V[:, :k], sig


def test_sin_theta_wider_iterate():
    """Definition 1 with a d x r iterate: columns outside span(U) and its
    complement's relevant directions leave the angles alone; a column along a
    missing direction removes that angle."""
    k = 3
    th = np.array([0.3, 0.1, 0.2])
    d = 4 * k
    U = np.zeros((d, k)); U[:k] = np.eye(k)
    Z = np.zeros((d, k + 2)); Z[:k, :k] = np.diag(np.cos(th)); Z[k:2 * k, :k] = np.diag(np.sin(th))
    Z[3 * k, k] = 1.0; Z[3 * k + 1, k + 1] = 1.0          # unrelated extra directions
    assert abs(oracle.sin_theta(Z, U) - np.sin(th).max()) < 1e-14
    # adding e_{k+1}, the direction that z_1 leans into, puts e_1 into the span;
    # an orthonormal basis of that span is e_{k+1}, z_2, z_3, e_1 (e_1 last, so a
    # distance that read only the first k columns would see an angle of 90 degrees)
    Z2 = np.zeros((d, k + 1)); Z2[:, 1:k] = Z[:, 1:k]; Z2[k, 0] = 1.0; Z2[0, k] = 1.0
    assert np.abs(Z2.T @ Z2 - np.eye(k + 1)).max() < 1e-15
    assert abs(oracle.sin_theta(Z2, U) - np.sin(th[1:]).max()) < 1e-14
    Z3 = np.eye(d)[:, :2 * k]
    assert oracle.sin_theta(Z3, U) < 1e-15


def test_oversampled_rate():
    """Iteration rank r above the target rank k (Algorithm 1's input; the
    appendix on the eigengap): with p = 1 the run is subspace iteration, and
    tan theta_k shrinks by lambda_{r+1} / lambda_k per round, so the gap that
    matters is the one after lambda_r.  At rank k the same data converge at
    lambda_{k+1} / lambda_k, here 0.97 per round."""
    n, d, k, r, m = 2400, 60, 4, 8, 4
    A, lam, Uk, sig = _cluster(n, d, k, r)
    assert np.abs(lam - sig ** 2).max() < 1e-13 * lam[0]
    offs = synth.equal_offsets(n, m)
    Y0 = synth.gaussian_start(d, r, 5)
    ro = oracle.localpower(A, offs, r, [1] * 16, "sign", Y0, U_ref=Uk)
    tan = [x / math.sqrt(1 - x * x) for x in ro["sin_hist"]]
    q = lam[r] / lam[k - 1]
    for t in range(6, 13):
        assert abs(tan[t + 1] / tan[t] / q - 1) < 0.02
    rk = oracle.localpower(A, offs, k, [1] * 16, "sign", Y0[:, :k], U_ref=Uk)
    assert rk["sin_hist"][-1] > 0.5 and ro["sin_hist"][-1] < 1e-11


def test_oversampled_ritz_top_k():
    """The top k Ritz pairs of the converged rank-r iterate are the top k
    eigenpairs of M."""
    n, d, k, r, m = 2400, 60, 4, 8, 4
    A, lam, Uk, _ = _cluster(n, d, k, r)
    ro = oracle.localpower(A, synth.equal_offsets(n, m), r, [1] * 30, "opt",
                           synth.gaussian_start(d, r, 5))
    rl, Zr, _ = oracle.ritz(A, ro["Z"])
    assert np.abs(rl[:k] - lam[:k]).max() < 1e-13 * lam[0]
    assert oracle.sin_theta(Zr[:, :k], Uk) < 1e-11


# ---------------------------------------------------------------- eta (Definition 2)

def test_eta_closed_form():
    """Two partitions along the axes: s1 rows [a, 0], s2 rows [0, b] give
    M_1 = diag(a^2, 0), M_2 = diag(0, b^2), M = diag(p1 a^2, p2 b^2), so
    eta = max(|M_1 - M|, |M_2 - M|) / |M| in closed form (diagonal matrices)."""
    for a, b, s1, s2 in ((2.0, 1.0, 25, 75), (1.0, 2.0, 25, 75), (1.0, 1.0, 50, 50), (3.0, 0.5, 10, 90)):
        A = np.vstack([np.tile([a, 0.0], (s1, 1)), np.tile([0.0, b], (s2, 1))])
        p1, p2 = s1 / (s1 + s2), s2 / (s1 + s2)
        Mn = max(p1 * a * a, p2 * b * b)
        e1 = max(a * a * (1 - p1), p2 * b * b)
        e2 = max(p1 * a * a, b * b * (1 - p2))
        assert abs(oracle.eta(A, [0, s1, s1 + s2]) - max(e1, e2) / Mn) < 1e-14 * max(e1, e2) / Mn


def test_eta_grows_with_m():
    """Uniform partitions of one matrix: smaller local samples (larger m) put the
    local matrices further from M (the paper's local-sample-size experiment)."""
    A = synth.lowrank_plus_noise(4096, 32, synth.spectrum_c1(32, 4), 0.05, 11).numpy()
    e = [oracle.eta(A, synth.equal_offsets(4096, m)) for m in (2, 8, 32)]
    assert e[0] < e[1] < e[2]


# ---------------------------------------------------------------- rho (Definition 3)

def test_residual_error_opt_brute_force_and_closed_form():
    """min over orthogonal O of ||Z_i O - Z_1||_2 (k = 2): a dense grid over all
    rotations and reflections never beats the oracle's value, which equals
    2 sin(theta_max / 2) of the principal angles."""
    rng = np.random.default_rng(4)
    for _ in range(25):
        Z1 = _rand_orth(rng, 7, 2)
        Zi = oracle.orth(Z1 + 0.6 * rng.standard_normal((7, 2)))
        got = oracle.residual_error([Z1, Zi], True)
        best = min(np.linalg.norm(Zi @ R - Z1, 2)
                   for a in np.linspace(0, 2 * np.pi, 2001)
                   for R in (np.array([[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]]),
                             np.array([[np.cos(a), np.sin(a)], [np.sin(a), -np.cos(a)]])))
        assert got <= best + 1e-12 and best - got < 2e-3
        assert abs(got - 2 * np.sin(np.arcsin(oracle.sin_theta(Zi, Z1)) / 2)) < 1e-12
    # without OPT it is the plain spectral norm of the difference: a sign flip costs 2
    Z1 = _rand_orth(rng, 7, 3)
    assert abs(oracle.residual_error([Z1, Z1 * np.array([1, -1, 1])], False) - 2.0) < 1e-12
    assert oracle.residual_error([Z1, Z1 * np.array([1, -1, 1])], True) < 1e-12


def test_residual_error_zero_at_p1_and_grows_with_p():
    """rho is 0 when every node starts the step from the broadcast Z (p = 1), and
    the spread of the local iterates grows with the local steps between
    communications; OPT keeps it below the plain difference."""
    w = synth.make_small(3000, 40, 4, 6, seed=2, noise=0.3)
    A = w.A.numpy()
    r1 = oracle.localpower(A, w.offsets, 4, [1] * 3, "sign", w.Y0)
    assert max(r1["rho"]) == 0.0
    last = {}
    for p in (2, 4, 8):
        ro = oracle.localpower(A, w.offsets, 4, [p] * 6, "opt", w.Y0)
        rs = oracle.localpower(A, w.offsets, 4, [p] * 6, "sign", w.Y0)
        assert ro["rho"][-1] <= rs["rho"][-1] + 1e-15
        last[p] = ro["rho"][-1]
    assert last[2] < last[4] < last[8]
