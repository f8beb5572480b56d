"""LocalPower in plain NumPy float64 (oracle; test infrastructure only).

Notation follows the paper: A_i (s_i x d) is the i-th row partition of A,
M_i = A_i^T A_i / s_i, p_i = s_i / n, M = sum_i p_i M_i = A^T A / n.
A run is a list of communication rounds; round r performs p_r local
iterations on every node and ends with one aggregation (Algorithm 1 with the
communication set I_T = {0, p, 2p, ...}, in the form of the update rule
Eqs. (V), (Y), (Z) of the appendix).
"""

from __future__ import annotations

from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

AMBIGUOUS_SIGN = 1e-8


def partition_setup(offsets: Sequence[int]):
    """Sizes s_i, weights p_i = s_i / n and the base node.

    The base node is the one holding the most samples (Section 3, OPT
    paragraph; the update rule assumes node 1 = argmax_i p_i); ties go to the
    lowest index.
    """
    o = np.asarray(offsets, dtype=np.int64)
    if o.ndim != 1 or len(o) < 2 or o[0] != 0 or np.any(np.diff(o) <= 0):
        raise ValueError("offsets must start at 0 and increase strictly")
    s = np.diff(o)
    n = int(o[-1])
    w = s.astype(np.float64) / float(n)
    base = int(np.argmax(s))  # numpy returns the first maximum
    return s, w, base


def orth(Y: np.ndarray) -> np.ndarray:
    """orth(Y): the Q of the thin QR factorisation Y = QR with R_jj > 0.

    The paper's orth is "a QR factorisation" (Notation; Eq. (Z)) and leaves
    the column signs open; the positive-diagonal factor is the unique choice.
    Householder QR from LAPACK, then column signs flipped where R_jj < 0.
    """
    Q, R = np.linalg.qr(Y, mode="reduced")
    sgn = np.sign(np.diag(R))
    sgn[sgn == 0] = 1.0
    return Q * sgn[None, :]


def local_multiply(A_i: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """Y_i = M_i Z = (1/s_i) A_i^T (A_i Z)  (Eq. (power_yi))."""
    return (A_i.T @ (A_i @ Z)) / float(A_i.shape[0])


def sign_fix(Z_i: np.ndarray, Z_b: np.ndarray) -> np.ndarray:
    """Diagonal of D_i = argmin_{D in D_k} ||Z_i D - Z_b||_F  (Eq. (opt:d)).

    D[j, j] = sgn(<Z_i[:, j], Z_b[:, j]>), with sgn(0) taken as +1.
    """
    c = np.sum(Z_i * Z_b, axis=0)
    return np.where(c >= 0.0, 1.0, -1.0)


def sign_ambiguous(Z_i: np.ndarray, Z_b: np.ndarray) -> np.ndarray:
    """Columns whose sign decision sits within rounding of zero."""
    c = np.sum(Z_i * Z_b, axis=0)
    scale = np.linalg.norm(Z_i, axis=0) * np.linalg.norm(Z_b, axis=0)
    return np.abs(c) < AMBIGUOUS_SIGN * scale


def opt_matrix(Z_i: np.ndarray, Z_b: np.ndarray) -> np.ndarray:
    """O_i = argmin_{O in O_k} ||Z_i O - Z_b||_F = W1 W2^T  (Eq. (opt:o)),

    where W1 Sigma W2^T is the SVD of Z_i^T Z_b.
    """
    W1, _, W2t = np.linalg.svd(Z_i.T @ Z_b)
    return W1 @ W2t


def sin_theta(Z: np.ndarray, U: np.ndarray) -> float:
    """sin theta_k(Z, U) = ||(I - Z Z^T) U||_2  (Definition 1 and the
    experimental section's form), evaluated as the largest singular value of
    U - Z (Z^T U) so that tiny angles keep their relative accuracy."""
    W = U - Z @ (Z.T @ U)
    return float(np.linalg.norm(W, 2))


def projection_distance(Z: np.ndarray, U: np.ndarray) -> float:
    """dist(Z, U) = ||Z Z^T - U U^T||_2 written out (Definition 1); d x d."""
    return float(np.linalg.norm(Z @ Z.T - U @ U.T, 2))


def residual_error(Z_list: Sequence[np.ndarray], use_opt: bool) -> float:
    """rho (Definition 3) of a set of local iterates: max_i ||Z_i - Z_1||_2 without
    OPT, max_i min_O ||Z_i O - Z_1||_2 over orthogonal O with OPT.  The minimiser
    is the polar factor of Z_i^T Z_1 (the Procrustes rotation of Eq. (opt:o)),
    which minimises the spectral distance too for matrices with orthonormal
    columns."""
    Z1 = Z_list[0]
    out = 0.0
    for Zi in Z_list:
        D = Zi @ opt_matrix(Zi, Z1) - Z1 if use_opt else Zi - Z1
        out = max(out, float(np.linalg.norm(D, 2)))
    return out


def _blocks(A: np.ndarray, offsets: Sequence[int]) -> List[np.ndarray]:
    o = np.asarray(offsets, dtype=np.int64)
    return [A[o[i]:o[i + 1]] for i in range(len(o) - 1)]


def localpower(A: np.ndarray, offsets: Sequence[int], k: int, p_sched: Sequence[int],
               mode: str, Y0: np.ndarray, U_ref: Optional[np.ndarray] = None,
               local_orth: Callable[[np.ndarray], np.ndarray] = orth,
               Z_init: Optional[np.ndarray] = None) -> Dict[str, object]:
    """Run LocalPower for len(p_sched) communication rounds.

    Round r with p = p_sched[r]:
      1. broadcast: Z_i <- Z on every node;
      2. p local iterations on every node: V_i = M_i Z_i, and between local
         iterations Z_i <- orth(V_i) (Algorithm 1, local computation);
      3. alignment of the inputs of the last local iteration against the base
         node's: D_i = I when p = 1 or mode is vanilla (the remark after the
         sign-fixing paragraph), the sign matrix (Eq. (opt:d)) for "sign",
         the Procrustes rotation (Eq. (opt:o)) for "opt";
      4. aggregation Y = sum_i p_i V_i D_i  (Eq. (Y)), then Z = orth(Y).
    The start is Z = orth(Y0) (Algorithm 1, initialisation), unless Z_init
    supplies an already orthonormal start.

    Returns a dict with Z, per-round sign vectors, ambiguity counts, the
    residual error rho (Definition 3) of each round's last local step and
    (when U_ref is given) the per-round sin theta history.
    """
    if mode not in ("vanilla", "sign", "opt"):
        raise ValueError(mode)
    A = np.asarray(A, dtype=np.float64)
    s, w, b = partition_setup(offsets)
    m = len(s)
    if k < 1 or k > A.shape[1] or np.any(s < k):
        raise ValueError("need 1 <= k <= d and every s_i >= k")
    blocks = _blocks(A, offsets)
    Z = np.array(Z_init, dtype=np.float64) if Z_init is not None else orth(np.asarray(Y0, np.float64))
    hist: List[float] = []
    rho: List[float] = []
    signs: List[Optional[np.ndarray]] = []
    ambiguous = 0
    local_iters = 0
    for p in p_sched:
        p = int(p)
        if p < 1:
            raise ValueError("p must be >= 1")
        Zi = [Z for _ in range(m)]
        Zlast = Zi
        V: List[np.ndarray] = []
        for step in range(1, p + 1):
            Zlast = Zi
            V = [local_multiply(blocks[i], Zi[i]) for i in range(m)]
            local_iters += 1
            if step < p:
                Zi = [local_orth(V[i]) for i in range(m)]
        # residual error at the last local step (the largest of the round; 0 at p = 1)
        rho.append(residual_error(Zlast, mode == "opt"))
        if p == 1 or mode == "vanilla":
            D = [np.eye(k) for _ in range(m)]
            signs.append(None)
        elif mode == "sign":
            sv = [sign_fix(Zlast[i], Zlast[b]) for i in range(m)]
            ambiguous += int(sum(int(np.sum(sign_ambiguous(Zlast[i], Zlast[b]))) for i in range(m)))
            D = [np.diag(v) for v in sv]
            signs.append(np.array(sv, dtype=np.int8))
        else:
            D = [opt_matrix(Zlast[i], Zlast[b]) for i in range(m)]
            signs.append(None)
        Y = np.zeros_like(V[0])
        for i in range(m):
            Y += w[i] * (V[i] @ D[i])
        Z = orth(Y)
        if U_ref is not None:
            hist.append(sin_theta(Z, U_ref))
    return {"Z": Z, "Y": Y, "sin_hist": hist, "rho": rho, "signs": signs, "ambiguous": ambiguous,
            "rounds": len(p_sched), "local_iters": local_iters, "base": b}


def dpi(A: np.ndarray, Y0: np.ndarray, T: int, U_ref: Optional[np.ndarray] = None):
    """Distributed power iteration written on the whole matrix: T times
    Y = M Z with M = A^T A / n, then Z = orth(Y)  (Eq. (power); the server's
    aggregate sum_i p_i M_i Z equals M Z)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    Z = orth(np.asarray(Y0, np.float64))
    hist = []
    for _ in range(T):
        Z = orth((A.T @ (A @ Z)) / n)
        if U_ref is not None:
            hist.append(sin_theta(Z, U_ref))
    return Z, hist


def power_iteration(Mmat: np.ndarray, Y0: np.ndarray, steps: int, Z_init=None) -> np.ndarray:
    """Single-node subspace iteration Z <- orth(M Z) for `steps` steps on an
    explicit d x d matrix (Eq. (power))."""
    Z = np.array(Z_init, np.float64) if Z_init is not None else orth(np.asarray(Y0, np.float64))
    for _ in range(steps):
        Z = orth(Mmat @ Z)
    return Z


def ritz(A: np.ndarray, Z: np.ndarray):
    """Rayleigh-Ritz on span(Z): H = Z^T M Z, H = Q diag(lam) Q^T.

    Returns (lam descending, Z Q, sigma = sqrt(n * lam)): lam are Ritz values
    of M (the paper's sigma_j are eigenvalues of M, Lemma 1), sigma the
    corresponding singular values of A.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    MZ = (A.T @ (A @ Z)) / n
    H = Z.T @ MZ
    H = 0.5 * (H + H.T)
    lam, Q = np.linalg.eigh(H)
    order = np.argsort(lam)[::-1]
    lam = lam[order]
    Q = Q[:, order]
    return lam, Z @ Q, np.sqrt(np.maximum(n * lam, 0.0))


def eta(A: np.ndarray, offsets: Sequence[int]) -> float:
    """eta = max_i ||M_i - M||_2 / ||M||_2  (Definition 2); d x d matrices."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    Mmat = A.T @ A / n
    nm = np.linalg.norm(Mmat, 2)
    return max(float(np.linalg.norm(B.T @ B / B.shape[0] - Mmat, 2)) / nm
               for B in _blocks(A, offsets))
