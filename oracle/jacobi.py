"""Cyclic Jacobi eigensolver for small symmetric matrices (oracle helper).

Textbook cyclic-by-row Jacobi (Golub and Van Loan, "Matrix Computations",
the symmetric Schur decomposition and cyclic Jacobi).  Pure Python loops: only
for tiny d, as an independent route to the truth U_k = top eigenvectors of
A^T A that the paper measures against (experimental section).
"""

from __future__ import annotations

import math

import numpy as np


def _sym_schur(S, p, q):
    """(c, s) such that the rotation in the (p, q) plane zeroes S[p, q]."""
    if S[p][q] == 0.0:
        return 1.0, 0.0
    tau = (S[q][q] - S[p][p]) / (2.0 * S[p][q])
    if tau >= 0:
        t = 1.0 / (tau + math.sqrt(1.0 + tau * tau))
    else:
        t = -1.0 / (-tau + math.sqrt(1.0 + tau * tau))
    c = 1.0 / math.sqrt(1.0 + t * t)
    return c, t * c


def jacobi_eig(S_in, tol: float = 1e-15, max_sweeps: int = 60):
    """Eigen-decomposition S = V diag(lam) V^T, lam sorted descending."""
    S = [list(map(float, row)) for row in np.asarray(S_in, dtype=np.float64)]
    n = len(S)
    V = [[1.0 if i == j else 0.0 for j in range(n)] for i in range(n)]
    fro = math.sqrt(sum(S[i][j] ** 2 for i in range(n) for j in range(n)))
    for _ in range(max_sweeps):
        off = math.sqrt(sum(S[i][j] ** 2 for i in range(n) for j in range(n) if i != j))
        if off <= tol * fro:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                c, s = _sym_schur(S, p, q)
                if s == 0.0:
                    continue
                # S <- J^T S J with J the rotation in the (p, q) plane
                for k in range(n):
                    skp, skq = S[k][p], S[k][q]
                    S[k][p] = c * skp - s * skq
                    S[k][q] = s * skp + c * skq
                for k in range(n):
                    spk, sqk = S[p][k], S[q][k]
                    S[p][k] = c * spk - s * sqk
                    S[q][k] = s * spk + c * sqk
                for k in range(n):
                    vkp, vkq = V[k][p], V[k][q]
                    V[k][p] = c * vkp - s * vkq
                    V[k][q] = s * vkp + c * vkq
    lam = np.array([S[i][i] for i in range(n)])
    Vm = np.array(V)
    order = np.argsort(lam)[::-1]
    return lam[order], Vm[:, order]
