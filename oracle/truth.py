"""Ground truth U_k: top-k eigenvectors of M = A^T A / n (oracle helper).

The quantity LocalPower approximates (Introduction: the top-k right singular
vectors of A; Eq. (power): M = A^T A / n).  Written as its definition with
LAPACK's symmetric eigensolver on the float64 Gram of the stored values.
"""

from __future__ import annotations

import numpy as np


def top_k(A: np.ndarray, k: int, block_rows: int = 1 << 16):
    """Returns (U_k d x k, lam_all descending) for M = A^T A / n.

    The Gram matrix is accumulated over row blocks (float64) so that float32
    or bfloat16 inputs are upcast block by block.
    """
    n, d = A.shape
    G = np.zeros((d, d), dtype=np.float64)
    for r0 in range(0, n, block_rows):
        B = np.asarray(A[r0:r0 + block_rows], dtype=np.float64)
        G += B.T @ B
    G /= n
    lam, V = np.linalg.eigh(G)
    order = np.argsort(lam)[::-1]
    return V[:, order[:k]], lam[order]
