"""Comparison helpers shared by the parity tests (no method arithmetic)."""

import numpy as np
import torch


def host(x) -> np.ndarray:
    if isinstance(x, torch.Tensor):
        return x.detach().to("cpu", torch.float64).numpy() if x.dtype != torch.int8 else x.cpu().numpy()
    return np.asarray(x)


def sign_normalise(Z: np.ndarray) -> np.ndarray:
    """Flip columns so that each column's largest-magnitude entry is positive."""
    idx = np.argmax(np.abs(Z), axis=0)
    s = np.sign(Z[idx, np.arange(Z.shape[1])])
    s[s == 0] = 1.0
    return Z * s


def sin_theta_np(Z: np.ndarray, U: np.ndarray) -> float:
    W = U - Z @ (Z.T @ U)
    return float(np.linalg.norm(W, 2))


def to_device(w, dtype=None):
    """Move a workload's A to cuda:0 (optionally changing the stored dtype)."""
    A = w.A
    if dtype is not None:
        A = A.to(dtype)
    return A.to("cuda:0").contiguous()


def upcast(A_dev: torch.Tensor) -> np.ndarray:
    """Exact FP64 copy of the stored values (FP32/BF16 -> FP64 is exact)."""
    return A_dev.to("cpu").to(torch.float64).numpy()


def rule_schedule(changes, p0, target):
    """The stop rule as include/lp.h states it, applied to a list of changes:
    returns the p of every round and whether the last round settled at p = 1."""
    p, prev_c, prev_q, ps = p0, -1.0, -1.0, []
    for c in changes:
        ps.append(p)
        q = c / prev_c if prev_c > 0 else -1.0
        qe = max(q, prev_q) if (q >= 0 and prev_q >= 0) else -1.0
        ratio = 0 <= qe < 1
        est = c * qe / (1 - qe) if ratio else c
        settled = c == 0 or (ratio and est <= 0.5 * target)
        prev_q, prev_c = q, c
        if settled and p == 1:
            return ps, True
        if p > 1 and (settled or q > 0.5):
            p, prev_c, prev_q = max(1, p // 2), -1.0, -1.0
    return ps, False


CAPTURE = None   # pytest's capture manager, set by conftest.py


def progress(msg: str) -> None:
    """Print a progress line of a long step on the real stdout, past pytest's
    capture (plain print when there is no capture manager)."""
    if CAPTURE is not None:
        with CAPTURE.global_and_fixture_disabled():
            print(msg, flush=True)
    else:
        print(msg, flush=True)
