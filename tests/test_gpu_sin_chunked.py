"""The per-round sin theta (chunk partials on FP64 matrix cores, lambda_max of
the k x k residual Gram by repeated squaring) against the oracle's SVD form, at
ragged and exact multiples of the 64-row chunk, k from 1 to 64, a reference
narrower than the iterate, and the degenerate cases (reference = the iterate,
reference orthogonal to it: every principal angle equal)."""

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lp(gpu_lib):
    import paper_2002_08014_amd as lp
    return lp


def _run(lp, d, k, U, seed):
    """Two rounds of p = 1 on a small FP64 problem with U as the reference; returns
    the last sin_hist entry and the final iterate."""
    w = synth.make_small(max(4 * d, 64), d, k, 2, seed=seed, dtype=torch.float64,
                         p_sched=[1, 1])
    A = w.A.to("cuda:0")
    P = lp.lp_create(A, w.offsets, k)
    r = lp.lp_run(P, k, [1, 1], "sign", w.Y0, U_ref=torch.as_tensor(U))
    return r["sin_hist"][-1], host(r["Z"])


@pytest.mark.parametrize("d,k,k_ref", [(1, 1, 1), (63, 5, 5), (64, 16, 16), (65, 16, 9),
                                       (200, 33, 33), (1000, 64, 64), (1000, 64, 17),
                                       (4096, 32, 32)])
def test_chunked_sin_theta_against_svd(lp, d, k, k_ref):
    print(f"sin chunked: d={d} k={k} k_ref={k_ref}", flush=True)
    rng = np.random.default_rng(d * 131 + k)
    U = oracle.orth(rng.standard_normal((d, k_ref)))
    got, Z = _run(lp, d, k, U, seed=d + k)
    want = oracle.sin_theta(Z, U)
    assert abs(got - want) <= 1e-12 + 1e-12 * want


def test_chunked_sin_theta_degenerate(lp):
    """U = the iterate itself gives 0 (to rounding); U orthogonal to the iterate
    gives 1 with all k angles equal (the largest eigenvalue has multiplicity k)."""
    print("sin chunked: degenerate", flush=True)
    d, k = 300, 12
    w = synth.make_small(1200, d, k, 2, seed=5, dtype=torch.float64, p_sched=[1, 1])
    A = w.A.to("cuda:0")
    P = lp.lp_create(A, w.offsets, k)
    Z = host(lp.lp_run(P, k, [1, 1], "sign", w.Y0)["Z"])
    same = lp.lp_run(P, k, [1, 1], "sign", w.Y0, U_ref=torch.as_tensor(Z))["sin_hist"][-1]
    assert same <= 1e-14
    Q, _ = np.linalg.qr(np.hstack([Z, np.random.default_rng(1).standard_normal((d, k))]))
    U = Q[:, k:]                     # orthonormal and orthogonal to Z
    ortho = lp.lp_run(P, k, [1, 1], "sign", w.Y0, U_ref=torch.as_tensor(U))["sin_hist"][-1]
    assert abs(ortho - 1.0) <= 1e-12
