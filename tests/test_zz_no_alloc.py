"""lp_orth_noalloc (the allocation-free variant of lp_orth, scratch in static
device memory) against lp_orth through the C ABI: two calls in a row, the
second with a smaller input, each equal to lp_orth's result on the same input
(the same CholeskyQR2 kernels, so the results agree to the last bit; the bar is
the FP64 tolerance 1e-10 of the orth parity tests, checked at 1e-14), and the
oracle's orth within 1e-12; a batch over the static limit is refused."""

import numpy as np
import pytest
import torch

import oracle
from tests._util import host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lp(gpu_lib):
    import paper_2002_08014_amd as lp
    return lp


def _reference(lp, Y):
    """lp_orth on a problem of the same d (its workspace provides the scratch)."""
    b, d, k = Y.shape
    A = torch.zeros(b * k + b, d, dtype=torch.float64, device="cuda:0")
    offs = [i * (k + 1) for i in range(b + 1)]
    P = lp.lp_create(A, offs, k)
    Q, flags = lp.lp_orth(P, Y)
    torch.cuda.synchronize()
    return Q, flags


def test_orth_noalloc_matches_lp_orth_twice(lp):
    rng = np.random.default_rng(17)
    for b, d, k in ((8, 1000, 24), (3, 500, 10)):
        print(f"lp_orth_noalloc batch={b} d={d} k={k}", flush=True)
        Yh = rng.standard_normal((b, d, k)) * rng.uniform(0.1, 10.0, (b, 1, k))
        Y = torch.as_tensor(Yh, device="cuda:0").contiguous()
        Q, flags = lp.lp_orth_noalloc(Y)
        torch.cuda.synchronize()
        Qr, flags_r = _reference(lp, Y)
        assert int(flags.sum()) == 0 and int(flags_r.sum()) == 0
        assert float((Q - Qr).abs().max()) <= 1e-14
        Qh = host(Q)
        for i in range(b):
            assert np.abs(Qh[i] - oracle.orth(Yh[i])).max() < 1e-12


def test_orth_noalloc_in_place_and_limit(lp):
    rng = np.random.default_rng(18)
    Yh = rng.standard_normal((2, 300, 7))
    Y = torch.as_tensor(Yh, device="cuda:0").contiguous()
    Q, _ = lp.lp_orth_noalloc(Y, Q=Y)          # Q may alias Y
    torch.cuda.synchronize()
    for i in range(2):
        assert np.abs(host(Q)[i] - oracle.orth(Yh[i])).max() < 1e-12
    big = torch.empty(64, 4096, 64, dtype=torch.float64, device="cuda:0")
    with pytest.raises(lp.LPError) as e:
        lp.lp_orth_noalloc(big)
    assert e.value.status == -1
