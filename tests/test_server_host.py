"""Host-side checks of the serving entry points that need no GPU: the
footprint of a job and the validation of job descriptions."""

import ctypes

import numpy as np
import pytest



@pytest.fixture(scope="module")
def L():
    import paper_2002_08014_amd._lib as lib
    return lib


def _job(lib, n=4096, d=256, k=16, m=4, p0=4, target=1e-4, max_rounds=50, dtype=1):
    offs = np.linspace(0, n, m + 1).astype(np.int64)
    y0 = np.zeros((d, k))
    job = lib.Job(ctypes.sizeof(lib.Job), 0x1000, dtype, n, d, d, offs.ctypes.data, m, k, p0, 1,
                  target, max_rounds, y0.ctypes.data, 0x2000)
    return job, (offs, y0)


def test_footprint_is_workspace_plus_job_buffers(L):
    lib = L.load()
    job, keep = _job(L)
    fp = ctypes.c_size_t()
    assert lib.lp_server_footprint(ctypes.byref(job), ctypes.byref(fp)) == 0
    ws = L.lp_workspace_size(__import__("torch").float32, 4096, 256, keep[0], 16)
    dk8 = ((256 * 16 * 8 + 255) // 256) * 256
    assert fp.value == ((ws + 255) // 256) * 256 + 2 * dk8 + 256


@pytest.mark.parametrize("field,value", [("k", 0), ("k", 65), ("p0", 0), ("max_rounds", 0),
                                         ("target", 0.0), ("mode", 7), ("lda", 100)])
def test_invalid_jobs_are_refused(L, field, value):
    lib = L.load()
    job, keep = _job(L)
    setattr(job, field, value)
    fp = ctypes.c_size_t()
    assert lib.lp_server_footprint(ctypes.byref(job), ctypes.byref(fp)) == L.LP_EINVAL


def test_partition_smaller_than_k_is_refused(L):
    lib = L.load()
    job, keep = _job(L, n=4096, k=16, m=4)
    offs = np.array([0, 8, 2000, 3000, 4096], dtype=np.int64)
    job.offsets = offs.ctypes.data
    fp = ctypes.c_size_t()
    assert lib.lp_server_footprint(ctypes.byref(job), ctypes.byref(fp)) == L.LP_EINVAL
