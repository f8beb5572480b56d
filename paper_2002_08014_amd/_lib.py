"""ctypes binding of liblp.so (argument marshalling only).

Each function has the name of the C entry point it calls (include/lp.h) and
takes torch tensors for device buffers; every step of the computation runs in
the HIP library.  The library is loaded after torch so that it binds to the
HIP runtime torch already loaded (one runtime per process).  A missing or
unloadable library raises: there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblp.so")

LP_OK, LP_EINVAL, LP_ENOMEM, LP_EDEVICE, LP_EBREAKDOWN, LP_ENOTCONV, LP_EBUSY = 0, -1, -2, -3, -4, -5, -6
DTYPES = {torch.float64: 0, torch.float32: 1, torch.bfloat16: 2}
MODES = {"vanilla": 0, "sign": 1, "opt": 2}

EXPORTS = ("lp_strerror", "lp_last_error", "lp_workspace_size", "lp_create", "lp_destroy",
           "lp_set_tuning", "lp_get_tuning", "lp_autotune", "lp_run", "lp_local_multiply", "lp_orth", "lp_align",
           "lp_sin_theta", "lp_bandwidth_probe", "lp_copy_probe")


class LPError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


class Tuning(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32),
                ("local_kernel", ctypes.c_int32),
                ("chunk_rows", ctypes.c_int64),
                ("cached_loads", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class RunOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32),
                ("U_ref", ctypes.c_void_p),
                ("sin_hist", ctypes.POINTER(ctypes.c_double)),
                ("signs_out", ctypes.POINTER(ctypes.c_int8)),
                ("z0_orthonormal", ctypes.c_int32),
                ("use_graph", ctypes.c_int32),
                ("time_local", ctypes.c_int32)]


class RunStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32),
                ("local_iters", ctypes.c_int32),
                ("breakdowns", ctypes.c_int32),
                ("near_singular", ctypes.c_int32),
                ("ms_total", ctypes.c_double),
                ("bytes_A", ctypes.c_double),
                ("ms_local", ctypes.c_double),
                ("local_launches", ctypes.c_int32),
                ("graph_rounds", ctypes.c_int32)]


_LIB: Optional[ctypes.CDLL] = None


def load() -> ctypes.CDLL:
    """Load liblp.so (raises if it is not built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.lp_strerror.restype = ctypes.c_char_p
    L.lp_strerror.argtypes = [i32]
    L.lp_last_error.restype = ctypes.c_char_p
    L.lp_last_error.argtypes = []
    L.lp_workspace_size.restype = i32
    L.lp_workspace_size.argtypes = [i32, i64, i64, vp, i32, i32, ctypes.POINTER(sz)]
    L.lp_create.restype = i32
    L.lp_create.argtypes = [ctypes.POINTER(vp), vp, i32, i64, i64, i64, vp, i32, i32, vp, sz, vp]
    L.lp_destroy.restype = i32
    L.lp_destroy.argtypes = [vp]
    L.lp_set_tuning.restype = i32
    L.lp_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.lp_get_tuning.restype = i32
    L.lp_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.lp_autotune.restype = i32
    L.lp_autotune.argtypes = [vp, i32, ctypes.c_char_p, ctypes.POINTER(Tuning)]
    L.lp_run.restype = i32
    L.lp_run.argtypes = [vp, i32, vp, i32, i32, vp, vp, vp, ctypes.POINTER(RunOpts),
                         ctypes.POINTER(RunStats)]
    L.lp_local_multiply.restype = i32
    L.lp_local_multiply.argtypes = [vp, i32, vp, vp]
    L.lp_orth.restype = i32
    L.lp_orth.argtypes = [vp, i32, i32, vp, vp, vp]
    L.lp_align.restype = i32
    L.lp_align.argtypes = [vp, i32, i32, i32, vp, vp, vp]
    L.lp_bandwidth_probe.restype = i32
    L.lp_bandwidth_probe.argtypes = [vp, sz, i32, ctypes.POINTER(ctypes.c_double), vp]
    L.lp_copy_probe.restype = i32
    L.lp_copy_probe.argtypes = [vp, vp, sz, i32, ctypes.POINTER(ctypes.c_double), vp]
    L.lp_sin_theta.restype = i32
    L.lp_sin_theta.argtypes = [vp, vp, i64, i32, ctypes.POINTER(ctypes.c_double), vp]
    _LIB = L
    return L


def _check(status: int, where: str) -> None:
    if status != LP_OK:
        L = load()
        raise LPError(status, where, f"{L.lp_strerror(status).decode()} ({L.lp_last_error().decode()})")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(x, like_device) -> torch.Tensor:
    t = torch.as_tensor(x, dtype=torch.float64, device=like_device)
    return t.contiguous()


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------

def lp_workspace_size(dtype: torch.dtype, n: int, d: int, offsets: Sequence[int], k_max: int) -> int:
    L = load()
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    out = ctypes.c_size_t(0)
    _check(L.lp_workspace_size(DTYPES[dtype], n, d, offs.ctypes.data, len(offs) - 1, k_max,
                               ctypes.byref(out)), "lp_workspace_size")
    return int(out.value)


class Problem:
    """A created problem: keeps A, the workspace tensor and the handle alive."""

    def __init__(self, handle, A, workspace, offsets, k_max, stream):
        self.handle = handle
        self.A = A
        self.workspace = workspace
        self.offsets = offsets
        self.k_max = k_max
        self.stream = stream

    @property
    def n(self):
        return int(self.A.shape[0])

    @property
    def d(self):
        return int(self.A.shape[1])

    @property
    def m(self):
        return len(self.offsets) - 1

    def __del__(self):
        try:
            if self.handle:
                load().lp_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


def lp_create(A: torch.Tensor, offsets: Sequence[int], k_max: int,
              stream: Optional[torch.cuda.Stream] = None) -> Problem:
    """A: device n x d tensor (float64/float32/bfloat16), rows contiguous."""
    L = load()
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D tensor with contiguous rows")
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    n, d = A.shape
    ws_bytes = lp_workspace_size(A.dtype, n, d, offs, k_max)
    ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=A.device)
    h = ctypes.c_void_p(None)
    st = stream if stream is not None else torch.cuda.current_stream(A.device)
    _check(L.lp_create(ctypes.byref(h), _ptr(A), DTYPES[A.dtype], n, d, A.stride(0),
                       offs.ctypes.data, len(offs) - 1, k_max, _ptr(ws), ws.numel(),
                       _stream_handle(st)), "lp_create")
    return Problem(h, A, ws, offs, k_max, st)


def lp_destroy(P: Problem) -> None:
    if P.handle:
        _check(load().lp_destroy(P.handle), "lp_destroy")
        P.handle = None


def lp_set_tuning(P: Problem, local_kernel: int = 0, chunk_rows: int = 0,
                  cached_loads: bool = False) -> None:
    t = Tuning(ctypes.sizeof(Tuning), local_kernel, chunk_rows, 1 if cached_loads else 0, 0)
    _check(load().lp_set_tuning(P.handle, ctypes.byref(t)), "lp_set_tuning")


def lp_get_tuning(P: Problem) -> dict:
    t = Tuning()
    _check(load().lp_get_tuning(P.handle, ctypes.byref(t)), "lp_get_tuning")
    return {"local_kernel": t.local_kernel, "chunk_rows": t.chunk_rows,
            "cached_loads": bool(t.cached_loads)}


def lp_autotune(P: Problem, k: int, cache_path: Optional[str] = None) -> dict:
    """Time the local-multiply candidates for rank k, apply the fastest, return it."""
    t = Tuning()
    _check(load().lp_autotune(P.handle, k, cache_path.encode() if cache_path else None,
                              ctypes.byref(t)), "lp_autotune")
    return {"local_kernel": t.local_kernel, "chunk_rows": t.chunk_rows,
            "cached_loads": bool(t.cached_loads)}


def lp_run(P: Problem, k: int, p_sched: Sequence[int], mode: str, Y0, ritz: bool = False,
           U_ref: Optional[torch.Tensor] = None, record_signs: bool = False,
           z0_orthonormal: bool = False, use_graph: bool = True, time_local: bool = False):
    """Returns dict(Z, ritz, sin_hist, signs, stats); Z is a device d x k float64 tensor."""
    L = load()
    dev = P.A.device
    sched = np.ascontiguousarray(np.asarray(p_sched, dtype=np.int32))
    T = len(sched)
    Y0d = _dev_f64(Y0, dev)
    Z = torch.empty(P.d, k, dtype=torch.float64, device=dev)
    rz = torch.empty(k, dtype=torch.float64, device=dev) if ritz else None
    opts = RunOpts()
    opts.struct_size = ctypes.sizeof(RunOpts)
    opts.z0_orthonormal = 1 if z0_orthonormal else 0
    opts.use_graph = 1 if use_graph else 0
    opts.time_local = 1 if time_local else 0
    hist = None
    if U_ref is not None:
        Ud = _dev_f64(U_ref, dev)
        hist = np.zeros(T, dtype=np.float64)
        opts.U_ref = Ud.data_ptr()
        opts.sin_hist = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    signs = None
    if record_signs:
        signs = np.zeros((T, P.m, k), dtype=np.int8)
        opts.signs_out = signs.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
    stats = RunStats()
    _check(L.lp_run(P.handle, k, sched.ctypes.data, T, MODES[mode], _ptr(Y0d), _ptr(Z), _ptr(rz),
                    ctypes.byref(opts), ctypes.byref(stats)), "lp_run")
    return {"Z": Z, "ritz": rz, "sin_hist": hist, "signs": signs,
            "stats": {f: getattr(stats, f) for f, _ in RunStats._fields_}}


def lp_local_multiply(P: Problem, k: int, Z) -> torch.Tensor:
    """Returns device m x d x k float64: Y[i] = A_i^T (A_i Z) (Z rounded to the working precision)."""
    L = load()
    Zd = _dev_f64(Z, P.A.device)
    Y = torch.empty(P.m, P.d, k, dtype=torch.float64, device=P.A.device)
    _check(L.lp_local_multiply(P.handle, k, _ptr(Zd), _ptr(Y)), "lp_local_multiply")
    return Y


def lp_orth(P: Problem, Y: torch.Tensor):
    """Batched orth of Y (batch x d x k float64 device); returns (Q, breakdown flags)."""
    L = load()
    Y = Y.contiguous()
    if Y.dim() == 2:
        Y = Y[None]
    b, d, k = Y.shape
    Q = torch.empty_like(Y)
    flags = torch.zeros(b, dtype=torch.int32, device=Y.device)
    _check(L.lp_orth(P.handle, k, b, _ptr(Y), _ptr(Q), _ptr(flags)), "lp_orth")
    return Q, flags


def lp_align(P: Problem, mode: str, Zi: torch.Tensor, Zb: torch.Tensor) -> torch.Tensor:
    """Sign vectors (batch x k int8) or Procrustes matrices (batch x k x k float64)."""
    L = load()
    Zi = Zi.contiguous()
    b, d, k = Zi.shape
    if mode == "sign":
        out = torch.empty(b, k, dtype=torch.int8, device=Zi.device)
    else:
        out = torch.empty(b, k, k, dtype=torch.float64, device=Zi.device)
    _check(L.lp_align(P.handle, k, b, MODES[mode], _ptr(Zi), _ptr(Zb.contiguous()), _ptr(out)),
           "lp_align")
    return out


def lp_sin_theta(Z: torch.Tensor, U: torch.Tensor, stream: Optional[torch.cuda.Stream] = None) -> float:
    L = load()
    Zd, Ud = Z.contiguous(), U.contiguous()
    out = ctypes.c_double(0.0)
    _check(L.lp_sin_theta(_ptr(Zd), _ptr(Ud), Zd.shape[0], Zd.shape[1], ctypes.byref(out),
                          _stream_handle(stream)), "lp_sin_theta")
    return float(out.value)


def lp_bandwidth_probe(buf: torch.Tensor, iters: int = 5,
                       stream: Optional[torch.cuda.Stream] = None) -> float:
    """Best-of-`iters` read bandwidth (GB/s) over the bytes of a device tensor."""
    L = load()
    nbytes = (buf.numel() * buf.element_size()) // 16 * 16
    out = ctypes.c_double(0.0)
    _check(L.lp_bandwidth_probe(_ptr(buf), nbytes, iters, ctypes.byref(out), _stream_handle(stream)),
           "lp_bandwidth_probe")
    return float(out.value)


def lp_copy_probe(dst: torch.Tensor, src: torch.Tensor, iters: int = 5,
                  stream: Optional[torch.cuda.Stream] = None) -> float:
    """Best-of-`iters` copy bandwidth (GB/s, read + written bytes) from src to dst."""
    L = load()
    nbytes = min(dst.numel() * dst.element_size(), src.numel() * src.element_size()) // 16 * 16
    out = ctypes.c_double(0.0)
    _check(L.lp_copy_probe(_ptr(dst), _ptr(src), nbytes, iters, ctypes.byref(out),
                           _stream_handle(stream)), "lp_copy_probe")
    return float(out.value)
