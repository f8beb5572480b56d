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
           "lp_set_tuning", "lp_get_tuning", "lp_autotune", "lp_run", "lp_solve", "lp_gram_bytes",
           "lp_gram_enable", "lp_gram_disable", "lp_eta", "lp_local_multiply", "lp_profile_local_multiply",
           "lp_orth", "lp_orth_noalloc",
           "lp_align",
           "lp_sin_theta", "lp_sin_theta_r", "lp_generate", "lp_bandwidth_probe", "lp_copy_probe", "lp_server_footprint",
           "lp_server_create", "lp_server_submit", "lp_server_poll", "lp_server_wait",
           "lp_server_destroy")


class LPError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


class Tuning(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32),
                ("local_kernel", ctypes.c_int32),
                ("chunk_rows", ctypes.c_int64),
                ("cached_loads", ctypes.c_int32),
                ("split_operands", ctypes.c_int32)]


class RunOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32),
                ("U_ref", ctypes.c_void_p),
                ("sin_hist", ctypes.POINTER(ctypes.c_double)),
                ("signs_out", ctypes.POINTER(ctypes.c_int8)),
                ("z0_orthonormal", ctypes.c_int32),
                ("use_graph", ctypes.c_int32),
                ("time_local", ctypes.c_int32),
                ("split_rounds", ctypes.c_int32),
                ("k_ref", ctypes.c_int32),
                ("rho_out", ctypes.POINTER(ctypes.c_double)),
                ("seed", ctypes.c_uint64)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32),
                ("p0", ctypes.c_int32),
                ("target", ctypes.c_double),
                ("max_rounds", ctypes.c_int32),
                ("z0_orthonormal", ctypes.c_int32),
                ("p_used", ctypes.POINTER(ctypes.c_int32)),
                ("change_out", ctypes.POINTER(ctypes.c_double)),
                ("seed", ctypes.c_uint64)]


class SolveStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32),
                ("local_iters", ctypes.c_int32),
                ("breakdowns", ctypes.c_int32),
                ("near_singular", ctypes.c_int32),
                ("p_final", ctypes.c_int32),
                ("change", ctypes.c_double),
                ("estimate", ctypes.c_double),
                ("ms_total", ctypes.c_double)]


class RunStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32),
                ("local_iters", ctypes.c_int32),
                ("breakdowns", ctypes.c_int32),
                ("near_singular", ctypes.c_int32),
                ("ms_total", ctypes.c_double),
                ("bytes_A", ctypes.c_double),
                ("ms_local", ctypes.c_double),
                ("local_launches", ctypes.c_int32),
                ("graph_rounds", ctypes.c_int32),
                ("split_rounds", ctypes.c_int32)]


class Job(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32),
                ("A", ctypes.c_void_p),
                ("dtype", ctypes.c_int32),
                ("n", ctypes.c_int64),
                ("d", ctypes.c_int64),
                ("lda", ctypes.c_int64),
                ("offsets", ctypes.c_void_p),
                ("m", ctypes.c_int32),
                ("k", ctypes.c_int32),
                ("p0", ctypes.c_int32),
                ("mode", ctypes.c_int32),
                ("target", ctypes.c_double),
                ("max_rounds", ctypes.c_int32),
                ("Y0", ctypes.c_void_p),
                ("Z_out", ctypes.c_void_p),
                ("stream", ctypes.c_void_p),
                ("gen_seed", ctypes.c_uint64),
                ("gen_gap", ctypes.c_double),
                ("gen_decay", ctypes.c_double),
                ("single_bf16", ctypes.c_int32)]


class JobResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64),
                ("status", ctypes.c_int32),
                ("rounds", ctypes.c_int32),
                ("local_iters", ctypes.c_int32),
                ("p_final", ctypes.c_int32),
                ("change", ctypes.c_double),
                ("estimate", ctypes.c_double),
                ("ms_queued", ctypes.c_double),
                ("ms_total", ctypes.c_double)]


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
    L.lp_solve.restype = i32
    L.lp_gram_bytes.restype = i32
    L.lp_gram_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.lp_gram_enable.restype = i32
    L.lp_gram_enable.argtypes = [vp, vp, ctypes.c_size_t]
    L.lp_gram_disable.restype = i32
    L.lp_eta.restype = i32
    L.lp_eta.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.lp_gram_disable.argtypes = [vp]
    L.lp_solve.argtypes = [vp, i32, i32, vp, vp, vp, ctypes.POINTER(SolveOpts),
                           ctypes.POINTER(SolveStats)]
    L.lp_run.argtypes = [vp, i32, vp, i32, i32, vp, vp, vp, ctypes.POINTER(RunOpts),
                         ctypes.POINTER(RunStats)]
    L.lp_local_multiply.restype = i32
    L.lp_local_multiply.argtypes = [vp, i32, vp, vp]
    L.lp_profile_local_multiply.restype = i32
    L.lp_profile_local_multiply.argtypes = [vp, i32, vp, vp, i32, ctypes.POINTER(i32)]
    L.lp_orth.restype = i32
    L.lp_orth.argtypes = [vp, i32, i32, vp, vp, vp]
    L.lp_orth_noalloc.restype = i32
    L.lp_orth_noalloc.argtypes = [i32, i32, i64, vp, vp, vp, vp]
    L.lp_align.restype = i32
    L.lp_align.argtypes = [vp, i32, i32, i32, vp, vp, vp]
    L.lp_bandwidth_probe.restype = i32
    L.lp_bandwidth_probe.argtypes = [vp, sz, i32, ctypes.POINTER(ctypes.c_double), vp]
    L.lp_copy_probe.restype = i32
    L.lp_copy_probe.argtypes = [vp, vp, sz, i32, ctypes.POINTER(ctypes.c_double), vp]
    L.lp_sin_theta.restype = i32
    L.lp_sin_theta.argtypes = [vp, vp, i64, i32, ctypes.POINTER(ctypes.c_double), vp]
    L.lp_generate.restype = i32
    L.lp_generate.argtypes = [vp, i32, i64, i64, i64, i32, ctypes.c_double, ctypes.c_double,
                              ctypes.c_uint64, vp, vp]
    L.lp_sin_theta_r.restype = i32
    L.lp_sin_theta_r.argtypes = [vp, i32, vp, i32, i64, ctypes.POINTER(ctypes.c_double), vp]
    L.lp_server_footprint.restype = i32
    L.lp_server_footprint.argtypes = [ctypes.POINTER(Job), ctypes.POINTER(sz)]
    L.lp_server_create.restype = i32
    L.lp_server_create.argtypes = [ctypes.POINTER(vp), sz, i32]
    L.lp_server_submit.restype = i32
    L.lp_server_submit.argtypes = [vp, ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_uint64)]
    L.lp_server_poll.restype = i32
    L.lp_server_poll.argtypes = [vp, ctypes.POINTER(JobResult), i32, ctypes.POINTER(i32)]
    L.lp_server_wait.restype = i32
    L.lp_server_wait.argtypes = [vp, i32, ctypes.c_double]
    L.lp_server_destroy.restype = i32
    L.lp_server_destroy.argtypes = [vp]
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
        self.gram_buffer = None   # device buffer of the local-Gram form while it is on

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


def lp_gram_bytes(P: Problem) -> int:
    nb = ctypes.c_size_t(0)
    _check(load().lp_gram_bytes(P.handle, ctypes.byref(nb)), "lp_gram_bytes")
    return int(nb.value)


def lp_gram_enable(P: Problem) -> None:
    """Switch the problem to the local-Gram form (M_i = A_i^T A_i formed once, FP32);
    the buffer is a device tensor kept on the Problem."""
    nb = lp_gram_bytes(P)
    buf = torch.empty(max(nb, 256), dtype=torch.uint8, device=P.A.device)
    _check(load().lp_gram_enable(P.handle, _ptr(buf), buf.numel()), "lp_gram_enable")
    P.gram_buffer = buf


def lp_gram_disable(P: Problem) -> None:
    _check(load().lp_gram_disable(P.handle), "lp_gram_disable")
    P.gram_buffer = None


def lp_eta(P: Problem, iters: int = 300):
    """(eta, per-partition ||M_i - M|| / ||M||) of Definition 2; needs lp_gram_enable."""
    out = ctypes.c_double(0.0)
    per = np.zeros(P.m, dtype=np.float64)
    _check(load().lp_eta(P.handle, int(iters), ctypes.byref(out),
                         per.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "lp_eta")
    return float(out.value), per


def lp_destroy(P: Problem) -> None:
    if P.handle:
        _check(load().lp_destroy(P.handle), "lp_destroy")
        P.handle = None


def lp_set_tuning(P: Problem, local_kernel: int = 0, chunk_rows: int = 0,
                  cached_loads: bool = False, split_operands: bool = False) -> None:
    t = Tuning(ctypes.sizeof(Tuning), local_kernel, chunk_rows, 1 if cached_loads else 0,
               1 if split_operands else 0)
    _check(load().lp_set_tuning(P.handle, ctypes.byref(t)), "lp_set_tuning")


def lp_get_tuning(P: Problem) -> dict:
    t = Tuning()
    _check(load().lp_get_tuning(P.handle, ctypes.byref(t)), "lp_get_tuning")
    return {"local_kernel": t.local_kernel, "chunk_rows": t.chunk_rows,
            "cached_loads": bool(t.cached_loads), "split_operands": bool(t.split_operands)}


def lp_autotune(P: Problem, k: int, cache_path: Optional[str] = None) -> dict:
    """Time the local-multiply candidates for rank k, apply the fastest, return it."""
    t = Tuning()
    _check(load().lp_autotune(P.handle, k, cache_path.encode() if cache_path else None,
                              ctypes.byref(t)), "lp_autotune")
    return {"local_kernel": t.local_kernel, "chunk_rows": t.chunk_rows,
            "cached_loads": bool(t.cached_loads), "split_operands": bool(t.split_operands)}


def lp_run(P: Problem, k: int, p_sched: Sequence[int], mode: str, Y0, ritz: bool = False,
           U_ref: Optional[torch.Tensor] = None, record_signs: bool = False,
           z0_orthonormal: bool = False, use_graph: bool = True, time_local: int = 0,
           split_rounds: Optional[bool] = None, record_rho: bool = False, seed: int = 0):
    """Returns dict(Z, ritz, sin_hist, signs, stats); Z is a device d x k float64 tensor.
    time_local: 0 no events, 1 (or True) every local multiply timed, 2 the first
    one of every round only.  split_rounds: partitions in two halves on two streams
    (None: the library decides, True: always, False: never).  k is the iteration
    rank; U_ref may have fewer columns (the target rank), and sin_hist then holds
    sin theta of the rank-k iterate against it.  record_rho: the residual error of
    Definition 3 at every round's last local step (rho).  Y0 None: the library draws
    the Gaussian start from `seed`."""
    L = load()
    dev = P.A.device
    sched = np.ascontiguousarray(np.asarray(p_sched, dtype=np.int32))
    T = len(sched)
    Y0d = None if Y0 is None else _dev_f64(Y0, dev)
    Z = torch.empty(P.d, k, dtype=torch.float64, device=dev)
    rz = torch.empty(k, dtype=torch.float64, device=dev) if ritz else None
    opts = RunOpts()
    opts.struct_size = ctypes.sizeof(RunOpts)
    opts.z0_orthonormal = 1 if z0_orthonormal else 0
    opts.use_graph = 1 if use_graph else 0
    opts.time_local = int(time_local)
    opts.split_rounds = 0 if split_rounds is None else (1 if split_rounds else 2)
    opts.seed = int(seed)
    hist = None
    if U_ref is not None:
        Ud = _dev_f64(U_ref, dev)
        hist = np.zeros(T, dtype=np.float64)
        if Ud.dim() != 2 or Ud.shape[0] != P.d or not 1 <= Ud.shape[1] <= k:
            raise ValueError("U_ref must be d x k_ref with 1 <= k_ref <= k")
        opts.U_ref = Ud.data_ptr()
        opts.k_ref = Ud.shape[1]
        opts.sin_hist = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    rho = None
    if record_rho:
        rho = np.zeros(T, dtype=np.float64)
        opts.rho_out = rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    signs = None
    if record_signs:
        signs = np.zeros((T, P.m, k), dtype=np.int8)
        opts.signs_out = signs.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
    stats = RunStats()
    _check(L.lp_run(P.handle, k, sched.ctypes.data, T, MODES[mode], _ptr(Y0d), _ptr(Z), _ptr(rz),
                    ctypes.byref(opts), ctypes.byref(stats)), "lp_run")
    return {"Z": Z, "ritz": rz, "sin_hist": hist, "rho": rho, "signs": signs,
            "stats": {f: getattr(stats, f) for f, _ in RunStats._fields_}}


def lp_solve(P: Problem, k: int, mode: str, Y0, p0: int, target: float, max_rounds: int,
             ritz: bool = False, z0_orthonormal: bool = False, seed: int = 0):
    """LocalPower with the truth-free stop rule and a decaying p (lp_solve).
    Returns dict(Z, ritz, p_used, changes, stats, status); status is LP_OK when the
    iterates settled at p = 1 and LP_ENOTCONV when max_rounds ran out (Z is then
    the last iterate); other failures raise LPError."""
    L = load()
    dev = P.A.device
    Y0d = None if Y0 is None else _dev_f64(Y0, dev)
    Z = torch.empty(P.d, k, dtype=torch.float64, device=dev)
    rz = torch.empty(k, dtype=torch.float64, device=dev) if ritz else None
    p_used = np.zeros(max_rounds, dtype=np.int32)
    changes = np.zeros(max_rounds, dtype=np.float64)
    o = SolveOpts()
    o.struct_size = ctypes.sizeof(SolveOpts)
    o.p0, o.target, o.max_rounds = int(p0), float(target), int(max_rounds)
    o.z0_orthonormal = 1 if z0_orthonormal else 0
    o.p_used = p_used.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    o.change_out = changes.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    o.seed = int(seed)
    st = SolveStats()
    status = L.lp_solve(P.handle, k, MODES[mode], _ptr(Y0d), _ptr(Z), _ptr(rz), ctypes.byref(o),
                        ctypes.byref(st))
    if status not in (LP_OK, LP_ENOTCONV):
        _check(status, "lp_solve")
    n = st.rounds
    return {"Z": Z, "ritz": rz, "p_used": p_used[:n], "changes": changes[:n], "status": status,
            "stats": {f: getattr(st, f) for f, _ in SolveStats._fields_}}


def lp_local_multiply(P: Problem, k: int, Z) -> torch.Tensor:
    """Returns device m x d x k float64: Y[i] = A_i^T (A_i Z) (Z rounded to the working precision)."""
    L = load()
    Zd = _dev_f64(Z, P.A.device)
    Y = torch.empty(P.m, P.d, k, dtype=torch.float64, device=P.A.device)
    _check(L.lp_local_multiply(P.handle, k, _ptr(Zd), _ptr(Y)), "lp_local_multiply")
    return Y


def lp_profile_local_multiply(P: Problem, k: int, Z) -> np.ndarray:
    """Workgroup stamps of one two-pass local multiply: rows (pass, item, start us, end us)."""
    L = load()
    Zd = _dev_f64(Z, P.A.device)
    n = ctypes.c_int32(0)
    st = L.lp_profile_local_multiply(P.handle, k, _ptr(Zd), None, 0, ctypes.byref(n))
    if n.value <= 0:
        _check(st, "lp_profile_local_multiply")
    out = np.zeros((n.value, 4), dtype=np.float64)
    _check(L.lp_profile_local_multiply(P.handle, k, _ptr(Zd), out.ctypes.data, n.value, ctypes.byref(n)),
           "lp_profile_local_multiply")
    return out


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


def lp_orth_noalloc(Y: torch.Tensor, Q: Optional[torch.Tensor] = None,
                    flags: Optional[torch.Tensor] = None,
                    stream: Optional[torch.cuda.Stream] = None):
    """lp_orth without a problem or an allocation inside the library (its scratch is
    static device memory shared by every call on the GPU).  Y: batch x d x k (or
    d x k) float64 device; Q (same shape) and flags (int32[batch]) may be passed in,
    e.g. to stay allocation-free under graph capture.  Returns (Q, flags)."""
    L = load()
    Y3 = Y if Y.dim() == 3 else Y[None]
    if not Y3.is_contiguous():
        raise ValueError("Y must be contiguous")
    b, d, k = Y3.shape
    Q = torch.empty_like(Y) if Q is None else Q
    flags = torch.zeros(b, dtype=torch.int32, device=Y.device) if flags is None else flags
    _check(L.lp_orth_noalloc(k, b, d, _ptr(Y3), _ptr(Q), _ptr(flags), _stream_handle(stream)),
           "lp_orth_noalloc")
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
    """sin theta of a d x r iterate Z against a d x k reference U (k <= r); Definition 1."""
    L = load()
    Zd, Ud = Z.contiguous(), U.contiguous()
    out = ctypes.c_double(0.0)
    if Zd.shape[1] == Ud.shape[1]:
        _check(L.lp_sin_theta(_ptr(Zd), _ptr(Ud), Zd.shape[0], Zd.shape[1], ctypes.byref(out),
                              _stream_handle(stream)), "lp_sin_theta")
    else:
        if Zd.shape[0] != Ud.shape[0]:
            raise ValueError("Z and U need the same row count")
        _check(L.lp_sin_theta_r(_ptr(Zd), Zd.shape[1], _ptr(Ud), Ud.shape[1], Zd.shape[0],
                                ctypes.byref(out), _stream_handle(stream)), "lp_sin_theta_r")
    return float(out.value)


def lp_generate(n: int, d: int, k: int, gap: float, decay: float, seed: int,
                dtype: Optional[torch.dtype] = torch.float32, basis: bool = True,
                device="cuda:0", stream: Optional[torch.cuda.Stream] = None):
    """The exact-truth matrix (n x d of `dtype`, or None when dtype is None) and its
    top-k right singular vectors (d x k float64 device, or None); lp_generate."""
    L = load()
    A = torch.empty(n, d, dtype=dtype, device=device) if dtype is not None else None
    U = torch.empty(d, k, dtype=torch.float64, device=device) if basis else None
    _check(L.lp_generate(_ptr(A), DTYPES[dtype] if dtype is not None else 1, n, d, d, k,
                         float(gap), float(decay), int(seed), _ptr(U), _stream_handle(stream)),
           "lp_generate")
    return A, U


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


# ----------------------------------------------------------------------------- serving

class Server:
    """A LocalPower job server on the current device (lp_server_*).

    submit() keeps A, the start matrix and the output alive until the job's
    result has been polled; poll() returns finished jobs with their Z."""

    def __init__(self, hbm_budget_bytes: int, max_active: int = 8):
        L = load()
        h = ctypes.c_void_p()
        _check(L.lp_server_create(ctypes.byref(h), int(hbm_budget_bytes), int(max_active)),
               "lp_server_create")
        self.handle = h
        self._jobs = {}

    @staticmethod
    def _job(A: Optional[torch.Tensor], offsets: Sequence[int], k: int, p0: int, mode: str,
             target: float, max_rounds: int, Y0, Z_out: Optional[torch.Tensor],
             stream: Optional[torch.cuda.Stream] = None, gen=None, single_bf16: bool = False):
        """gen = (n, d, dtype, seed, gap, decay) when A is None (generated at admission);
        Y0 None draws the start from the generation seed (gen[3], or 0)."""
        offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        if A is not None:
            if A.dim() != 2 or A.stride(1) != 1:
                raise ValueError("A must be a 2-D tensor with contiguous rows")
            if not A.is_cuda:
                raise ValueError("A must be a device tensor")
            n, d = A.shape
            dt, lda, dev = DTYPES[A.dtype], A.stride(0), A.device
            seed, gap, decay = (int(gen[3]), float(gen[4]), float(gen[5])) if gen else (0, 1.0, 1.0)
        else:
            n, d, dtype, seed, gap, decay = gen
            dt, lda, dev = DTYPES[dtype], d, torch.device("cuda", torch.cuda.current_device())
        y0 = None
        if Y0 is not None:
            y0 = np.ascontiguousarray(np.asarray(Y0, dtype=np.float64))
            if y0.shape != (d, k):
                raise ValueError("Y0 must be d x k")
        Z = Z_out if Z_out is not None else torch.empty(d, k, dtype=torch.float64, device=dev)
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        job = Job(ctypes.sizeof(Job), None if A is None else A.data_ptr(), dt, n, d, lda,
                  offs.ctypes.data, len(offs) - 1, k, p0, MODES[mode], float(target), int(max_rounds),
                  None if y0 is None else y0.ctypes.data, Z.data_ptr(), st.cuda_stream,
                  int(seed), float(gap), float(decay), 1 if single_bf16 else 0)
        return job, (A, offs, y0, Z)

    @staticmethod
    def footprint(A: Optional[torch.Tensor], offsets: Sequence[int], k: int, gen=None) -> int:
        d = A.shape[1] if A is not None else gen[1]
        job, keep = Server._job(A, offsets, k, 1, "sign", 1e-4, 1, np.zeros((d, k)), None, gen=gen)
        out = ctypes.c_size_t()
        _check(load().lp_server_footprint(ctypes.byref(job), ctypes.byref(out)), "lp_server_footprint")
        return out.value

    def submit(self, A: Optional[torch.Tensor], offsets: Sequence[int], k: int, Y0, p0: int = 4,
               mode: str = "sign", target: float = 1e-4, max_rounds: int = 200,
               Z_out: Optional[torch.Tensor] = None, stream: Optional[torch.cuda.Stream] = None,
               gen=None, single_bf16: bool = False) -> int:
        """Queue a job.  A None: gen = (n, d, dtype, seed, gap, decay) describes the
        exact-truth matrix the server generates at admission (lp_generate).  The job
        waits for the work queued on `stream` (default: the current stream) first."""
        job, keep = self._job(A, offsets, k, p0, mode, target, max_rounds, Y0, Z_out, stream, gen,
                              single_bf16)
        jid = ctypes.c_uint64()
        _check(load().lp_server_submit(self.handle, ctypes.byref(job), ctypes.byref(jid)),
               "lp_server_submit")
        self._jobs[jid.value] = keep
        return jid.value

    def poll(self, max_results: int = 256) -> list:
        buf = (JobResult * max_results)()
        n = ctypes.c_int32()
        _check(load().lp_server_poll(self.handle, buf, max_results, ctypes.byref(n)), "lp_server_poll")
        out = []
        for r in buf[:n.value]:
            keep = self._jobs.pop(r.id)
            out.append({"id": r.id, "status": r.status, "rounds": r.rounds, "local_iters": r.local_iters,
                        "p_final": r.p_final, "change": r.change, "estimate": r.estimate,
                        "ms_queued": r.ms_queued, "ms_total": r.ms_total, "Z": keep[3]})
        return out

    def wait(self, min_done: int, timeout_s: float = 60.0) -> bool:
        st = load().lp_server_wait(self.handle, int(min_done), float(timeout_s))
        if st == LP_EBUSY:
            return False
        _check(st, "lp_server_wait")
        return True

    def close(self) -> None:
        if self.handle is not None:
            _check(load().lp_server_destroy(self.handle), "lp_server_destroy")
            self.handle = None
            self._jobs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
