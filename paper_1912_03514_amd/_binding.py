"""ctypes binding of libmihs (include/mihs.h).

Argument marshalling only: torch tensors supply device memory and the current
stream; every step of the solver runs in the HIP library.  If libmihs.so has
not been built the binding raises instead of falling back to anything else.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import threading
import weakref
from typing import Dict, List, Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmihs.so")

F64, F32 = 0, 1
SKETCH_KINDS = {"gaussian": 0, "srht": 1, "countsketch": 2, "count_gauss": 3}
PRECISIONS = {"plain": 0, "fp64": 0, "mixed": 1}
INNER_SOLVERS = {"cg": 0, "aab": 1}

MIHS_OK = 0
STATUS_NAMES = {0: "converged", 1: "max_iter", -5: "breakdown", -6: "barrier_timeout"}


class MihsError(RuntimeError):
    pass


class Info(ctypes.Structure):
    _fields_ = [
        ("outer_iters", ctypes.c_int64),
        ("inner_iters_total", ctypes.c_int64),
        ("inner_iters_max", ctypes.c_int64),
        ("rel_step", ctypes.c_double),
        ("grad_norm", ctypes.c_double),
        ("status", ctypes.c_int32),
        ("elapsed_us", ctypes.c_int32),
    ]


INFO_BYTES = ctypes.sizeof(Info)  # 48


class Tuning(ctypes.Structure):
    _fields_ = [("cg_cols", ctypes.c_int32), ("a_dma", ctypes.c_int32),
                ("inner_weight", ctypes.c_double), ("measured", ctypes.c_int32),
                ("exact", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"cg_cols": self.cg_cols, "a_dma": self.a_dma, "inner_weight": self.inner_weight,
                "measured": self.measured, "exact": self.exact}


TUNE_MAX_CANDIDATES = 16


class Problem(ctypes.Structure):
    _fields_ = [
        ("A", ctypes.c_void_p), ("b", ctypes.c_void_p), ("SA", ctypes.c_void_p),
        ("X", ctypes.c_void_p), ("info", ctypes.c_void_p),
        ("n", ctypes.c_int64), ("d", ctypes.c_int64), ("lda", ctypes.c_int64),
        ("m", ctypes.c_int64), ("ldsa", ctypes.c_int64),
    ]


_i64, _u32, _dbl, _vp, _int, _sz = (ctypes.c_int64, ctypes.c_uint32, ctypes.c_double,
                                     ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t)

_SIGS = {
    "mihs_momentum_cor4": (_int, [_dbl, _i64, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)]),
    "mihs_momentum_thm1": (_int, [_dbl, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)]),
    "mihs_lambda_from_log": (_int, [_dbl, ctypes.POINTER(_dbl)]),
    "mihs_create": (_int, [ctypes.POINTER(_vp), _int]),
    "mihs_destroy": (_int, [_vp]),
    "mihs_calibrate_rows": (_int, [_vp, ctypes.POINTER(ctypes.c_int32)]),
    "mihs_set_row_weights": (_int, [_vp, ctypes.POINTER(ctypes.c_int32)]),
    "mihs_get_row_weights": (_int, [_vp, ctypes.POINTER(ctypes.c_int32)]),
    "mihs_row_split": (_int, [_i64, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(_i64)]),
    "mihs_status_string": (ctypes.c_char_p, [_int]),
    "mihs_sketch_workspace_size": (_int, [_vp, _i64, _i64, _i64, _i64, _int, _int, _int,
                                          ctypes.POINTER(_sz)]),
    "mihs_sketch": (_int, [_vp, _vp, _int, _i64, _i64, _i64, _int, _i64, _i64, _u32, _int, _vp,
                           _i64, _vp, _sz, _vp]),
    "mihs_solve_workspace_size": (_int, [_vp, _i64, _i64, _i64, _int, ctypes.POINTER(_sz)]),
    "mihs_solve": (_int, [_vp, _vp, _int, _i64, _i64, _i64, _vp, _dbl, _vp, _i64, _i64, _int,
                          _dbl, _dbl, _dbl, _dbl, _i64, _i64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "mihs_solve_noalloc": (_int, [_vp, _vp, _int, _i64, _i64, _i64, _vp, _dbl, _vp, _i64, _i64,
                                  _int, _dbl, _dbl, _dbl, _dbl, _i64, _i64, _vp, _vp, _vp, _vp]),
    "mihs_solve_inner": (_int, [_vp, _vp, _int, _i64, _i64, _i64, _vp, _dbl, _vp, _i64, _i64,
                                _int, _int, _dbl, _dbl, _dbl, _dbl, _i64, _i64, _vp, _vp, _vp,
                                _vp, _sz, _vp]),
    "mihs_solve_dual_workspace_size": (_int, [_vp, _i64, _i64, _i64, _int, ctypes.POINTER(_sz)]),
    "mihs_solve_pd_workspace_size": (_int, [_vp, _i64, _i64, _i64, _i64, _int,
                                            ctypes.POINTER(_sz)]),
    "mihs_solve_pd": (_int, [_vp, _vp, _int, _i64, _i64, _i64, _vp, _dbl, _vp, _i64, _i64, _vp,
                             _i64, _i64, _int, _int, _dbl, _dbl, _dbl, _dbl, _i64, _dbl, _dbl,
                             _i64, _i64, _vp, _vp, _vp, _sz, _vp]),
    "mihs_solve_pd_dual_workspace_size": (_int, [_vp, _i64, _i64, _i64, _i64, _int,
                                                 ctypes.POINTER(_sz)]),
    "mihs_solve_pd_dual": (_int, [_vp, _vp, _int, _i64, _i64, _i64, _vp, _dbl, _vp, _i64, _i64,
                                  _vp, _i64, _i64, _int, _int, _dbl, _dbl, _dbl, _dbl, _i64,
                                  _dbl, _dbl, _i64, _i64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "mihs_transpose": (_int, [_vp, _vp, _int, _i64, _i64, _i64, _vp, _i64, _vp]),
    "mihs_solve_dual": (_int, [_vp, _vp, _int, _i64, _i64, _i64, _vp, _dbl, _vp, _i64, _i64,
                               _int, _dbl, _dbl, _dbl, _dbl, _i64, _i64, _vp, _vp, _vp, _vp,
                               _sz, _vp]),
    "mihs_estimate_sd_workspace_size": (_int, [_vp, _i64, _i64, _i64, _int,
                                               ctypes.POINTER(_sz)]),
    "mihs_estimate_sd": (_int, [_vp, _vp, _i64, _i64, _i64, _int, _int, _dbl, _i64,
                                ctypes.c_uint32, _dbl, _i64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "mihs_solve_multi_workspace_size": (_int, [_vp, _i64, _i64, _i64, _i64, _int,
                                               ctypes.POINTER(_sz)]),
    "mihs_solve_multi": (_int, [_vp, _vp, _int, _i64, _i64, _i64, _vp, _i64, _i64, _dbl, _vp,
                                _i64, _i64, _int, _dbl, _dbl, _dbl, _dbl, _i64, _i64, _vp, _vp,
                                _vp, _sz, _vp]),
    "mihs_solve_batched_workspace_size": (_int, [_vp, _vp, _i64, _i64, _int, ctypes.POINTER(_sz)]),
    "mihs_solve_batched": (_int, [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _i64, _int, _dbl, _dbl,
                                  _i64, _i64, _vp, _sz, _vp]),
    "mihs_batched_default_tuning": (None, [_vp]),
    "mihs_batched_plan_create": (_int, [_vp, _vp, _i64, _vp, _vp, _vp, _i64, _int, _dbl, _dbl,
                                        _i64, _i64, _vp, _vp, _sz, _vp, ctypes.POINTER(_vp)]),
    "mihs_batched_plan_run": (_int, [_vp, _vp]),
    "mihs_batched_schedule": (_int, [ctypes.c_int32, _vp, _vp, _i64, _i64, _vp, _vp, _vp, _vp,
                                     _vp]),
    "mihs_batched_plan_destroy": (_int, [_vp]),
    "mihs_tune_batched": (_int, [_vp, _vp, _i64, _vp, _vp, _vp, _i64, _int, _dbl, _dbl, _i64,
                                 _i64, _i64, ctypes.c_int32, _vp, _sz, _vp, _vp, _vp, _vp]),
    "mihs_tuning_cache_save": (_int, [_vp, ctypes.c_char_p]),
    "mihs_tuning_cache_load": (_int, [_vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]),
    "mihs_batched_cached_tuning": (_int, [_vp, _vp, _i64, _i64, _vp]),
    "mihs_solve_backward_workspace_size": (_int, [_vp, _i64, _i64, _i64, _i64, _int,
                                                  ctypes.POINTER(_sz)]),
    "mihs_solve_backward": (_int, [_vp, _vp, _int, _i64, _i64, _i64, _vp, _i64, _i64, _dbl, _int,
                                   _vp, _vp, _i64, _dbl, _dbl, _dbl, _dbl, _i64, _i64, _vp, _vp,
                                   _vp, _vp, _vp, _vp, _sz, _vp]),
}

EXPORTED = tuple(_SIGS)

_lib = None
_lock = threading.Lock()
_handles: Dict[int, int] = {}
_plans = weakref.WeakSet()  # live BatchedSolver objects, released at exit
_closed = False


def release_all():
    """Destroy every live batched plan and every handle (host memory only) while
    the process is still whole; runs at exit too (atexit handlers run before the
    HIP runtime is torn down), so no destructor calls into the library at
    interpreter shutdown.  The binding cannot be used afterwards."""
    global _closed
    with _lock:
        if _closed or _lib is None:
            _closed = True
            return
        _closed = True
        for s in list(_plans):
            s.close()
        for dev, h in list(_handles.items()):
            _lib.mihs_destroy(h)
        _handles.clear()


atexit.register(release_all)


def load_library(path: str = LIB_PATH):
    """Load libmihs.so (no GPU work).  Raises if it is missing."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise MihsError(f"{path} is not built; run `python -m paper_1912_03514_amd.build`")
            lib = ctypes.CDLL(path)
            for name, (res, args) in _SIGS.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def _check(rc: int, what: str):
    if rc != MIHS_OK:
        msg = load_library().mihs_status_string(rc).decode()
        raise MihsError(f"{what} failed with {rc}: {msg}")


def handle(device: Optional[int] = None) -> int:
    if _closed:
        raise MihsError("libmihs handles were released at exit")
    dev = torch.cuda.current_device() if device is None else int(device)
    with _lock:
        h = _handles.get(dev)
    if h is None:
        lib = load_library()
        hp = _vp()
        _check(lib.mihs_create(ctypes.byref(hp), dev), "mihs_create")
        # per-XCD row shares of the gradient pass, measured once per handle;
        # when the measurement cannot run the handle keeps equal shares
        lib.mihs_calibrate_rows(hp.value, None)
        with _lock:
            _handles[dev] = hp.value
        h = hp.value
    return h


_W8 = ctypes.c_int32 * 8


def row_weights(device: Optional[int] = None) -> Tuple[int, ...]:
    """The handle's 8 per-XCD row weights of the gradient pass
    (mihs_get_row_weights)."""
    w = _W8()
    _check(load_library().mihs_get_row_weights(handle(device), w), "mihs_get_row_weights")
    return tuple(w)


def set_row_weights(weights: Optional[Sequence[int]], device: Optional[int] = None) -> None:
    """Set the 8 per-XCD row weights (each 1..64); None restores equal weights
    (mihs_set_row_weights)."""
    w = None if weights is None else _W8(*[int(v) for v in weights])
    _check(load_library().mihs_set_row_weights(handle(device), w), "mihs_set_row_weights")


def calibrate_rows(device: Optional[int] = None) -> Tuple[int, ...]:
    """Measure the per-XCD streaming rates again and set the weights from them
    (mihs_calibrate_rows); returns the new weights."""
    w = _W8()
    _check(load_library().mihs_calibrate_rows(handle(device), w), "mihs_calibrate_rows")
    return tuple(w)


def row_split(n: int, G: int, weights: Sequence[int]) -> List[int]:
    """First row of each of G workgroups (and n at the end) for these weights
    (mihs_row_split, host only)."""
    out = (_i64 * (int(G) + 1))()
    _check(load_library().mihs_row_split(int(n), int(G), _W8(*[int(v) for v in weights]), out),
           "mihs_row_split")
    return list(out)


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise MihsError(f"unsupported dtype {t.dtype}")


def _row_aligned(t: torch.Tensor) -> torch.Tensor:
    """Rows must start on 16-byte boundaries; copy into a padded buffer if not."""
    es = t.element_size()
    if t.stride(1) == 1 and t.data_ptr() % 16 == 0 and (t.stride(0) * es) % 16 == 0:
        return t
    n, d = t.shape
    per = 16 // es
    ld = (d + per - 1) // per * per
    buf = torch.zeros((n, ld), dtype=t.dtype, device=t.device)
    buf[:, :d] = t
    return buf[:, :d]


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def momentum(sd: float, m: int) -> Tuple[float, float]:
    """Corollary 4 momentum (alpha, beta) for statistical dimension sd and a
    sketch of m rows, from mihs_momentum_cor4."""
    a, b = _dbl(), _dbl()
    if load_library().mihs_momentum_cor4(float(sd), int(m), ctypes.byref(a), ctypes.byref(b)):
        raise ValueError("need 0 < sd < m")
    return a.value, b.value


def momentum_thm1(eps: float) -> Tuple[float, float]:
    """Theorem 1 momentum (alpha*, beta*) for embedding distortion eps, from
    mihs_momentum_thm1."""
    a, b = _dbl(), _dbl()
    if load_library().mihs_momentum_thm1(float(eps), ctypes.byref(a), ctypes.byref(b)):
        raise ValueError("need 0 < eps < 1")
    return a.value, b.value


def lambda_from_log(log_lambda: float) -> float:
    """lambda of the log(lambda) parametrisation, from mihs_lambda_from_log."""
    v = _dbl()
    _check(load_library().mihs_lambda_from_log(float(log_lambda), ctypes.byref(v)),
           "mihs_lambda_from_log")
    return v.value


def mihs_sketch(A: torch.Tensor, kind: str, m: int, seed: int, precision: str = "plain",
                m2: int = 0, out: Optional[torch.Tensor] = None,
                workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """SA = S A on the GPU (see include/mihs.h).  Returns an (m or m2) x d tensor,
    float64 for the plain path and float32 for the mixed path.  `out` (rows x d of
    that type, 16-byte aligned rows) and `workspace` (uint8, at least
    sketch_workspace_bytes) may be given to run without allocating, e.g. inside a
    captured graph."""
    if A.dim() != 2 or not A.is_cuda:
        raise MihsError("A must be a 2-D device tensor")
    A = _row_aligned(A)
    lib = load_library()
    h = handle(A.device.index)
    n, d = A.shape
    k = SKETCH_KINDS[kind]
    p = PRECISIONS[precision]
    rows = m2 if kind == "count_gauss" else m
    sa_dtype = torch.float32 if p == 1 else torch.float64
    if out is None:
        ld = (d + 3) // 4 * 4
        SA = torch.zeros((rows, ld), dtype=sa_dtype, device=A.device)[:, :d]
    else:
        if out.shape != (rows, d) or out.dtype != sa_dtype or out.stride(1) != 1:
            raise MihsError(f"out must be a {rows} x {d} {sa_dtype} tensor with unit column stride")
        SA = out
    ws_n = _sz()
    _check(lib.mihs_sketch_workspace_size(h, n, d, m, m2, k, _dtype_code(A), p, ctypes.byref(ws_n)),
           "mihs_sketch_workspace_size")
    if workspace is None:
        ws = _workspace(ws_n.value, A.device)
    else:
        if workspace.numel() < ws_n.value:
            raise MihsError("sketch workspace too small")
        ws = workspace
    _check(lib.mihs_sketch(h, A.data_ptr(), _dtype_code(A), n, d, A.stride(0), k, m, m2,
                           seed & 0xFFFFFFFF, p, SA.data_ptr(), SA.stride(0), ws.data_ptr(),
                           ws.numel(), _stream(A.device)), "mihs_sketch")
    return SA


def info_to_dict(raw: torch.Tensor) -> list:
    host = raw.cpu().numpy().tobytes()
    out = []
    for i in range(len(host) // INFO_BYTES):
        s = Info.from_buffer_copy(host[i * INFO_BYTES:(i + 1) * INFO_BYTES])
        out.append({"outer_iters": s.outer_iters, "inner_iters_total": s.inner_iters_total,
                    "inner_iters_max": s.inner_iters_max, "rel_step": s.rel_step,
                    "grad_norm": s.grad_norm, "status": s.status,
                    "status_name": STATUS_NAMES.get(s.status, str(s.status)),
                    "elapsed_us": s.elapsed_us})
    return out


class SolveWorkspace:
    """Preallocated device buffers for repeated solves of one shape."""

    def __init__(self, n: int, d: int, m: int, precision: str, device):
        lib = load_library()
        self.h = handle(device.index if hasattr(device, "index") else device)
        ws_n = _sz()
        _check(lib.mihs_solve_workspace_size(self.h, n, d, m, PRECISIONS[precision],
                                             ctypes.byref(ws_n)), "mihs_solve_workspace_size")
        self.ws = _workspace(ws_n.value, device)
        self.info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=device)


def mihs_solve(A: torch.Tensor, b: torch.Tensor, lam: float, SA: torch.Tensor, alpha: float,
               beta: float, eps_sub: float = 1e-2, tol: float = 1e-10, max_outer: int = 200,
               max_inner: int = 1000, x0: Optional[torch.Tensor] = None,
               x_prev: Optional[torch.Tensor] = None, precision: Optional[str] = None,
               workspace: Optional[SolveWorkspace] = None, sync: bool = True,
               inner: str = "cg"):
    """M-IHS on the GPU (see include/mihs.h); inner is "cg" or "aab" (AAb_Solver,
    Algorithm 6).  Returns (x, info) where info is a dict (sync=True) or the raw
    device record (sync=False)."""
    if precision is None:
        precision = "mixed" if SA.dtype == torch.float32 else "plain"
    p = PRECISIONS[precision]
    inn = INNER_SOLVERS[inner]
    A = _row_aligned(A)
    SA = _row_aligned(SA)
    n, d = A.shape
    m = SA.shape[0]
    dev = A.device
    if b.dtype != torch.float64 or b.numel() != n or not b.is_contiguous():
        raise MihsError("b must be a contiguous float64 vector of length n")
    x = torch.zeros(d, dtype=torch.float64, device=dev) if x0 is None else x0.clone()
    if workspace is None:
        workspace = SolveWorkspace(n, d, m, precision, dev)
    lib = load_library()
    rc = lib.mihs_solve_inner(workspace.h, A.data_ptr(), _dtype_code(A), n, d, A.stride(0),
                              b.data_ptr(), float(lam), SA.data_ptr(), m, SA.stride(0), p, inn,
                              float(alpha), float(beta), float(eps_sub), float(tol),
                              int(max_outer), int(max_inner), x.data_ptr(),
                              x_prev.data_ptr() if x_prev is not None else None,
                              workspace.info.data_ptr(), workspace.ws.data_ptr(),
                              workspace.ws.numel(), _stream(dev))
    _check(rc, "mihs_solve_inner")
    if not sync:
        return x, workspace.info
    torch.cuda.synchronize(dev)
    return x, info_to_dict(workspace.info)[0]


NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024  # MIHS_NOALLOC_SCRATCH_BYTES


def mihs_solve_noalloc(A: torch.Tensor, b: torch.Tensor, lam: float, SA: torch.Tensor,
                       alpha: float, beta: float, X: torch.Tensor, info: torch.Tensor,
                       eps_sub: float = 1e-2, tol: float = 1e-10, max_outer: int = 200,
                       max_inner: int = 1000, x_prev: Optional[torch.Tensor] = None,
                       precision: Optional[str] = None):
    """mihs_solve_noalloc (see include/mihs.h): M-IHS with the library's static
    scratch instead of a workspace.  The caller passes every buffer: A, b, SA
    (16-byte aligned rows), X (d float64: in x^1, out the solution) and info
    (INFO_BYTES uint8); nothing is allocated or copied, and nothing waits."""
    if precision is None:
        precision = "mixed" if SA.dtype == torch.float32 else "plain"
    n, d = A.shape
    m = SA.shape[0]
    if X.dtype != torch.float64 or X.numel() != d or not X.is_contiguous():
        raise MihsError("X must be a contiguous float64 vector of length d")
    if info.dtype != torch.uint8 or info.numel() < INFO_BYTES:
        raise MihsError("info must hold one record")
    if b.dtype != torch.float64 or b.numel() != n or not b.is_contiguous():
        raise MihsError("b must be a contiguous float64 vector of length n")
    for name, t in (("A", A), ("SA", SA)):
        if t.stride(1) != 1 or t.data_ptr() % 16 or (t.stride(0) * t.element_size()) % 16:
            raise MihsError(f"{name} must have unit column stride and 16-byte aligned rows")
    lib = load_library()
    rc = lib.mihs_solve_noalloc(handle(A.device.index), A.data_ptr(), _dtype_code(A), n, d,
                                A.stride(0), b.data_ptr(), float(lam), SA.data_ptr(), m,
                                SA.stride(0), PRECISIONS[precision], float(alpha), float(beta),
                                float(eps_sub), float(tol), int(max_outer), int(max_inner),
                                X.data_ptr(), x_prev.data_ptr() if x_prev is not None else None,
                                info.data_ptr(), _stream(A.device))
    _check(rc, "mihs_solve_noalloc")
    return X


def mihs_solve_dual(At: torch.Tensor, b: torch.Tensor, lam: float, SAt: torch.Tensor,
                    alpha: float, beta: float, eps_sub: float = 1e-2, tol: float = 1e-10,
                    max_outer: int = 200, max_inner: int = 1000,
                    nu0: Optional[torch.Tensor] = None, precision: Optional[str] = None,
                    sync: bool = True):
    """Dual M-IHS for n <= d (see include/mihs.h).  At is A^T (d x n), SAt its
    sketch (m x n).  Returns (x, nu, info): x = A^T nu in R^d, nu in R^n."""
    if precision is None:
        precision = "mixed" if SAt.dtype == torch.float32 else "plain"
    p = PRECISIONS[precision]
    At = _row_aligned(At)
    SAt = _row_aligned(SAt)
    d, n = At.shape
    m = SAt.shape[0]
    dev = At.device
    if b.dtype != torch.float64 or b.numel() != n or not b.is_contiguous():
        raise MihsError("b must be a contiguous float64 vector of length n")
    nu = torch.zeros(n, dtype=torch.float64, device=dev) if nu0 is None else nu0.clone()
    x = torch.empty(d, dtype=torch.float64, device=dev)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=dev)
    lib = load_library()
    h = handle(dev.index)
    ws_n = _sz()
    _check(lib.mihs_solve_dual_workspace_size(h, n, d, m, p, ctypes.byref(ws_n)),
           "mihs_solve_dual_workspace_size")
    ws = _workspace(ws_n.value, dev)
    rc = lib.mihs_solve_dual(h, At.data_ptr(), _dtype_code(At), n, d, At.stride(0), b.data_ptr(),
                             float(lam), SAt.data_ptr(), m, SAt.stride(0), p, float(alpha),
                             float(beta), float(eps_sub), float(tol), int(max_outer),
                             int(max_inner), nu.data_ptr(), x.data_ptr(), info.data_ptr(),
                             ws.data_ptr(), ws.numel(), _stream(dev))
    _check(rc, "mihs_solve_dual")
    if not sync:
        return x, nu, (info, ws)
    torch.cuda.synchronize(dev)
    return x, nu, info_to_dict(info)[0]


def mihs_estimate_sd(SA: torch.Tensor, lam: float, T: int = 2, seed: int = 0,
                     eps_tr: float = 0.5, max_inner: int = 1000,
                     precision: Optional[str] = None, want_z: bool = False,
                     inner: str = "aab"):
    """Inexact Hutchinson estimate of the statistical dimension from a sketch SA
    (m x d), Algorithm 5 (see include/mihs.h); inner is "aab" (AAb_Solver, the
    paper's choice) or "cg".  Returns (sd, infos) or, with want_z, (sd, Z, infos)
    where row l of Z (T x d) solves ((SA)^T SA + lambda I) z = v^l."""
    if precision is None:
        precision = "mixed" if SA.dtype == torch.float32 else "plain"
    p = PRECISIONS[precision]
    inn = INNER_SOLVERS[inner]
    SA = _row_aligned(SA)
    m, d = SA.shape
    dev = SA.device
    sd = torch.zeros((), dtype=torch.float64, device=dev)
    Z = torch.empty((T, d), dtype=torch.float64, device=dev) if want_z else None
    info = torch.zeros(INFO_BYTES * T, dtype=torch.uint8, device=dev)
    lib = load_library()
    h = handle(dev.index)
    ws_n = _sz()
    _check(lib.mihs_estimate_sd_workspace_size(h, m, d, int(T), p, ctypes.byref(ws_n)),
           "mihs_estimate_sd_workspace_size")
    ws = _workspace(ws_n.value, dev)
    rc = lib.mihs_estimate_sd(h, SA.data_ptr(), m, d, SA.stride(0), p, inn, float(lam), int(T),
                              int(seed) & 0xFFFFFFFF, float(eps_tr), int(max_inner),
                              sd.data_ptr(), Z.data_ptr() if Z is not None else None,
                              info.data_ptr(), ws.data_ptr(), ws.numel(), _stream(dev))
    _check(rc, "mihs_estimate_sd")
    torch.cuda.synchronize(dev)
    infos = info_to_dict(info)
    return (float(sd), Z, infos) if want_z else (float(sd), infos)


def mihs_transpose(M: torch.Tensor) -> torch.Tensor:
    """M^T as a new row-major tensor, on the library's transpose kernel."""
    M = _row_aligned(M)
    rows, cols = M.shape
    per = 16 // M.element_size()
    ld = (rows + per - 1) // per * per
    out = torch.empty((cols, ld), dtype=M.dtype, device=M.device)
    lib = load_library()
    _check(lib.mihs_transpose(handle(M.device.index), M.data_ptr(), _dtype_code(M), rows, cols,
                              M.stride(0), out.data_ptr(), ld, _stream(M.device)),
           "mihs_transpose")
    return out[:, :rows]


def mihs_sketch_two_stage(M: torch.Tensor, kind1: str, m1: int, seed1: int, kind2: str,
                          m2: int, seed2: int, precision: str = "plain"):
    """The two sketches of Primal-Dual M-IHS (Algorithms 3, 4): Q = (S M)^T
    (cols x m1) and WQ = W Q (m2 x m1), from mihs_sketch and mihs_transpose."""
    SM = mihs_sketch(M, kind1, m1, seed1, precision=precision)
    Q = mihs_transpose(SM)
    WQ = mihs_sketch(Q, kind2, m2, seed2, precision=precision)
    return Q, WQ


def _pd_call(fn_ws, fn, Aop, rows, cols, b, lam, Q, WQ, alpha1, beta1, alpha2, beta2, M,
             eps_sub, tol, max_outer, max_inner, x, extra, precision, inner, dev):
    p = PRECISIONS[precision]
    inn = INNER_SOLVERS[inner]
    if Q.dim() != 2 or Q.shape[0] != cols:
        raise MihsError(f"Q must have one row per outer unknown ({cols}), got {tuple(Q.shape)}")
    if WQ.dim() != 2 or WQ.shape[1] != Q.shape[1]:
        raise MihsError("WQ must have as many columns as Q")
    Q = _row_aligned(Q)
    WQ = _row_aligned(WQ)
    m1 = Q.shape[1]
    m2 = WQ.shape[0]
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=dev)
    lib = load_library()
    h = handle(dev.index)
    n_, d_ = (rows, cols) if fn == "mihs_solve_pd" else (cols, rows)
    ws_n = _sz()
    _check(getattr(lib, fn_ws)(h, n_, d_, m1, m2, p, ctypes.byref(ws_n)), fn_ws)
    ws = _workspace(ws_n.value, dev)
    args = [h, Aop.data_ptr(), _dtype_code(Aop), n_, d_, Aop.stride(0), b.data_ptr(), float(lam),
            Q.data_ptr(), m1, Q.stride(0), WQ.data_ptr(), m2, WQ.stride(0), p, inn,
            float(alpha1), float(beta1), float(alpha2), float(beta2), int(M), float(eps_sub),
            float(tol), int(max_outer), int(max_inner), x.data_ptr()]
    args += [e.data_ptr() for e in extra]
    args += [info.data_ptr(), ws.data_ptr(), ws.numel(), _stream(dev)]
    _check(getattr(lib, fn)(*args), fn)
    return info, ws


def mihs_solve_pd(A: torch.Tensor, b: torch.Tensor, lam: float, Q: torch.Tensor,
                  WQ: torch.Tensor, alpha1: float, beta1: float, alpha2: float, beta2: float,
                  M: int = 25, eps_sub: float = 0.1, tol: float = 1e-10, max_outer: int = 100,
                  max_inner: int = 1000, x0: Optional[torch.Tensor] = None,
                  precision: Optional[str] = None, inner: str = "aab", sync: bool = True):
    """Primal-Dual M-IHS for n >= d (Algorithm 4; see include/mihs.h).  Q = (S A)^T
    (d x m1), WQ = W Q (m2 x m1).  Returns (x, info)."""
    if precision is None:
        precision = "mixed" if Q.dtype == torch.float32 else "plain"
    A = _row_aligned(A)
    n, d = A.shape
    dev = A.device
    if b.dtype != torch.float64 or b.numel() != n or not b.is_contiguous():
        raise MihsError("b must be a contiguous float64 vector of length n")
    x = torch.zeros(d, dtype=torch.float64, device=dev) if x0 is None else x0.clone()
    info, ws = _pd_call("mihs_solve_pd_workspace_size", "mihs_solve_pd", A, n, d, b, lam, Q, WQ,
                        alpha1, beta1, alpha2, beta2, M, eps_sub, tol, max_outer, max_inner, x,
                        [], precision, inner, dev)
    if not sync:
        return x, (info, ws)
    torch.cuda.synchronize(dev)
    return x, info_to_dict(info)[0]


def mihs_solve_pd_dual(At: torch.Tensor, b: torch.Tensor, lam: float, Q: torch.Tensor,
                       WQ: torch.Tensor, alpha1: float, beta1: float, alpha2: float,
                       beta2: float, M: int = 25, eps_sub: float = 0.1, tol: float = 1e-10,
                       max_outer: int = 100, max_inner: int = 1000,
                       precision: Optional[str] = None, inner: str = "aab", sync: bool = True):
    """Primal-Dual M-IHS for n <= d (Algorithm 3; see include/mihs.h).  At = A^T
    (d x n), Q = (S A^T)^T (n x m1), WQ = W Q.  Returns (x, nu, info)."""
    if precision is None:
        precision = "mixed" if Q.dtype == torch.float32 else "plain"
    At = _row_aligned(At)
    d, n = At.shape
    dev = At.device
    if b.dtype != torch.float64 or b.numel() != n or not b.is_contiguous():
        raise MihsError("b must be a contiguous float64 vector of length n")
    nu = torch.zeros(n, dtype=torch.float64, device=dev)
    x = torch.empty(d, dtype=torch.float64, device=dev)
    info, ws = _pd_call("mihs_solve_pd_dual_workspace_size", "mihs_solve_pd_dual", At, d, n, b,
                        lam, Q, WQ, alpha1, beta1, alpha2, beta2, M, eps_sub, tol, max_outer,
                        max_inner, nu, [x], precision, inner, dev)
    if not sync:
        return x, nu, (info, ws)
    torch.cuda.synchronize(dev)
    return x, nu, info_to_dict(info)[0]


def mihs_solve_backward(A: torch.Tensor, SA: torch.Tensor, lam: float, Xstar: torch.Tensor,
                        Gbar: torch.Tensor, alpha: float, beta: float, eps_sub: float = 1e-2,
                        tol: float = 1e-12, max_outer: int = 300, max_inner: int = 1000,
                        want_dB: bool = True, precision: Optional[str] = None,
                        want_dloglam: bool = False):
    """Adjoint M-IHS solves W = (A^T A + lambda I)^{-1} Gbar; dB = A W;
    dlambda = -sum X*.W.  Returns (W, dB or None, dlambda (0-d tensor), infos),
    or with want_dloglam (W, dB, dlambda, dloglambda, infos)."""
    if precision is None:
        precision = "mixed" if SA.dtype == torch.float32 else "plain"
    p = PRECISIONS[precision]
    A = _row_aligned(A)
    SA = _row_aligned(SA)
    n, d = A.shape
    m = SA.shape[0]
    dev = A.device
    Xs = Xstar.reshape(d, -1).contiguous().to(torch.float64)
    Gb = Gbar.reshape(d, -1).contiguous().to(torch.float64)
    k = Gb.shape[1]
    W = torch.zeros((d, k), dtype=torch.float64, device=dev)
    dB = torch.zeros((n, k), dtype=torch.float64, device=dev) if want_dB else None
    dlam = torch.zeros((), dtype=torch.float64, device=dev)
    dll = torch.zeros((), dtype=torch.float64, device=dev) if want_dloglam else None
    info = torch.zeros(INFO_BYTES * k, dtype=torch.uint8, device=dev)
    lib = load_library()
    h = handle(dev.index)
    ws_n = _sz()
    _check(lib.mihs_solve_backward_workspace_size(h, n, d, m, k, p, ctypes.byref(ws_n)),
           "mihs_solve_backward_workspace_size")
    ws = _workspace(ws_n.value, dev)
    rc = lib.mihs_solve_backward(h, A.data_ptr(), _dtype_code(A), n, d, A.stride(0),
                                 SA.data_ptr(), m, SA.stride(0), float(lam), p, Xs.data_ptr(),
                                 Gb.data_ptr(), k, float(alpha), float(beta), float(eps_sub),
                                 float(tol), int(max_outer), int(max_inner), W.data_ptr(),
                                 dB.data_ptr() if dB is not None else None, dlam.data_ptr(),
                                 dll.data_ptr() if dll is not None else None,
                                 info.data_ptr(), ws.data_ptr(), ws.numel(), _stream(dev))
    _check(rc, "mihs_solve_backward")
    torch.cuda.synchronize(dev)
    if want_dloglam:
        return W, dB, dlam, dll, info_to_dict(info)
    return W, dB, dlam, info_to_dict(info)


def mihs_solve_batched(problems, lambdas: torch.Tensor, alphas: torch.Tensor,
                       betas: torch.Tensor, eps_sub: float = 1e-2, tol: float = 1e-10,
                       max_outer: int = 300, max_inner: int = 1000,
                       precision: Optional[str] = None, sync: bool = True):
    """Lambda-path solves of many problems in one launch (see include/mihs.h).

    problems: list of (A, b, SA) device tensors (A float64, n_k x d_k with d_k <= 1024).
    lambdas, alphas, betas: nprob x nlam float64 device tensors.
    Returns (list of d_k x nlam solution tensors, list of per-problem info lists)."""
    nprob = len(problems)
    if lambdas.shape[0] != nprob or lambdas.dim() != 2:
        raise MihsError("lambdas must be nprob x nlam")
    nlam = lambdas.shape[1]
    if precision is None:
        precision = "mixed" if problems[0][2].dtype == torch.float32 else "plain"
    p = PRECISIONS[precision]
    dev = problems[0][0].device
    lam = lambdas.to(torch.float64).contiguous()
    alp = alphas.to(torch.float64).contiguous()
    bet = betas.to(torch.float64).contiguous()
    keep, xs, infos = [], [], []
    table = (Problem * nprob)()
    for i, (A, b, SA) in enumerate(problems):
        A = _row_aligned(A)
        SA = _row_aligned(SA)
        if A.dtype != torch.float64:
            raise MihsError("batched problems take float64 A")
        n, d = A.shape
        X = torch.zeros((d, nlam), dtype=torch.float64, device=dev)
        info = torch.zeros(INFO_BYTES * nlam, dtype=torch.uint8, device=dev)
        keep += [A, b, SA]
        xs.append(X)
        infos.append(info)
        table[i] = Problem(A.data_ptr(), b.data_ptr(), SA.data_ptr(), X.data_ptr(),
                           info.data_ptr(), n, d, A.stride(0), SA.shape[0], SA.stride(0))
    lib = load_library()
    h = handle(dev.index)
    ws_n = _sz()
    _check(lib.mihs_solve_batched_workspace_size(h, ctypes.cast(table, _vp), nprob, nlam, p,
                                                 ctypes.byref(ws_n)),
           "mihs_solve_batched_workspace_size")
    ws = _workspace(ws_n.value, dev)
    rc = lib.mihs_solve_batched(h, None, ctypes.cast(table, _vp), nprob, lam.data_ptr(),
                                alp.data_ptr(), bet.data_ptr(), nlam, p, float(eps_sub),
                                float(tol), int(max_outer), int(max_inner), ws.data_ptr(),
                                ws.numel(), _stream(dev))
    _check(rc, "mihs_solve_batched")
    if not sync:
        return xs, infos, (keep, ws)
    torch.cuda.synchronize(dev)
    return xs, [info_to_dict(t) for t in infos]


def batched_schedule(shapes, nlam: int, num_cu: int, tuning: Optional[dict] = None,
                     cost=None) -> dict:
    """The batched launch's schedule for problems of the given (n, d) shapes on
    num_cu workgroups, computed on the host (no device): team0, tsize, tcg per
    entry (problem-major, one entry per 16 lambdas)."""
    lib = load_library()
    nprob = len(shapes)
    n = (ctypes.c_int64 * nprob)(*[int(s[0]) for s in shapes])
    d = (ctypes.c_int64 * nprob)(*[int(s[1]) for s in shapes])
    tn = Tuning()
    lib.mihs_batched_default_tuning(ctypes.byref(tn))
    if tuning is not None:
        tn = Tuning(int(tuning["cg_cols"]), int(tuning["a_dma"]), float(tuning["inner_weight"]),
                    int(tuning.get("measured", 0)), int(tuning.get("exact", 0)))
    count = nprob * ((nlam + 15) // 16)
    c = None
    if cost is not None:
        if len(cost) != count:
            raise MihsError(f"cost needs {count} values")
        c = (ctypes.c_double * count)(*[float(v) for v in cost])
    t0, ts, tc = ((ctypes.c_int32 * count)() for _ in range(3))
    _check(lib.mihs_batched_schedule(int(num_cu), n, d, nprob, int(nlam), ctypes.byref(tn), c,
                                     t0, ts, tc), "mihs_batched_schedule")
    return {"team0": list(t0), "tsize": list(ts), "tcg": list(tc)}


def tuning_cache_save(path: str, device: Optional[int] = None) -> None:
    """Write the batched launch shapes tuned in this process (on `device`) to a
    JSON tuning-cache file (mihs_tuning_cache_save)."""
    _check(load_library().mihs_tuning_cache_save(handle(device), os.fsencode(path)),
           "mihs_tuning_cache_save")


def tuning_cache_load(path: str, device: Optional[int] = None) -> int:
    """Take the shapes of a tuning-cache file written on the same kind of
    device (mihs_tuning_cache_load); returns how many were taken."""
    n = ctypes.c_int32()
    _check(load_library().mihs_tuning_cache_load(handle(device), os.fsencode(path),
                                                 ctypes.byref(n)), "mihs_tuning_cache_load")
    return n.value


def sketch_workspace_bytes(n: int, d: int, m: int, kind: str, precision: str = "plain",
                           a_dtype: torch.dtype = torch.float64, m2: int = 0,
                           device: Optional[int] = None) -> int:
    """Workspace bytes of one mihs_sketch call of this shape."""
    lib = load_library()
    h = handle(device)
    ws_n = _sz()
    _check(lib.mihs_sketch_workspace_size(h, n, d, m, m2, SKETCH_KINDS[kind],
                                          F32 if a_dtype == torch.float32 else F64,
                                          PRECISIONS[precision], ctypes.byref(ws_n)),
           "mihs_sketch_workspace_size")
    return ws_n.value


class BatchedSolver:
    """A planned batched lambda-path solve (mihs_batched_plan_create/run).

    problems: list of (A, b, SA) device tensors as for mihs_solve_batched.  The
    plan records their addresses: new values may be written into A, b or SA in
    place between runs.  run() zeroes X (x^1 = 0) and enqueues the solve on the
    current stream without synchronising or allocating, so it can be captured
    (capture() returns a replayable torch.cuda.CUDAGraph).  tune() runs the
    library's autotuner on these problems and re-plans with its choice."""

    def __init__(self, problems, lambdas: torch.Tensor, alphas: torch.Tensor,
                 betas: torch.Tensor, eps_sub: float = 1e-2, tol: float = 1e-10,
                 max_outer: int = 300, max_inner: int = 1000, precision: Optional[str] = None,
                 tuning: Optional[dict] = None):
        nprob = len(problems)
        if lambdas.dim() != 2 or lambdas.shape[0] != nprob:
            raise MihsError("lambdas must be nprob x nlam")
        self.nprob, self.nlam = nprob, lambdas.shape[1]
        if precision is None:
            precision = "mixed" if problems[0][2].dtype == torch.float32 else "plain"
        self.precision = PRECISIONS[precision]
        self.dev = problems[0][0].device
        self.params = (float(eps_sub), float(tol), int(max_outer), int(max_inner))
        self.lam = lambdas.to(torch.float64).contiguous()
        self.alp = alphas.to(torch.float64).contiguous()
        self.bet = betas.to(torch.float64).contiguous()
        ds = [int(A.shape[1]) for A, _, _ in problems]
        # every X in one buffer (one fill restarts them all), every info record in another
        self.X_all = torch.zeros(sum(ds) * self.nlam, dtype=torch.float64, device=self.dev)
        self.info_all = torch.zeros(INFO_BYTES * self.nlam * nprob, dtype=torch.uint8,
                                    device=self.dev)
        self.xs, self._keep = [], []
        self.table = (Problem * nprob)()
        off = 0
        for i, (A, b, SA) in enumerate(problems):
            A = _row_aligned(A)
            SA = _row_aligned(SA)
            if A.dtype != torch.float64:
                raise MihsError("batched problems take float64 A")
            n, d = A.shape
            X = self.X_all[off:off + d * self.nlam].view(d, self.nlam)
            off += d * self.nlam
            info = self.info_all[i * INFO_BYTES * self.nlam:(i + 1) * INFO_BYTES * self.nlam]
            self._keep += [A, b, SA]
            self.xs.append(X)
            self.table[i] = Problem(A.data_ptr(), b.data_ptr(), SA.data_ptr(), X.data_ptr(),
                                    info.data_ptr(), n, d, A.stride(0), SA.shape[0],
                                    SA.stride(0))
        lib = load_library()
        self.h = handle(self.dev.index)
        ws_n = _sz()
        _check(lib.mihs_solve_batched_workspace_size(self.h, ctypes.cast(self.table, _vp), nprob,
                                                     self.nlam, self.precision,
                                                     ctypes.byref(ws_n)),
               "mihs_solve_batched_workspace_size")
        self.ws = _workspace(ws_n.value, self.dev)
        self.plan = None
        self._make_plan(tuning)
        _plans.add(self)

    def _make_plan(self, tuning: Optional[dict]):
        lib = load_library()
        if self.plan is not None:
            lib.mihs_batched_plan_destroy(self.plan)
            self.plan = None
        tn = None
        if tuning is not None:
            tn = Tuning(int(tuning["cg_cols"]), int(tuning["a_dma"]), float(tuning["inner_weight"]),
                        int(tuning.get("measured", 0)), int(tuning.get("exact", 0)))
        eps_sub, tol, max_outer, max_inner = self.params
        plan = _vp()
        _check(lib.mihs_batched_plan_create(
            self.h, ctypes.cast(self.table, _vp), self.nprob, self.lam.data_ptr(),
            self.alp.data_ptr(), self.bet.data_ptr(), self.nlam, self.precision, eps_sub, tol,
            max_outer, max_inner, ctypes.byref(tn) if tn is not None else None,
            self.ws.data_ptr(), self.ws.numel(), _stream(self.dev), ctypes.byref(plan)),
            "mihs_batched_plan_create")
        self.plan = plan

    def cached_tuning(self) -> Optional[dict]:
        """The shape the handle keeps for this problem set (from an earlier
        tune() or a loaded tuning cache), or None."""
        t = Tuning()
        rc = load_library().mihs_batched_cached_tuning(self.h, ctypes.cast(self.table, _vp),
                                                       self.nprob, self.nlam, ctypes.byref(t))
        return t.as_dict() if rc == MIHS_OK else None

    def tune(self, trial_outer: int = 8, measure: bool = True, allow_exact: bool = False,
             cache: Optional[str] = None) -> dict:
        """Autotune the launch shape on these problems (blocking; overwrites X)
        and re-plan with the choice: coordinate descent on trial_outer-iteration
        trials of the inexact-CG shapes (with allow_exact also exact Cholesky
        sub-solves), then (measure) full runs of the best of each kind and a
        schedule sized from the faster one's per-problem times.  Returns the
        choice and the trial times.  With `cache` (a tuning-cache file) a shape
        stored there for this problem set is used without tuning (if it obeys
        allow_exact), and a new one is written there after tuning."""
        lib = load_library()
        if cache is not None:
            if os.path.exists(cache):
                tuning_cache_load(cache, self.dev.index)
            got = self.cached_tuning()
            if got is not None and (allow_exact or not got["exact"]):
                self._make_plan(got)
                return {"best": got, "trial_ms": [], "from_cache": True}
        eps_sub, tol, max_outer, max_inner = self.params
        best = Tuning()
        times = (ctypes.c_float * TUNE_MAX_CANDIDATES)()
        nc = ctypes.c_int32()
        _check(lib.mihs_tune_batched(
            self.h, ctypes.cast(self.table, _vp), self.nprob, self.lam.data_ptr(),
            self.alp.data_ptr(), self.bet.data_ptr(), self.nlam, self.precision, eps_sub, tol,
            int(trial_outer), int(max_outer) if measure else 0, max_inner,
            1 if allow_exact else 0, self.ws.data_ptr(),
            self.ws.numel(), _stream(self.dev),
            ctypes.byref(best), times, ctypes.byref(nc)), "mihs_tune_batched")
        self._make_plan(best.as_dict())
        if cache is not None:
            tuning_cache_save(cache, self.dev.index)
        return {"best": best.as_dict(), "trial_ms": [round(times[i], 3) for i in range(nc.value)]}

    def run(self):
        """x^1 = 0 and the solve, enqueued on the current stream (no sync)."""
        self.X_all.zero_()
        _check(load_library().mihs_batched_plan_run(self.plan, _stream(self.dev)),
               "mihs_batched_plan_run")

    def capture(self) -> "torch.cuda.CUDAGraph":
        """Capture run() in a graph (warm it up eagerly first)."""
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream(device=self.dev)
        s.wait_stream(torch.cuda.current_stream(self.dev))
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                self.run()
        torch.cuda.current_stream(self.dev).wait_stream(s)
        return g

    def infos(self) -> list:
        raw = info_to_dict(self.info_all)
        return [raw[i * self.nlam:(i + 1) * self.nlam] for i in range(self.nprob)]

    def close(self):
        """Free the plan (host memory only); the solver cannot run afterwards."""
        if self.plan is not None and _lib is not None:
            _lib.mihs_batched_plan_destroy(self.plan)
        self.plan = None

    def __del__(self):
        # at interpreter shutdown the atexit hook has already released the plan
        if not _closed:
            try:
                self.close()
            except Exception:
                pass


def mihs_solve_multi(A: torch.Tensor, B: torch.Tensor, lam: float, SA: torch.Tensor,
                     alpha: float, beta: float, eps_sub: float = 1e-2, tol: float = 1e-10,
                     max_outer: int = 300, max_inner: int = 1000, X0: Optional[torch.Tensor] = None,
                     precision: Optional[str] = None, sync: bool = True):
    """Solve for k right-hand sides B (n x k float64) sharing A, SA and lambda.
    Returns (X (d x k), infos)."""
    if precision is None:
        precision = "mixed" if SA.dtype == torch.float32 else "plain"
    p = PRECISIONS[precision]
    A = _row_aligned(A)
    SA = _row_aligned(SA)
    n, d = A.shape
    m = SA.shape[0]
    dev = A.device
    Bm = B.reshape(n, -1).to(torch.float64).contiguous()
    k = Bm.shape[1]
    X = (torch.zeros((d, k), dtype=torch.float64, device=dev) if X0 is None
         else X0.reshape(d, k).to(torch.float64).clone().contiguous())
    info = torch.zeros(INFO_BYTES * k, dtype=torch.uint8, device=dev)
    lib = load_library()
    h = handle(dev.index)
    ws_n = _sz()
    _check(lib.mihs_solve_multi_workspace_size(h, n, d, m, k, p, ctypes.byref(ws_n)),
           "mihs_solve_multi_workspace_size")
    ws = _workspace(ws_n.value, dev)
    rc = lib.mihs_solve_multi(h, A.data_ptr(), _dtype_code(A), n, d, A.stride(0), Bm.data_ptr(), k,
                              Bm.stride(0), float(lam), SA.data_ptr(), m, SA.stride(0), p,
                              float(alpha), float(beta), float(eps_sub), float(tol),
                              int(max_outer), int(max_inner), X.data_ptr(), info.data_ptr(),
                              ws.data_ptr(), ws.numel(), _stream(dev))
    _check(rc, "mihs_solve_multi")
    if not sync:
        return X, info
    torch.cuda.synchronize(dev)
    return X, info_to_dict(info)


class MIHSRidge(torch.autograd.Function):
    """x*(B, lambda) = (A^T A + lambda I)^{-1} A^T B as a differentiable op of B and
    log(lambda); the backward is an adjoint M-IHS solve on the same sketch.
    A and SA are constants (dL/dA is not computed).

        X = MIHSRidge.apply(B, log_lam, A, SA, alpha, beta, solver_kwargs)
    """

    @staticmethod
    def forward(ctx, B, log_lam, A, SA, alpha, beta, kw):
        kw = dict(kw or {})
        lam = lambda_from_log(float(log_lam.detach()))
        X, infos = mihs_solve_multi(A, B.detach(), lam, SA, alpha, beta, **kw)
        ctx.save_for_backward(X)
        ctx.A, ctx.SA, ctx.lam, ctx.alpha, ctx.beta, ctx.kw = A, SA, lam, alpha, beta, kw
        ctx.infos = infos
        return X

    @staticmethod
    def backward(ctx, gX):
        (X,) = ctx.saved_tensors
        kw = {k: v for k, v in ctx.kw.items() if k in ("eps_sub", "tol", "max_outer", "max_inner",
                                                      "precision")}
        _, dB, _, dloglam, _ = mihs_solve_backward(ctx.A, ctx.SA, ctx.lam, X, gX.contiguous(),
                                                   ctx.alpha, ctx.beta, want_dB=True,
                                                   want_dloglam=True, **kw)
        return dB, dloglam, None, None, None, None, None
