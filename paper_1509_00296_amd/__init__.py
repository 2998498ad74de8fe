"""Python binding of the gfx950 FRSVT library (libfrsvt.so, C ABI in
include/frsvt.h).

Argument marshalling only: every step of every call runs in the library's
HIP kernels.  PyTorch supplies device memory and the current HIP stream.
The binding refuses to run without the built library or without a gfx950
device; there is no CPU fallback.

Names follow the C ABI: ``svt``, ``frsvt``, ``wsvt``, ``wsvt_batched``,
``rpca_ialm``.  Matrices are torch tensors on the GPU (float64 or float32);
a row-major tensor is handed to the library as the column-major view of its
transpose, which the operators commute with (SVT(A^T) = SVT(A)^T, and the
orientation rule of FRSVT makes the same holds for a fixed Omega).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfrsvt.so")

F64, F32, MIXED_BF16 = 0, 1, 2
OK, NOT_CONVERGED, MAX_ITER = 0, 1, 2
ERR_HIP, ERR_OOM, ERR_NONFINITE, ERR_UNSUPPORTED = -100, -101, -102, -104

_i32, _i64, _u64, _dbl, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p


class FRSVTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class RpcaOpts(ctypes.Structure):
    _fields_ = [("tol", _dbl), ("max_iter", _i32), ("mu0", _dbl), ("rho", _dbl),
                ("mu_bar_factor", _dbl), ("use_frsvt", _i32), ("p", _i32), ("q", _i32),
                ("l0", _i32), ("seed", _u64)]


class RpcaStats(ctypes.Structure):
    _fields_ = [("iters", _i32), ("converged", _i32), ("residual", _dbl), ("norm2", _dbl),
                ("seconds", _dbl), ("ranks", _i32 * 64), ("residuals", _dbl * 64)]


class WsvtRule(ctypes.Structure):
    _fields_ = [("c", _dbl), ("noise_var", _dbl), ("eps", _dbl), ("tau", _dbl)]


_lib = None


def library(path: str | None = None) -> ctypes.CDLL:
    """Load libfrsvt.so (built in-tree by build.py); raises if it is missing."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"libfrsvt.so not built at {p}: run paper_1509_00296_amd/build.py")
    lib = ctypes.CDLL(p)
    lib.frsvt_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, _vp]
    lib.frsvt_destroy.argtypes = [_vp]
    lib.frsvt_set_stream.argtypes = [_vp, _vp]
    lib.frsvt_status_string.argtypes = [ctypes.c_int]
    lib.frsvt_status_string.restype = ctypes.c_char_p
    lib.frsvt_last_error.argtypes = [_vp]
    lib.frsvt_last_error.restype = ctypes.c_char_p
    lib.frsvt_workspace_bytes.argtypes = [_vp]
    lib.frsvt_workspace_bytes.restype = _i64
    lib.svt.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _i64, _dbl, _vp, _i64,
                        ctypes.POINTER(_i32)]
    lib.frsvt.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _i64, _dbl, _i32, _i32, _i32, _vp,
                          _i32, _i64, _u64, _u64, _vp, _i64, _vp, _i64, ctypes.POINTER(_i32)]
    lib.wsvt.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _i64, _vp, _vp, _i64,
                         ctypes.POINTER(_i32)]
    lib.wsvt_batched.argtypes = [_vp, _i64, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(WsvtRule), _vp]
    lib.frsvt_rpca_default_opts.argtypes = [ctypes.POINTER(RpcaOpts)]
    lib.frsvt_rpca_default_opts.restype = None
    lib.rpca_ialm.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _i64, _dbl,
                              ctypes.POINTER(RpcaOpts), _vp, _i64, _vp, _i64,
                              ctypes.POINTER(RpcaStats)]
    if path is None:
        _lib = lib
    return lib


def status_string(code: int) -> str:
    return library().frsvt_status_string(code).decode()


class Handle:
    """A library handle bound to one device; rebound to torch's current
    stream before every call."""

    def __init__(self, device: int = 0):
        import torch
        self.lib = library()
        self.device = device
        self.ptr = _vp()
        stream = torch.cuda.current_stream(device).cuda_stream
        rc = self.lib.frsvt_create(ctypes.byref(self.ptr), device, stream)
        if rc != 0:
            raise FRSVTError(rc, "frsvt_create: " + status_string(rc))

    def bind_current_stream(self):
        import torch
        self.lib.frsvt_set_stream(self.ptr, torch.cuda.current_stream(self.device).cuda_stream)

    def workspace_bytes(self) -> int:
        return int(self.lib.frsvt_workspace_bytes(self.ptr))

    def close(self):
        if self.ptr:
            self.lib.frsvt_destroy(self.ptr)
            self.ptr = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_handles: dict = {}


def handle(device: int | None = None) -> Handle:
    import torch
    if device is None:
        device = torch.cuda.current_device()
    if device not in _handles:
        _handles[device] = Handle(device)
    h = _handles[device]
    h.bind_current_stream()
    return h


def _check(h: Handle, rc: int, name: str, ok=(OK,)):
    if rc in ok:
        return rc
    detail = h.lib.frsvt_last_error(h.ptr).decode() if rc <= -100 else ""
    raise FRSVTError(rc, f"{name}: {status_string(rc)} {detail}".strip())


def _prec(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _colmajor(t):
    """(m, n, ld, transposed) of a 2-D tensor seen as a column-major matrix.
    A row-major tensor is described as its transpose."""
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    m, n = t.shape
    s0, s1 = t.stride()
    if s0 == 1 and (s1 >= max(m, 1) or n == 1):
        return m, n, max(s1, m, 1), False
    if s1 == 1 and (s0 >= max(n, 1) or m == 1):
        return n, m, max(s0, n, 1), True
    raise ValueError("tensor must have a unit stride in one dimension")


def _like(A, transposed):
    """An output with the same memory order as A."""
    import torch
    m, n = A.shape
    if transposed:
        return torch.empty((m, n), dtype=A.dtype, device=A.device)
    return torch.empty((n, m), dtype=A.dtype, device=A.device).t()


def svt(A, tau: float, *, return_rank: bool = False):
    """Exact SVT X = U S_tau(Sigma) V^T (Def. 1)."""
    h = handle(A.device.index)
    m, n, lda, tr = _colmajor(A)
    X = _like(A, tr)
    _, _, ldx, _ = _colmajor(X)
    r = _i32()
    rc = h.lib.svt(h.ptr, _prec(A), m, n, A.data_ptr(), lda, float(tau), X.data_ptr(), ldx,
                   ctypes.byref(r) if return_rank else None)
    _check(h, rc, "svt")
    return (X, int(r.value)) if return_rank else X


def wsvt(A, w, *, return_rank: bool = False):
    """Weighted SVT with thresholds w (descending-sigma order, float64 GPU tensor)."""
    import torch
    h = handle(A.device.index)
    m, n, lda, tr = _colmajor(A)
    w = w.to(device=A.device, dtype=torch.float64).contiguous()
    if w.numel() < min(m, n):
        raise ValueError("need min(m, n) weights")
    X = _like(A, tr)
    _, _, ldx, _ = _colmajor(X)
    r = _i32()
    rc = h.lib.wsvt(h.ptr, _prec(A), m, n, A.data_ptr(), lda, w.data_ptr(), X.data_ptr(), ldx,
                    ctypes.byref(r) if return_rank else None)
    _check(h, rc, "wsvt")
    return (X, int(r.value)) if return_rank else X


def wsvt_batched(rows, cols, offsets, A_packed, *, c: float = 2.8, noise_var: float = 0.01,
                 eps: float = 1e-8, tau: float = 0.0, X_packed=None, ranks=None):
    """Weighted SVT of a ragged batch in one persistent launch.  rows, cols
    (int32), offsets (int64) and A_packed (float32) are GPU tensors; each
    matrix is column-major at its offset.  Weights follow the patch-group
    rule w_i = c sqrt(cols) / (sqrt(max(s_i^2 - cols noise_var, 0)) + eps)
    (c <= 0: constant threshold tau).  Returns (X_packed, ranks)."""
    import torch
    h = handle(A_packed.device.index)
    count = rows.numel()
    for t, dt in ((rows, torch.int32), (cols, torch.int32), (offsets, torch.int64),
                  (A_packed, torch.float32)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise TypeError("rows/cols int32, offsets int64, A_packed float32, contiguous GPU tensors")
    if X_packed is None:
        X_packed = torch.empty_like(A_packed)
    if ranks is None:
        ranks = torch.empty(count, dtype=torch.int32, device=A_packed.device)
    rule = WsvtRule(c, noise_var, eps, tau)
    rc = h.lib.wsvt_batched(h.ptr, count, rows.data_ptr(), cols.data_ptr(), offsets.data_ptr(),
                            A_packed.data_ptr(), X_packed.data_ptr(), ctypes.byref(rule),
                            ranks.data_ptr())
    _check(h, rc, "wsvt_batched")
    return X_packed, ranks


def wsvt_tuning() -> list:
    """Lanes per Jacobi pair chosen by the batched-WSVT autotuner per size bucket."""
    h = handle()
    g = (_i32 * 3)()
    h.lib.frsvt_wsvt_tuning(h.ptr, g)
    return list(g)


def frsvt(A, tau: float, k: int, p: int, q: int, Q_prev=None, *, seed: int = 0,
          counter: int = 0, return_basis: bool = True):
    """FRSVT (Alg. 1).  Returns (X, Q~ (mhat x r), r); with Q_prev (mhat x r_prev,
    orthonormal columns) the basis is propagated and only p samples are drawn."""
    import torch
    h = handle(A.device.index)
    m, n, lda, tr = _colmajor(A)
    mh = min(m, n)
    X = _like(A, tr)
    _, _, ldx, _ = _colmajor(X)
    if Q_prev is not None:
        Qp = Q_prev.to(dtype=A.dtype)
        if Qp.shape[0] != mh:
            raise ValueError("Q_prev must have min(m, n) rows")
        Qp = Qp.t().contiguous().t() if Qp.stride(0) != 1 else Qp
        rp = Qp.shape[1]
        qptr, ldq = Qp.data_ptr(), max(Qp.stride(1), mh)
        lcap = min(rp + p, mh)
    else:
        qptr, rp, ldq = None, 0, mh
        lcap = min(max(k + p, 1), mh)
    Qout = torch.empty((max(lcap, 1), mh), dtype=A.dtype, device=A.device).t()
    r = _i32()
    rc = h.lib.frsvt(h.ptr, _prec(A), m, n, A.data_ptr(), lda, float(tau), int(k), int(p), int(q),
                     qptr, int(rp), int(ldq), int(seed) & (2**64 - 1), int(counter) & (2**64 - 1),
                     X.data_ptr(), ldx, Qout.data_ptr() if return_basis else None, mh,
                     ctypes.byref(r))
    _check(h, rc, "frsvt")
    rr = int(r.value)
    return X, Qout[:, :rr], rr


@dataclass
class RpcaResult:
    L: object
    S: object
    iters: int
    converged: bool
    residual: float
    norm2: float
    seconds: float
    ranks: list = field(default_factory=list)
    residuals: list = field(default_factory=list)


def rpca_ialm(O, lam: float, *, use_frsvt: bool = True, tol: float = 1e-7, max_iter: int = 60,
              mu0: float = 0.0, rho: float = 1.5, mu_bar_factor: float = 1e7, p: int = 5,
              q: int = 1, l0: int = 0, seed: int = 0) -> RpcaResult:
    """Inexact-ALM RPCA (the host of Sec. 4.1) with FRSVT + range propagation
    or exact SVT.  O is a GPU tensor (m x n)."""
    h = handle(O.device.index)
    m, n, ldo, tr = _colmajor(O)
    L = _like(O, tr)
    S = _like(O, tr)
    _, _, ldl, _ = _colmajor(L)
    _, _, lds, _ = _colmajor(S)
    op = RpcaOpts()
    h.lib.frsvt_rpca_default_opts(ctypes.byref(op))
    op.tol, op.max_iter, op.mu0, op.rho, op.mu_bar_factor = tol, max_iter, mu0, rho, mu_bar_factor
    op.use_frsvt, op.p, op.q, op.l0, op.seed = int(use_frsvt), p, q, l0, seed
    st = RpcaStats()
    rc = h.lib.rpca_ialm(h.ptr, _prec(O), m, n, O.data_ptr(), ldo, float(lam), ctypes.byref(op),
                         L.data_ptr(), ldl, S.data_ptr(), lds, ctypes.byref(st))
    _check(h, rc, "rpca_ialm", ok=(OK, MAX_ITER))
    k = min(st.iters, 64)
    return RpcaResult(L, S, st.iters, bool(st.converged), st.residual, st.norm2, st.seconds,
                      list(st.ranks[:k]), list(st.residuals[:k]))
