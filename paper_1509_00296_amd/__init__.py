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
ERR_SCRATCH = -106
NOALLOC_SCRATCH_BYTES = 64 << 20

_i32, _i64, _u64, _dbl, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p


class FRSVTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class RpcaOpts(ctypes.Structure):
    _fields_ = [("tol", _dbl), ("max_iter", _i32), ("mu0", _dbl), ("rho", _dbl),
                ("mu_bar_factor", _dbl), ("use_frsvt", _i32), ("p", _i32), ("q", _i32),
                ("l0", _i32), ("seed", _u64), ("ap", _i32), ("ap_a", _i32), ("ap_rho", _dbl),
                ("ap_gamma", _dbl), ("keep", _i32), ("q_init", ctypes.c_void_p), ("r_init", _i32),
                ("q_final", ctypes.c_void_p), ("resid_check", _i32)]


class LrrOpts(ctypes.Structure):
    _fields_ = [("tol", _dbl), ("max_iter", _i32), ("mu0", _dbl), ("rho", _dbl), ("mu_max", _dbl),
                ("use_frsvt", _i32), ("p", _i32), ("q", _i32), ("seed", _u64)]


class LrrStats(ctypes.Structure):
    _fields_ = [("iters", _i32), ("converged", _i32), ("rank", _i32), ("primal", _dbl), ("dual", _dbl),
                ("seconds", _dbl)]


class TensorOpts(ctypes.Structure):
    _fields_ = [("tol", _dbl), ("max_iter", _i32), ("mu0", _dbl), ("rho", _dbl), ("mu_max", _dbl),
                ("use_frsvt", _i32), ("p", _i32), ("q", _i32), ("seed", _u64)]


class TensorStats(ctypes.Structure):
    _fields_ = [("iters", _i32), ("converged", _i32), ("rank", _i32 * 3), ("resid", _dbl), ("mu0", _dbl),
                ("seconds", _dbl)]


class RpcaStats(ctypes.Structure):
    _fields_ = [("iters", _i32), ("converged", _i32), ("residual", _dbl), ("norm2", _dbl),
                ("seconds", _dbl), ("ranks", _i32 * 64), ("residuals", _dbl * 64),
                ("widths", _i32 * 64), ("resid_est", _dbl * 64)]


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
    lib.frsvt_noalloc.argtypes = lib.frsvt.argtypes
    lib.frsvt_set_option.argtypes = [_vp, ctypes.c_int, ctypes.c_int]
    lib.rpca_unrolled_saved_bytes.argtypes = [ctypes.c_int, _i32, _i32, _i64, _i64, _i32, _i32]
    lib.rpca_unrolled_saved_bytes.restype = _i64
    lib.rpca_unrolled_schedule.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _i64, _dbl, _dbl, _dbl, _i32,
                                           ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)]
    lib.rpca_unrolled_fwd.argtypes = [_vp, ctypes.c_int, _i32, _i32, _i64, _i64, _vp, _i64, _i64, _vp, _vp,
                                      _dbl, _dbl, _dbl, _i32, _i32, _i32, _u64, _vp, _i64, _i64, _vp, _i64]
    lib.rpca_unrolled_bwd.argtypes = [_vp, ctypes.c_int, _i32, _i32, _i64, _i64, _vp, _i64, _i64, _vp, _vp,
                                      _i32, _i32, _i32, _u64, _vp, _i64, _vp, _i64, _i64, _vp, _vp]
    lib.rpca_sliding.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _i64, _i32, _dbl, _i32, _i32, _i32,
                                 _u64, _dbl, _i32, _dbl, _vp, _i64, _vp, _i64, _vp, _vp]
    lib.wsvt.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _i64, _vp, _vp, _i64,
                         ctypes.POINTER(_i32)]
    lib.wsvt_batched.argtypes = [_vp, _i64, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(WsvtRule), _vp]
    lib.frsvt_rpca_default_opts.argtypes = [ctypes.POINTER(RpcaOpts)]
    lib.frsvt_rpca_default_opts.restype = None
    lib.rpca_ialm.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _i64, _dbl,
                              ctypes.POINTER(RpcaOpts), _vp, _i64, _vp, _i64,
                              ctypes.POINTER(RpcaStats)]
    lib.frsvt_lrr_default_opts.argtypes = [ctypes.POINTER(LrrOpts)]
    lib.frsvt_lrr_default_opts.restype = None
    lib.lrr_ialm.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _i64, _dbl, ctypes.POINTER(LrrOpts), _vp, _i64,
                             _vp, _i64, ctypes.POINTER(LrrStats)]
    lib.frsvt_tensor_default_opts.argtypes = [ctypes.POINTER(TensorOpts)]
    lib.frsvt_tensor_default_opts.restype = None
    lib.tensor_rpca.argtypes = [_vp, ctypes.c_int, _i64, _i64, _i64, _vp, ctypes.POINTER(_dbl), _dbl,
                                ctypes.POINTER(TensorOpts), _vp, _vp, ctypes.POINTER(TensorStats)]
    lib.frsvt_fwd.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _i64, _dbl, _i32, _i32, _i32, _u64,
                              _u64, _vp, _i64, _vp, _i64, _vp]
    lib.frsvt_vjp.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _i64, _dbl, _i32, _i32, _i32, _u64,
                              _u64, _vp, _i64, _vp, _vp, _i64, _vp, _i64, _vp]
    lib.rpca_dual_step.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64,
                                   _dbl, _dbl, _dbl, _vp, _i64, _vp, _i64, _vp, _i64]
    lib.rpca_dual_step_vjp.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _i64, _vp, _i64, _vp,
                                       _i64, _dbl, _dbl, _dbl, _vp, _i64, _vp, _i64, _vp, _i64, _vp,
                                       _i64, _vp, _i64, _vp]
    lib.rpca_init.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _i64, _dbl, _dbl, _vp, _i64, _vp,
                              _i64, ctypes.POINTER(_dbl)]
    lib.frsvt_wsvt_tuning.argtypes = [_vp, _vp]
    lib.frsvt_wsvt_work.argtypes = [_vp, _vp]
    lib.frsvt_last_info.argtypes = [_vp, ctypes.POINTER(_i32), ctypes.c_int]
    lib.frsvt_trace_enable.argtypes = [_vp, ctypes.c_int]
    lib.frsvt_trace_read.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(_dbl), ctypes.POINTER(_i64)]
    lib.frsvt_trace_name.argtypes = [ctypes.c_int]
    lib.frsvt_trace_name.restype = ctypes.c_char_p
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
    """The handle of (device, torch's current stream): work issued on
    different streams uses different handles, so their workspaces never
    overlap."""
    import torch
    if device is None:
        device = torch.cuda.current_device()
    key = (device, torch.cuda.current_stream(device).cuda_stream)
    if key not in _handles:
        _handles[key] = Handle(device)
    h = _handles[key]
    h.bind_current_stream()
    return h


def handles(device: int = 0) -> list:
    """Every handle created on a device (one per stream used)."""
    return [h for (d, _), h in _handles.items() if d == device]


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


def wsvt_work() -> list:
    """Jacobi work of the last batched WSVT call: [sum of the column length
    over examined pairs, the same over applied rotations, rotations]."""
    h = handle()
    w = (ctypes.c_int64 * 3)()
    _check(h, h.lib.frsvt_wsvt_work(h.ptr, w), "frsvt_wsvt_work")
    return list(w)


def frsvt(A, tau: float, k: int, p: int, q: int, Q_prev=None, *, seed: int = 0,
          counter: int = 0, return_basis: bool = True, out=None, noalloc: bool = False,
          want_rank: bool = True):
    """FRSVT (Alg. 1).  Returns (X, Q~ (mhat x r), r); with Q_prev (mhat x r_prev,
    orthonormal columns) the basis is propagated and only p samples are drawn.
    out = (X, Qout) supplies the output buffers (X like A, Qout column-major
    mhat x l); noalloc calls frsvt_noalloc, whose workspace is the library's
    fixed device scratch.  want_rank=False leaves the rank on the device
    (no host wait: the call can be captured in a graph); r is then -1 and
    the basis is returned at its full width l."""
    import torch
    h = handle(A.device.index)
    m, n, lda, tr = _colmajor(A)
    mh = min(m, n)
    X = _like(A, tr) if out is None else out[0]
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
    if out is None:
        Qout = torch.empty((max(lcap, 1), mh), dtype=A.dtype, device=A.device).t()
    else:
        Qout = out[1]
        if Qout.shape[0] != mh or Qout.shape[1] < lcap or Qout.stride(0) != 1 or Qout.stride(1) != mh:
            raise ValueError("out[1] must be column-major mhat x l with leading dimension mhat")
        if X.shape != A.shape or X.dtype != A.dtype or _colmajor(X)[3] != tr:
            raise ValueError("out[0] must have the shape, dtype and memory order of A")
    r = _i32()
    fn = h.lib.frsvt_noalloc if noalloc else h.lib.frsvt
    rc = fn(h.ptr, _prec(A), m, n, A.data_ptr(), lda, float(tau), int(k), int(p), int(q),
            qptr, int(rp), int(ldq), int(seed) & (2**64 - 1), int(counter) & (2**64 - 1),
            X.data_ptr(), ldx, Qout.data_ptr() if return_basis else None, mh,
            ctypes.byref(r) if want_rank else None)
    _check(h, rc, "frsvt_noalloc" if noalloc else "frsvt")
    if not want_rank:
        return X, Qout, -1
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
    widths: list = field(default_factory=list)
    resid_est: list = field(default_factory=list)
    Q: object = None


def rpca_ialm(O, lam: float, *, use_frsvt: bool = True, tol: float = 1e-7, max_iter: int = 60,
              mu0: float = 0.0, rho: float = 1.5, mu_bar_factor: float = 1e7, p: int = 5,
              q: int = 1, l0: int = 0, seed: int = 0, ap: bool = False, ap_a: int = 2,
              ap_rho: float = 0.05, ap_gamma: float = 1.0, keep: int = 0, q_init=None,
              return_basis: bool = False, resid_check: bool = False) -> RpcaResult:
    """Inexact-ALM RPCA (the host of Sec. 4.1) with FRSVT + range propagation
    or exact SVT.  O is a GPU tensor (m x n).  With ap the sketch widths follow
    adaptive rank prediction (Sec. 2.3, Eq. 7: a, rho, gamma) instead of p
    new samples per iteration.  keep > 0 selects partial SVT (the keep largest
    singular values unshrunk: the truncated nuclear norm).  q_init (GPU, mhat x
    r, orthonormal columns) is the first call's propagated basis and
    return_basis returns the last one in .Q (semi-online use).  resid_check
    stops each iteration's sampling at the first new sample whose residual
    estimate (Prop. 4) is at most the threshold."""
    import torch
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
    op.ap, op.ap_a, op.ap_rho, op.ap_gamma = int(ap), ap_a, ap_rho, ap_gamma
    op.keep = keep
    op.resid_check = int(resid_check)
    mh = min(m, n)
    qi = None
    if q_init is not None:
        if q_init.dim() != 2 or q_init.shape[0] != mh or q_init.dtype != O.dtype or \
                q_init.device != O.device:
            raise ValueError("q_init must be a GPU tensor of shape (min(m, n), r) with the dtype of O")
        qi = q_init.t().contiguous().t()          # column-major, leading dimension mhat
        op.q_init, op.r_init = qi.data_ptr(), qi.shape[1]
    qf = None
    if return_basis and use_frsvt:
        qf = torch.empty((mh, mh), dtype=O.dtype, device=O.device).t()   # column-major
        op.q_final = qf.data_ptr()
    st = RpcaStats()
    rc = h.lib.rpca_ialm(h.ptr, _prec(O), m, n, O.data_ptr(), ldo, float(lam), ctypes.byref(op),
                         L.data_ptr(), ldl, S.data_ptr(), lds, ctypes.byref(st))
    _check(h, rc, "rpca_ialm", ok=(OK, MAX_ITER))
    k = min(st.iters, 64)
    Qf = qf[:, :st.ranks[k - 1]] if (qf is not None and k > 0) else None
    return RpcaResult(L, S, st.iters, bool(st.converged), st.residual, st.norm2, st.seconds,
                      list(st.ranks[:k]), list(st.residuals[:k]),
                      list(st.widths[:k]) if use_frsvt else [],
                      list(st.resid_est[:k]) if use_frsvt else [], Qf)


def rpca_sliding(frames, n: int, lam=None, *, keep: int = 1, l: int = 3, q: int = 2,
                 seed: int = 0, tol: float = 1e-7, max_iter: int = 60, rho: float = 1.5):
    """Semi-online low-rank + sparse decomposition of a frame sequence (Sec. 4,
    Type B of Table 6) through rpca_sliding: consecutive windows of n frames
    (the columns of frames, m x F on the GPU), each by the partial-SVT iALM
    (the keep largest singular values unshrunk) with FRSVT, the sketch width
    bounded by l and q power iterations; each window starts from the previous
    window's propagated basis.  lam defaults to 1/sqrt(max(m, n)).  Frames
    past the last whole window are left out (zero in L and S).  Returns L, S
    and the per-window results."""
    import torch
    h = handle(frames.device.index)
    F = frames if (frames.stride(0) == 1) else frames.t().contiguous().t()
    m, nf, ldf, tr = _colmajor(F)
    if tr:
        raise ValueError("frames must be a column-major (or contiguous-column) m x F tensor")
    lam = 1.0 / float(max(m, n)) ** 0.5 if lam is None else lam
    L = torch.zeros((nf, m), dtype=F.dtype, device=F.device).t()
    S = torch.zeros((nf, m), dtype=F.dtype, device=F.device).t()
    nw = nf // n if n >= 1 else 0
    mh = min(m, n)
    st = (RpcaStats * max(nw, 1))()
    bases = torch.zeros((max(nw, 1), l, mh), dtype=F.dtype, device=F.device)
    rc = h.lib.rpca_sliding(h.ptr, _prec(F), m, nf, F.data_ptr(), ldf, int(n), float(lam), int(keep), int(l),
                            int(q), int(seed) & (2**64 - 1), float(tol), int(max_iter), float(rho), L.data_ptr(),
                            m, S.data_ptr(), m, st, bases.data_ptr())
    _check(h, rc, "rpca_sliding")
    runs = []
    for w in range(nw):
        k = min(st[w].iters, 64)
        r = st[w].ranks[k - 1] if k > 0 else 0
        Qw = bases[w].t()[:, :r]                       # column-major mhat x r
        runs.append(RpcaResult(L[:, w * n:(w + 1) * n], S[:, w * n:(w + 1) * n], st[w].iters,
                               bool(st[w].converged), st[w].residual, st[w].norm2, st[w].seconds,
                               list(st[w].ranks[:k]), list(st[w].residuals[:k]), list(st[w].widths[:k]),
                               list(st[w].resid_est[:k]), Qw))
    return L, S, runs


# ---------------------------------------------------------------------------
# Adjoint: the fresh-sketch FRSVT with saved state, its vector-Jacobian
# product, and the unrolled inexact-ALM pieces.
# ---------------------------------------------------------------------------
def _in_order(t, transposed: bool):
    """t with the memory order of a tensor whose _colmajor flag is `transposed`."""
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    try:
        if _colmajor(t)[3] == transposed:
            return t
    except ValueError:
        pass
    return t.contiguous() if transposed else t.t().contiguous().t()


def _ptr(t):
    return None if t is None else t.data_ptr()


def frsvt_fwd(A, tau: float, k: int, p: int, q: int, *, seed: int = 0, counter: int = 0):
    """Fresh-sketch FRSVT that keeps the adjoint's state.  Returns (X, Q, factors):
    Q is the mhat x l basis of B = Q^T Ahat, factors = [sigma (l), U_B (l*l)] in
    float64 on the device."""
    import torch
    h = handle(A.device.index)
    m, n, lda, tr = _colmajor(A)
    mh = min(m, n)
    l = min(k + p, mh)
    X = _like(A, tr)
    _, _, ldx, _ = _colmajor(X)
    Q = torch.empty((l, mh), dtype=A.dtype, device=A.device).t()
    fac = torch.empty(l + l * l, dtype=torch.float64, device=A.device)
    rc = h.lib.frsvt_fwd(h.ptr, _prec(A), m, n, A.data_ptr(), lda, float(tau), int(k), int(p), int(q),
                         int(seed) & (2**64 - 1), int(counter) & (2**64 - 1), X.data_ptr(), ldx,
                         Q.data_ptr(), mh, fac.data_ptr())
    _check(h, rc, "frsvt_fwd")
    return X, Q, fac


def frsvt_vjp(A, tau: float, k: int, p: int, q: int, Q, factors, X_bar, *, seed: int = 0,
              counter: int = 0):
    """(A_bar, tau_bar) of the frsvt_fwd call with the same arguments, for the
    upstream gradient X_bar; tau_bar is a 0-dim float64 device tensor."""
    import torch
    h = handle(A.device.index)
    m, n, lda, tr = _colmajor(A)
    Xb = _in_order(X_bar.to(dtype=A.dtype), tr)
    _, _, ldxb, _ = _colmajor(Xb)
    Ab = _like(A, tr)
    _, _, ldab, _ = _colmajor(Ab)
    tb = torch.empty((), dtype=torch.float64, device=A.device)
    mh = min(m, n)
    Qc = Q if Q.stride(0) == 1 else Q.t().contiguous().t()
    rc = h.lib.frsvt_vjp(h.ptr, _prec(A), m, n, A.data_ptr(), lda, float(tau), int(k), int(p), int(q),
                         int(seed) & (2**64 - 1), int(counter) & (2**64 - 1), Qc.data_ptr(),
                         max(Qc.stride(1), mh), factors.data_ptr(), Xb.data_ptr(), ldxb,
                         Ab.data_ptr(), ldab, tb.data_ptr())
    _check(h, rc, "frsvt_vjp")
    return Ab, tb


OPT_QRCP_TRUNCATE = 1


def set_option(option: int, value: int, device: int | None = None) -> None:
    """Handle option (frsvt_set_option), e.g. OPT_QRCP_TRUNCATE."""
    h = handle(device)
    _check(h, h.lib.frsvt_set_option(h.ptr, int(option), int(value)), "frsvt_set_option")


def last_info(count: int = 8) -> list:
    """Status words of the last thresholding step (frsvt_last_info)."""
    h = handle()
    info = (_i32 * 8)()
    h.lib.frsvt_last_info(h.ptr, info, count)
    return list(info[:count])


def rpca_init(O, lam: float, mu0: float = 0.0):
    """Starting point of the inexact-ALM loop: (Y0, A0, norm2, mu0, J)."""
    h = handle(O.device.index)
    m, n, ldo, tr = _colmajor(O)
    Y0, A0 = _like(O, tr), _like(O, tr)
    out = (_dbl * 3)()
    rc = h.lib.rpca_init(h.ptr, _prec(O), m, n, O.data_ptr(), ldo, float(lam), float(mu0),
                         Y0.data_ptr(), _colmajor(Y0)[2], A0.data_ptr(), _colmajor(A0)[2], out)
    _check(h, rc, "rpca_init")
    return Y0, A0, out[0], out[1], out[2]


def dual_step(O, L, Y, lam: float, mu: float, mu_next: float, *, want_S: bool = False,
              want_Y: bool = True, want_A: bool = True):
    """(S, Y_next, A_next) of one unrolled iALM step (None where not wanted)."""
    h = handle(O.device.index)
    m, n, ldo, tr = _colmajor(O)
    L, Y = _in_order(L, tr), _in_order(Y, tr)
    outs = [_like(O, tr) if w else None for w in (want_S, want_Y, want_A)]
    lds = [_colmajor(t)[2] if t is not None else m for t in outs]
    rc = h.lib.rpca_dual_step(h.ptr, _prec(O), m, n, O.data_ptr(), ldo, L.data_ptr(),
                              _colmajor(L)[2], Y.data_ptr(), _colmajor(Y)[2], float(lam), float(mu),
                              float(mu_next), _ptr(outs[0]), lds[0], _ptr(outs[1]), lds[1],
                              _ptr(outs[2]), lds[2])
    _check(h, rc, "rpca_dual_step")
    return tuple(outs)


def dual_step_vjp(O, L, Y, lam: float, mu: float, mu_next: float, S_bar=None, Y_next_bar=None,
                  A_next_bar=None, *, lam_bar=None):
    """(L_bar, Y_bar, lam_bar) of dual_step; lam_bar is a 0-dim float64 device
    tensor (or the given one, overwritten)."""
    import torch
    h = handle(O.device.index)
    m, n, ldo, tr = _colmajor(O)
    L, Y = _in_order(L, tr), _in_order(Y, tr)
    ups = [None if t is None else _in_order(t.to(dtype=O.dtype), tr) for t in (S_bar, Y_next_bar, A_next_bar)]
    lds = [_colmajor(t)[2] if t is not None else m for t in ups]
    Lb, Yb = _like(O, tr), _like(O, tr)
    if lam_bar is None:
        lam_bar = torch.empty((), dtype=torch.float64, device=O.device)
    rc = h.lib.rpca_dual_step_vjp(h.ptr, _prec(O), m, n, O.data_ptr(), ldo, L.data_ptr(),
                                  _colmajor(L)[2], Y.data_ptr(), _colmajor(Y)[2], float(lam),
                                  float(mu), float(mu_next), _ptr(ups[0]), lds[0], _ptr(ups[1]),
                                  lds[1], _ptr(ups[2]), lds[2], Lb.data_ptr(), _colmajor(Lb)[2],
                                  Yb.data_ptr(), _colmajor(Yb)[2], lam_bar.data_ptr())
    _check(h, rc, "rpca_dual_step_vjp")
    return Lb, Yb, lam_bar


def _torch():
    import torch
    return torch


class _FRSVTFn(_torch().autograd.Function):
    """X = FRSVT_tau(A) for a fixed sketch (seed, counter), differentiable in
    A and tau through frsvt_vjp."""

    @staticmethod
    def forward(ctx, A, tau, k, p, q, seed, counter):
        torch = _torch()
        tv = float(tau)
        X, Q, fac = frsvt_fwd(A, tv, k, p, q, seed=seed, counter=counter)
        ctx.save_for_backward(A, Q, fac)
        ctx.cfg = (tv, k, p, q, seed, counter)
        ctx.tau_meta = (tau.device, tau.dtype) if torch.is_tensor(tau) else None
        return X

    @staticmethod
    def backward(ctx, X_bar):
        A, Q, fac = ctx.saved_tensors
        tv, k, p, q, seed, counter = ctx.cfg
        Ab, tb = frsvt_vjp(A, tv, k, p, q, Q, fac, X_bar, seed=seed, counter=counter)
        gtau = None
        if ctx.tau_meta is not None and ctx.needs_input_grad[1]:
            gtau = tb.to(device=ctx.tau_meta[0], dtype=ctx.tau_meta[1])
        return (Ab if ctx.needs_input_grad[0] else None), gtau, None, None, None, None, None


def frsvt_ad(A, tau, k: int, p: int, q: int, *, seed: int = 0, counter: int = 0):
    """Differentiable FRSVT (fresh sketch): gradients flow to A and, when tau is a
    tensor, to tau."""
    return _FRSVTFn.apply(A, tau, k, p, q, seed, counter)


class _UnrolledFn(_torch().autograd.Function):
    """T unrolled inexact-ALM steps on a batch of instances with learnable
    per-step SVT thresholds taus[t] and shrink thresholds lams[t] shared by
    the batch (rpca_unrolled_fwd / rpca_unrolled_bwd: the steps, the mu
    schedule, the side streams and the batch sums all run in the library).
    Output L_T, shape (B, m, n)."""

    @staticmethod
    def forward(ctx, taus, lams, O, lam, rho, mu_bar_factor, k, p, q, seed):
        torch = _torch()
        h = handle(O.device.index)
        Oc = O.contiguous()
        B, m, n = Oc.shape
        # instance b is row-major m x n: the column-major n x m matrix at b*m*n
        td = taus.detach().to(device=O.device, dtype=torch.float64).contiguous()
        ld = lams.detach().to(device=O.device, dtype=torch.float64).contiguous()
        T = td.numel()
        nbytes = h.lib.rpca_unrolled_saved_bytes(_prec(Oc), B, T, n, m, k, p)
        if nbytes < 0:
            raise ValueError("invalid unrolled RPCA sizes")
        saved = torch.empty(nbytes, dtype=torch.uint8, device=O.device)
        L = torch.empty_like(Oc)
        rc = h.lib.rpca_unrolled_fwd(h.ptr, _prec(Oc), B, T, n, m, Oc.data_ptr(), n, m * n, td.data_ptr(),
                                     ld.data_ptr(), float(lam), float(rho), float(mu_bar_factor), int(k), int(p),
                                     int(q), int(seed) & (2**64 - 1), L.data_ptr(), n, m * n, saved.data_ptr(),
                                     nbytes)
        _check(h, rc, "rpca_unrolled_fwd")
        ctx.state = (Oc, td, ld, saved, nbytes, k, p, q, seed, taus.device)
        return L

    @staticmethod
    def backward(ctx, L_bar):
        torch = _torch()
        Oc, td, ld, saved, nbytes, k, p, q, seed, pdev = ctx.state
        h = handle(Oc.device.index)
        B, m, n = Oc.shape
        T = td.numel()
        Lb = L_bar.to(dtype=Oc.dtype).contiguous()
        gt = torch.empty(T, dtype=torch.float64, device=Oc.device)
        gl = torch.empty(T, dtype=torch.float64, device=Oc.device)
        rc = h.lib.rpca_unrolled_bwd(h.ptr, _prec(Oc), B, T, n, m, Oc.data_ptr(), n, m * n, td.data_ptr(),
                                     ld.data_ptr(), int(k), int(p), int(q), int(seed) & (2**64 - 1),
                                     saved.data_ptr(), nbytes, Lb.data_ptr(), n, m * n, gt.data_ptr(),
                                     gl.data_ptr())
        _check(h, rc, "rpca_unrolled_bwd")
        ctx.state = None
        return gt.to(pdev), gl.to(pdev), None, None, None, None, None, None, None, None


class UnrolledRPCA(_torch().nn.Module):
    """Differentiable unrolled inexact-ALM RPCA (FRSVT thresholding) with
    learnable per-step thresholds tau_t (SVT) and lam_t (shrink).  mu_t
    follows the iALM schedule of each instance: mu_0 = 1.25 / ||O||_2,
    mu_{t+1} = rho mu_t (capped at mu_bar_factor mu_0); instance b draws its
    sketches with seed + b."""

    def __init__(self, taus, lams, *, k: int = 5, p: int = 5, q: int = 1, rho: float = 1.5,
                 mu_bar_factor: float = 1e7, seed: int = 0, lam_ialm: float | None = None):
        torch = _torch()
        super().__init__()
        self.tau = torch.nn.Parameter(torch.as_tensor(taus, dtype=torch.float64).clone())
        self.lam = torch.nn.Parameter(torch.as_tensor(lams, dtype=torch.float64).clone())
        self.k, self.p, self.q, self.rho, self.mu_bar_factor = k, p, q, rho, mu_bar_factor
        self.seed = seed
        self.lam_ialm = lam_ialm

    @staticmethod
    def default_schedule(O, steps: int = 10, rho: float = 1.5, lam: float | None = None,
                         mu_bar_factor: float = 1e7):
        """tau_t = 1/mu_t and lam_t = lam/mu_t of the plain iALM on instance O
        (rpca_unrolled_schedule)."""
        h = handle(O.device.index)
        m, n, ldo, _ = _colmajor(O)
        lam = lam if lam is not None else 1.0 / max(m, n) ** 0.5
        tv, lv = (_dbl * steps)(), (_dbl * steps)()
        rc = h.lib.rpca_unrolled_schedule(h.ptr, _prec(O), m, n, O.data_ptr(), ldo, float(lam), float(rho),
                                          float(mu_bar_factor), int(steps), tv, lv)
        _check(h, rc, "rpca_unrolled_schedule")
        return list(tv), list(lv)

    def forward(self, O):
        """O: (B, m, n) GPU tensor.  Returns L_T, shape (B, m, n)."""
        B, m, n = O.shape
        lam = self.lam_ialm if self.lam_ialm is not None else 1.0 / max(m, n) ** 0.5
        return _UnrolledFn.apply(self.tau, self.lam, O, lam, self.rho, self.mu_bar_factor, self.k, self.p,
                                 self.q, self.seed)


@dataclass
class LrrResult:
    Z: object
    E: object
    iters: int
    converged: bool
    rank: int
    primal: float
    dual: float
    seconds: float


def lrr_ialm(X, lam: float, *, use_frsvt: bool = True, p: int = 5, q: int = 1, seed: int = 0,
             tol: float = 1e-8, max_iter: int = 1000, mu0: float = 1e-6, rho: float = 1.1,
             mu_max: float = 1e10) -> LrrResult:
    """Low-rank representation (Type A of Table 6), min ||Z||_* + lam ||E||_{2,1}
    s.t. X = X Z + E, by its inexact ALM with the J step by FRSVT + range
    propagation (or exact SVT).  X is a float64 GPU tensor (d x n samples)."""
    import torch
    h = handle(X.device.index)
    if X.dtype != torch.float64:
        raise TypeError("lrr_ialm takes float64 data")
    Xc = X.t().contiguous().t() if X.stride(0) != 1 else X
    d, n = Xc.shape
    ldx = max(Xc.stride(1), d, 1)
    Z = torch.empty((n, n), dtype=X.dtype, device=X.device).t()
    E = torch.empty((n, d), dtype=X.dtype, device=X.device).t()
    op = LrrOpts()
    h.lib.frsvt_lrr_default_opts(ctypes.byref(op))
    op.tol, op.max_iter, op.mu0, op.rho, op.mu_max = tol, max_iter, mu0, rho, mu_max
    op.use_frsvt, op.p, op.q, op.seed = int(use_frsvt), p, q, seed
    st = LrrStats()
    rc = h.lib.lrr_ialm(h.ptr, F64, d, n, Xc.data_ptr(), ldx, float(lam), ctypes.byref(op), Z.data_ptr(), n,
                        E.data_ptr(), d, ctypes.byref(st))
    _check(h, rc, "lrr_ialm", ok=(OK, MAX_ITER))
    return LrrResult(Z, E, st.iters, bool(st.converged), st.rank, st.primal, st.dual, st.seconds)


@dataclass
class TensorResult:
    L: object
    E: object
    iters: int
    converged: bool
    rank: tuple
    resid: float
    mu0: float
    seconds: float


def tensor_rpca(O, alpha, lam: float, *, use_frsvt: bool = True, p: int = 5, q: int = 1, seed: int = 0,
                tol: float = 1e-7, max_iter: int = 100, mu0: float = 0.0, rho: float = 1.5,
                mu_max: float = 1e10) -> TensorResult:
    """Low-rank + sparse decomposition of a 3-way tensor (Type C of Table 6,
    alignment fixed): min sum_i alpha_i ||L_(i)||_* + lam ||E||_1 s.t.
    O = L + E, each mode's SVT by FRSVT + range propagation (or exact SVT).
    O is a float64 GPU tensor of shape (I1, I2, I3); it is used in
    column-major order (first index fastest), copied once if it is not
    stored that way.  L and E come back with O's shape."""
    import torch
    h = handle(O.device.index)
    if O.dtype != torch.float64 or O.dim() != 3:
        raise TypeError("tensor_rpca takes a 3-way float64 tensor")
    I1, I2, I3 = O.shape
    Oc = O.permute(2, 1, 0).contiguous().permute(2, 1, 0)
    L = torch.empty((I3, I2, I1), dtype=O.dtype, device=O.device).permute(2, 1, 0)
    E = torch.empty((I3, I2, I1), dtype=O.dtype, device=O.device).permute(2, 1, 0)
    if len(alpha) != 3:
        raise ValueError("alpha holds one weight per mode")
    al = (_dbl * 3)(*[float(a) for a in alpha])
    op = TensorOpts()
    h.lib.frsvt_tensor_default_opts(ctypes.byref(op))
    op.tol, op.max_iter, op.mu0, op.rho, op.mu_max = tol, max_iter, mu0, rho, mu_max
    op.use_frsvt, op.p, op.q, op.seed = int(use_frsvt), p, q, seed
    st = TensorStats()
    rc = h.lib.tensor_rpca(h.ptr, F64, I1, I2, I3, Oc.data_ptr(), al, float(lam), ctypes.byref(op),
                           L.data_ptr(), E.data_ptr(), ctypes.byref(st))
    _check(h, rc, "tensor_rpca", ok=(OK, MAX_ITER))
    return TensorResult(L, E, st.iters, bool(st.converged), tuple(st.rank), st.resid, st.mu0, st.seconds)
