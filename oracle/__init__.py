"""Plain FP64 CPU oracle for fast randomized SVT (arXiv:1509.00296).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  It wraps
``frsvt_oracle.c`` (plain C, no BLAS) through ctypes and shares no code with
the GPU library; the two never import each other.

Every function takes and returns numpy float64 arrays; matrices cross the
ctypes boundary in column-major (Fortran) order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "frsvt_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, single thread)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp,
                               _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_OMP_LIB_PATH = os.path.join(_HERE, "liboracle_omp.so")


def build_openmp(force: bool = False) -> str:
    """The same source compiled with -fopenmp (for the all-core CPU
    baseline only): the parallel loops split independent output columns, so
    the results equal the plain build's bit for bit."""
    if force or not os.path.exists(_OMP_LIB_PATH) or \
            os.path.getmtime(_OMP_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _OMP_LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-o", tmp,
                               _SRC, "-lm"])
        os.replace(tmp, _OMP_LIB_PATH)
    return _OMP_LIB_PATH


def threads() -> int:
    """Threads of the active oracle build (1 for the plain build)."""
    return int(_L().orc_threads())


_libs: dict = {}
_active = [None]


def _bind(path: str):
    if path not in _libs:
        lib = ctypes.CDLL(path)
        lib.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        lib.orc_threads.argtypes = []
        lib.orc_threads.restype = ctypes.c_int
        lib.orc_uniform53.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        lib.orc_uniform53.restype = ctypes.c_double
        lib.orc_gaussian_matrix.argtypes = [ctypes.c_uint64, ctypes.c_uint64, _i64, _i64, _dp, _i64]
        lib.orc_qr.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64, _dp, _i64]
        lib.orc_qrcp_basis.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64]
        lib.orc_qrcp_basis.restype = _i64
        lib.orc_svd.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64, _dp, _dp, _i64]
        lib.orc_svt.argtypes = [_i64, _i64, _dp, _i64, ctypes.c_double, _dp, _i64, _i64p]
        lib.orc_wsvt.argtypes = [_i64, _i64, _dp, _i64, _dp, _dp, _i64, _i64p]
        lib.orc_frsvt.argtypes = [_i64, _i64, _dp, _i64, ctypes.c_double, ctypes.c_int,
                                  _dp, _i64, _i64, _dp, _i64, _i64, _dp, _i64, _dp, _i64,
                                  _i64p, _dp, _i64p]
        lib.orc_rpca_ialm.argtypes = [_i64, _i64, _dp, _i64, ctypes.c_double, ctypes.c_int,
                                      _i64, ctypes.c_int, ctypes.c_uint64, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, _dp, _i64, _dp, _i64, _i64p, _dp,
                                      ctypes.POINTER(ctypes.c_int)]
        lib.orc_rpca_ialm_ap.argtypes = [_i64, _i64, _dp, _i64, ctypes.c_double, ctypes.c_int,
                                         _i64, ctypes.c_int, ctypes.c_uint64, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, _i64, ctypes.c_double,
                                         ctypes.c_double, _i64, _dp, _i64, _dp, _i64p, _dp, _i64,
                                         _dp, _i64, _i64p, _i64p, _dp, _dp,
                                         ctypes.POINTER(ctypes.c_int)]
        lib.orc_rpca_ialm_rc.argtypes = [_i64, _i64, _dp, _i64, ctypes.c_double, ctypes.c_int,
                                         _i64, ctypes.c_int, ctypes.c_uint64, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, _i64, ctypes.c_double,
                                         ctypes.c_double, _i64, _dp, _i64, _dp, _i64p, ctypes.c_int,
                                         _dp, _i64, _dp, _i64, _i64p, _i64p, _dp, _dp,
                                         ctypes.POINTER(ctypes.c_int)]
        lib.orc_residual_check.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64, _i64, _dp, _i64, _i64,
                                           ctypes.c_double, ctypes.c_double, _dp]
        lib.orc_residual_check.restype = _i64
        lib.orc_lrr_ialm.argtypes = [_i64, _i64, _dp, _i64, ctypes.c_double, ctypes.c_int, _i64,
                                     ctypes.c_int, ctypes.c_uint64, ctypes.c_double, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp, _i64,
                                     _dp, _i64, _i64p, ctypes.POINTER(ctypes.c_int)]
        lib.orc_psvt.argtypes = [_i64, _i64, _dp, _i64, ctypes.c_double, _i64, _dp, _i64, _i64p]
        lib.orc_residual_estimate.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64, _i64, _dp,
                                              ctypes.c_double]
        lib.orc_residual_estimate.restype = ctypes.c_double
        lib.orc_svt_vjp.argtypes = [_i64, _i64, _dp, _i64, ctypes.c_double, _dp, _i64, _dp,
                                    _i64, _dp]
        lib.orc_wsvt_rule.argtypes = [_i64, _i64, _dp, _i64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, _dp, _i64, _i64p]
        _libs[path] = lib
    return _libs[path]


def _L():
    if _active[0] is None:
        override = os.environ.get("FRSVT_ORACLE_LIB")
        if override:
            _active[0] = override
        else:
            if not os.path.exists(_LIB_PATH):
                build()
            _active[0] = _LIB_PATH
    return _bind(_active[0])


class use_library:
    """Context manager: route every call in this module to another build of
    the oracle source (the mutation tests compile deliberately broken copies
    on the CPU and check that the pins reject them)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        self.prev = _active[0]
        _bind(self.path)
        _active[0] = self.path
        return self

    def __exit__(self, *exc):
        _active[0] = self.prev
        return False


def _f(a) -> np.ndarray:
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


class OracleError(RuntimeError):
    pass


def _check(rc: int, name: str):
    if rc < 0:
        raise OracleError(f"{name}: argument {-rc} invalid")


# ---------------------------------------------------------------- random numbers

def philox4x32_10(ctr, key) -> np.ndarray:
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    _L().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def uniform53(a: int, b: int) -> float:
    return float(_L().orc_uniform53(a, b))


def gaussian_matrix(seed: int, counter: int, rows: int, cols: int) -> np.ndarray:
    om = np.zeros((rows, cols), dtype=np.float64, order="F")
    _L().orc_gaussian_matrix(seed, counter, rows, cols, _p(om), max(rows, 1))
    return om


# ---------------------------------------------------------------- factorizations

def qr(A):
    A = _f(A)
    m, n = A.shape
    Q = np.zeros((m, n), order="F")
    R = np.zeros((n, n), order="F")
    _check(_L().orc_qr(m, n, _p(A), max(m, 1), _p(Q), max(m, 1), _p(R), max(n, 1)), "qr")
    return Q, R


def qrcp_basis(A):
    A = _f(A)
    m, n = A.shape
    Q = np.zeros((m, min(m, n)), order="F")
    s = _L().orc_qrcp_basis(m, n, _p(A), m, _p(Q), m)
    return np.asfortranarray(Q[:, :s])


def svd(A):
    """Thin SVD by one-sided Jacobi: returns U, S, V, sweeps (A = U diag(S) V^T)."""
    A = _f(A)
    m, n = A.shape
    k = min(m, n)
    U = np.zeros((m, k), order="F")
    S = np.zeros(k)
    V = np.zeros((n, k), order="F")
    rc = _L().orc_svd(m, n, _p(A), m, _p(U), m, _p(S), _p(V), n)
    _check(rc, "svd")
    return U, S, V, rc


# ---------------------------------------------------------------- operators

def svt(A, tau: float):
    A = _f(A)
    m, n = A.shape
    X = np.zeros((m, n), order="F")
    r = _i64()
    _check(_L().orc_svt(m, n, _p(A), m, tau, _p(X), m, ctypes.byref(r)), "svt")
    return X, int(r.value)


def wsvt(A, w):
    A = _f(A)
    m, n = A.shape
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    assert w.shape[0] >= min(m, n)
    X = np.zeros((m, n), order="F")
    r = _i64()
    _check(_L().orc_wsvt(m, n, _p(A), m, _p(w), _p(X), m, ctypes.byref(r)), "wsvt")
    return X, int(r.value)


def wsvt_rule(A, c: float = 2.8, noise_var: float = 0.01, eps: float = 1e-8, tau: float = 0.0):
    """Weighted SVT with w_i = c sqrt(n) / (sqrt(max(sigma_i^2 - n noise_var, 0)) + eps)."""
    A = _f(A)
    m, n = A.shape
    X = np.zeros((m, n), order="F")
    r = _i64()
    _check(_L().orc_wsvt_rule(m, n, _p(A), m, c, noise_var, eps, tau, _p(X), m, ctypes.byref(r)),
           "wsvt_rule")
    return X, int(r.value)


def frsvt(A, tau: float, q: int, Omega, Qprev=None):
    """FRSVT (Alg. 1) with an explicit Gaussian matrix.

    Omega is nhat x l (fresh) or nhat x p (range propagation with Qprev,
    mhat x r_prev).  Returns X, Q~ (mhat x r), r, sigma (length s), s.
    """
    A = _f(A)
    m, n = A.shape
    mh, nh = min(m, n), max(m, n)
    Om = _f(Omega)
    assert Om.shape[0] == nh
    nomega = Om.shape[1]
    X = np.zeros((m, n), order="F")
    Qout = np.zeros((mh, mh), order="F")
    sigma = np.zeros(mh)
    r = _i64()
    s = _i64()
    if Qprev is None:
        qp, rp, ldq = None, 0, mh
    else:
        Qp = _f(Qprev)
        qp, rp, ldq = _p(Qp), Qp.shape[1], mh
    rc = _L().orc_frsvt(m, n, _p(A), m, tau, q, _p(Om), nh, nomega, qp, ldq, rp,
                        _p(X), m, _p(Qout), mh, ctypes.byref(r), _p(sigma), ctypes.byref(s))
    _check(rc, "frsvt")
    rr, ss = int(r.value), int(s.value)
    return X, np.asfortranarray(Qout[:, :rr]), rr, sigma[:ss].copy(), ss


def rpca_ialm(O, lam: float, mode: str = "frsvt", p: int = 5, q: int = 1, seed: int = 0,
              tol: float = 1e-7, max_iter: int = 60, mu0: float = 0.0, rho: float = 1.5,
              mu_bar_factor: float = 1e7, ap: bool = False, ap_a: int = 2, ap_rho: float = 0.05,
              ap_gamma: float = 1.0, keep: int = 0, q_init=None, resid_check: bool = False):
    """Inexact-ALM RPCA; mode 'exact' (SVT by full SVD) or 'frsvt' (FRSVT + RP),
    with the sketch widths of adaptive rank prediction (Sec. 2.3, Eq. 7) when
    ap is set.

    keep > 0 selects partial SVT (the keep largest singular values unshrunk);
    q_init (mhat x r) is the first call's propagated basis (semi-online use);
    resid_check stops each iteration's sampling at the first new sample whose
    residual estimate (Prop. 4, alpha = 20) is at most the threshold 1/mu.

    Returns dict(L, S, ranks, widths, resid_est, resid, iters, converged, Q)
    with Q the last propagated basis."""
    O = _f(O)
    m, n = O.shape
    L = np.zeros((m, n), order="F")
    S = np.zeros((m, n), order="F")
    ranks = np.zeros(max_iter, dtype=np.int64)
    widths = np.zeros(max_iter, dtype=np.int64)
    resid_est = np.zeros(max_iter)
    resid = np.zeros(max_iter)
    mh = min(m, n)
    Qf = np.zeros((mh, mh), order="F")
    rf = _i64()
    if q_init is None:
        Qi, ri = np.zeros((mh, 1), order="F"), 0
    else:
        Qi = _f(q_init)
        assert Qi.shape[0] == mh
        ri = Qi.shape[1]
    it = ctypes.c_int()
    rc = _L().orc_rpca_ialm_rc(m, n, _p(O), m, lam, 0 if mode == "exact" else 1, p, q, seed,
                               tol, max_iter, mu0, rho, mu_bar_factor, int(ap), ap_a, ap_rho,
                               ap_gamma, keep, _p(Qi), ri, _p(Qf), ctypes.byref(rf),
                               int(resid_check), _p(L), m, _p(S), m, ranks.ctypes.data_as(_i64p),
                               widths.ctypes.data_as(_i64p), _p(resid_est), _p(resid),
                               ctypes.byref(it))
    _check(rc, "rpca_ialm")
    k = int(it.value)
    return dict(L=L, S=S, ranks=ranks[:k], widths=widths[:k], resid_est=resid_est[:k],
                resid=resid[:k], iters=k, converged=(rc == 0),
                Q=np.asfortranarray(Qf[:, :int(rf.value)]))


def residual_check(A, Qt, Om, tau: float, alpha: float = 20.0):
    """Sequential residual check (Sec. 3.2): (samples kept, estimates of the
    samples checked).  Qt (mhat x r) may have r = 0 columns; Om is nhat x c."""
    A, Om = _f(A), _f(Om)
    m, n = A.shape
    mh = min(m, n)
    r = 0 if Qt is None else Qt.shape[1]
    Qb = np.zeros((mh, max(r, 1)), order="F") if r == 0 else _f(Qt)
    c = Om.shape[1]
    est = np.full(c, np.nan)
    kept = _L().orc_residual_check(m, n, _p(A), m, _p(Qb), mh, r, _p(Om), Om.shape[0], c, tau, alpha,
                                   _p(est))
    return int(kept), est


def psvt(A, tau: float, keep: int):
    """Partial SVT: the keep largest singular values unshrunk, the rest
    soft-thresholded by tau.  Returns X, rank."""
    A = _f(A)
    m, n = A.shape
    X = np.zeros((m, n), order="F")
    r = _i64()
    _check(_L().orc_psvt(m, n, _p(A), m, tau, keep, _p(X), m, ctypes.byref(r)), "psvt")
    return X, int(r.value)


def residual_estimate(A, Qt, omega, alpha: float = 20.0) -> float:
    """Prop. 4: alpha sqrt(2/pi) ||(I - Q~ Q~^T) Ahat omega||_2, an upper
    bound on sigma_{r+1}(Ahat) with probability >= 1 - 1/alpha."""
    A = _f(A)
    m, n = A.shape
    mh = min(m, n)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    assert om.shape == (max(m, n),)
    if Qt is None or Qt.shape[1] == 0:
        Q, r = np.zeros((mh, 1), order="F"), 0
    else:
        Q = _f(Qt)
        r = Q.shape[1]
    return float(_L().orc_residual_estimate(m, n, _p(A), m, _p(Q), mh, r, _p(om), alpha))


def svt_vjp(A, tau: float, Xbar):
    A = _f(A)
    Xb = _f(Xbar)
    m, n = A.shape
    Ab = np.zeros((m, n), order="F")
    tb = ctypes.c_double()
    _check(_L().orc_svt_vjp(m, n, _p(A), m, tau, _p(Xb), m, _p(Ab), m, ctypes.byref(tb)),
           "svt_vjp")
    return Ab, float(tb.value)


# ---------------------------------------------------------------------------
# Unrolled inexact-ALM with learnable thresholds (test infrastructure for the
# adjoint).  The iALM loop of the RPCA host (Sec. 4.1 of the paper, the
# standard inexact ALM): L-update by thresholding, then the S-update by
# elementwise shrinkage, then the multiplier update.  In the unrolled form the
# SVT threshold of step t is a free parameter tau_t (in place of 1/mu_t) and
# the shrink threshold is lam_t (in place of lam/mu_t); mu_t keeps the plain
# schedule, which also scales the multiplier terms.
# ---------------------------------------------------------------------------
def shrink(V, t: float):
    """Elementwise soft shrinkage sgn(v) max(|v| - t, 0)."""
    return np.sign(V) * np.maximum(np.abs(V) - t, 0.0)


def dual_step(O, L, Y, lam: float, mu: float, mu_next: float):
    """S, Y_next, A_next of one iALM step after the thresholding."""
    O, L, Y = (np.asarray(x, dtype=np.float64) for x in (O, L, Y))
    S = shrink(O - L + Y / mu, lam)
    Yn = Y + mu * (O - L - S)
    An = O - S + Yn / mu_next
    return S, Yn, An


def rpca_start(O, lam: float, norm2: float | None = None, mu0: float = 0.0):
    """Y0 = O / J, A0 = O + Y0 / mu0 with J = max(||O||_2, ||O||_inf / lam) and
    mu0 = 1.25 / ||O||_2 (S_0 = 0).  Returns (Y0, A0, norm2, mu0)."""
    O = np.asarray(O, dtype=np.float64)
    if norm2 is None:
        norm2 = float(svd(O)[1][0])
    J = max(norm2, float(np.abs(O).max()) / lam)
    mu = mu0 if mu0 > 0 else 1.25 / norm2
    Y0 = O / J
    return Y0, O + Y0 / mu, norm2, mu


def rpca_unrolled(O, taus, lams, k: int = 5, p: int = 5, q: int = 1, seed: int = 0,
                  rho: float = 1.5, mu_bar_factor: float = 1e7, lam: float | None = None,
                  norm2: float | None = None):
    """L_T of len(taus) unrolled steps; step t thresholds with FRSVT (fresh
    sketch, l = min(k + p, mhat), q power iterations, Omega drawn with
    counter t from `seed`)."""
    O = np.asarray(O, dtype=np.float64)
    m, n = O.shape
    mh, nh = min(m, n), max(m, n)
    lam = lam if lam is not None else 1.0 / np.sqrt(max(m, n))
    Y, A, _, mu = rpca_start(O, lam, norm2)
    mu_bar = mu * mu_bar_factor
    l = min(k + p, mh)
    T = len(taus)
    L = None
    for t in range(T):
        L = frsvt(A, float(taus[t]), q, gaussian_matrix(seed, t, nh, l))[0]
        if t + 1 == T:
            break
        mu_next = min(rho * mu, mu_bar)
        _, Y, A = dual_step(O, L, Y, float(lams[t]), mu, mu_next)
        mu = mu_next
    return L


def lrr_ialm(X, lam: float, mode: str = "exact", p: int = 5, q: int = 1, seed: int = 0,
             tol: float = 1e-8, max_iter: int = 1000, mu0: float = 1e-6, rho: float = 1.1,
             mu_max: float = 1e10):
    """Low-rank representation (Type A of Table 6) by its inexact ALM: the J
    step by exact SVT (mode 'exact') or FRSVT + range propagation ('frsvt').
    Returns dict(Z, E, ranks, iters, converged)."""
    X = _f(X)
    d, n = X.shape
    Z = np.zeros((n, n), order="F")
    E = np.zeros((d, n), order="F")
    ranks = np.zeros(max_iter, dtype=np.int64)
    it = ctypes.c_int()
    rc = _L().orc_lrr_ialm(d, n, _p(X), d, lam, 0 if mode == "exact" else 1, p, q, seed, tol,
                           max_iter, mu0, rho, mu_max, _p(Z), n, _p(E), d,
                           ranks.ctypes.data_as(_i64p), ctypes.byref(it))
    _check(rc, "lrr_ialm")
    k = int(it.value)
    return dict(Z=Z, E=E, ranks=ranks[:k], iters=k, converged=(rc == 0))


# ---------------------------------------------------------------- tensor host (Type C)

def unfold(T, mode: int) -> np.ndarray:
    """Mode-`mode` unfolding (mode in 0, 1, 2) of a 3-way array: rows indexed
    by that mode, columns by the other two with the earlier one varying
    fastest (the convention of the tensor notation the paper refers to)."""
    T = np.asarray(T, dtype=np.float64)
    return np.asfortranarray(np.moveaxis(T, mode, 0).reshape(T.shape[mode], -1, order="F"))


def fold(M, mode: int, shape) -> np.ndarray:
    """Inverse of unfold."""
    rest = [s for i, s in enumerate(shape) if i != mode]
    T = np.asarray(M).reshape([shape[mode]] + rest, order="F")
    return np.asfortranarray(np.moveaxis(T, 0, mode))


def tensor_rpca(O, alpha, lam: float, mode: str = "exact", p: int = 5, q: int = 1, seed: int = 0,
                tol: float = 1e-7, max_iter: int = 100, mu0: float = 0.0, rho: float = 1.5,
                mu_max: float = 1e10):
    """Low-rank + sparse decomposition of a 3-way tensor (Type C of Table 6
    with the alignment fixed to the identity): min sum_i alpha_i ||L_(i)||_*
    + lam ||E||_1 s.t. O = L + E, by an inexact ALM over one copy L_i of L
    per mode, each tied to O by its own constraint O = L_i + E:

      L_i = fold_i(SVT_{alpha_i / mu}(unfold_i(O - E + Y_i / mu)))
      E   = shrink_{lam / (3 mu)}(mean_i(O - L_i + Y_i / mu))
      Y_i = Y_i + mu (O - L_i - E),  mu = min(rho mu, mu_max)

    from E = Y_i = 0, mu0 = 1.25 / ||O_(1)||_2 unless given; stop when
    max_i ||O - L_i - E||_F / ||O||_F < tol.  The SVT of mode i is exact
    (mode 'exact') or FRSVT with range propagation ('frsvt': first sketch
    ceil(0.1 mhat_i) columns, then r_i + p; q power iterations; the Gaussian
    matrix of mode i in iteration t drawn with seed + i and counter t).
    Returns dict(L = mean of the L_i, E, Ls, ranks (iters x 3), iters,
    converged, resid)."""
    O = np.asfortranarray(np.asarray(O, dtype=np.float64))
    shape = O.shape
    assert len(shape) == 3
    alpha = [float(a) for a in alpha]
    normO = np.linalg.norm(O)
    if mu0 <= 0.0:
        mu0 = 1.25 / svd(unfold(O, 0))[1][0]
    mu = mu0
    E = np.zeros(shape, order="F")
    Y = [np.zeros(shape, order="F") for _ in range(3)]
    Ls = [None] * 3
    Qs = [None] * 3
    rprev = [-1, -1, -1]
    ranks, resid = [], []
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        rk = []
        for i in range(3):
            M = unfold(O - E + Y[i] / mu, i)
            if mode == "exact":
                X, r = svt(M, alpha[i] / mu)
            else:
                mh, nh = min(M.shape), max(M.shape)
                l0 = max(1, int(np.ceil(0.1 * mh)))
                Qp = Qs[i] if rprev[i] > 0 else None
                nom = l0 if rprev[i] < 0 else p
                if Qp is not None and rprev[i] + nom > mh:
                    nom = mh - rprev[i]
                if nom < 1 and Qp is None:
                    nom = 1
                Om = gaussian_matrix(seed + i, it - 1, nh, nom)
                X, Qs[i], r, _, _ = frsvt(M, alpha[i] / mu, q, Om, Qp)
                rprev[i] = r
            Ls[i] = fold(X, i, shape)
            rk.append(r)
        V = sum(O - Ls[i] + Y[i] / mu for i in range(3)) / 3.0
        E = np.asfortranarray(shrink(V, lam / (3.0 * mu)))
        res = 0.0
        for i in range(3):
            Z = O - Ls[i] - E
            Y[i] = Y[i] + mu * Z
            res = max(res, np.linalg.norm(Z) / normO)
        ranks.append(rk)
        resid.append(res)
        mu = min(rho * mu, mu_max)
        if res < tol:
            converged = True
            break
    L = (Ls[0] + Ls[1] + Ls[2]) / 3.0
    return dict(L=L, E=E, Ls=Ls, Y=Y, ranks=np.array(ranks, dtype=np.int64).reshape(-1, 3), iters=it,
                converged=converged, resid=np.array(resid), mu0=mu0)
