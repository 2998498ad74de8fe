"""Pins for the oracle's iALM RPCA host and its exact-SVT gradient."""
import numpy as np
import pytest

from paper_1509_00296_amd import synth


@pytest.fixture(scope="module")
def small_rpca():
    O, L, S = synth.rpca(seed=3, m=3000, n=60, rank=3, frac=0.10)
    return O, L, S


def test_ialm_exact_recovers_and_meets_kkt(orc, small_rpca):
    O, L, S = small_rpca
    lam = 1.0 / np.sqrt(max(O.shape))
    out = orc.rpca_ialm(O, lam, mode="exact", tol=1e-7, max_iter=60)
    assert out["converged"]
    nrmse = np.linalg.norm(out["L"] - L) / np.linalg.norm(L)
    assert nrmse < 1e-4
    assert out["ranks"][-1] == 3
    # the residual decreases after the first iterations
    res = out["resid"]
    assert np.all(np.diff(res[3:]) < 0)
    # KKT of min ||L||_* + lam ||S||_1 s.t. O = L + S: the dual certificate
    # Y = O - S - SVT... is rebuilt from the solution: Y = mu (O - L - S) is not
    # returned, so check the subgradient of the sparse part instead: the
    # residual of the constraint is tiny and S is exactly zero off-support.
    assert np.linalg.norm(O - out["L"] - out["S"]) / np.linalg.norm(O) < 1e-7


def test_ialm_frsvt_matches_exact_iterations(orc, small_rpca):
    O, L, S = small_rpca
    lam = 1.0 / np.sqrt(max(O.shape))
    ex = orc.rpca_ialm(O, lam, mode="exact", tol=1e-7, max_iter=60)
    fr = orc.rpca_ialm(O, lam, mode="frsvt", p=5, q=1, seed=11, tol=1e-7, max_iter=60)
    assert fr["converged"]
    assert abs(fr["iters"] - ex["iters"]) <= 1       # Table 5: equal iteration counts
    n_ex = np.linalg.norm(ex["L"] - L) / np.linalg.norm(L)
    n_fr = np.linalg.norm(fr["L"] - L) / np.linalg.norm(L)
    assert n_fr <= 2 * n_ex + 1e-9
    assert fr["ranks"][-1] == 3


def _fd_svt(orc, A, tau, D, h):
    Xp, _ = orc.svt(A + h * D, tau)
    Xm, _ = orc.svt(A - h * D, tau)
    return (Xp - Xm) / (2 * h)


@pytest.mark.parametrize("m,n", [(14, 9), (9, 14), (10, 10)])
def test_svt_vjp_matches_central_differences(orc, m, n):
    rng = np.random.default_rng(m * n)
    A = rng.standard_normal((m, n)) * 2
    tau = 1.3
    for _ in range(3):
        D = rng.standard_normal((m, n))
        Xbar = rng.standard_normal((m, n))
        Abar, _ = orc.svt_vjp(A, tau, Xbar)
        fd = np.sum(Xbar * _fd_svt(orc, A, tau, D, 1e-5))
        assert np.sum(Abar * D) == pytest.approx(fd, rel=1e-6, abs=1e-8)
    # tau direction
    Xbar = rng.standard_normal((m, n))
    _, tb = orc.svt_vjp(A, tau, Xbar)
    Xp, _ = orc.svt(A, tau + 1e-5)
    Xm, _ = orc.svt(A, tau - 1e-5)
    assert tb == pytest.approx(np.sum(Xbar * (Xp - Xm)) / 2e-5, rel=1e-6, abs=1e-8)


def test_svt_jacobian_symmetric_psd_contraction(orc):
    # SVT is the proximal map of a convex function: its Jacobian is symmetric
    # with eigenvalues in [0, 1]
    rng = np.random.default_rng(21)
    A = rng.standard_normal((12, 8)) * 2
    tau = 1.0
    for _ in range(10):
        D1, D2 = rng.standard_normal((2, 12, 8))
        J1, _ = orc.svt_vjp(A, tau, D1)
        J2, _ = orc.svt_vjp(A, tau, D2)
        assert np.sum(D1 * J2) == pytest.approx(np.sum(J1 * D2), rel=1e-10, abs=1e-12)
        q = np.sum(D1 * J1)
        assert -1e-12 <= q <= np.sum(D1 * D1) + 1e-12


def test_svt_tau_derivative_closed_form(orc):
    rng = np.random.default_rng(22)
    A = rng.standard_normal((15, 10)) * 2
    tau = 1.5
    u, s, vt = np.linalg.svd(A, full_matrices=False)
    r = int(np.sum(s > tau))
    UV = u[:, :r] @ vt[:r]
    _, tb = orc.svt_vjp(A, tau, UV)
    assert tb == pytest.approx(-r, rel=1e-12)


def test_svt_vjp_straddling_pair_guard(orc):
    """A pair of singular values straddling tau closer than 1e-12 (relative)
    takes the divided difference 1/2 instead of f(s_i)/(s_i - s_j) (here 1/6);
    the VJP stays a contraction (SVT is 1-Lipschitz) and finite.  A is
    diagonal so that its singular vectors are the coordinate axes."""
    import numpy as np
    rng = np.random.default_rng(8)
    m, n, tau = 12, 9, 2.0
    s = np.array([9.0, 7.0, 5.0, tau + 1e-13, tau - 5e-13, 1.0, 0.5, 0.2, 0.1])
    A = np.zeros((m, n))
    A[np.arange(n), np.arange(n)] = s
    Xb = rng.standard_normal((m, n))
    Ab, tb = orc.svt_vjp(A, tau, Xb)
    assert np.all(np.isfinite(Ab)) and np.isfinite(tb)
    assert np.linalg.norm(Ab) <= np.linalg.norm(Xb) * (1 + 1e-9)
    ga = (s[3] - tau) / (s[3] + s[4])
    want = 0.5 * 0.5 * (Xb[3, 4] + Xb[4, 3]) + ga * 0.5 * (Xb[3, 4] - Xb[4, 3])
    assert abs(Ab[3, 4] - want) <= 1e-12
    # a pair above tau: symmetric part 1, antisymmetric (f_0 + f_1)/(s_0 + s_1)
    ga01 = (s[0] + s[1] - 2 * tau) / (s[0] + s[1])
    want01 = 0.5 * (Xb[0, 1] + Xb[1, 0]) + ga01 * 0.5 * (Xb[0, 1] - Xb[1, 0])
    assert abs(Ab[0, 1] - want01) <= 1e-12
