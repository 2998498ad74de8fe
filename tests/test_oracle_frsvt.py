"""Pins for the oracle's FRSVT (Alg. 1): Prop. 1, exact recovery when the rank
is at most l, the pseudo-contraction per draw of Omega (Prop. 2 + Lemma 2),
the average bound of Thm. 3, the span identity of range propagation and the
fixed point of propagation."""
import numpy as np
import pytest

from paper_1509_00296_amd.synth import haar


def _lowrank(rng, m, n, s):
    k = len(s)
    return (haar(rng, m, k) * np.asarray(s, float)) @ haar(rng, n, k).T


def test_prop1_orthonormal_left_factor(orc):
    # S_tau(Q B) = Q S_tau(B) for any Q with orthonormal columns (m x l, l <= m)
    rng = np.random.default_rng(0)
    for (m, l, n) in [(40, 6, 25), (30, 30, 12), (50, 9, 9)]:
        Q = haar(rng, m, l)
        B = rng.standard_normal((l, n)) * 3
        lhs, r1 = orc.svt(Q @ B, 2.0)
        SB, r2 = orc.svt(B, 2.0)
        assert r1 == r2
        assert np.linalg.norm(lhs - Q @ SB) <= 1e-13 * max(np.linalg.norm(lhs), 1.0)


@pytest.mark.parametrize("m,n", [(120, 70), (70, 120)])
@pytest.mark.parametrize("extra", [0, 4])
@pytest.mark.parametrize("q", [0, 1, 2])
def test_exact_recovery_when_rank_le_l(orc, m, n, extra, q):
    rng = np.random.default_rng(m + 10 * extra + q)
    s = np.array([50.0, 30.0, 20.0, 8.0, 3.0, 1.5])
    A = _lowrank(rng, m, n, s)
    tau = 2.0
    l = len(s) + extra
    Om = orc.gaussian_matrix(77, q, max(m, n), l)
    X, Qt, r, sig, sdim = orc.frsvt(A, tau, q, Om)
    Xe, re = orc.svt(A, tau)
    assert r == re == 5
    assert np.linalg.norm(X - Xe) / np.linalg.norm(Xe) < 1e-12
    assert np.allclose(sig[:6], s, rtol=1e-12)
    assert sdim == len(s)           # QR_CP drops the numerically null samples
    assert np.abs(Qt.T @ Qt - np.eye(r)).max() < 1e-13


def test_full_sampling_is_exact(orc):
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 25)) * 2
    Om = orc.gaussian_matrix(5, 0, 40, 25)
    X, _, r, _, _ = orc.frsvt(A, 1.5, 1, Om)
    Xe, re = orc.svt(A, 1.5)
    assert r == re
    assert np.linalg.norm(X - Xe) / np.linalg.norm(Xe) < 1e-13


def test_projection_identities_per_draw(orc):
    """tau = 0 gives P_Q A; then S_tau(P_Q A) is the FRSVT result (Prop. 1) and
    Prop. 2 with Lemma 2 bounds its distance to S_tau(A) for this Omega."""
    rng = np.random.default_rng(4)
    A = _lowrank(rng, 60, 45, [20, 15, 10, 7, 5, 3, 2, 1, 0.5]) + 0.05 * rng.standard_normal((60, 45))
    k, p, tau = 4, 3, 1.2
    for seed in range(10):
        Om = orc.gaussian_matrix(seed, 0, 60, k + p)
        PQA, _, _, _, _ = orc.frsvt(A, 0.0, 0, Om)
        X, _, _, _, _ = orc.frsvt(A, tau, 0, Om)
        SPQA, _ = orc.svt(PQA, tau)
        assert np.linalg.norm(X - SPQA) <= 1e-12 * np.linalg.norm(X)
        SA, _ = orc.svt(A, tau)
        lhs = np.sum((SA - X) ** 2)
        PA = A - SA
        PPQA = PQA - SPQA
        assert lhs <= np.sum((A - PQA) ** 2) - np.sum((PA - PPQA) ** 2) + 1e-10
        sig = np.linalg.svd(A, compute_uv=False)
        # Lemma 2: the dual gap is at least sum_{j>l} min(sigma_j, tau)^2
        assert np.sum((PA - PPQA) ** 2) >= np.sum(np.minimum(sig[k + p:], tau) ** 2) - 1e-10
        # Eckart-Young: a rank-l projection loses at least the tail energy
        assert np.sum((A - PQA) ** 2) >= np.sum(sig[k + p:] ** 2) - 1e-10


def test_thm3_average_bound_q0(orc):
    rng = np.random.default_rng(5)
    m, n = 50, 40
    sig_true = 10.0 * 0.7 ** np.arange(min(m, n))
    A = (haar(rng, m, 40) * sig_true) @ haar(rng, n, 40).T
    k, p, tau = 5, 4, 0.8
    SA, _ = orc.svt(A, tau)
    errs = []
    for seed in range(200):
        Om = orc.gaussian_matrix(1000 + seed, 0, m, k + p)
        X, _, _, _, _ = orc.frsvt(A, tau, 0, Om)
        errs.append(np.sum((SA - X) ** 2))
    tail = sig_true[k:]
    bound = (1 + k / (p - 1)) * np.sum(tail ** 2) - np.sum(np.minimum(tail, tau) ** 2)
    assert np.mean(errs) <= bound
    # and the power scheme helps on average (Thm. 2 / Cor. 1 trend)
    errs2 = []
    for seed in range(60):
        Om = orc.gaussian_matrix(1000 + seed, 0, m, k + p)
        X, _, _, _, _ = orc.frsvt(A, tau, 2, Om)
        errs2.append(np.sum((SA - X) ** 2))
    assert np.mean(errs2) < np.mean(errs[:60])


@pytest.mark.parametrize("q", [0, 1, 2])
def test_range_propagation_span_identity(orc, q):
    """With Q~ given, FRSVT equals S_tau of the projection of A onto
    span((A A^T)^q [Q~, A Omega_p]) (Alg. 1 with range propagation and power iterations)."""
    rng = np.random.default_rng(6 + q)
    m, n = 30, 80                      # m <= n: Ahat = A
    A = _lowrank(rng, m, n, [30, 20, 12, 6, 3, 2, 1]) + 0.1 * rng.standard_normal((m, n))
    Qt = haar(rng, m, 3)
    p = 4
    Om = orc.gaussian_matrix(9, 1, n, p)
    X, _, r, _, s = orc.frsvt(A, 1.0, q, Om, Qprev=Qt)
    assert s == 7
    M = np.hstack([Qt, A @ Om])
    for _ in range(q):
        M = A @ (A.T @ M)
    Qm, _ = np.linalg.qr(M)
    Xref, rref = orc.svt(Qm @ (Qm.T @ A), 1.0)
    assert r == rref
    assert np.linalg.norm(X - Xref) / np.linalg.norm(Xref) < 1e-11


def test_range_propagation_fixed_point(orc):
    rng = np.random.default_rng(8)
    m, n = 90, 50
    s = np.array([40.0, 25.0, 15.0, 0.6, 0.4, 0.2])
    A = _lowrank(rng, m, n, s)
    tau = 1.0
    u, sv, vt = np.linalg.svd(A.T, full_matrices=False)   # Ahat = A^T (m > n)
    Qt = u[:, :3]                                         # exact top singular vectors
    Om = orc.gaussian_matrix(3, 2, m, 2)
    X, Qo, r, _, _ = orc.frsvt(A, tau, 1, Om, Qprev=Qt)
    Xe, _ = orc.svt(A, tau)
    assert r == 3
    assert np.linalg.norm(X - Xe) / np.linalg.norm(Xe) < 1e-12
    # the propagated basis spans the same top-3 space
    assert np.linalg.norm(Qo @ Qo.T - Qt @ Qt.T) < 1e-12


def test_orientation_and_special_thresholds(orc):
    rng = np.random.default_rng(9)
    A = rng.standard_normal((25, 60))
    Om = orc.gaussian_matrix(4, 0, 60, 8)
    X1, _, r1, _, _ = orc.frsvt(A, 1.0, 2, Om)
    X2, _, r2, _, _ = orc.frsvt(A.T, 1.0, 2, Om)      # same oriented problem
    assert r1 == r2 and np.abs(X1 - X2.T).max() < 1e-13
    s1 = np.linalg.svd(A, compute_uv=False)[0]
    X3, Q3, r3, _, _ = orc.frsvt(A, 1.01 * s1, 2, Om)
    assert r3 == 0 and np.abs(X3).max() == 0.0 and Q3.shape == (25, 0)
