"""Pins for the oracle's exact SVT (Def. 1, Eq. (3)) and weighted SVT against
closed forms, the optimality condition of Problem (2), the dual projection
(Def. 3, Lemma 1), the pseudo-contractions (Props. 2-3) and brute force."""
import numpy as np
import pytest

from paper_1509_00296_amd.synth import haar


def _known(rng, m, n, s):
    k = len(s)
    U, V = haar(rng, m, k), haar(rng, n, k)
    return U, np.asarray(s, float), V, (U * s) @ V.T


@pytest.mark.parametrize("m,n", [(40, 25), (25, 40), (30, 30)])
def test_svt_closed_form_known_sigma(orc, m, n):
    rng = np.random.default_rng(m * 7 + n)
    s = np.array([9.0, 7.5, 5.0, 3.0, 2.0, 0.5])
    U, s, V, A = _known(rng, m, n, s)
    tau = 2.5
    X, r = orc.svt(A, tau)
    ref = (U * np.maximum(s - tau, 0)) @ V.T
    assert r == 4
    assert np.linalg.norm(X - ref) / np.linalg.norm(ref) < 1e-14


def test_svt_optimality_condition(orc):
    # A - X* = tau (U1 V1^T + W), ||W||_2 <= 1, U1^T W = 0, W V1 = 0
    rng = np.random.default_rng(11)
    A = rng.standard_normal((35, 20)) * 3.0
    tau = 4.0
    X, r = orc.svt(A, tau)
    u, s, vt = np.linalg.svd(X, full_matrices=False)
    U1, V1 = u[:, :r], vt[:r].T
    assert np.all(s[:r] > 1e-8) and np.all(s[r:] < 1e-10)
    W = (A - X) / tau - U1 @ V1.T
    assert np.linalg.norm(W, 2) <= 1.0 + 1e-12
    assert np.abs(U1.T @ W).max() < 1e-12
    assert np.abs(W @ V1).max() < 1e-12


def test_svt_special_cases(orc):
    rng = np.random.default_rng(2)
    A = rng.standard_normal((12, 9))
    s1 = np.linalg.svd(A, compute_uv=False)[0]
    X0, r0 = orc.svt(A, 0.0)
    assert r0 == 9 and np.abs(X0 - A).max() < 1e-13
    Xbig, rbig = orc.svt(A, s1 * 1.0001)
    assert rbig == 0 and np.abs(Xbig).max() == 0.0
    # diagonal input: SVT is the scalar soft shrinkage of the diagonal
    d = np.array([3.0, -2.0, 0.5, -0.1])
    X, r = orc.svt(np.diag(d), 0.75)
    assert r == 2
    assert np.allclose(X, np.diag(np.sign(d) * np.maximum(np.abs(d) - 0.75, 0)), atol=1e-15)


def _objective(X, A, tau):
    return tau * np.linalg.svd(X, compute_uv=False).sum() + 0.5 * np.sum((X - A) ** 2)


def test_svt_brute_force_tiny(orc):
    rng = np.random.default_rng(4)
    for shape in [(2, 2), (3, 2)]:
        A = rng.standard_normal(shape) * 2
        tau = 0.9
        X, _ = orc.svt(A, tau)
        f0 = _objective(X, A, tau)
        # dense grid around X* and random perturbations never do better
        grid = np.linspace(-0.3, 0.3, 7)
        for _ in range(400):
            D = rng.choice(grid, size=shape)
            assert _objective(X + D, A, tau) >= f0 - 1e-12
        for scale in (1e-1, 1e-3, 1e-6):
            for _ in range(200):
                assert _objective(X + scale * rng.standard_normal(shape), A, tau) >= f0 - 1e-12


def test_dual_projection_def3_lemma1(orc):
    rng = np.random.default_rng(9)
    A = rng.standard_normal((20, 14)) * 2
    tau = 1.7
    X, _ = orc.svt(A, tau)
    P = A - X                              # X + P_tau(X) = X decomposition
    u, s, vt = np.linalg.svd(A, full_matrices=False)
    assert np.abs(P - (u * np.minimum(s, tau)) @ vt).max() < 1e-13   # Def. 3
    assert np.linalg.norm(P, 2) <= tau * (1 + 1e-13)
    # Lemma 1: P_tau(A) is the closest point of the spectral ball
    for _ in range(100):
        Z = rng.standard_normal(A.shape)
        Z *= rng.uniform(0.2, 1.0) * tau / np.linalg.norm(Z, 2)
        assert np.sum((A - Z) ** 2) >= np.sum((A - P) ** 2) - 1e-12


def test_pseudo_contraction_props_2_3(orc):
    rng = np.random.default_rng(10)
    tau = 1.0
    for _ in range(30):
        A = rng.standard_normal((15, 10)) * 2
        B = A + rng.standard_normal((15, 10)) * rng.uniform(0.01, 2.0)
        SA, _ = orc.svt(A, tau)
        SB, _ = orc.svt(B, tau)
        PA, PB = A - SA, B - SB
        lhs = np.sum((SA - SB) ** 2)
        rhs = np.sum((A - B) ** 2) - np.sum((PA - PB) ** 2)
        assert lhs <= rhs + 1e-10                                   # Prop. 2
        lhs2 = np.linalg.norm(SA - SB, 2)
        assert lhs2 <= 2 * np.linalg.norm(A - B, 2) - np.linalg.norm(PA - PB, 2) + 1e-10  # Prop. 3
        assert lhs2 <= np.linalg.norm(A - B, 2) + 1e-10             # non-expansive


def test_wsvt_constant_weights_equal_svt(orc):
    rng = np.random.default_rng(12)
    A = rng.standard_normal((18, 11)) * 3
    X, r = orc.svt(A, 2.0)
    Xw, rw = orc.wsvt(A, np.full(11, 2.0))
    assert r == rw and np.abs(X - Xw).max() < 1e-14


def test_wsvt_closed_form_and_objective(orc):
    rng = np.random.default_rng(13)
    s = np.array([10.0, 6.0, 4.0, 1.0])
    U, s, V, A = _known(rng, 16, 9, s)
    w = np.array([1.0, 2.0, 5.0, 6.0, 7.0, 8.0, 9.0, 9.5, 9.9])   # non-descending
    X, r = orc.wsvt(A, w)
    ref = (U * np.maximum(s - w[:4], 0)) @ V.T
    assert r == 2 and np.abs(X - ref).max() < 1e-13

    # with non-descending weights WSVT minimises sum_i w_i sigma_i(X) + 1/2||X-A||^2
    def obj(Y):
        return np.dot(w, np.linalg.svd(Y, compute_uv=False)) + 0.5 * np.sum((Y - A) ** 2)
    f0 = obj(X)
    for scale in (1e-1, 1e-3):
        for _ in range(200):
            assert obj(X + scale * rng.standard_normal(X.shape)) >= f0 - 1e-10


def test_wsvt_rule_reduces_to_explicit_weights(orc):
    # the rule's weights depend only on each singular value: recomputing them
    # from the exact spectrum and calling the explicit-weight WSVT must agree
    rng = np.random.default_rng(14)
    for (m, n) in [(64, 40), (49, 90), (100, 30)]:
        s = np.array([50.0, 20.0, 10.0, 5.0])
        _, _, _, L = _known(rng, m, n, s)
        A = L + 0.1 * rng.standard_normal((m, n))
        sig = np.linalg.svd(A, compute_uv=False)
        sh = np.sqrt(np.maximum(sig ** 2 - n * 0.01, 0.0))
        w = 2.8 * np.sqrt(n) / (sh + 1e-8)
        Xr, rr = orc.wsvt_rule(A, 2.8, 0.01, 1e-8)
        Xw, rw = orc.wsvt(A, w)
        assert rr == rw
        assert np.abs(Xr - Xw).max() < 1e-12
        # the weights are non-descending here, so this is the WNNM optimum
        assert np.all(np.diff(w) >= 0)
    # c <= 0 is plain SVT with threshold tau
    A = rng.standard_normal((30, 20)) * 3
    Xs, rs = orc.svt(A, 2.0)
    Xr, rr = orc.wsvt_rule(A, 0.0, 0.0, 0.0, 2.0)
    assert rs == rr and np.abs(Xs - Xr).max() < 1e-14
