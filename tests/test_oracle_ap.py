"""Adaptive rank prediction (Sec. 2.3, Eq. 7) in the oracle's iALM loop.

Pins: with a = p, ceil(rho mhat) = p and gamma = 1 the rule is the fixed
rule (l_{i+1} = r_i + p), so the two runs must agree bit for bit; with the
bound b at the true rank the loop must still recover L (the propagated basis
alone once r = b) and never sketch wider than b; and the adaptive run must
reach the exact-SVT iALM solution within the iALM tolerance."""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def orc():
    import oracle
    return oracle


@pytest.fixture(scope="module")
def problem():
    from paper_1509_00296_amd import synth
    O, L, S = synth.rpca(seed=3, m=3000, n=60, rank=3, frac=0.10)
    return O, L, 1.0 / math.sqrt(3000)


def test_ap_reduces_to_fixed_rule(orc, problem):
    O, _, lam = problem
    ap = orc.rpca_ialm(O, lam, mode="frsvt", p=3, q=1, seed=17, ap=True, ap_a=3, ap_rho=3 / 60)
    fx = orc.rpca_ialm(O, lam, mode="frsvt", p=3, q=1, seed=17)
    assert ap["iters"] == fx["iters"]
    assert np.array_equal(ap["ranks"], fx["ranks"])
    assert np.array_equal(ap["widths"], fx["widths"])
    assert np.array_equal(ap["L"], fx["L"]) and np.array_equal(ap["S"], fx["S"])


def test_ap_bounded_width_recovers(orc, problem):
    O, Lgt, lam = problem
    out = orc.rpca_ialm(O, lam, mode="frsvt", q=1, seed=17, ap=True, ap_gamma=0.05)  # b = 3
    w, r = out["widths"], out["ranks"]
    assert out["converged"]
    assert w.max() <= 3 and np.all(r <= w)
    assert r[-1] == 3
    assert np.linalg.norm(out["L"] - Lgt) / np.linalg.norm(Lgt) < 1e-4


def test_ap_matches_exact_ialm(orc, problem):
    O, Lgt, lam = problem
    ap = orc.rpca_ialm(O, lam, mode="frsvt", q=1, seed=17, ap=True)
    ex = orc.rpca_ialm(O, lam, mode="exact")
    assert ap["converged"] and ex["converged"]
    # the widths stay near the rank: a beside it once the rank is found
    assert ap["widths"].max() <= 6
    assert np.linalg.norm(ap["L"] - ex["L"]) / np.linalg.norm(ex["L"]) < 1e-6
    assert np.linalg.norm(ap["L"] - Lgt) / np.linalg.norm(Lgt) < 1e-4


def test_residual_estimate_prop4(orc):
    """Prop. 4 (with Lemma 3): for Q~ spanning the top-r left singular
    vectors of Ahat, ||(I - Q~Q~^T) Ahat omega|| <= sigma_{r+1} ||omega||
    always, and alpha sqrt(2/pi) ||(I - Q~Q~^T) Ahat omega|| >= sigma_{r+1}
    with probability >= 1 - 1/alpha; a basis of the whole range gives 0."""
    rng = np.random.default_rng(5)
    m, n, r, alpha = 400, 120, 5, 20.0
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.geomspace(100.0, 0.1, n)
    A = np.asfortranarray((U * s) @ V.T)          # m > n: Ahat = A^T, its left vectors are V
    Q = np.asfortranarray(V[:, :r])
    c = alpha * math.sqrt(2.0 / math.pi)
    hits = 0
    for _ in range(200):
        om = rng.standard_normal(m)
        est = orc.residual_estimate(A, Q, om, alpha)
        assert est / c <= s[r] * np.linalg.norm(om) * (1 + 1e-12)
        hits += est >= s[r]
    assert hits >= 190
    full = orc.residual_estimate(A, np.asfortranarray(V), rng.standard_normal(m), alpha)
    assert full <= 1e-10 * s[0]


def test_rpca_reports_residual_estimate(orc, problem):
    O, _, lam = problem
    out = orc.rpca_ialm(O, lam, mode="frsvt", q=1, seed=17, ap=True, ap_gamma=0.05)  # b = 3
    est, w, r = out["resid_est"], out["widths"], out["ranks"]
    # a sample is drawn exactly when the width exceeds the propagated rank
    prev = np.concatenate([[0], r[:-1]])
    assert np.array_equal(est < 0, w == prev)
    assert np.all(est[est >= 0] > 0)


# ---------------------------------------------------------------------------
# Partial SVT (the truncated nuclear norm's proximal step, Type B of Table 6)
# ---------------------------------------------------------------------------
def test_psvt_definition_on_diagonal(orc):
    s = np.array([9.0, 5.0, 3.0, 1.5, 0.5])
    A = np.zeros((7, 5))
    A[np.arange(5), np.arange(5)] = s
    X, r = orc.psvt(A, 2.0, 2)
    want = np.array([9.0, 5.0, 1.0, 0.0, 0.0])
    assert np.allclose(np.diag(X[:5]), want, atol=1e-14) and abs(X).sum() - want.sum() < 1e-12
    assert r == 3


def test_psvt_special_cases_and_invariance(orc):
    rng = np.random.default_rng(9)
    A = rng.standard_normal((40, 25))
    X0, r0 = orc.psvt(A, 1.5, 0)
    Xs, rs = orc.svt(A, 1.5)
    assert r0 == rs and np.abs(X0 - Xs).max() < 1e-12
    Xk, rk = orc.psvt(A, 100.0, 25)          # every singular value kept
    assert rk == 25 and np.abs(Xk - A).max() < 1e-11
    U, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    V, _ = np.linalg.qr(rng.standard_normal((25, 25)))
    X1, _ = orc.psvt(A, 1.5, 3)
    X2, _ = orc.psvt(U @ A @ V.T, 1.5, 3)
    assert np.abs(U @ X1 @ V.T - X2).max() < 1e-11


def test_rpca_partial_svt_recovers_rank_one(orc):
    """Type B: a rank-1 scene over n = 5 frames with 5 % sparse outliers; the
    partial-SVT iALM (k = 1) with FRSVT (widths up to l = 3, q = 2) and the
    exact PSVT iALM reach nearly the same L, and leaving the largest singular
    value unshrunk recovers the scene better than SVT does with so few
    frames (the degradation the section describes)."""
    from paper_1509_00296_amd import synth
    O, Lgt, _ = synth.rpca(seed=11, m=6000, n=5, rank=1, frac=0.05)
    lam = 1.0 / math.sqrt(6000)
    fr = orc.rpca_ialm(O, lam, mode="frsvt", q=2, seed=3, keep=1, ap=True, ap_a=2, ap_gamma=0.6)
    ex = orc.rpca_ialm(O, lam, mode="exact", keep=1)
    sv = orc.rpca_ialm(O, lam, mode="exact")
    assert fr["converged"] and ex["converged"]
    assert fr["widths"].max() <= 3
    assert np.linalg.norm(fr["L"] - ex["L"]) / np.linalg.norm(ex["L"]) < 1e-3
    err = lambda d: np.linalg.norm(d["L"] - Lgt) / np.linalg.norm(Lgt)
    assert err(ex) < 0.85 * err(sv)


def test_rpca_initial_basis(orc):
    """Starting from the previous solve's propagated basis (semi-online use)
    reaches the same solution."""
    from paper_1509_00296_amd import synth
    O, _, _ = synth.rpca(seed=3, m=3000, n=60, rank=3, frac=0.10)
    lam = 1.0 / math.sqrt(3000)
    a = orc.rpca_ialm(O, lam, mode="frsvt", q=1, seed=17)
    assert a["Q"].shape == (60, a["ranks"][-1])
    assert np.abs(a["Q"].T @ a["Q"] - np.eye(a["Q"].shape[1])).max() < 1e-12
    b = orc.rpca_ialm(O, lam, mode="frsvt", q=1, seed=17, q_init=a["Q"])
    assert b["converged"] and b["widths"][0] == a["ranks"][-1] + 5
    assert np.linalg.norm(b["L"] - a["L"]) / np.linalg.norm(a["L"]) < 1e-6


def test_ap_saturated_iteration_oversamples_more(orc, problem):
    """Sec. 2.3: when the rank reaches the predicted width the rule predicts
    optimistically with the larger rate ceil(rho mhat); otherwise it adds
    only a.  With a = 1 and rho = 0.5 (30 columns at mhat = 60) the run whose
    rank grows from 1 to 3 must sketch at least 30 columns once after the
    first call, and stays within the rank plus one elsewhere."""
    O, Lgt, lam = problem
    out = orc.rpca_ialm(O, lam, mode="frsvt", q=1, seed=17, ap=True, ap_a=1, ap_rho=0.5)
    w, r = out["widths"], out["ranks"]
    assert out["converged"]
    assert w[1:].max() >= 30
    assert np.sum(w[1:] > r[:-1] + 1) == 1
    assert np.linalg.norm(out["L"] - Lgt) / np.linalg.norm(Lgt) < 1e-4
