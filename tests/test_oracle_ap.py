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
