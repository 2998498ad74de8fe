"""The residual check that steers sampling (Sec. 3.2 after Prop. 4), in the
oracle: new samples are taken in order and sampling stops at the first whose
estimate alpha sqrt(2/pi) ||(I - Q_j Q_j^T) y_j|| (alpha = 20) against the
basis it would extend is at most the threshold.

Pins: on a matrix with known singular values and a clear drop below tau,
the check stops exactly after the samples that span the missing directions
and never leaves a direction above tau outside the kept basis; tau = 0
never stops; a propagated basis spanning the whole range stops at the first
sample; in the iALM on an exactly low-rank input it shrinks the widths to
r + 1 and reaches the same L, and on the video-like data (10 % outliers) it
never stops early, so the run equals the unchecked one bit for bit."""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def orc():
    import oracle
    return oracle


def _matrix(rng, m=400, n=120, top=8):
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.concatenate([100.0 * 0.8 ** np.arange(top), 1e-4 * 0.9 ** np.arange(n - top)])
    return np.asfortranarray((U * s) @ V.T), V, s     # m > n: Ahat = A^T, left vectors V


def test_check_stops_after_the_missing_directions(orc):
    rng = np.random.default_rng(11)
    A, V, s = _matrix(rng)
    tau, r, c = 1.0, 3, 12                          # s[7] = 21 > tau > s[8] = 1e-4
    Qt = np.asfortranarray(V[:, :r])
    Ahat = A.T
    stops = 0
    for trial in range(200):
        Om = np.asfortranarray(rng.standard_normal((A.shape[0], c)))
        kept, est = orc.residual_check(A, Qt, Om, tau)
        assert 1 <= kept <= c
        # the kept basis [Q~, Ahat Omega(:, :kept)] leaves nothing above tau
        B, _ = np.linalg.qr(np.hstack([Qt, Ahat @ Om[:, :kept]]))
        resid = np.linalg.norm(Ahat - B @ (B.T @ Ahat), 2)
        assert resid <= tau
        # the samples before the stop each saw a direction above tau
        assert np.all(est[:kept - 1] > tau)
        stops += kept == 8 - r + 1
    # five samples to span directions 3..7, the sixth finds only the tail
    assert stops >= 190


def test_check_zero_threshold_never_stops(orc):
    rng = np.random.default_rng(12)
    A, V, _ = _matrix(rng)
    Om = np.asfortranarray(rng.standard_normal((A.shape[0], 7)))
    kept, est = orc.residual_check(A, np.asfortranarray(V[:, :2]), Om, 0.0)
    assert kept == 7 and np.all(est > 0)


def test_check_full_range_stops_at_first_sample(orc):
    rng = np.random.default_rng(13)
    m, n, r = 300, 90, 6
    U, _ = np.linalg.qr(rng.standard_normal((m, r)))
    W, _ = np.linalg.qr(rng.standard_normal((n, r)))
    A = np.asfortranarray((U * np.linspace(50, 5, r)) @ W.T)   # rank 6, Ahat = A^T
    Om = np.asfortranarray(rng.standard_normal((m, 5)))
    kept, est = orc.residual_check(A, np.asfortranarray(W), Om, 1e-6)
    assert kept == 1 and est[0] <= 1e-10
    # without the propagated basis the first r samples span the range
    kept0, est0 = orc.residual_check(A, None, np.asfortranarray(rng.standard_normal((m, 9))), 1e-6)
    assert kept0 == r + 1 and np.all(est0[:r] > 1.0)


def test_ialm_check_on_exact_low_rank_input(orc):
    from paper_1509_00296_amd import synth
    O, Lgt, _ = synth.rpca(seed=3, m=60, n=3000, rank=3, frac=0.0)
    lam = 1.0 / math.sqrt(3000)
    a = orc.rpca_ialm(O, lam, mode="frsvt", p=5, q=1, seed=17)
    b = orc.rpca_ialm(O, lam, mode="frsvt", p=5, q=1, seed=17, resid_check=True)
    assert b["converged"] and b["iters"] == a["iters"]
    assert np.all(b["widths"] == 4) and a["widths"].max() > 4
    assert np.linalg.norm(b["L"] - a["L"]) <= 1e-12 * np.linalg.norm(a["L"])
    assert np.linalg.norm(b["L"] - Lgt) <= 1e-12 * np.linalg.norm(Lgt)


def test_ialm_check_prunes_first_sketch_only(orc):
    """2000 x 200, 0.05 % outliers: the first sketch (l0 = 20) stops after 6
    samples; later iterations keep all p = 5 (the outliers keep the residual
    estimate above 1/mu); the solution is the unchecked run's."""
    from paper_1509_00296_amd import synth
    O, Lgt, _ = synth.rpca(seed=3, m=2000, n=200, rank=3, frac=0.0005)
    lam = 1.0 / math.sqrt(2000)
    a = orc.rpca_ialm(O, lam, mode="frsvt", p=5, q=1, seed=17)
    b = orc.rpca_ialm(O, lam, mode="frsvt", p=5, q=1, seed=17, resid_check=True)
    assert a["widths"][0] == 20 and b["widths"][0] == 6
    assert np.array_equal(a["widths"][1:], b["widths"][1:])
    assert b["iters"] == a["iters"] and np.array_equal(a["ranks"], b["ranks"])
    assert np.linalg.norm(b["L"] - a["L"]) <= 1e-12 * np.linalg.norm(a["L"])


def test_ialm_check_inactive_on_video_like_data(orc):
    from paper_1509_00296_amd import synth
    O, _, _ = synth.rpca(seed=3, m=3000, n=60, rank=3, frac=0.10)
    lam = 1.0 / math.sqrt(3000)
    a = orc.rpca_ialm(O, lam, mode="frsvt", p=5, q=1, seed=17)
    b = orc.rpca_ialm(O, lam, mode="frsvt", p=5, q=1, seed=17, resid_check=True)
    assert np.array_equal(a["widths"], b["widths"])
    assert np.array_equal(a["L"], b["L"]) and np.array_equal(a["S"], b["S"])
