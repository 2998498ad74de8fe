"""Pins of the oracle's unrolled inexact-ALM pieces (the S- and multiplier
updates with free thresholds, and the unrolled loop), against special cases
whose values follow from the definitions alone and against the oracle's
pinned iALM with exact SVT."""
import numpy as np
import pytest


def test_shrink_matches_definition(orc):
    v = np.array([-3.0, -1.0, -0.5, 0.0, 0.5, 1.0, 3.0])
    assert np.array_equal(orc.shrink(v, 1.0), [-2.0, 0.0, 0.0, 0.0, 0.0, 0.0, 2.0])


def test_dual_step_special_cases(orc):
    rng = np.random.default_rng(3)
    O, L, Y = (rng.standard_normal((7, 5)) for _ in range(3))
    mu, mun = 0.8, 1.2
    # lam = 0: S = O - L + Y/mu, so O - L - S = -Y/mu and the multiplier vanishes
    S, Yn, An = orc.dual_step(O, L, Y, 0.0, mu, mun)
    assert np.allclose(S, O - L + Y / mu, atol=1e-15)
    assert np.abs(Yn).max() < 1e-14
    assert np.allclose(An, O - S, atol=1e-14)
    # lam above every |entry|: S = 0, Y_next = Y + mu (O - L)
    S, Yn, An = orc.dual_step(O, L, Y, 1e3, mu, mun)
    assert np.array_equal(S, np.zeros_like(S))
    assert np.allclose(Yn, Y + mu * (O - L), atol=1e-14)
    assert np.allclose(An, O + Yn / mun, atol=1e-14)


def test_unrolled_with_full_basis_is_exact_ialm(orc):
    """With l = mhat the FRSVT range is the whole short side, so FRSVT is exact
    SVT; with tau_t = 1/mu_t and lam_t = lam/mu_t the unrolled steps are the
    plain iALM iterations."""
    rng = np.random.default_rng(11)
    m, n, r = 40, 24, 2
    O = rng.uniform(size=(m, r)) @ rng.uniform(size=(r, n))
    mask = rng.uniform(size=(m, n)) < 0.05
    O[mask] += rng.uniform(-1, 1, size=mask.sum())
    lam = 1.0 / np.sqrt(m)
    T = 6
    norm2 = orc.svd(O)[1][0]
    mu0 = 1.25 / norm2
    mus = [mu0 * 1.5 ** t for t in range(T)]
    taus = [1.0 / mu for mu in mus]
    lams = [lam / mu for mu in mus]
    L_unr = orc.rpca_unrolled(O, taus, lams, k=n, p=0, q=1, seed=4, lam=lam)
    ref = orc.rpca_ialm(O, lam, mode="exact", tol=1e-300, max_iter=T)
    assert ref["iters"] == T
    assert np.linalg.norm(L_unr - ref["L"]) <= 1e-11 * np.linalg.norm(ref["L"])


def test_unrolled_fd_is_smooth_at_default_schedule(orc):
    """Central differences at h and h/2 agree to second order: the unrolled
    map is smooth at these thresholds (no singular value or entry at a kink)."""
    rng = np.random.default_rng(5)
    m, n = 36, 20
    O = rng.uniform(size=(m, 3)) @ rng.uniform(size=(3, n))
    O[rng.uniform(size=(m, n)) < 0.05] += 0.7
    lam = 1.0 / np.sqrt(m)
    norm2 = orc.svd(O)[1][0]
    mus = [1.25 / norm2 * 1.5 ** t for t in range(4)]
    taus = np.array([1.0 / mu for mu in mus])
    lams = np.array([lam / mu for mu in mus])
    W = rng.standard_normal((m, n))
    f = lambda tt: np.sum(W * orc.rpca_unrolled(O, tt, lams, k=3, p=3, q=1, seed=2, lam=lam,
                                                 norm2=norm2))
    e = np.zeros(4)
    e[1] = 1.0
    d1 = (f(taus + 1e-4 * e) - f(taus - 1e-4 * e)) / 2e-4
    d2 = (f(taus + 5e-5 * e) - f(taus - 5e-5 * e)) / 1e-4
    assert abs(d1 - d2) <= 1e-6 * max(1.0, abs(d1))
