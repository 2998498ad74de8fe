"""Pins of the oracle's tensor host (Type C of Table 6 with the alignment
fixed to the identity): the unfolding convention by brute force, the
optimality conditions that each step of the inexact ALM meets exactly, the
reduction to matrix RPCA when all weight sits on one mode, and exact
recovery of a low-multilinear-rank tensor from sparse corruption."""
import numpy as np
import pytest

import oracle as orc
from paper_1509_00296_amd import synth


def test_unfold_matches_index_formula_and_folds_back():
    rng = np.random.default_rng(0)
    I1, I2, I3 = 3, 4, 5
    T = np.asfortranarray(rng.standard_normal((I1, I2, I3)))
    M = [orc.unfold(T, i) for i in range(3)]
    assert [m.shape for m in M] == [(I1, I2 * I3), (I2, I1 * I3), (I3, I1 * I2)]
    for a in range(I1):
        for b in range(I2):
            for c in range(I3):
                assert M[0][a, b + I2 * c] == T[a, b, c]
                assert M[1][b, a + I1 * c] == T[a, b, c]
                assert M[2][c, a + I1 * b] == T[a, b, c]
    for i in range(3):
        assert np.array_equal(orc.fold(M[i], i, T.shape), T)


def _data(seed=1, shape=(12, 10, 50), ranks=(2, 2, 3)):
    O, L, S = synth.tensor_lowrank(seed, shape, ranks, 0.05)
    lam = 1.0 / np.sqrt(max(shape[0] * shape[1], shape[2]))
    return O, L, S, lam


@pytest.mark.parametrize("alpha", [(1 / 3, 1 / 3, 1 / 3), (0.15, 0.15, 0.7)])
def test_each_step_meets_its_optimality_condition(alpha):
    """After K iterations and one more: the L_i step is the proximal map of
    alpha_i ||.||_* on unfolding i, so Y_i + mu (O - E - L_i) (with the
    previous E and mu) lies in alpha_i times the nuclear norm's
    subdifferential at L_i(i): spectral norm <= alpha_i and inner product
    alpha_i ||L_i(i)||_*.  The E step makes sum_i Y_i (updated) a
    subgradient of lam ||.||_1 at E: |.| <= lam, = lam sgn(E) on E's support."""
    O, _, _, lam = _data()
    K = 6
    a = orc.tensor_rpca(O, alpha, lam, max_iter=K)
    b = orc.tensor_rpca(O, alpha, lam, max_iter=K + 1)
    assert a["iters"] == K and b["iters"] == K + 1
    mu = a["mu0"] * 1.5 ** K
    for i in range(3):
        Li = orc.unfold(b["Ls"][i], i)
        G = orc.unfold(a["Y"][i] + mu * (O - a["E"] - b["Ls"][i]), i)
        s = np.linalg.svd(G, compute_uv=False)
        nuc = np.linalg.svd(Li, compute_uv=False).sum()
        assert s[0] <= alpha[i] * (1 + 1e-9)
        assert abs(np.sum(G * Li) - alpha[i] * nuc) <= 1e-9 * max(1.0, alpha[i] * nuc)
        assert nuc > 0
    W = b["Y"][0] + b["Y"][1] + b["Y"][2]
    supp = b["E"] != 0
    assert supp.sum() > 0 and (~supp).sum() > 0
    assert np.abs(W).max() <= lam * (1 + 1e-9)
    assert np.allclose(W[supp], lam * np.sign(b["E"][supp]), rtol=1e-9, atol=0)


def test_all_weight_on_one_mode_is_matrix_rpca_of_its_unfolding():
    """alpha = (1, 0, 0): L_2 and L_3 are free copies, so the optimum is the
    RPCA solution of the mode-1 unfolding with the same lam.  The two are
    different inexact ALMs that stop at feasibility; each lands within
    O(rho - 1) of the minimiser, so both run with slow growth rho = 1.02
    (at rho = 1.1 they differ by 3e-4, at 1.02 by 2e-5)."""
    O, _, _, lam = _data(seed=2, shape=(10, 6, 40))
    t = orc.tensor_rpca(O, (1.0, 0.0, 0.0), lam, tol=1e-11, max_iter=3000, rho=1.02)
    assert t["converged"]
    r = orc.rpca_ialm(orc.unfold(O, 0), lam, mode="exact", tol=1e-11, max_iter=3000, rho=1.02,
                      mu_bar_factor=1e12)
    Lm = orc.fold(r["L"], 0, O.shape)
    assert np.linalg.norm(t["L"] - Lm) / np.linalg.norm(Lm) < 1e-4
    Sm = orc.fold(r["S"], 0, O.shape)
    assert np.linalg.norm(t["E"] - Sm) / np.linalg.norm(Sm) < 2e-3


@pytest.mark.parametrize("mode", ["exact", "frsvt"])
def test_exact_recovery_of_low_multilinear_rank(mode):
    O, L, S, lam = _data()
    out = orc.tensor_rpca(O, (0.15, 0.15, 0.7), lam, mode=mode, max_iter=100)
    assert out["converged"]
    assert list(out["ranks"][-1]) == [2, 2, 3]
    assert np.linalg.norm(out["L"] - L) / np.linalg.norm(L) < 1e-6
    assert np.linalg.norm(out["E"] - S) / np.linalg.norm(S) < 1e-5
    for i in range(3):
        assert np.linalg.norm(out["Ls"][i] - out["L"]) / np.linalg.norm(L) < 1e-6


def test_frsvt_mode_agrees_with_exact_mode():
    O, _, _, lam = _data(seed=3)
    ex = orc.tensor_rpca(O, (1 / 3, 1 / 3, 1 / 3), lam, mode="exact", tol=1e-9)
    fr = orc.tensor_rpca(O, (1 / 3, 1 / 3, 1 / 3), lam, mode="frsvt", tol=1e-9)
    assert ex["converged"] and fr["converged"]
    assert np.linalg.norm(fr["L"] - ex["L"]) / np.linalg.norm(ex["L"]) < 1e-7
