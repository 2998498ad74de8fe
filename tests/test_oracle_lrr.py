"""Low-rank representation (Type A of Table 6) in the oracle.

Pins: for data drawn from independent subspaces without corruption the LRR
problem's solution is the shape-interaction matrix Z = V V^T of the skinny
SVD X = U S V^T with E = 0 (the closed form of the LRR paper), which both
the exact-SVT and the FRSVT inexact ALM must reach; FRSVT with a sketch as
wide as the matrix is exact SVT, so on corrupted data it must reproduce the
exact-SVT run."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def orc():
    import oracle
    return oracle


def _subspaces(seed, d=80, K=3, dim=4, N=20):
    rng = np.random.default_rng(seed)
    blocks = []
    for _ in range(K):
        U, _ = np.linalg.qr(rng.standard_normal((d, dim)))
        blocks.append(U @ rng.standard_normal((dim, N)))
    return np.hstack(blocks), rng


@pytest.mark.parametrize("mode", ["exact", "frsvt"])
def test_lrr_clean_subspaces_closed_form(orc, mode):
    X, _ = _subspaces(1)
    out = orc.lrr_ialm(X, 100.0, mode=mode, p=5, q=1, seed=3)
    assert out["converged"]
    _, s, Vt = np.linalg.svd(X, full_matrices=False)
    r = int((s > 1e-9 * s[0]).sum())
    assert r == 12
    Zs = Vt[:r].T @ Vt[:r]
    assert np.linalg.norm(out["Z"] - Zs) / np.linalg.norm(Zs) < 1e-7
    assert np.abs(out["E"]).max() < 1e-8
    # block-diagonal: no affinity between samples of different subspaces
    off = np.ones((60, 60), bool)
    for k in range(3):
        off[20 * k:20 * k + 20, 20 * k:20 * k + 20] = False
    assert np.abs(out["Z"][off]).max() < 1e-7


def test_lrr_full_width_frsvt_is_exact(orc):
    X, rng = _subspaces(2)
    bad = rng.choice(60, 6, replace=False)
    X[:, bad] += 3.0 * rng.standard_normal((80, 6))
    ex = orc.lrr_ialm(X, 0.1, mode="exact", max_iter=400)
    fr = orc.lrr_ialm(X, 0.1, mode="frsvt", p=60, q=0, seed=5, max_iter=400)
    assert ex["converged"] and np.linalg.norm(ex["E"]) > 1.0
    assert ex["iters"] == fr["iters"]
    assert np.linalg.norm(fr["Z"] - ex["Z"]) / np.linalg.norm(ex["Z"]) < 1e-8
    assert np.linalg.norm(fr["E"] - ex["E"]) / np.linalg.norm(ex["E"]) < 1e-8
