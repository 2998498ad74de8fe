"""Pins for the oracle's dense factorizations (Householder QR, QR with column
pivoting, one-sided Jacobi SVD) against closed forms and library routines."""
import numpy as np
import pytest

from paper_1509_00296_amd.synth import haar


@pytest.mark.parametrize("m,n", [(7, 7), (40, 9), (300, 15), (5, 1)])
def test_qr_properties(orc, m, n):
    A = np.random.default_rng(m * n).standard_normal((m, n))
    Q, R = orc.qr(A)
    assert np.abs(Q.T @ Q - np.eye(n)).max() < 1e-14
    assert np.abs(np.tril(R, -1)).max() == 0.0
    assert np.linalg.norm(Q @ R - A) / np.linalg.norm(A) < 1e-14
    # unique up to column signs: compare with numpy's LAPACK QR
    Qn, Rn = np.linalg.qr(A)
    d = np.sign(np.diag(R)) * np.sign(np.diag(Rn))
    assert np.abs(Q * d - Qn).max() < 1e-12


def test_qr_rank_deficient_stays_orthonormal(orc):
    rng = np.random.default_rng(0)
    A = rng.standard_normal((50, 3)) @ rng.standard_normal((3, 8))
    A[:, 5] = 0.0
    Q, R = orc.qr(A)
    assert np.abs(Q.T @ Q - np.eye(8)).max() < 1e-13
    assert np.linalg.norm(Q @ R - A) / np.linalg.norm(A) < 1e-14


def test_qrcp_rank_and_range(orc):
    rng = np.random.default_rng(1)
    A = rng.standard_normal((60, 4)) @ rng.standard_normal((4, 12))
    Q = orc.qrcp_basis(A)
    assert Q.shape == (60, 4)   # s = min(l, r) = 4
    assert np.abs(Q.T @ Q - np.eye(4)).max() < 1e-14
    assert np.linalg.norm(A - Q @ (Q.T @ A)) / np.linalg.norm(A) < 1e-13
    # full rank input keeps every column
    B = rng.standard_normal((60, 12))
    assert orc.qrcp_basis(B).shape == (60, 12)
    # pivoting: the first basis vector is the direction of the largest column
    C = np.zeros((6, 3))
    C[:, 0] = [1, 0, 0, 0, 0, 0]
    C[:, 1] = [0, 5, 0, 0, 0, 0]
    C[:, 2] = [0, 0, 2, 0, 0, 0]
    Qc = orc.qrcp_basis(C)
    assert abs(abs(Qc[1, 0]) - 1.0) < 1e-15


@pytest.mark.parametrize("m,n,k", [(80, 50, 50), (50, 80, 50), (200, 200, 200), (300, 40, 40)])
def test_svd_known_singular_values(orc, m, n, k):
    rng = np.random.default_rng(m + n)
    s = np.sort(rng.uniform(0.1, 10.0, k))[::-1]
    U0, V0 = haar(rng, m, k), haar(rng, n, k)
    A = (U0 * s) @ V0.T
    U, S, V, sweeps = orc.svd(A)
    assert 0 < sweeps < 1000
    # the input itself is formed with rounding of order k u ||A||
    assert np.abs(S - s).max() / s[0] < 1e-15 * k
    kk = min(m, n)
    assert np.abs(U.T @ U - np.eye(kk)).max() < 1e-13
    assert np.abs(V.T @ V - np.eye(kk)).max() < 1e-13
    assert np.linalg.norm(U @ np.diag(S) @ V.T - A) / np.linalg.norm(A) < 5e-16 * k
    # singular subspaces: U diag(S) matches up to signs since s is simple
    d = np.sign(np.sum(U[:, :k] * U0, axis=0))
    assert np.abs(U[:, :k] * d - U0).max() < 1e-10


def test_svd_closed_forms(orc):
    # 2 x 2: singular values of [[a, b], [0, c]] from the characteristic polynomial
    a, b, c = 3.0, 4.0, 2.0
    M = np.array([[a, b], [0.0, c]])
    t = a * a + b * b + c * c
    d = np.sqrt(t * t - 4 * (a * c) ** 2)
    ref = np.sqrt([(t + d) / 2, (t - d) / 2])
    assert np.allclose(orc.svd(M)[1], ref, rtol=1e-15, atol=0)
    # diagonal: |d_i| sorted
    D = np.diag([-1.5, 7.0, 0.0, 2.0])
    assert np.array_equal(orc.svd(D)[1], [7.0, 2.0, 1.5, 0.0])
    # rank one a b^T: sigma_1 = |a| |b|, others zero
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal(30), rng.standard_normal(12)
    S = orc.svd(np.outer(x, y))[1]
    assert S[0] == pytest.approx(np.linalg.norm(x) * np.linalg.norm(y), rel=1e-14)
    assert np.abs(S[1:]).max() < 1e-13 * S[0]


def test_svd_vs_lapack(orc):
    rng = np.random.default_rng(5)
    for shape in [(33, 17), (17, 33), (64, 64)]:
        A = rng.standard_normal(shape)
        assert np.allclose(orc.svd(A)[1], np.linalg.svd(A, compute_uv=False), rtol=1e-13,
                           atol=1e-13)


def test_svd_zero_and_deficient_complete_bases(orc):
    Z = np.zeros((9, 4))
    U, S, V, _ = orc.svd(Z)
    assert np.all(S == 0)
    assert np.abs(U.T @ U - np.eye(4)).max() < 1e-15
    assert np.abs(V.T @ V - np.eye(4)).max() < 1e-15


def test_openmp_build_matches_plain_build(orc):
    """The all-core CPU baseline runs the oracle's source built with -fopenmp:
    its parallel loops split independent output columns, so every value is
    computed in the same order and the results equal the plain build's."""
    import math
    from paper_1509_00296_amd import synth
    O, _, _ = synth.rpca(seed=4, m=2000, n=60, rank=3, frac=0.1)
    lam = 1.0 / math.sqrt(2000)
    a = orc.rpca_ialm(O, lam, mode="frsvt", max_iter=4, seed=5)
    A = np.asfortranarray(np.random.default_rng(2).standard_normal((300, 120)))
    Xa, ra = orc.svt(A, 3.0)
    with orc.use_library(orc.build_openmp()):
        assert orc.threads() >= 1
        b = orc.rpca_ialm(O, lam, mode="frsvt", max_iter=4, seed=5)
        Xb, rb = orc.svt(A, 3.0)
    assert np.array_equal(a["L"], b["L"]) and np.array_equal(a["S"], b["S"])
    assert ra == rb and np.array_equal(Xa, Xb)
