"""Low-rank representation (Type A of Table 6) on the GPU against the oracle:
the same iteration count and final rank, Z and E within 1e-10 (clean data,
both J-step modes; corrupted data with FRSVT in the J step, the method of
the paper).

One case keeps a looser bar, for a reason that lies in the exact-SVT
comparator, not in the LRR loop: the library's exact SVT takes the singular
values from the Gram matrix A A^T (Cholesky, then one-sided Jacobi on the
factor), which resolves them down to about sqrt(4 l u) sigma_1 (1.5e-7
sigma_1 at l = 60; smaller pivots of the semidefinite Cholesky are zero).
On corrupted data the late J inputs of the exact loop hold a singular value
between the threshold 1/mu (down to 1e-10) and that resolution: the oracle's
Jacobi SVD of the matrix itself keeps it (final rank 14), the Gram route
drops it (13), and Z moves by about its size (measured 2.1e-8), hence 1e-7
there.  The FRSVT J step meets the same data at 4.9e-12 (its small SVD
works on the l x l core, whose spectrum stays above the resolution).
Measured (GPU vs oracle, relative Frobenius): clean 1.4e-14 (exact) and
2.6e-14 (FRSVT); corrupted 4.9e-12 (FRSVT).  The LRR loop itself is well
conditioned: the oracle's own Z moves by 1e-14 (clean) and 2e-12
(corrupted) under a 1e-15 relative perturbation of X."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_00296_amd as m
    return m


@pytest.fixture(scope="module")
def orc():
    import oracle
    return oracle


def _say(msg):
    print(msg, flush=True)


def _subspaces(seed, d=80, K=3, dim=4, N=20):
    rng = np.random.default_rng(seed)
    blocks = []
    for _ in range(K):
        U, _ = np.linalg.qr(rng.standard_normal((d, dim)))
        blocks.append(U @ rng.standard_normal((dim, N)))
    return np.hstack(blocks), rng


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.mark.parametrize("mode,corrupt", [("exact", False), ("frsvt", False), ("exact", True), ("frsvt", True)])
def test_lrr_matches_oracle(fr, orc, mode, corrupt):
    X, rng = _subspaces(2 if corrupt else 1)
    lam = 100.0
    if corrupt:
        bad = rng.choice(60, 6, replace=False)
        X[:, bad] += 3.0 * rng.standard_normal((80, 6))
        lam = 0.1
    _say(f"case lrr {mode} corrupt={corrupt} 80x60")
    Xd = torch.from_numpy(np.asfortranarray(X)).cuda()
    res = fr.lrr_ialm(Xd, lam, use_frsvt=(mode == "frsvt"), p=5, q=1, seed=3, max_iter=1000)
    out = orc.lrr_ialm(X, lam, mode=mode, p=5, q=1, seed=3, max_iter=1000)
    assert res.converged and out["converged"]
    assert res.iters == out["iters"]
    Zg = res.Z.cpu().numpy()
    Eg = res.E.cpu().numpy()
    # the exact-SVT comparator on corrupted data: see the module docstring
    tol = 1e-7 if (corrupt and mode == "exact") else 1e-10
    assert _rel(Zg, out["Z"]) <= tol
    assert _rel(Eg, out["E"]) <= tol or np.abs(out["E"]).max() < 1e-12
    # the GPU's own result meets the equality constraint X = XZ + E to the
    # stopping tolerance (its dual residual Z - J is not observable here)
    assert np.abs(X - X @ Zg - Eg).max() < 1e-8
    # The final J-step rank counts singular values above 1/mu_max = 1e-10;
    # those below the stopping tolerance's scale (~1e-8) are rounding-level
    # and may fall either side of it.  What is unique is the rank of Z above
    # that noise; the reported ranks may differ only by values inside it.
    so = np.linalg.svd(out["Z"], compute_uv=False)
    sg = np.linalg.svd(Zg, compute_uv=False)
    r_robust = int((so > 1e-4 * so[0]).sum())
    assert r_robust == int((sg > 1e-4 * sg[0]).sum())
    noise = int(((so > 1e-12) & (so <= 1e-6)).sum())
    assert r_robust <= res.rank and abs(res.rank - int(out["ranks"][-1])) <= noise
    if not corrupt:
        assert res.rank == out["ranks"][-1] == 12


def test_lrr_iteration_limit(fr, orc):
    """A run stopped by the iteration limit (200 iterations, threshold 1/mu
    near 5e-3, rank settled at 11): the same partial iterate."""
    X, rng = _subspaces(2)
    bad = rng.choice(60, 6, replace=False)
    X[:, bad] += 3.0 * rng.standard_normal((80, 6))
    _say("case lrr frsvt limit 80x60")
    res = fr.lrr_ialm(torch.from_numpy(np.asfortranarray(X)).cuda(), 0.1, p=5, q=1, seed=3, max_iter=200)
    out = orc.lrr_ialm(X, 0.1, mode="frsvt", p=5, q=1, seed=3, max_iter=200)
    assert not res.converged and not out["converged"] and res.iters == out["iters"] == 200
    assert res.rank == out["ranks"][-1] == 11
    assert _rel(res.Z.cpu().numpy(), out["Z"]) <= 1e-10
    assert _rel(res.E.cpu().numpy(), out["E"]) <= 1e-10


def test_lrr_zero_data(fr):
    """X = 0: Z = E = 0 after one iteration (both residuals vanish)."""
    _say("case lrr zero")
    X = torch.zeros((30, 20), dtype=torch.float64, device="cuda")
    res = fr.lrr_ialm(X, 0.1)
    assert res.converged and res.iters == 1 and res.rank == 0
    assert float(res.Z.abs().max()) == 0.0 and float(res.E.abs().max()) == 0.0


def test_lrr_full_workload_matches_oracle_summary(fr):
    """The 2016 x 640 workload bench.py times (10 nine-dimensional subspaces,
    64 corrupted columns, lambda = 0.1, FRSVT J step, p = 5, q = 1, seed 11)
    against the oracle's full run, stored as a summary by
    tests/golden/make_lrr_golden.py (the oracle takes minutes): the same
    iteration count and rank sequence, the Frobenius norms and the top 100
    singular values of Z within 1e-10, and 400 fixed entries of Z and of E
    within 1e-10 of the respective Frobenius norm."""
    import json
    import os
    from paper_1509_00296_amd import synth
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "lrr_2016x640_seed0.json")
    g = json.load(open(path))
    _say("case lrr 2016x640 full workload")
    X, _, _ = synth.subspaces(seed=0)
    res = fr.lrr_ialm(torch.from_numpy(X).cuda(), 0.1, use_frsvt=True, p=5, q=1, seed=11)
    assert res.converged == g["converged"] and res.iters == g["iters"]
    assert res.rank == g["ranks"][-1]
    Z = res.Z.cpu().numpy()
    E = res.E.cpu().numpy()
    assert abs(np.linalg.norm(Z) - g["Z_fro"]) <= 1e-10 * g["Z_fro"]
    assert abs(np.linalg.norm(E) - g["E_fro"]) <= 1e-10 * g["E_fro"]
    sz = np.linalg.svd(Z, compute_uv=False)[:100]
    so = np.array(g["Z_sigma_top100"])
    assert np.abs(sz - so).max() <= 1e-10 * so[0]
    dz = max(abs(Z[i, j] - v) for i, j, v in g["Z_samples"])
    de = max(abs(E[i, j] - v) for i, j, v in g["E_samples"])
    _say(f"  max sample deviation Z {dz:.2e}, E {de:.2e}")
    assert dz <= 1e-10 * g["Z_fro"]
    assert de <= 1e-10 * g["E_fro"]
