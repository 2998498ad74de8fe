"""GPU parity of the large (matrix-core) path and of the precision form.

* FP64 large path (l > 32 or a wide short side): matrix-core f64 GEMMs,
  multi-kernel CholeskyQR, Jacobi of a 110 x 110 core -- against the oracle
  at <= 1e-10.
* Precision form (FRSVT_MIXED_BF16): bfloat16 sketch/power products with
  float accumulation, float projection and reconstruction, double
  Gram/Cholesky/small SVD.  Compared with the FP64 oracle fed the same
  bfloat16-rounded Omega; the total relative error and the error inside the
  signal subspace are checked against first-order bounds derived from the
  bfloat16 rounding of A and of the product operands (derivation in
  test_precision_workload_full_size), and the rank must be the oracle's.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_00296_amd as fr
    fr.handle(0)
    return fr


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build()
    return oracle


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def bf16_round(x):
    """float64 -> float32 -> bfloat16 (round to nearest even) -> float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("m,n,k,p,q", [(1200, 700, 100, 10, 2), (700, 1200, 40, 8, 1),
                                       (900, 900, 60, 10, 0)])
def test_frsvt_f64_large_path(fr, orc, m, n, k, p, q):
    from paper_1509_00296_amd import synth
    _say(f"case frsvt f64 large path {m}x{n} l={k + p} q={q}")
    A = synth.single_svt(seed=m + n, m=m, n=n, rank=k, noise_std=0.05, smax=200.0, smin=5.0)
    X, Qt, r = fr.frsvt(torch.from_numpy(A).cuda(), 2.0, k, p, q, seed=7, counter=1)
    Om = orc.gaussian_matrix(7, 1, max(m, n), k + p)
    Xo, Qo, ro, _, _ = orc.frsvt(A, 2.0, q, Om)
    assert r == ro
    assert _rel(X.cpu().numpy(), Xo) <= 1e-10
    Qg = Qt.cpu().numpy()
    assert np.abs(Qg.T @ Qg - np.eye(r)).max() < 1e-12


@pytest.mark.parametrize("n", [2048])
def test_frsvt_mixed_bf16_error_bounds(fr, orc, n):
    """The precision form at 2048 x 2048 (same spectrum as the 8192 workload,
    tau = 5, l = 110, q = 2) against the FP64 oracle fed the same
    bfloat16-rounded Omega, with the first-order bounds of the full-size test
    below; the all-float run of the same call against the FP64 oracle."""
    from paper_1509_00296_amd import synth
    _say(f"case frsvt mixed bf16 {n}x{n} l=110 q=2")
    A = synth.precision(seed=1, n=n, rank=100, noise_std=0.1)
    tau, k, p, q, seed = 5.0, 100, 10, 2, 31
    X32, _, r32 = fr.frsvt(torch.from_numpy(A.astype(np.float32)).cuda(), tau, k, p, q,
                           seed=seed, counter=0)
    _mixed_against_oracle(fr, orc, A, tau, k, p, q, seed)
    # the all-float run of the same call: float32 rounding of A, of the
    # products and of the reconstruction, u32 times the spread of the signal
    Om64 = orc.gaussian_matrix(seed, 0, n, k + p)
    Xo64, _, _, _, _ = orc.frsvt(A, tau, q, Om64)
    tot32 = _rel(X32.double().cpu().numpy(), Xo64)
    _say(f"float run: total rel err {tot32:.3e}")
    assert tot32 <= 5e-3


@pytest.fixture(scope="module")
def c3_data():
    from paper_1509_00296_amd import synth
    return synth.precision(seed=0, n=8192, rank=100, noise_std=0.1)


def _bf16_error_norm(A, iters=30):
    """||bf16(A) - A||_2 by power iteration on the CPU (the rounding error
    the bfloat16 products see in A)."""
    E = bf16_round(A) - A
    x = np.random.default_rng(0).standard_normal(A.shape[1])
    for _ in range(iters):
        y = E.T @ (E @ x)
        x = y / np.linalg.norm(y)
    return float(np.sqrt(np.linalg.norm(E.T @ (E @ x))))


def _mixed_against_oracle(fr, orc, A, tau, k, p, q, seed, fp64_check=False):
    """The precision form of FRSVT (and optionally the all-FP64 GPU run)
    against the oracle fed the same bfloat16-rounded Omega, with the
    first-order bounds derived in test_precision_workload_full_size."""
    import ctypes
    n = A.shape[0]
    if fp64_check:
        X64, _, r64 = fr.frsvt(torch.from_numpy(A).cuda(), tau, k, p, q, seed=seed, counter=0)
        X64 = X64.cpu().numpy()
    lib, h = fr.library(), fr.handle(0)
    Af = torch.from_numpy(A.astype(np.float32)).cuda()
    Xm = torch.empty((n, n), dtype=torch.float32, device="cuda").t()
    r = ctypes.c_int32()
    rc = lib.frsvt(h.ptr, fr.MIXED_BF16, n, n, Af.data_ptr(), n, tau, k, p, q, None, 0, n, seed, 0,
                   Xm.data_ptr(), n, None, n, ctypes.byref(r))
    assert rc == 0
    Xm = Xm.double().cpu().numpy()
    del Af
    _say(f"  oracle runs at {n}x{n}")
    Om = orc.gaussian_matrix(seed, 0, n, k + p)
    if fp64_check:
        Xo, _, ro, _, _ = orc.frsvt(A, tau, q, Om)
        assert r64 == ro
        e64 = _rel(X64, Xo)
        _say(f"  FP64 GPU vs oracle {e64:.3e}")
        assert e64 <= 1e-10
    Xob, Qob, rob, sob, _ = orc.frsvt(A, tau, q, bf16_round(Om))
    tot = _rel(Xm, Xob)
    # the signal subspace: the oracle's left singular vectors of X whose
    # singular value of B lies above the noise edge; V_s = X^T U_s / f_s
    edge = 2 * 0.1 * np.sqrt(n)
    ks = int(np.sum(sob > edge))
    Us = Qob[:, :ks]
    fs = sob[:ks] - tau
    Vs = (Xob.T @ Us) / fs
    sig_err = np.linalg.norm(Us.T @ (Xm - Xob) @ Vs) / np.linalg.norm(Xob)
    # first-order predictions
    ub = 2.0 ** -8
    eps = _bf16_error_norm(A) + edge * ub
    xf = np.linalg.norm(Xob)
    pred_tot = np.sqrt(ks) * eps / xf
    pred_sig = float(np.sum((eps / sob[:ks]) ** 2 * sob[:ks])) / xf
    _say(f"  mixed vs oracle(bf16 Omega): total {tot:.3e} (first order {pred_tot:.3e}, ratio "
         f"{tot / pred_tot:.2f}), signal ({ks} directions) {sig_err:.3e} (first order {pred_sig:.3e}, "
         f"ratio {sig_err / pred_sig:.2f}); eps_A + sigma_b u_b = {eps:.3e}; r mixed {r.value} oracle {rob}")
    assert r.value == rob
    assert tot <= 3.0 * pred_tot
    assert sig_err <= 3.0 * pred_sig


def test_precision_workload_full_size(fr, orc, c3_data):
    """8192 x 8192, rank 100 (s_i = 1000 0.95^i), noise 0.1, tau = 5,
    k = 100, p = 10, q = 2: the all-FP64 GPU run matches the oracle to
    1e-10; the precision form is checked against the FP64 oracle fed the same
    bfloat16-rounded Omega with first-order bounds.

    First order: the bfloat16 products see A + E_A (E_A the rounding of A,
    eps_A = ||E_A||_2) and their operand Z = A^T Q rounded to u_b = 2^-8 of
    each entry; in the last power step the component of the basis direction
    j outside the signal subspace is then about (eps_A + sigma_b u_b) /
    sigma_j (sigma_b = 2 * 0.1 * sqrt(8192) ~ 18.1 the noise edge), and the
    thresholded result, 1-Lipschitz, moves by that angle times sigma_j - tau
    per signal direction: total error <= sqrt(ks) (eps_A + sigma_b u_b) /
    ||X||_F.  Inside the signal subspace (U_s^T (X~ - X) V_s) a rotation of
    angle a_j enters at second order, sum_j a_j^2 sigma_j.  The bounds below
    are those predictions times 3 (measured ratios to the predictions:
    total 0.78, signal 0.59 here; 0.43 and 0.22 at 2048 x 2048); the rank is
    the oracle's (every sampled direction lies above tau = 5)."""
    _say("case precision workload 8192x8192: GPU runs and the oracle (about two minutes)")
    _mixed_against_oracle(fr, orc, c3_data, 5.0, 100, 10, 2, 1000, fp64_check=True)


@pytest.mark.parametrize("m,n,k,p,q", [(1500, 900, 190, 10, 1), (900, 1400, 150, 6, 0)])
def test_frsvt_f64_wide_sketch(fr, orc, m, n, k, p, q):
    """Sketch widths between 128 and 256 columns: the Cholesky on its global
    workspace (sixteen wavefronts), the triangular solve and product with the
    wider LDS stride, against the oracle at <= 1e-10."""
    from paper_1509_00296_amd import synth
    _say(f"case frsvt f64 wide sketch {m}x{n} l={k + p} q={q}")
    A = synth.single_svt(seed=m + 3 * n, m=m, n=n, rank=k - 20, noise_std=0.05, smax=200.0, smin=5.0)
    X, Qt, r = fr.frsvt(torch.from_numpy(A).cuda(), 2.0, k, p, q, seed=11, counter=3)
    Om = orc.gaussian_matrix(11, 3, max(m, n), k + p)
    Xo, Qo, ro, _, _ = orc.frsvt(A, 2.0, q, Om)
    assert r == ro
    assert _rel(X.cpu().numpy(), Xo) <= 1e-10
    Qg = Qt.cpu().numpy()
    assert np.abs(Qg.T @ Qg - np.eye(r)).max() < 1e-12


def test_frsvt_width_above_256_rejected(fr):
    """A sketch wider than 256 columns (below the short side) is refused
    before any launch."""
    A = torch.zeros((1200, 600), dtype=torch.float64, device="cuda")
    with pytest.raises(fr.FRSVTError):
        fr.frsvt(A, 1.0, 290, 10, 1, seed=1)
