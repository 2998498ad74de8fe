"""GPU parity of the large (matrix-core) path and of the precision form.

* FP64 large path (l > 32 or a wide short side): matrix-core f64 GEMMs,
  multi-kernel CholeskyQR, Jacobi of a 110 x 110 core -- against the oracle
  at <= 1e-10.
* Precision form (FRSVT_MIXED_BF16): bfloat16 sketch/power products with
  float accumulation, float projection and reconstruction, double
  Gram/Cholesky/small SVD.  Compared with the FP64 oracle fed the same
  bfloat16-rounded Omega; the total relative error and the error inside the
  signal subspace are checked against the bounds stated here (derivation in
  the design notes: total <= 5e-2, signal <= 2e-3 at these spectra).
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


def _signal_error(Xg, Xo, A, edge):
    """Error of Xg against Xo inside the oracle's singular subspace of the
    directions whose singular value in A exceeds the noise edge."""
    u, s, vt = np.linalg.svd(Xo, full_matrices=False)
    sa = np.linalg.svd(A, compute_uv=False)
    ks = int(np.sum(sa > edge))
    U, V = u[:, :ks], vt[:ks].T
    D = U.T @ (Xg - Xo) @ V
    return np.linalg.norm(D) / np.linalg.norm(Xo), ks


@pytest.mark.parametrize("n", [2048])
def test_frsvt_mixed_bf16_error_bounds(fr, orc, n):
    from paper_1509_00296_amd import synth
    _say(f"case frsvt mixed bf16 {n}x{n} l=110 q=2")
    A = synth.precision(seed=1, n=n, rank=100, noise_std=0.1)
    tau, k, p, q, seed = 5.0, 100, 10, 2, 31
    X32, _, r32 = fr.frsvt(torch.from_numpy(A.astype(np.float32)).cuda(), tau, k, p, q,
                           seed=seed, counter=0)
    # the precision form through the same entry point
    import ctypes
    lib = fr.library()
    h = fr.handle(0)
    Af = torch.from_numpy(A.astype(np.float32)).cuda()
    Xm = torch.empty((n, n), dtype=torch.float32, device="cuda").t()
    Qo_buf = torch.empty((110, n), dtype=torch.float32, device="cuda").t()
    r = ctypes.c_int32()
    rc = lib.frsvt(h.ptr, fr.MIXED_BF16, n, n, Af.data_ptr(), n, tau, k, p, q, None, 0, n, seed, 0,
                   Xm.data_ptr(), n, Qo_buf.data_ptr(), n, ctypes.byref(r))
    assert rc == 0
    Om = bf16_round(orc.gaussian_matrix(seed, 0, n, k + p))
    Xo, _, ro, sig, _ = orc.frsvt(A, tau, q, Om)
    tot = _rel(Xm.double().cpu().numpy(), Xo)
    edge = 2 * 0.1 * np.sqrt(n)
    sig_err, ks = _signal_error(Xm.double().cpu().numpy(), Xo, A, edge)
    _say(f"mixed: r={r.value} oracle r={ro} total rel err {tot:.3e} signal ({ks} dirs) {sig_err:.3e}")
    assert abs(r.value - ro) <= 2
    assert tot <= 5e-2
    assert sig_err <= 2e-3
    # the all-float run of the same call, for comparison
    Om64 = orc.gaussian_matrix(seed, 0, n, k + p)
    Xo64, _, _, _, _ = orc.frsvt(A, tau, q, Om64)
    tot32 = _rel(X32.double().cpu().numpy(), Xo64)
    _say(f"float run: total rel err {tot32:.3e}")
    assert tot32 <= 5e-3


@pytest.fixture(scope="module")
def c3_data():
    from paper_1509_00296_amd import synth
    return synth.precision(seed=0, n=8192, rank=100, noise_std=0.1)


def test_precision_workload_full_size(fr, orc, c3_data):
    """8192 x 8192, rank 100 (s_i = 1000 0.95^i), noise 0.1, tau = 5,
    k = 100, p = 10, q = 2: the all-FP64 GPU run matches the oracle to
    1e-10; the precision form stays inside the stated bounds against the
    oracle fed the same bfloat16-rounded Omega."""
    import ctypes
    A = c3_data
    n, tau, k, p, q, seed = 8192, 5.0, 100, 10, 2, 1000
    _say("case precision workload 8192x8192: GPU runs")
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
    _say("case precision workload: oracle (FP64, two runs of about a minute)")
    Om = orc.gaussian_matrix(seed, 0, n, k + p)
    Xo, _, ro, _, _ = orc.frsvt(A, tau, q, Om)
    assert r64 == ro
    e64 = _rel(X64, Xo)
    Xob, _, rob, _, _ = orc.frsvt(A, tau, q, bf16_round(Om))
    tot = _rel(Xm, Xob)
    _say(f"precision workload: FP64 GPU vs oracle {e64:.3e}; mixed vs oracle(bf16 Omega) {tot:.3e}, "
         f"r mixed {r.value} oracle {rob}")
    assert e64 <= 1e-10
    assert tot <= 5e-2
