"""FP32 RPCA (the float32 form of the video workload) against the FP64 oracle.

The oracle runs in FP64 on the same float32 input (widened exactly), with
the same Gaussian test matrices.  FP32 storage rounds every iterate to
u32 = 2^-24 relative, so the comparison bar is derived from that unit, not
from the FP64 bar:

* iterates: per iteration the rounding of A, Y, L and S adds a few u32 of
  ||O||; the thresholding and shrinkage steps are non-expansive and the
  multiplier term Y/mu is divided by rho = 1.5 each iteration, so the
  accumulated deviation stays below about 3 rho/(rho - 1) u32 ||O|| =
  9 u32 ||O|| -> relative L error <= 16 u32 = 9.5e-7 (bound 1e-6), and the
  S error, measured against ||S|| ~ ||L|| / 4.6 at these data, <= 5e-6;
* the stopping test: the FP32 residual ||O - L - S||_F / ||O||_F has a
  rounding floor of a few 1e-8, close to tol = 1e-7, so the FP32 run may
  need more iterations than the FP64 one (it stays on the floor for a few
  iterations before it dips below tol).  The ranks agree over the oracle's
  iterations; the FP32 run must still reach tol within 60 iterations and
  report a residual below it.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U32 = 2.0 ** -24


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


def _check(res, out, Lgt, it_slack):
    _say(f"  iters gpu {res.iters} oracle {out['iters']}, residual gpu {res.residual:.3e}")
    assert res.converged and res.residual < 1e-7
    assert out["iters"] <= res.iters <= out["iters"] + it_slack
    k = out["iters"]
    assert res.ranks[:k] == list(out["ranks"][:k])
    L = res.L.cpu().numpy().astype(np.float64)
    S = res.S.cpu().numpy().astype(np.float64)
    eL, eS = _rel(L, out["L"]), _rel(S, out["S"])
    _say(f"  rel L {eL:.3e} ({eL / U32:.1f} u32), rel S {eS:.3e}")
    assert eL <= 1e-6
    assert eS <= 5e-6
    assert _rel(L, Lgt) <= 1e-6


@pytest.mark.parametrize("m,n", [(3000, 60), (60, 3000)])
def test_rpca_f32_frsvt_matches_oracle(fr, orc, m, n):
    from paper_1509_00296_amd import synth
    _say(f"case rpca f32 frsvt {m}x{n}")
    O, Lgt, _ = synth.rpca(seed=3, m=m, n=n, rank=3, frac=0.10)
    O32 = np.asfortranarray(O.astype(np.float32))
    lam = 1.0 / np.sqrt(max(m, n))
    res = fr.rpca_ialm(torch.from_numpy(O32).cuda(), lam, use_frsvt=True, seed=2024)
    out = orc.rpca_ialm(O32.astype(np.float64), lam, mode="frsvt", p=5, q=1, seed=2024)
    assert res.widths[:out["iters"]] == list(out["widths"][:out["iters"]])
    _check(res, out, Lgt, it_slack=4)


def test_rpca_f32_exact_svt_matches_oracle(fr, orc):
    """Exact SVT in the loop, FP32: the residual sits on its rounding floor
    just above tol for several iterations (S21) before it dips below."""
    from paper_1509_00296_amd import synth
    _say("case rpca f32 exact 3000x60")
    O, Lgt, _ = synth.rpca(seed=3, m=3000, n=60, rank=3, frac=0.10)
    O32 = np.asfortranarray(O.astype(np.float32))
    lam = 1.0 / np.sqrt(3000)
    res = fr.rpca_ialm(torch.from_numpy(O32).cuda(), lam, use_frsvt=False)
    out = orc.rpca_ialm(O32.astype(np.float64), lam, mode="exact")
    _check(res, out, Lgt, it_slack=32)


def test_rpca_f32_video_shape_matches_oracle(fr, orc):
    """The full 76800 x 200 workload in FP32 against the FP64 oracle run on
    the same float32 input (the oracle takes about a minute)."""
    from paper_1509_00296_amd import synth
    _say("case rpca f32 76800x200")
    O, Lgt, _ = synth.rpca(seed=0)
    O32 = np.asfortranarray(O.astype(np.float32))
    lam = 1.0 / np.sqrt(76800)
    res = fr.rpca_ialm(torch.from_numpy(O32).cuda(), lam, use_frsvt=True, seed=2024)
    out = orc.rpca_ialm(O32.astype(np.float64), lam, mode="frsvt", p=5, q=1, seed=2024)
    assert res.widths[:out["iters"]] == list(out["widths"][:out["iters"]])
    _check(res, out, Lgt, it_slack=4)
