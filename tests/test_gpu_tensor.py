"""3-way tensor host (Type C of Table 6, alignment fixed) on the GPU against
the oracle: the same iteration count and per-mode ranks, L and E within
1e-10 (relative Frobenius), over shapes that put each unfolding's short side
on either index, both SVT forms, and the 32 x 22 x 3000 gait-sequence shape
(mode 3 on the large path)."""
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


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _check(fr, orc, O, alpha, lam, mode, **kw):
    Od = torch.from_numpy(O).cuda()
    res = fr.tensor_rpca(Od, alpha, lam, use_frsvt=(mode == "frsvt"), seed=5, **kw)
    out = orc.tensor_rpca(O, alpha, lam, mode=mode, seed=5, **kw)
    assert res.converged == out["converged"]
    assert res.iters == out["iters"]
    assert list(res.rank) == list(out["ranks"][-1])
    assert abs(res.mu0 - out["mu0"]) <= 1e-12 * out["mu0"]
    assert _rel(res.L.cpu().numpy(), out["L"]) <= 1e-10
    assert _rel(res.E.cpu().numpy(), out["E"]) <= 1e-10
    return res, out


# (shape, Tucker ranks, lambda * sqrt(max(I1 I2, I3)), alpha): the first has
# every unfolding wide, the second a tall mode-1 unfolding (short side I2 I3),
# the third a wide mode-3 unfolding (short side I3), the fourth frontal slices
# above 8192 values (the update pass deals them out element by element
# instead of one slice per workgroup); each recovers L
@pytest.mark.parametrize("shape,ranks,c,alpha", [((12, 10, 50), (2, 2, 3), 1.0, (0.15, 0.15, 0.7)),
                                                 ((60, 6, 8), (2, 2, 2), 2.0, (0.5, 0.25, 0.25)),
                                                 ((7, 33, 9), (2, 2, 2), 1.0, (0.15, 0.15, 0.7)),
                                                 ((100, 90, 3), (2, 2, 2), 2.0, (0.4, 0.4, 0.2))])
@pytest.mark.parametrize("mode", ["exact", "frsvt"])
def test_tensor_rpca_matches_oracle(fr, orc, shape, ranks, c, alpha, mode):
    from paper_1509_00296_amd import synth
    _say(f"case tensor {mode} {shape}")
    O, L, _ = synth.tensor_lowrank(4, shape, ranks, 0.05)
    lam = c / np.sqrt(max(shape[0] * shape[1], shape[2]))
    res, _ = _check(fr, orc, O, alpha, lam, mode)
    assert res.converged and list(res.rank) == list(ranks)
    assert _rel(res.L.cpu().numpy(), L) < 1e-6


def test_tensor_rpca_iteration_limit_and_weights(fr, orc):
    """Unequal weights, a zero weight (that mode's SVT keeps everything) and
    a run stopped by the iteration limit."""
    from paper_1509_00296_amd import synth
    _say("case tensor limit/weights")
    O, _, _ = synth.tensor_lowrank(6, (10, 8, 30), (2, 2, 2), 0.05)
    res, out = _check(fr, orc, O, (0.0, 0.4, 0.6), 0.05, "exact", max_iter=7)
    assert res.iters == 7 and not res.converged


def test_tensor_rpca_gait_shape(fr, orc):
    from paper_1509_00296_amd import synth
    _say("case tensor frsvt 32x22x3000")
    O, L, _ = synth.tensor_lowrank(0)
    lam = 0.5 / np.sqrt(32 * 22)
    res, out = _check(fr, orc, O, (0.15, 0.15, 0.7), lam, "frsvt")
    assert res.converged and list(res.rank) == [3, 3, 5]
    assert _rel(res.L.cpu().numpy(), L) < 1e-6


def test_tensor_rpca_zero_tensor(fr):
    """O = 0: the minimiser is L = E = 0, returned without iterating."""
    _say("case tensor zero")
    O = torch.zeros((5, 4, 6), dtype=torch.float64, device="cuda")
    res = fr.tensor_rpca(O, (0.3, 0.3, 0.4), 0.1)
    assert res.converged and res.iters == 0
    assert float(res.L.abs().max()) == 0.0 and float(res.E.abs().max()) == 0.0
