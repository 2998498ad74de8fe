"""The single-SVT workload's FRSVT call (500 x 300, l = 15, q = 2) captured
in a HIP graph through frsvt_noalloc (no allocation, no host wait): every
replay -- with eager library work and synchronisations between replays --
equals the eager call bit for bit."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_frsvt_graph_replay_matches_eager():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_00296_amd as fr
    from paper_1509_00296_amd import synth
    _say("case frsvt graph capture 500x300")
    A = torch.from_numpy(synth.single_svt(seed=0)).cuda()
    s = torch.cuda.Stream()
    X = torch.empty((300, 500), dtype=torch.float64, device="cuda").t()
    Q = torch.empty((15, 300), dtype=torch.float64, device="cuda").t()
    with torch.cuda.stream(s):
        fr.handle(0)                     # the stream's handle, created outside the capture
        Xe, Qe, re = fr.frsvt(A, 1.0, 10, 5, 2, seed=7, counter=3)
        fr.frsvt(A, 1.0, 10, 5, 2, seed=7, counter=3, noalloc=True, out=(X, Q), want_rank=False)
    s.synchronize()
    assert np.array_equal(X.cpu().numpy(), Xe.cpu().numpy())
    g = torch.cuda.CUDAGraph()
    X.zero_()
    with torch.cuda.graph(g, stream=s):
        fr.frsvt(A, 1.0, 10, 5, 2, seed=7, counter=3, noalloc=True, out=(X, Q), want_rank=False)
    for rep in range(4):
        X.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(X.cpu().numpy(), Xe.cpu().numpy()), f"replay {rep}"
        # eager library work between replays (another call on the same stream)
        with torch.cuda.stream(s):
            fr.frsvt(A, 2.0, 10, 5, 2, seed=9, counter=1, noalloc=True, out=(X, Q), want_rank=False)
        s.synchronize()
