"""Host logic on the CPU: the benchmark's one-GPU contract and the synthetic
inputs of the low-rank representation and tensor workloads."""
import os
import subprocess
import sys

import numpy as np

from paper_1509_00296_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    for argv, env in ((["--gpus", "2"], {}), (["--gpus", "1"], {"WORLD_SIZE": "2"})):
        proc = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv],
                              env=dict(os.environ, **env), capture_output=True, text=True, timeout=120)
        assert proc.returncode == 2
        assert "one GPU" in proc.stderr and proc.stdout == ""


def test_subspaces_generator():
    X, labels, bad = synth.subspaces(seed=3, d=200, groups=4, per_group=16, dim=3, corrupt=0.125)
    assert X.shape == (200, 64) and X.flags.f_contiguous
    assert np.array_equal(labels, np.repeat(np.arange(4), 16))
    assert bad.size == 8 and len(set(bad.tolist())) == 8
    clean = np.setdiff1d(np.arange(64), bad)
    for g in range(4):
        cols = [j for j in clean if labels[j] == g]
        s = np.linalg.svd(X[:, cols], compute_uv=False)
        assert s[2] > 1e-8 * s[0] and s[3] < 1e-10 * s[0]      # each clean group spans dim = 3
    s = np.linalg.svd(X[:, bad], compute_uv=False)
    assert s[-1] > 1e-3 * s[0]                                 # corrupted columns leave the subspaces


def test_tensor_lowrank_generator():
    O, L, S = synth.tensor_lowrank(seed=1, shape=(6, 5, 40), ranks=(2, 3, 4), frac=0.05)
    assert O.shape == (6, 5, 40) and O.flags.f_contiguous
    assert np.count_nonzero(S) == round(0.05 * O.size)
    assert np.abs(S).max() <= 1.0 and abs(L.mean() - 1.0) < 1e-12
    assert np.array_equal(O, L + S)
    for mode, r in enumerate((2, 3, 4)):
        M = np.moveaxis(L, mode, 0).reshape(L.shape[mode], -1, order="F")
        s = np.linalg.svd(M, compute_uv=False)
        assert s[r - 1] > 1e-10 * s[0] and (len(s) == r or s[r] < 1e-10 * s[0])
