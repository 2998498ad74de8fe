"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws test data (numpy PCG64 streams keyed by a seed).  It
holds none of the thresholding method's arithmetic; both the GPU library's
tests and the CPU oracle's tests take their inputs from here.

Workloads (all sizes are the defaults; every generator takes smaller sizes
for fast tests):

* ``single_svt``   500 x 300, rank-10 Haar factors, s = linspace(100, 10, 10),
                   plus iid N(0, 0.01^2) noise (the single-SVT test of Sec. 4.1).
* ``rpca``         76800 x 200 (320 x 240 video frames as columns, 200 frames):
                   L = P R^T with P, R iid U[0,1] of rank 3, S with exactly
                   floor(0.1 m n) entries at uniformly random positions, values
                   U[-1, 1]; O = L + S (the RPCA test of Sec. 4.1, Table 5).
* ``precision``    8192 x 8192, rank-100 Haar factors, s_i = 1000 * 0.95^i
                   (i = 0..99), plus iid noise of standard deviation 0.1.
* ``patch_groups`` ragged batch of patch-group matrices, rows in
                   {49, 64, 81, 100}, cols in [30, 90], rank-4 Haar signal with
                   s = (50, 20, 10, 5) plus iid N(0, 0.1^2) noise.
* ``rpca_batch``   unrolled-RPCA batch: instances built like ``rpca``.
* ``subspaces``    low-rank representation input: 10 random 9-dimensional
                   subspaces of R^2016, 64 samples each (the 2016 x 640 shape
                   of the face-clustering experiment), 10 % of the columns
                   corrupted by Gaussian noise of about a sample's norm.
"""
from __future__ import annotations

import numpy as np


def haar(rng: np.random.Generator, n: int, k: int) -> np.ndarray:
    """n x k matrix with Haar-distributed orthonormal columns: the Q of a QR of
    iid N(0,1), columns multiplied by sign(diag R) (Mezzadri 2007)."""
    g = rng.standard_normal((n, k))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def single_svt(seed: int = 0, m: int = 500, n: int = 300, rank: int = 10,
               noise_std: float = 0.01, smax: float = 100.0, smin: float = 10.0):
    rng = np.random.default_rng(seed)
    U = haar(rng, m, rank)
    V = haar(rng, n, rank)
    s = np.linspace(smax, smin, rank)
    A = (U * s) @ V.T
    if noise_std > 0:
        A = A + noise_std * rng.standard_normal((m, n))
    return np.asfortranarray(A)


def rpca(seed: int = 0, m: int = 76800, n: int = 200, rank: int = 3, frac: float = 0.10,
         dtype=np.float64):
    """Returns (O, L, S) as Fortran-ordered arrays."""
    rng = np.random.default_rng(seed)
    P = rng.random((m, rank))
    R = rng.random((n, rank))
    L = np.asfortranarray(P @ R.T)
    count = int(np.floor(frac * m * n))
    pos = rng.choice(m * n, size=count, replace=False)
    S = np.zeros(m * n)
    S[pos] = rng.uniform(-1.0, 1.0, size=count)
    S = S.reshape((m, n), order="F")
    O = L + S
    return (np.asfortranarray(O.astype(dtype)), np.asfortranarray(L.astype(dtype)),
            np.asfortranarray(S.astype(dtype)))


def precision(seed: int = 0, n: int = 8192, rank: int = 100, noise_std: float = 0.1,
              dtype=np.float64):
    rng = np.random.default_rng(seed)
    U = haar(rng, n, rank)
    V = haar(rng, n, rank)
    s = 1000.0 * 0.95 ** np.arange(rank)
    A = (U * s) @ V.T
    A += noise_std * rng.standard_normal((n, n))
    return np.asfortranarray(A.astype(dtype))


def patch_groups(seed: int = 0, count: int = 8192, rows_choices=(49, 64, 81, 100),
                 cols_range=(30, 90), signal=(50.0, 20.0, 10.0, 5.0), noise_std: float = 0.1):
    """Ragged batch packed column-major back to back.

    Returns (rows int32[count], cols int32[count], offsets int64[count],
    packed float32[total])."""
    rng = np.random.default_rng(seed)
    rows = rng.choice(np.asarray(rows_choices), size=count).astype(np.int32)
    cols = rng.integers(cols_range[0], cols_range[1] + 1, size=count).astype(np.int32)
    sizes = rows.astype(np.int64) * cols.astype(np.int64)
    offsets = np.zeros(count, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)[:-1]
    packed = np.empty(int(sizes.sum()), dtype=np.float32)
    s = np.asarray(signal)
    k = len(s)
    for j in range(count):
        r, c = int(rows[j]), int(cols[j])
        X = (haar(rng, r, k) * s) @ haar(rng, c, k).T + noise_std * rng.standard_normal((r, c))
        packed[offsets[j]:offsets[j] + r * c] = X.reshape(-1, order="F")
    return rows, cols, offsets, packed


def rpca_batch(seed: int = 0, batch: int = 16, m: int = 4096, n: int = 256, rank: int = 5,
               frac: float = 0.05, dtype=np.float32):
    """Returns (O, L) of shape (batch, m, n), each instance column-major."""
    Os, Ls = [], []
    for b in range(batch):
        O, L, _ = rpca(seed * 1000 + b, m, n, rank, frac, np.float64)
        Os.append(O)
        Ls.append(L)
    # (batch, n, m) in C order, viewed as (batch, m, n): instance b is column-major
    cm = lambda xs: np.stack([x.T for x in xs]).astype(dtype).transpose(0, 2, 1)
    return cm(Os), cm(Ls)


def subspaces(seed: int = 0, d: int = 2016, groups: int = 10, per_group: int = 64, dim: int = 9,
              corrupt: float = 0.1, noise_scale: float = 1.0):
    """Union of `groups` random `dim`-dimensional subspaces of R^d with
    `per_group` samples each (columns grouped in order; unit-variance
    coefficients, so a sample's norm is about sqrt(dim)); a fraction `corrupt`
    of the columns (exact count, random positions) gets an added iid Gaussian
    corruption of about the same norm (entries N(0, noise_scale^2 dim / d)).  Returns (X d x n column-major, labels n, the
    corrupted column indices)."""
    rng = np.random.default_rng(seed)
    n = groups * per_group
    X = np.empty((d, n), order="F")
    labels = np.repeat(np.arange(groups), per_group)
    for g in range(groups):
        U = haar(rng, d, dim)
        X[:, g * per_group:(g + 1) * per_group] = U @ rng.standard_normal((dim, per_group))
    bad = np.sort(rng.choice(n, int(round(corrupt * n)), replace=False))
    scale = noise_scale * np.sqrt(dim / d)
    X[:, bad] += scale * rng.standard_normal((d, bad.size))
    return X, labels, bad


def tensor_lowrank(seed: int = 0, shape=(32, 22, 3000), ranks=(3, 3, 5), frac: float = 0.05):
    """3-way O = L + S: L = G x1 U1 x2 U2 x3 U3 with iid U[0,1] core and
    factors, scaled to mean 1; S holds exactly `frac` of the entries at random
    positions with values U[-1, 1].  Arrays are column-major (first index
    fastest).  Returns (O, L, S)."""
    rng = np.random.default_rng(seed)
    I1, I2, I3 = shape
    G = rng.random(ranks)
    U = [rng.random((s, r)) for s, r in zip(shape, ranks)]
    L = np.einsum("abc,ia,jb,kc->ijk", G, U[0], U[1], U[2])
    L /= L.mean()
    N = I1 * I2 * I3
    S = np.zeros(N)
    idx = rng.choice(N, int(round(frac * N)), replace=False)
    S[idx] = rng.uniform(-1.0, 1.0, idx.size)
    S = S.reshape(shape, order="F")
    f = lambda a: np.asfortranarray(a)
    return f(L + S), f(L), f(S)
