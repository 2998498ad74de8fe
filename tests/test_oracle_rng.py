"""Pins for the oracle's random test matrix Omega (Alg. 1's sampling steps)."""
import os

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(orc, ctr, key, expect):
    # published Random123 known-answer vectors, not produced by this code
    assert list(orc.philox4x32_10(ctr, key)) == expect


def test_uniform53_open_interval(orc):
    lo = orc.uniform53(0, 0)
    hi = orc.uniform53(0xFFFFFFFF, 0xFFFFFFFF)
    assert lo == 0.5 * 2.0 ** -53
    # (2^53 - 1/2) 2^-53 is a tie between 1 - 2^-53 and 1; it rounds to 1.0
    assert hi == 1.0
    assert 0.0 < lo < hi <= 1.0
    # 27 + 26 bits: the step between neighbouring codes is 2^-53
    assert orc.uniform53(0, 1 << 6) - lo == 2.0 ** -53
    assert orc.uniform53(1 << 5, 0) - lo == 2.0 ** -27


def test_gaussian_distribution(orc):
    om = orc.gaussian_matrix(1234, 7, 200_000, 5)
    x = om.ravel()
    n = x.size
    assert abs(x.mean()) < 5.0 / np.sqrt(n)
    assert abs(x.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    # columns (cos / sin halves of Box-Muller and different pairs) uncorrelated
    c = np.corrcoef(om.T)
    assert np.abs(c - np.eye(5)).max() < 5.0 / np.sqrt(om.shape[0])


def test_gaussian_counter_and_seed_streams_differ(orc):
    a = orc.gaussian_matrix(1, 0, 1000, 4)
    b = orc.gaussian_matrix(1, 1, 1000, 4)
    c = orc.gaussian_matrix(2, 0, 1000, 4)
    assert abs(np.corrcoef(a.ravel(), b.ravel())[0, 1]) < 0.1
    assert abs(np.corrcoef(a.ravel(), c.ravel())[0, 1]) < 0.1
    # a matrix with more columns extends the one with fewer (same counters)
    d = orc.gaussian_matrix(1, 0, 1000, 7)
    assert np.array_equal(d[:, :4], a)


def test_gaussian_entry_from_words(orc):
    # Omega(k, 2j+e) is the e-th Box-Muller output of Philox(k, j, counter)
    seed, counter = 0x1234_5678_9ABC, 0x2_0000_0003
    om = orc.gaussian_matrix(seed, counter, 9, 5)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for k in (0, 3, 8):
        for j in range(3):
            x = orc.philox4x32_10([k, j, counter & 0xFFFFFFFF, counter >> 32], key)
            u1 = orc.uniform53(int(x[0]), int(x[1]))
            u2 = orc.uniform53(int(x[2]), int(x[3]))
            r = np.sqrt(-2.0 * np.log(u1))
            assert om[k, 2 * j] == pytest.approx(r * np.cos(2 * np.pi * u2), rel=1e-15, abs=1e-15)
            if 2 * j + 1 < 5:
                assert om[k, 2 * j + 1] == pytest.approx(r * np.sin(2 * np.pi * u2),
                                                         rel=1e-15, abs=1e-15)
