"""Pins of the oracle's random numbers: Philox4x32-10 known answers and the
Gaussian test matrix against the normal law."""
import os

import numpy as np
import pytest
import scipy.stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(x, 16) for x in line.split()])
    return rows


@pytest.mark.parametrize("row", _kat())
def test_philox_known_answers(row):
    ctr = np.array(row[0:4], np.uint32)
    key = row[4] | (row[5] << 32)
    out = oracle.philox(key, ctr)[0]
    assert [int(x) for x in out] == row[6:10]


def test_philox_counter_sensitivity():
    # every counter word and both key words change the output block
    base = np.zeros(4, np.uint32)
    ref = oracle.philox(7, base)[0]
    for w in range(4):
        c = base.copy()
        c[w] = 1
        assert not np.array_equal(oracle.philox(7, c)[0], ref)
    assert not np.array_equal(oracle.philox(7 + (1 << 32), base)[0], ref)
    assert not np.array_equal(oracle.philox(8, base)[0], ref)


def test_philox_words_uniform():
    n = 1 << 15
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n)
    z = oracle.philox(3, ctr).ravel()
    # 16 equal bins of the 32-bit range
    hist = np.bincount(z >> 28, minlength=16)
    assert scipy.stats.chisquare(hist).pvalue > 1e-6


def test_gaussian_omega_is_standard_normal():
    om = oracle.gaussian_omega(4000, 12, seed=5)
    assert om.shape == (4000, 12)
    flat = om.ravel()
    assert scipy.stats.kstest(flat, "norm").pvalue > 1e-6
    # columns uncorrelated (cosine/sine pairs included)
    c = np.corrcoef(om.T)
    off = c - np.diag(np.diag(c))
    assert np.max(np.abs(off)) < 6 / np.sqrt(4000)


def test_gaussian_omega_ragged_width_is_prefix():
    a = oracle.gaussian_omega(50, 7, seed=9)
    b = oracle.gaussian_omega(50, 8, seed=9)
    np.testing.assert_array_equal(a, b[:, :7])
