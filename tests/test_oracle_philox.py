"""Pins for the oracle's sketch generator (Philox4x64-10 + Box-Muller).

The Philox block function is pinned against numpy's independent library
implementation (``numpy.random.Philox``, which emits the block of
``counter + 1`` first); the Gaussian transform against distributional facts.
"""
import numpy as np
import pytest
from scipy import stats

from oracle.philox import gaussian, philox4x64_10

CASES = [
    ((0, 0), (0, 0, 0, 0)),
    ((123456789, 987654321), (5, 7, 9, 11)),
    ((2**64 - 1, 2**63), (2**64 - 1, 3, 0, 2**64 - 1)),
    ((1, 1), (41, 0, 0, 0)),
]


@pytest.mark.parametrize("key,ctr", CASES)
def test_philox_block_matches_numpy_library(key, ctr):
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(ctr, dtype=np.uint64))
    ref = [int(x) for x in bg.random_raw(4)]
    c0 = (ctr[0] + 1) % 2**64
    c1 = (ctr[1] + (1 if c0 == 0 else 0)) % 2**64
    got = [int(x) for x in philox4x64_10((c0, c1, ctr[2], ctr[3]), key)]
    assert got == ref


def test_philox_vectorised_equals_scalar():
    g = np.arange(5, dtype=np.uint64)[:, None]
    c = np.arange(3, dtype=np.uint64)[None, :]
    z = np.zeros((1, 1), dtype=np.uint64)
    vec = philox4x64_10((g, c, z, z), (7, 9))
    for i in range(5):
        for j in range(3):
            sc = philox4x64_10((i, j, 0, 0), (7, 9))
            assert [int(v[i, j]) for v in vec] == [int(x) for x in sc]


def test_gaussian_prefix_property_and_layout():
    big = gaussian(3, 5, 37, 11)
    small = gaussian(3, 5, 10, 4)
    assert big.flags["F_CONTIGUOUS"]
    np.testing.assert_array_equal(small, big[:10, :4])


def test_gaussian_streams_and_seeds_differ():
    a = gaussian(1, 1, 64, 8)
    assert not np.array_equal(a, gaussian(1, 2, 64, 8))
    assert not np.array_equal(a, gaussian(2, 1, 64, 8))


def test_gaussian_distribution():
    x = gaussian(11, 1, 4000, 25).ravel()
    assert abs(x.mean()) < 0.01
    assert abs(x.var() - 1.0) < 0.01
    assert stats.kstest(x, "norm").pvalue > 1e-3
    # the cos/sin halves of each Box-Muller pair are uncorrelated
    g = gaussian(11, 2, 4000, 25)
    assert abs(np.corrcoef(g[0::4].ravel(), g[1::4].ravel())[0, 1]) < 0.02


def test_gaussian_empty():
    assert gaussian(0, 0, 0, 5).shape == (0, 5)
