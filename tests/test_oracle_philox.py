"""Pins of the oracle's random matrices (oracle/philox.py)."""
import numpy as np
import pytest
from scipy import stats

from oracle import philox


def _numpy_block(ctr, key):
    """The four words NumPy's Philox bit generator (Philox4x64-10) returns
    for counter `ctr`: it adds one to its 256-bit counter before each block,
    so its state is set to ctr - 1."""
    value = sum(int(c) << (64 * i) for i, c in enumerate(ctr))
    value = (value - 1) % (1 << 256)
    words = np.array([(value >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64))
    st = bg.state
    st["state"]["counter"] = words
    st["buffer_pos"] = 4
    bg.state = st
    return bg.random_raw(4)


@pytest.mark.parametrize("ctr,key", [
    ((1, 0, 0, 0), (0, 0)),
    ((5, 7, 1, 0), (12345, 0)),
    ((0xFFFF_FFFF_FFFF, 3, 1, 0), (0, 0)),
    ((0, 2**63 + 5, 1, 9), (2**64 - 1, 2**40)),
    ((2**64 - 1, 2**64 - 1, 2**64 - 1, 2**64 - 1), (2**64 - 1, 2**64 - 1)),
    ((0, 0, 0, 0), (7, 0)),
])
def test_philox_words_match_numpy(ctr, key):
    mine = philox.philox4x64_10(np.array([ctr], dtype=np.uint64), np.array(key, dtype=np.uint64))[0]
    ref = _numpy_block(ctr, key)
    assert [int(v) for v in mine] == [int(v) for v in ref]


def test_philox_vectorised_equals_scalar():
    g = np.random.default_rng(3)
    ctr = g.integers(0, 2**63, size=(50, 4), dtype=np.uint64)
    key = np.array([11, 0], dtype=np.uint64)
    allw = philox.philox4x64_10(ctr, key)
    for i in range(0, 50, 7):
        assert np.array_equal(allw[i], philox.philox4x64_10(ctr[i:i + 1], key)[0])


def test_uniform_open_interval():
    w = np.array([0, 2**64 - 1, 2**12 - 1, 2**12], dtype=np.uint64)
    u = philox.uniform_from_words(w)
    assert np.all(u > 0) and np.all(u < 1)
    assert u[0] == 2.0 ** -53 and u[2] == u[0]
    assert u[1] == 1.0 - 2.0 ** -53
    assert u[3] == 3 * 2.0 ** -53


def test_gaussian_distribution():
    z = philox.gaussian_columns(0, 0, 50_000, 0, 4).ravel()
    assert abs(z.mean()) < 4.0 / np.sqrt(z.size) * 1.5
    assert abs(z.var() - 1.0) < 0.02
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_streams_independent_and_column_addressable():
    n = 1001
    r = philox.gaussian_columns(9, 0, n, 0, 12)
    c = philox.gaussian_columns(9, 1, n, 0, 12)
    corr = np.corrcoef(r.ravel(), c.ravel())[0, 1]
    assert abs(corr) < 0.05
    # columns are addressed, not drawn in sequence
    assert np.array_equal(philox.gaussian_columns(9, 0, n, 5, 12), r[:, 5:12])
    # rows likewise: a longer matrix starts with the shorter one
    assert np.array_equal(philox.gaussian_columns(9, 0, n + 6, 0, 12)[:n], r)
    # the seed matters
    assert not np.allclose(philox.gaussian_columns(10, 0, n, 0, 12), r)
