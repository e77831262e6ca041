"""Pins of the oracle's Philox4x32-10 generator and white-noise layout (CPU only)."""
import numpy as np
import pytest

from oracle import philox


def _kat_rows():
    rows = []
    with open("tests/golden/philox4x32_10_kat.txt") as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(t, 16) for t in line.split()])
    return rows


@pytest.mark.parametrize("row", _kat_rows())
def test_known_answer_vectors(row):
    ctr = [np.array([v], dtype=np.uint64) for v in row[0:4]]
    key = [np.array([v], dtype=np.uint64) for v in row[4:6]]
    out = philox.philox4x32_10(ctr, key)
    assert [int(x[0]) for x in out] == row[6:10]


def test_white_noise_is_standard_normal_and_prefix_stable():
    w = philox.white_noise(1301, 1 << 18)
    assert abs(w.mean()) < 5.0 / np.sqrt(w.size)
    assert abs(w.var() - 1.0) < 10.0 / np.sqrt(w.size)
    # fourth moment of N(0, 1) is 3
    assert abs((w**4).mean() - 3.0) < 0.05
    # value p depends only on (seed, p): a shorter draw is a prefix
    np.testing.assert_array_equal(philox.white_noise(1301, 1001), w[:1001])
    assert not np.array_equal(philox.white_noise(1302, 64), w[:64])
