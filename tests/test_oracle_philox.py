"""Pins of the oracle's Philox4x64-10: bitwise equality with numpy's
independent Philox bit generator (numpy advances its 256-bit counter by
one before producing each block of four words), and uniformity of the
word -> [0,1) map."""
import numpy as np
import pytest
from scipy import stats

from oracle.philox import philox4x64_10, selection_uniforms, word_to_uniform

CASES = [
    ((5, 0, 0, 0), (0, 0)),
    ((1, 2, 3, 4), (2**64 - 1, 17)),
    ((2**64 - 1, 3, 0, 9), (1, 2)),           # carry from word 0
    ((0, 4, 0, 9), (1, 2)),                   # borrow when undoing numpy's increment
    ((123456789, 98765, (7 << 32) | (29 << 1) | 1, 1023), (2024, 0)),
]


@pytest.mark.parametrize("ctr,key", CASES)
def test_matches_numpy_philox(ctr, key):
    v = (sum(int(x) << (64 * i) for i, x in enumerate(ctr)) - 1) % (2**256)
    prev = np.array([(v >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=prev, key=np.array(key, dtype=np.uint64))
    assert [int(x) for x in bg.random_raw(4)] == list(philox4x64_10(ctr, key))


def test_uniform_map_range():
    assert word_to_uniform(0) == 0.0
    assert word_to_uniform(2**64 - 1) == 1.0 - 2.0**-53


def test_selection_uniforms_are_uniform():
    u = np.concatenate([selection_uniforms(0, s, 0, 3, 1, 257) for s in range(40)])
    assert u.min() >= 0.0 and u.max() < 1.0
    counts, _ = np.histogram(u, bins=20, range=(0, 1))
    assert stats.chisquare(counts).pvalue > 1e-4


def test_selection_uniforms_are_addressed_by_counter():
    a = selection_uniforms(7, 11, 2, 5, 0, 9)
    b = selection_uniforms(7, 11, 2, 5, 0, 20)
    assert np.array_equal(a, b[:9])
    assert not np.array_equal(a, selection_uniforms(7, 11, 2, 5, 1, 9))
    assert not np.array_equal(a, selection_uniforms(7, 12, 2, 5, 0, 9))
