"""Pins for the oracle's Philox4x64-10 and its uniform/normal maps.

Philox is pinned against numpy's independent implementation of the same
published generator (numpy.random.Philox is Philox4x64-10; it increments the
counter before producing each block).  The uniform map is pinned by its exact
range, the Box-Muller normals by distribution tests.
"""

import math

import numpy as np
import pytest
from scipy import stats

from oracle import philox, sampling


def _numpy_block(counter, key):
    # numpy adds one (with carry) before generating, so hand it counter - 1
    c = [int(x) for x in counter]
    i = 0
    while i < 4:
        if c[i] == 0:
            c[i] = (1 << 64) - 1
            i += 1
        else:
            c[i] -= 1
            break
    ctr = np.array(c, dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=ctr)
    return tuple(int(x) for x in bg.random_raw(4))


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 2, 3, 4), (5, 7)),
    ((2**64 - 1, 2**64 - 1, 2**64 - 1, 2**64 - 1), (2**64 - 1, 2**64 - 1)),
    ((123456789, 7, philox.TAG_HOP, 0), (0x1703061160000001, 0)),
    ((0, 1, philox.TAG_NORMAL, 0), (42, 0)),
    ((2**63 + 5, 0, philox.TAG_UNIF, 0), (2**40 + 3, 0)),
])
def test_philox_matches_numpy(counter, key):
    assert philox.philox4x64_10(counter, key) == _numpy_block(counter, key)


def test_philox_many_random_counters():
    rng = np.random.default_rng(0)
    for _ in range(200):
        ctr = tuple(int(x) * 2 + 1 for x in rng.integers(0, 2**63, size=4, dtype=np.int64))
        key = tuple(int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64))
        assert philox.philox4x64_10(ctr, key) == _numpy_block(ctr, key)


def test_u01_range_and_exact_complement():
    lo = philox.u01(0)
    hi = philox.u01(2**64 - 1)
    assert lo == 2.0 ** -53 and lo > 0.0
    assert hi == 1.0 - 2.0 ** -53 and hi < 1.0
    rng = np.random.default_rng(1)
    for w in rng.integers(0, 2**63, size=1000, dtype=np.int64):
        y = philox.u01(int(w) * 2)
        one_minus = 1.0 - y
        # 1 - Y is exact: adding Y back recovers 1 exactly and the complement
        # is a multiple of 2^-53
        assert one_minus + y == 1.0
        assert (one_minus * 2.0**53) == math.floor(one_minus * 2.0**53)


def test_u01_is_uniform():
    ys = [philox.u01(philox.block(9, g, 0, philox.TAG_HOP)[1]) for g in range(4000)]
    assert stats.kstest(ys, "uniform").pvalue > 1e-4


def test_box_muller_normals():
    z = np.array([sampling.normal(77, g, c) for g in range(3000) for c in range(4)])
    assert abs(z.mean()) < 4.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 4.0 * math.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the cos and sin outputs of one pair are uncorrelated
    a = np.array([sampling.normal(77, g, 0) for g in range(3000)])
    b = np.array([sampling.normal(77, g, 1) for g in range(3000)])
    assert abs(np.corrcoef(a, b)[0, 1]) < 4.0 / math.sqrt(3000)


def test_box_muller_closed_form_point():
    # one block by hand: z0 = sqrt(-2 ln u1) cos(2 pi u2) with u1, u2 from words 0, 1
    w = philox.block(5, 11, 0, philox.TAG_NORMAL)
    u1, u2 = philox.u01(w[0]), philox.u01(w[1])
    assert sampling.normal(5, 11, 0) == math.sqrt(-2 * math.log(u1)) * math.cos(2 * math.pi * u2)
    u3, u4 = philox.u01(w[2]), philox.u01(w[3])
    assert sampling.normal(5, 11, 3) == math.sqrt(-2 * math.log(u3)) * math.sin(2 * math.pi * u4)
