"""Pins for the oracle's counter-based RNG (Philox4x64-10, Salmon et al. SC'11).

The paper gives each RANSAC thread an independent random state (Sec. III-C
(a)); the oracle replaces it by Philox4x64-10 keyed (seed, 0) with counter
(hypothesis, cluster tag, frame, 0).  Pinned against the published
known-answer vector and against numpy's independent Philox implementation."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            left, right = line.split("->")
            v = [int(s, 16) for s in left.split()]
            o = [int(s, 16) for s in right.split()]
            rows.append((v[:4], v[4:6], o))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_known_answer(ctr, key, expect):
    assert [int(x) for x in oracle.philox4x64_10(ctr, key)] == expect


def test_matches_numpy_philox():
    # numpy.random.Philox is Philox4x64-10 and increments its counter before
    # producing a block, so a state of (c - 1) yields block c.  Counters go in
    # as uint64 arrays: a list of Python ints above 2^63 would pass through
    # float64 and lose bits.
    rng = np.random.default_rng(1234)
    M = 2 ** 64
    for _ in range(300):
        ctr = [int(v) for v in rng.integers(0, M, size=4, dtype=np.uint64)]
        key = [int(v) for v in rng.integers(0, M, size=2, dtype=np.uint64)]
        c = ctr[0] + (ctr[1] << 64) + (ctr[2] << 128) + (ctr[3] << 192)
        c = (c - 1) % (1 << 256)
        prev = [(c >> (64 * i)) & (M - 1) for i in range(4)]
        bg = np.random.Philox(counter=np.array(prev, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
        want = [int(v) for v in bg.random_raw(4)]
        assert [int(v) for v in oracle.philox4x64_10(ctr, key)] == want


def test_small_counters_like_ransac():
    # the counters RANSAC actually uses: (h, tag, frame, 0)
    for h in (0, 1, 255, 1023):
        for tag in (0, 7, 1016144, 2 ** 32 - 2):
            ctr = [h, tag, 3, 0]
            c = h + (tag << 64) + (3 << 128)
            c -= 1
            prev = [(c >> (64 * i)) & (2 ** 64 - 1) for i in range(4)]
            want = [int(v) for v in np.random.Philox(counter=np.array(prev, dtype=np.uint64), key=np.array([0x5EED, 0], dtype=np.uint64)).random_raw(4)]
            assert [int(v) for v in oracle.philox4x64_10(ctr, [0x5EED, 0])] == want
