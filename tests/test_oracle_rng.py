"""Pins for oracle.rng, the counter stream behind the probe vectors
(Algorithm 1 step 1) and the range finder's test matrix (Section 2)."""
import os

import numpy as np
import pytest

from oracle import rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_vectors():
    out = []
    for line in open(os.path.join(GOLDEN, "splitmix64_vectors.txt")):
        if line.startswith("#") or not line.strip():
            continue
        parts = line.split()
        out.append((int(parts[0]), [int(h, 16) for h in parts[1:]]))
    return out


@pytest.mark.parametrize("state,expected", load_vectors())
def test_splitmix64_published_outputs(state, expected):
    got = rng.splitmix64_sequence(state, len(expected))
    assert [int(v) for v in got] == expected


def test_counter_stream_is_sequential_splitmix_from_key():
    # bits(i) for i = 0,1,2,... is the SplitMix64 sequence started at the key
    key = int(rng.key_for(77, 2))
    seq = rng.splitmix64_sequence(key, 5)
    np.testing.assert_array_equal(rng.bits(77, 2, np.arange(5)), seq)


def test_distributions():
    n = 200000
    r = rng.rademacher(5, rng.STREAM_PROBES, n, 1)[:, 0]
    assert set(np.unique(r)) == {-1.0, 1.0}
    assert abs(r.mean()) < 4.0 / np.sqrt(n)
    u = rng.uniform(5, 3, n, 1)
    assert u.min() > 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 4.0 * np.sqrt(1 / 12 / n)
    g = rng.gaussian(5, rng.STREAM_OMEGA, n, 1)[:, 0]
    assert abs(g.mean()) < 4.0 / np.sqrt(n)
    assert abs(g.var() - 1.0) < 4.0 * np.sqrt(2.0 / n)
    # kurtosis of a normal is 3
    assert abs(np.mean(g ** 4) / g.var() ** 2 - 3.0) < 0.1


def test_layout_row_major_and_streams_independent():
    a = rng.rademacher(9, rng.STREAM_PROBES, 7, 5)
    flat = rng.rademacher(9, rng.STREAM_PROBES, 35, 1)[:, 0]
    np.testing.assert_array_equal(a.reshape(-1), flat)
    b = rng.rademacher(9, rng.STREAM_OMEGA, 7, 5)
    assert not np.array_equal(a, b)
