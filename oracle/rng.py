"""Counter-based random stream for the method's own random draws: the probe
vectors of Algorithm 1 step 1 and the Gaussian test matrix of the randomized
range finder (Section 2).

Oracle module (test infrastructure).  The paper fixes only the distribution
(mean 0, variance 1; Rademacher in Section 3).  The generator is a reading:
SplitMix64's output function (Steele, Lea and Flood, OOPSLA 2014) used as a
counter hash, written here from its published definition.

    mix(z)   = SplitMix64 finalizer (xor-shift 30, *0xBF58476D1CE4E5B9,
               xor-shift 27, *0x94D049BB133111EB, xor-shift 31)
    key      = mix(seed + G * (stream + 1))            G = 0x9E3779B97F4A7C15
    bits(i)  = mix(key + G * (i + 1))                  (mod 2^64)

    rademacher(i) = +1 if bit 63 of bits(i) is 0 else -1
    uniform(i)    = ((bits(i) >> 11) + 1/2) * 2^-53        in (0, 1)
    gaussian(i)   = sqrt(-2 ln uniform(2i)) * cos(2 pi uniform(2i + 1))

A block of shape rows x cols uses index i = row * cols + col.
"""
from __future__ import annotations

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB

STREAM_OMEGA = 1   # Gaussian test matrix of the range finder
STREAM_PROBES = 2  # Hutchinson probe block

_U64 = np.uint64


def mix(z):
    """SplitMix64 finalizer on a uint64 array (wrap-around arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> _U64(30))) * _U64(M1)
        z = (z ^ (z >> _U64(27))) * _U64(M2)
    return z ^ (z >> _U64(31))


def splitmix64_sequence(state: int, count: int):
    """The sequential SplitMix64 generator (state += G, output mix(state))."""
    idx = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix(_U64(state) + _U64(GOLDEN) * idx)


def key_for(seed: int, stream: int):
    with np.errstate(over="ignore"):
        return mix(np.array([seed], dtype=np.uint64) + _U64(GOLDEN) * _U64(stream + 1))[0]


def bits(seed: int, stream: int, index):
    index = np.asarray(index, dtype=np.uint64)
    key = key_for(seed, stream)
    with np.errstate(over="ignore"):
        return mix(key + _U64(GOLDEN) * (index + _U64(1)))


def uniform_from_bits(u):
    return ((u >> _U64(11)).astype(np.float64) + 0.5) * 2.0 ** -53


def rademacher(seed: int, stream: int, rows: int, cols: int):
    idx = np.arange(rows * cols, dtype=np.uint64)
    u = bits(seed, stream, idx)
    v = 1.0 - 2.0 * (u >> _U64(63)).astype(np.float64)
    return v.reshape(rows, cols)


def uniform(seed: int, stream: int, rows: int, cols: int):
    idx = np.arange(rows * cols, dtype=np.uint64)
    return uniform_from_bits(bits(seed, stream, idx)).reshape(rows, cols)


def gaussian(seed: int, stream: int, rows: int, cols: int):
    idx = np.arange(rows * cols, dtype=np.uint64)
    u1 = uniform_from_bits(bits(seed, stream, 2 * idx))
    u2 = uniform_from_bits(bits(seed, stream, 2 * idx + _U64(1)))
    g = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return g.reshape(rows, cols)
