"""SplitMix64 counter-based generator (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

ChFSI draws random numbers in two places: the Lanczos start vector and, when
no start block is given, a random start block (Sec. 3.1 and Sec. 4.2).  Both
the oracle and the GPU library implement the same counter-based generator
from its published definition (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): the i-th output of a stream
seeded with S is the SplitMix64 finaliser applied to S + (i + 1) * gamma
with gamma = 0x9E3779B97F4A7C15.  Stream s uses the seed S + s * 2^48.

Complex entry p of a block (column-major index) is
(u(2p) - 1/2) + i (u(2p+1) - 1/2), with u(i) = (x_i >> 11) * 2^-53.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
C1 = np.uint64(0xBF58476D1CE4E5B9)
C2 = np.uint64(0x94D049BB133111EB)

STREAM_LANCZOS = 0
STREAM_START = 1


def mix(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= C1
        z ^= z >> np.uint64(27)
        z *= C2
        z ^= z >> np.uint64(31)
    return z


def raw(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    base = np.uint64((int(seed) + (int(stream) << 48)) & 0xFFFFFFFFFFFFFFFF)
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = base + idx * GOLDEN
    return mix(state)


def uniform(seed: int, stream: int, count: int) -> np.ndarray:
    x = raw(seed, stream, count)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def complex_block(seed: int, stream: int, n: int, k: int) -> np.ndarray:
    u = uniform(seed, stream, 2 * n * k) - 0.5
    z = u[0::2] + 1j * u[1::2]
    return np.asfortranarray(z.reshape(k, n).T)
