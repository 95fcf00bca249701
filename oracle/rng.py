"""Counter-based SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) and the random guess of Section
"An improved initial guess strategy" (factors uniform in [-1, 1]).

Draw c of a stream seeded with s is output number c + 1 of SplitMix64 started
at state s: x = s + (c + 1) * 0x9E3779B97F4A7C15 (mod 2^64), then the
xor-shift-multiply finaliser.  The uniform value is 2^-52 (z >> 11) - 1 in
[-1, 1), exact in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Pinned by the
generator's published first outputs for seed 0 in tests/test_oracle_rng.py.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters) -> np.ndarray:
    """Output number c + 1 of SplitMix64 seeded with `seed`, for each counter c."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (c + np.uint64(1)) * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def uniform_pm1(seed: int, counters) -> np.ndarray:
    z = splitmix64(seed, counters)
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0


def random_guess(o: int, v: int, rank: int, seed: int):
    """(gamma, rho, alpha, beta): element (row, r) of the m-th factor in this
    order is draw offset_m + row * rank + r, offset_m the sizes of the factors
    before it."""
    out, off = [], 0
    for n in (o, o, v, v):
        idx = off + np.arange(n * rank, dtype=np.uint64)
        out.append(uniform_pm1(seed, idx).reshape(n, rank))
        off += n * rank
    return tuple(out)
