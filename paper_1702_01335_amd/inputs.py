"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Holds none of the solver's arithmetic: only the counter-based generator that draws the
perturbation field r in [-1, 1) of the seeded initial states F = F^eq_rest (1 + eps r).
Both the HIP path and the oracle receive the same r as an input array.

splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014): z_k = seed + k * 0x9E3779B97F4A7C15 (k = 1, 2, ...), then
z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31;
the top 53 bits give u in [0, 1), and r = 2u - 1.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, n, offset=0):
    """n consecutive 64-bit outputs of splitmix64 started at counter ``offset`` + 1."""
    k = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over='ignore'):
        z = np.uint64(seed) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def perturbation(seed, shape):
    """r in [-1, 1) of the given shape (C order), from splitmix64(seed)."""
    n = int(np.prod(shape))
    u = (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return (2.0 * u - 1.0).reshape(shape)
