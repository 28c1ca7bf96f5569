"""SplitMix64 (Steele, Lea & Flood, OOPSLA 2014; Vigna's reference form).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The k-th output (k = 0, 1, ...) of a generator seeded with s is
    z = s + (k + 1) * 0x9E3779B97F4A7C15            (mod 2^64)
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    out = z ^ (z >> 31)
Written here from that definition only; the GPU side has its own copy.
"""

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def outputs(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+count-1 of the generator seeded with `seed`."""
    k = np.arange(start, start + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed % (1 << 64)) + (k + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed: int, count: int) -> np.ndarray:
    """xi = 2U - 1 with U = (out >> 11) * 2^-53, uniform on [-1, 1)."""
    u = (outputs(seed, count) >> np.uint64(11)).astype(np.float64) * 2.0**-53
    return 2.0 * u - 1.0
