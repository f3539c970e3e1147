"""Counter-based generator for the random vector the method itself draws
(start vector of the power method, paper Section 3.4).

SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): state + 0x9E3779B97F4A7C15, then the finaliser
z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
z ^= z >> 31.  The counter of composite node i on level l under seed s is
i + (l << 40) + (s << 48); the value is 2 * (z >> 11) * 2^-53 - 1 in [-1, 1).
Dirichlet nodes take 0.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(ctr: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = ctr.astype(np.uint64) + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform_pm1(n: int, level: int, seed: int) -> np.ndarray:
    ctr = (np.arange(n, dtype=np.uint64) + (np.uint64(level) << np.uint64(40))
           + (np.uint64(seed) << np.uint64(48)))
    z = splitmix64(ctr)
    return 2.0 * (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) - 1.0
