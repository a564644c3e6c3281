"""Counter-based splitmix64 (Steele, Lea & Flood, 2014).

``u64(seed, stream, counter)`` mixes the three words into one 64-bit state
and applies the splitmix64 finaliser, so every draw is addressable by its
counter and independent of call order.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK = (1 << 64) - 1


def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def u64(seed: int, stream: int, counter) -> np.ndarray:
    """64-bit draws for the given counters of one (seed, stream)."""
    base = ((seed & _MASK) * 0x2545F4914F6CDD1D + (stream & _MASK)) & _MASK
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(base) + (c + np.uint64(1)) * _GAMMA
    return _mix(z)


def uniform(seed: int, stream: int, counter) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits."""
    return (u64(seed, stream, counter) >> np.uint64(11)).astype(np.float64) * (
        1.0 / 9007199254740992.0)


class Stream:
    """Sequential view of one (seed, stream) pair."""

    def __init__(self, seed: int, stream: int = 0):
        self.seed, self.stream, self.n = seed, stream, 0

    def uniform(self, lo: float = 0.0, hi: float = 1.0, size=None):
        k = 1 if size is None else int(np.prod(size))
        v = uniform(self.seed, self.stream, np.arange(self.n, self.n + k))
        self.n += k
        v = lo + (hi - lo) * v
        return float(v[0]) if size is None else v.reshape(size)

    def integers(self, lo: int, hi_inclusive: int) -> int:
        span = hi_inclusive - lo + 1
        return lo + int(self.uniform() * span) % span
