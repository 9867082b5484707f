"""Counter-based SplitMix64 draws, vectorised over numpy uint64 arrays.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) keeps a 64-bit state that advances by the odd
constant GAMMA and returns a finalised copy of it.  The t-th output
(0-based) of the stream seeded with ``s`` is therefore a pure function of
(s, t):

    draw(s, t) = mix64(s + (t + 1) * GAMMA)            (mod 2**64)

which lets every consumer (CPU oracle, GPU drivers, tests) regenerate any
element of any stream independently.  This module holds the generator only;
it contains none of the ZX / GF(2) arithmetic.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_S30 = np.uint64(30)
_S27 = np.uint64(27)
_S31 = np.uint64(31)
_S11 = np.uint64(11)
_S53 = np.uint64(53)

MASK64 = (1 << 64) - 1


def mix64(z):
    """SplitMix64 output finaliser (two xor-shift-multiply rounds)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> _S30)) * _M1
        z = (z ^ (z >> _S27)) * _M2
    return z ^ (z >> _S31)


def stream_seed(seed: int, item: int, purpose: int) -> np.uint64:
    """64-bit seed of the stream for (workload seed, item id, purpose).

    seed < 2**24, item < 2**32, purpose < 2**8; the packed value is passed
    through the finaliser once so that neighbouring streams decorrelate.
    """
    if not (0 <= seed < 1 << 24 and 0 <= item < 1 << 32 and 0 <= purpose < 256):
        raise ValueError("stream id out of range")
    packed = (seed << 40) ^ (item << 8) ^ purpose
    return mix64(np.uint64(packed))


def draw(s, t):
    """t-th output of the SplitMix64 stream seeded with s (vectorised in t)."""
    t = np.asarray(t, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(s) + (t + np.uint64(1)) * GAMMA
    return mix64(state)


def unit(h):
    """Uniform double in [0, 1) from the top 53 bits of a draw."""
    return (np.asarray(h, dtype=np.uint64) >> _S11).astype(np.float64) * (2.0 ** -53)


def randint(h, lo: int, hi: int):
    """Uniform integer in [lo, hi] from the top 53 bits of a draw (hi-lo < 2047)."""
    span = hi - lo + 1
    if not (0 < span < 2048):
        raise ValueError("span out of range")
    top = np.asarray(h, dtype=np.uint64) >> _S11
    with np.errstate(over="ignore"):
        return (lo + ((top * np.uint64(span)) >> _S53)).astype(np.int64)


def bernoulli_threshold(p: float) -> np.uint64:
    """Integer threshold so that (draw >> 11) < threshold has probability p."""
    return np.uint64(int(p * float(1 << 53)))
