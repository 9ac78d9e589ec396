"""Counter-based SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014; the 64-bit finaliser is the
one Vigna publishes with xoshiro).

The i-th draw (i = 0, 1, ...) of a sequence whose state starts at ``s0`` is
``mix64(s0 + (i + 1) * GAMMA)`` with all arithmetic modulo 2**64, which is
exactly what the sequential generator returns.  Streams are addressed by a
64-bit counter base, so any element can be produced independently and in any
chunking; both sides of every comparison call this one implementation.
"""

from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(state0: int, n: int, offset: int = 0) -> np.ndarray:
    """Draws ``offset .. offset+n-1`` of the SplitMix64 sequence seeded with
    state ``state0`` (uint64 array)."""
    out = np.empty(n, dtype=np.uint64)
    s0 = np.uint64(state0 % (1 << 64))
    with np.errstate(over="ignore"):
        for lo in range(0, n, _CHUNK):
            hi = min(n, lo + _CHUNK)
            k = np.arange(offset + lo + 1, offset + hi + 1, dtype=np.uint64)
            out[lo:hi] = _mix64(s0 + k * GAMMA)
    return out


def _base(seed: int, stream: int) -> int:
    # seed in the top 20 bits, stream in the next 4, element index below 2**40
    if not (0 <= seed < (1 << 20)) or not (0 <= stream < 16):
        raise ValueError("seed must be in [0, 2**20) and stream in [0, 16)")
    return (seed << 44) + (stream << 40)


def u64_stream(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """Raw uint64 draws ``offset .. offset+n-1`` of (seed, stream)."""
    if offset + n > (1 << 40):
        raise ValueError("stream index exceeds 2**40")
    with np.errstate(over="ignore"):
        s0 = int((np.uint64(_base(seed, stream)) * GAMMA))
    return splitmix64(s0, n, offset)


def uniform_f64(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """Uniform [0, 1) doubles: the top 53 bits times 2**-53 (exact)."""
    out = np.empty(n, dtype=np.float64)
    for lo in range(0, n, _CHUNK):
        hi = min(n, lo + _CHUNK)
        z = u64_stream(seed, stream, hi - lo, offset + lo)
        out[lo:hi] = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return out


def uniform_f32(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """Uniform [0, 1) floats: the top 24 bits times 2**-24 (exact, no
    denormals)."""
    out = np.empty(n, dtype=np.float32)
    for lo in range(0, n, _CHUNK):
        hi = min(n, lo + _CHUNK)
        z = u64_stream(seed, stream, hi - lo, offset + lo)
        out[lo:hi] = (z >> np.uint64(40)).astype(np.float32) * np.float32(2.0 ** -24)
    return out
