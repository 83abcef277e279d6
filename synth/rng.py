"""Counter-based random numbers for the synthetic workloads.

The generator is SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): the j-th output of a stream
with key s is mix64(s + (j + 1) * GAMMA), so any position of a stream can be
computed directly.  That makes the draw vectorisable with numpy uint64
arithmetic (which wraps modulo 2**64) and independent of how a caller
chunks it.

Uniform doubles are (x >> 11) * 2**-53, in [0, 1).  Normal deviates use the
Box-Muller transform (Box & Muller 1958), cosine branch only.

This module holds no part of the cross-section lookup: it only draws numbers.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_S30, _S27, _S31, _S11 = (np.uint64(30), np.uint64(27), np.uint64(31),
                          np.uint64(11))
_TWO_M53 = 2.0 ** -53


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (a bijection of 64-bit words)."""
    z = np.asarray(z, dtype=np.uint64).copy()
    z ^= z >> _S30
    z *= _M1
    z ^= z >> _S27
    z *= _M2
    z ^= z >> _S31
    return z


def stream_key(seed: int, stream: int) -> np.uint64:
    """Key of substream `stream` under base seed `seed`.

    key = mix64(mix64(seed) + (stream + 1) * GAMMA): distinct substreams
    start at unrelated points of the 2**64 cycle.
    """
    with np.errstate(over="ignore"):
        s = mix64(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))
        s = s + np.uint64((stream + 1) & 0xFFFFFFFFFFFFFFFF) * GAMMA
        return mix64(s)[0]


class Stream:
    """A SplitMix64 stream read sequentially; `pos` counts words consumed."""

    def __init__(self, seed: int, stream: int):
        self.key = stream_key(seed, stream)
        self.pos = 0

    def u64(self, n: int) -> np.ndarray:
        j = np.arange(self.pos + 1, self.pos + 1 + n, dtype=np.uint64)
        self.pos += n
        with np.errstate(over="ignore"):
            return mix64(self.key + j * GAMMA)

    def uniform(self, n: int) -> np.ndarray:
        """n doubles uniform on [0, 1), 53 random bits each."""
        return (self.u64(n) >> _S11).astype(np.float64) * _TWO_M53

    def uniform_open0(self, n: int) -> np.ndarray:
        """n doubles uniform on (0, 1]: 1 - U."""
        return 1.0 - self.uniform(n)

    def normal(self, n: int) -> np.ndarray:
        """n standard normal deviates (Box-Muller, cosine branch)."""
        u1 = self.uniform_open0(n)
        u2 = self.uniform(n)
        return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)

    def lognormal(self, n: int) -> np.ndarray:
        """n lognormal(0, 1) deviates: exp(Z)."""
        return np.exp(self.normal(n))

    def log_uniform(self, n: int, a: float, b: float) -> np.ndarray:
        """n deviates log-uniform on [a, b): exp(ln a + U (ln b - ln a))."""
        la, lb = np.log(a), np.log(b)
        return np.exp(la + self.uniform(n) * (lb - la))

    def integers(self, n: int, lo: int, hi: int) -> np.ndarray:
        """n integers uniform on {lo, ..., hi} (inclusive): lo + floor(U (hi-lo+1))."""
        span = hi - lo + 1
        v = np.floor(self.uniform(n) * span).astype(np.int64)
        return (lo + np.minimum(v, span - 1)).astype(np.int64)

    def permutation(self, k: int) -> np.ndarray:
        """A random permutation of range(k): stable argsort of k uniforms."""
        return np.argsort(self.uniform(k), kind="stable")
