"""Counter-based random numbers for every seeded synthetic input.

The generator is SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a stateless counter
hash: draw ``i`` of a stream is ``mix(key + (i + 1) * GOLDEN)``, where ``key``
is derived from the integer seed and a short purpose tag ("pd", "noise",
"mask", ...).  Every draw is a pure function of (seed, tag, i), so any
subset of a stream can be regenerated in any order, on any side.

Uniform doubles take the top 53 bits; normal deviates use the Box-Muller
transform on pairs of uniforms.  Nothing here is specific to MRF.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser applied elementwise to uint64 values."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def _fnv1a64(tag: str) -> int:
    h = 0xCBF29CE484222325
    for b in tag.encode("utf-8"):
        h ^= b
        h = (h * 0x100000001B3) & _MASK64
    return h


def stream_key(seed: int, tag: str) -> np.uint64:
    """64-bit key of the sub-stream (seed, tag)."""
    base = (int(seed) * 0xD1B54A32D192ED03 + _fnv1a64(tag)) & _MASK64
    return mix64(np.array([base], dtype=np.uint64))[0]


def raw64(seed: int, tag: str, n: int, offset: int = 0) -> np.ndarray:
    """Draws offset .. offset+n-1 of the stream (seed, tag) as uint64."""
    key = stream_key(seed, tag)
    ctr = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(key + ctr * GOLDEN)


def uniform(seed: int, tag: str, n: int, lo: float = 0.0, hi: float = 1.0,
            offset: int = 0) -> np.ndarray:
    """Uniform doubles in [lo, hi)."""
    u = (raw64(seed, tag, n, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return lo + (hi - lo) * u


def normal(seed: int, tag: str, n: int, offset: int = 0) -> np.ndarray:
    """Standard normal deviates (Box-Muller, two uniforms per pair)."""
    m = (n + 1) // 2
    u = uniform(seed, tag, 2 * m, offset=2 * offset)
    u1 = 1.0 - u[0::2]            # (0, 1]: log is finite
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    out = np.empty(2 * m)
    out[0::2] = r * np.cos(2.0 * np.pi * u2)
    out[1::2] = r * np.sin(2.0 * np.pi * u2)
    return out[:n]


def randint(seed: int, tag: str, n: int, high: int, offset: int = 0) -> np.ndarray:
    """Integers uniform on {0, ..., high-1} (multiply-shift on 53-bit uniforms)."""
    u = uniform(seed, tag, n, offset=offset)
    return np.minimum((u * high).astype(np.int64), high - 1)


def permutation(seed: int, tag: str, n: int) -> np.ndarray:
    """A uniformly random permutation of 0..n-1 (sort of i.i.d. keys)."""
    keys = raw64(seed, tag, n)
    return np.argsort(keys, kind="stable")


def complex_gaussian(seed: int, tag: str, shape, sigma2) -> np.ndarray:
    """Circular complex Gaussian with E|x|^2 = sigma2 (Re, Im each sigma2/2)."""
    shape = tuple(np.atleast_1d(shape))
    n = int(np.prod(shape))
    g = normal(seed, tag, 2 * n).reshape(shape + (2,))
    s = np.sqrt(np.asarray(sigma2, dtype=np.float64) / 2.0)
    return (g[..., 0] + 1j * g[..., 1]) * s
