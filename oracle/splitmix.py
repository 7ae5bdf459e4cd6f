"""SplitMix64 as a counter-based generator, for the interface noise of the initial state.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Published definition: G. L. Steele, D. Lea, C. H. Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014 (the 64-bit finaliser with constants 0xBF58476D1CE4E5B9,
0x94D049BB133111EB and the golden-gamma increment 0x9E3779B97F4A7C15). The value for node
n under seed s is the (n+1)-th output of a SplitMix64 stream started at state s, that is
mix(s + (n + 1) * gamma); the uniform double in [0, 1) is the top 53 bits times 2^-53.
"""
import numpy as np

_GAMMA = 0x9E3779B97F4A7C15
_MASK = (1 << 64) - 1


def mix64(z):
    """The SplitMix64 output function on a Python int."""
    z &= _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def uniform(seed, n):
    """Uniform double in [0, 1) for counter n (Python ints, slow and plain)."""
    z = mix64((seed + (n + 1) * _GAMMA) & _MASK)
    return (z >> 11) * (1.0 / (1 << 53))


def uniform_array(seed, count):
    """uniform(seed, n) for n = 0..count-1, vectorised with numpy uint64 wrap-around."""
    with np.errstate(over="ignore"):
        n = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed & _MASK) + n * np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
