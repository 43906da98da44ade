"""SplitMix64 counter-based generator (oracle; test infrastructure).

Published definition (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014; constants as in Vigna's public-domain
reference): the i-th output (i = 0, 1, ...) of a generator seeded with s is
mix(s + (i+1) * 0x9E3779B97F4A7C15 mod 2^64) with
  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31.
Uniform doubles on [-1, 1) take the top 53 bits: 2 * (z >> 11) * 2^-53 - 1.
Used only where the method itself draws random numbers (the Lanczos start
vector of the eigenvalue estimate), so that both sides can form it.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_C1 = np.uint64(0xBF58476D1CE4E5B9)
_C2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, count):
    i = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _C1
        z = (z ^ (z >> np.uint64(27))) * _C2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed, count):
    z = splitmix64(seed, count)
    return 2.0 * (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 - 1.0
