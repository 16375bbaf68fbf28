"""SplitMix64 counter-based generator (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), oracle side.

Used only for the re-seed rule of Algorithm 1 step 2 / Algorithm 2 step 3: when
(r_0, r~_0) vanishes, x~_{-1} is replaced by a random vector.  Element i of that
vector is drawn from counter value i with the generator state
seed + (i+1)*gamma, gamma = 0x9E3779B97F4A7C15, and mapped to [-1, 1) from the
top 53 bits.  Complex vectors take the real part from counter 2i and the
imaginary part from counter 2i+1.

Pinned by the published first outputs of SplitMix64 seeded with 0.
"""
import numpy as np

_MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64(state: int) -> int:
    """The SplitMix64 output function applied to a 64-bit state value."""
    z = state & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def _uniform_pm1(seed: int, counters: np.ndarray) -> np.ndarray:
    out = np.empty(len(counters), dtype=np.float64)
    for j, c in enumerate(counters):
        v = splitmix64(seed + (int(c) + 1) * GAMMA)
        out[j] = 2.0 * ((v >> 11) * 2.0 ** -53) - 1.0
    return out


def reseed_vector(seed: int, n: int, complex_valued: bool) -> np.ndarray:
    """Random replacement for x~_{-1} (see module docstring)."""
    if complex_valued:
        re = _uniform_pm1(seed, 2 * np.arange(n))
        im = _uniform_pm1(seed, 2 * np.arange(n) + 1)
        return re + 1j * im
    return _uniform_pm1(seed, np.arange(n))
