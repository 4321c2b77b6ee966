"""Counter-based random numbers written out in plain Python for the tests.

An independent restatement (Python integers, no numpy, no oracle, no library)
of the two published generators both implementations draw from:

* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014): the value for counter ``idx`` of the stream
  ``seed`` is the (idx + 1)-th output of the generator started at ``seed``.
* Box-Muller (Box and Muller, 1958) on two 24-bit uniforms of one draw:
  u1 = (top 24 bits + 1) / 2^24 in (0, 1], u2 = low 24 bits / 2^24 in [0, 1),
  eta = r cos(theta) with r = sqrt(-2 ln u1), theta = 2 pi u2.

The noise term of Eq. (10) draws eta for spin i of global replica g at step t
from counter (g T + t) n + i of the stream keyed seed ^ NOISE_KEY.
"""
from __future__ import annotations

import math

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
NOISE_KEY = 0xD1B54A32D192ED03


def splitmix64(seed: int, idx: int) -> int:
    z = (seed + (idx + 1) * GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def box_muller(bits: int) -> tuple[float, float, float]:
    """(eta, r, theta) of one 64-bit draw, in float64."""
    u1 = ((bits >> 40) + 1) * 2.0 ** -24
    u2 = (bits & 0xFFFFFF) * 2.0 ** -24
    r = math.sqrt(-2.0 * math.log(u1))
    theta = 2.0 * math.pi * u2
    return r * math.cos(theta), r, theta


def noise(seed: int, idx: int) -> tuple[float, float, float]:
    """(eta, r, theta) for noise counter ``idx`` of SB seed ``seed``."""
    return box_muller(splitmix64(seed ^ NOISE_KEY, idx))


def noise_counter(g: int, T: int, t: int, n: int, i: int) -> int:
    return (g * T + t) * n + i
