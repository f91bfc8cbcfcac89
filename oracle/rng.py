"""Counter-based uniform numbers of the seeded initial guess (test
infrastructure only).

The paper starts every method from a uniformly random initial guess
(Section 2.4); the library can draw that guess itself from a seed.  Both
sides implement the same counter-based generator from its published
definition, so that the guess the GPU draws can be checked number by number:
Philox-4x64 with 10 rounds (J. K. Salmon, M. A. Moraes, R. O. Dror,
D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011).

One round maps a counter block (c0, c1, c2, c3) under a key (k0, k1) to

    (hi(M1 c2) ^ c1 ^ k0,  lo(M1 c2),  hi(M0 c0) ^ c3 ^ k1,  lo(M0 c0))

where hi/lo are the upper and lower 64 bits of the 128-bit product; the key
is advanced by the Weyl constants (W0, W1) before every round after the
first.  The stream used here: key = (seed, 0); block b (b = 0, 1, ...) is
the cipher of the counter (b + 1, 0, 0, 0) and yields outputs 4b .. 4b + 3;
output x becomes the double (x >> 11) * 2^-53 in [0, 1).

Pins: tests/test_oracle_rng.py compares the raw outputs with numpy's
independent Philox bit generator and the doubles with its Generator.random.
"""
from __future__ import annotations

import numpy as np

__all__ = ["philox4x64_10", "uniform01"]

_M0, _M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
_W0, _W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B
_MASK = (1 << 64) - 1


def philox4x64_10(counter, key):
    """The ten-round Philox-4x64 cipher of one counter block (Python ints)."""
    c0, c1, c2, c3 = (int(x) & _MASK for x in counter)
    k0, k1 = (int(x) & _MASK for x in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        c0, c1, c2, c3 = (p1 >> 64) ^ c1 ^ k0, p1 & _MASK, (p0 >> 64) ^ c3 ^ k1, p0 & _MASK
    return c0, c1, c2, c3


def raw_stream(seed, n):
    """The first n 64-bit outputs of the stream with key (seed, 0)."""
    out = []
    b = 0
    while len(out) < n:
        out.extend(philox4x64_10((b + 1, 0, 0, 0), (seed, 0)))
        b += 1
    return out[:n]


def uniform01(seed, n):
    """n doubles in [0, 1): output x of the stream mapped to (x >> 11) 2^-53."""
    return np.array([(x >> 11) * 2.0 ** -53 for x in raw_stream(seed, n)], dtype=np.float64)
