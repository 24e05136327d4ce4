"""Philox4x32-10 counter-based generator, plain NumPy (oracle).

The paper draws every per-particle parameter at random (Section 2, the
sentence after Eq. 1, and "Sampling the particles") but does not name a
generator.  This oracle uses Philox4x32 with 10 rounds as published by Salmon,
Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11):
each round multiplies counter words 0 and 2 by two fixed 32-bit multipliers
into 64-bit products, and the new counter is
(hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));
between rounds the key is bumped by two Weyl constants.

Counter layout used by the generator: (index, stream, pair_id_lo, pair_id_hi),
key = (seed_lo, seed_hi).  Streams: 0 geometry (x, y, z, uniform d), 1 photometry
(I0, Box-Muller words for a normal d), 3 / 4 noise of frame 1 / 2, 5 per-pair
scalars (the ppp draw).
"""

from __future__ import annotations

import numpy as np

PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint64(0x9E3779B9)
PHILOX_W1 = np.uint64(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

STREAM_GEOM = 0
STREAM_PHOTO = 1
STREAM_NOISE0 = 3
STREAM_PAIR = 5


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  All arguments are broadcastable arrays of
    values in [0, 2^32); returns four uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK32
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & _MASK32
            k1 = (k1 + PHILOX_W1) & _MASK32
        p0 = PHILOX_M0 * c0          # exact: both factors < 2^32
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK32
        hi1, lo1 = p1 >> _S32, p1 & _MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def draw(index, stream: int, pair_id: int, seed: int):
    """Four words for counter (index, stream, pair_id) under key ``seed``."""
    pid = int(pair_id)
    sd = int(seed)
    return philox4x32_10(index, stream, pid & 0xFFFFFFFF, (pid >> 32) & 0xFFFFFFFF,
                         sd & 0xFFFFFFFF, (sd >> 32) & 0xFFFFFFFF)


def uniform24(w):
    """Top 24 bits of a word as a float in [0, 1): exactly (w >> 8) * 2^-24."""
    return (np.asarray(w, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) * 2.0 ** -24


def uniform24_open0(w):
    """((w >> 8) + 1) * 2^-24 in (0, 1]; the argument of the Box-Muller log."""
    return ((np.asarray(w, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) + 1.0) * 2.0 ** -24
