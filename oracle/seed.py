"""Particle seeding, float64 definition (oracle).

Follows Section 2, "Sampling the particles": allocate H*W*ppp_max candidate
particles per image, draw their positions over the image domain, draw the
actual ppp uniformly from the configured range and mask the excess particles by
giving them zero intensity.  Per-particle parameters are drawn uniformly from
configured intervals (Section 2, the paragraph after Eq. 1); the diameter may
instead be a clipped normal.

Readings (the paper leaves these open): the particle count is
floor(H*W*ppp + 1/2); the masked particles are those with index >= n_active;
ppp is drawn once per image pair; positions are uniform over [0, W) x [0, H)
with pixel (r, c) centred at (c + 1/2, r + 1/2); z is the out-of-plane position
in sheet units.
"""

from __future__ import annotations

import math

import numpy as np

from . import philox as ph


def particle_count(H: int, W: int, ppp: float) -> int:
    """floor(H * W * ppp + 1/2), evaluated in float64."""
    return int(math.floor(float(H) * float(W) * float(ppp) + 0.5))


def pair_scalars(H: int, W: int, ppp_lo: float, ppp_hi: float, pair_id: int, seed: int):
    """The pair's drawn ppp and its active particle count (stream 5, index 0)."""
    n_max = particle_count(H, W, ppp_hi)
    w = ph.draw(0, ph.STREAM_PAIR, pair_id, seed)[0]
    u = float(ph.uniform24(w))
    ppp = float(ppp_lo) + (float(ppp_hi) - float(ppp_lo)) * u
    n_active = min(n_max, int(math.floor(float(H) * float(W) * ppp + 0.5)))
    return ppp, n_active, n_max


def box_muller_cos(w_a, w_b):
    """Standard normal sqrt(-2 ln u1) cos(2 pi u2), u1 in (0, 1], u2 in [0, 1)."""
    u1 = ph.uniform24_open0(w_a)
    u2 = ph.uniform24(w_b)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def seed_pair(H: int, W: int, pair_id: int, seed: int, ppp=(0.05, 0.05),
              d_dist: str = "uniform", d_params=(1.0, 5.0), I0=(0.8, 1.0), z=(-1.0, 1.0)):
    """All n_max candidate particles of one pair, float64.

    Returns dict x, y, z, d, I0 (arrays of n_max) plus ppp and n_active.
    """
    ppp_v, n_active, n_max = pair_scalars(H, W, ppp[0], ppp[1], pair_id, seed)
    i = np.arange(n_max, dtype=np.uint64)
    g = ph.draw(i, ph.STREAM_GEOM, pair_id, seed)
    h = ph.draw(i, ph.STREAM_PHOTO, pair_id, seed)
    x = ph.uniform24(g[0]) * W
    y = ph.uniform24(g[1]) * H
    zz = z[0] + (z[1] - z[0]) * ph.uniform24(g[2])
    if d_dist == "uniform":
        d = d_params[0] + (d_params[1] - d_params[0]) * ph.uniform24(g[3])
    elif d_dist == "normal":
        mu, sigma, lo, hi = d_params
        d = np.clip(mu + sigma * box_muller_cos(h[1], h[2]), lo, hi)
    else:
        raise ValueError(d_dist)
    I = I0[0] + (I0[1] - I0[0]) * ph.uniform24(h[0])
    I = np.where(np.arange(n_max) < n_active, I, 0.0)
    return {"x": x, "y": y, "z": zz, "d": d, "I0": I, "ppp": ppp_v, "n_active": n_active,
            "n_max": n_max}
