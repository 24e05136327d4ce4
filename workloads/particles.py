"""Free-standing particle sets for feeding one stage in isolation.

These are plain seeded draws (float32 SoA arrays), used where a test wants to
drive advection or rendering directly with positions it chose, instead of the
generator's own Philox seeding.
"""

from __future__ import annotations

import numpy as np


def random_particles(seed: int, n: int, H: int, W: int, d_range=(1.0, 5.0),
                     I0_range=(0.8, 1.0), z_range=(-1.0, 1.0), pad: float = 4.0,
                     zero_frac: float = 0.0):
    """``n`` particles with positions uniform over the frame grown by ``pad`` px."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, n, H, W, 0xBA11]))
    x = rng.uniform(-pad, W + pad, n).astype(np.float32)
    y = rng.uniform(-pad, H + pad, n).astype(np.float32)
    d = rng.uniform(d_range[0], d_range[1], n).astype(np.float32)
    I0 = rng.uniform(I0_range[0], I0_range[1], n).astype(np.float32)
    z = rng.uniform(z_range[0], z_range[1], n).astype(np.float32)
    if zero_frac > 0.0:
        I0[rng.random(n) < zero_frac] = 0.0
    return {"x": x, "y": y, "z": z, "d": d, "I0": I0}


def edge_case_particles(H: int, W: int, tile: int = 32, d: float = 2.5):
    """Particles placed where off-by-one mistakes show: exactly on pixel centres,
    on pixel edges, on tile borders, at and beyond the frame corners, half
    outside the frame, and one with zero intensity."""
    pts = []
    pts += [(0.5, 0.5), (W - 0.5, H - 0.5), (W / 2 + 0.5, H / 2 + 0.5)]          # pixel centres
    pts += [(1.0, 1.0), (float(W // 2), float(H // 3))]                        # pixel edges
    for t in range(tile, max(W, H), tile):                                      # tile borders
        if t < W:
            pts.append((float(t), H / 2 + 0.25))
        if t < H:
            pts.append((W / 3 + 0.125, float(t)))
    pts += [(-1.5, -1.5), (W + 1.0, H + 1.0), (-0.25, H / 2), (W / 2, H + 0.25)]  # outside / half out
    pts += [(-10.0, -10.0), (W + 20.0, 3.0)]                                   # fully outside
    n = len(pts) + 1
    x = np.array([p[0] for p in pts] + [W / 4 + 0.5], dtype=np.float32)
    y = np.array([p[1] for p in pts] + [H / 4 + 0.5], dtype=np.float32)
    dd = np.full(n, d, dtype=np.float32)
    I0 = np.full(n, 0.9, dtype=np.float32)
    I0[-1] = 0.0                                                               # masked
    z = np.linspace(-0.9, 0.9, n).astype(np.float32)
    return {"x": x, "y": y, "z": z, "d": dd, "I0": I0}
