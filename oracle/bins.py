"""Screen-tile membership of particles (oracle).

The paper renders each particle as a square patch of side 3*max(d)+1 pixels
around it and sums the patches (Section 2, "Efficient rasterization").
Reading: a particle's support is the set of pixel centres within 1.5*d_i of it
along each axis (abs(dx) <= 1.5 d and abs(dy) <= 1.5 d), whose side is at most
floor(3 d) + 1 pixels -- the paper's patch side.

A tile renderer needs, for every tile, the particles whose support (clipped to
the image) comes within ``apron`` pixels of the tile, because a blur of radius
``apron`` is applied afterwards.  Membership is an integer decided by floats, so
it is taken here in binary32, exactly as the kernels take it: dx is the binary32
difference (c + 1/2) - x and R is the binary32 product 1.5 * d.  Only particles
with positive intensity and diameter are binned (masked particles add exact
zeros, Section 2, "Sampling the particles").

Per tile the member set is unique; the order inside a tile is not part of the
result (the rendered sum does not depend on it), and this oracle lists members
in ascending particle index.
"""

from __future__ import annotations

import numpy as np

f32 = np.float32


def support_range_f32(p, R, n: int):
    """Integer range [lo, hi] of pixel indices k in [0, n) whose binary32 offset
    (k + 1/2) - p lies in [-R, R].  Empty ranges have lo > hi."""
    p = np.asarray(p, dtype=f32)
    R = np.asarray(R, dtype=f32)
    base = np.floor(p.astype(np.float64) - R.astype(np.float64)).astype(np.int64) - 2
    width = int(np.ceil(2.0 * float(R.max(initial=0.0)))) + 6 if p.size else 0
    k = base[:, None] + np.arange(width, dtype=np.int64)[None, :]
    dx = (k.astype(f32) + f32(0.5)) - p[:, None]          # binary32, one rounding
    inside = (np.abs(dx) <= R[:, None]) & (k >= 0) & (k < n)
    any_in = inside.any(axis=1)
    lo = np.where(any_in, base + np.argmax(inside, axis=1), 1)
    hi = np.where(any_in, base + width - 1 - np.argmax(inside[:, ::-1], axis=1), 0)
    return lo.astype(np.int64), hi.astype(np.int64)


def valid_mask(x, y, d, I0):
    x = np.asarray(x, dtype=f32)
    y = np.asarray(y, dtype=f32)
    d = np.asarray(d, dtype=f32)
    I0 = np.asarray(I0, dtype=f32)
    return (I0 > 0) & (d > 0) & np.isfinite(x) & np.isfinite(y) & np.isfinite(d)


def tile_grid(H: int, W: int, tile_h: int, tile_w: int):
    return (H + tile_h - 1) // tile_h, (W + tile_w - 1) // tile_w


def bin_frame(x, y, d, I0, H: int, W: int, tile_h: int, tile_w: int, apron: int):
    """Counts, exclusive offsets and member lists of every tile of one frame.

    Tiles are numbered row-major (ty * ntx + tx)."""
    nty, ntx = tile_grid(H, W, tile_h, tile_w)
    x = np.asarray(x, dtype=f32)
    y = np.asarray(y, dtype=f32)
    d = np.asarray(d, dtype=f32)
    ok = valid_mask(x, y, d, I0)
    idx = np.nonzero(ok)[0]
    R = f32(1.5) * d[idx]
    clo, chi = support_range_f32(x[idx], R, W)
    rlo, rhi = support_range_f32(y[idx], R, H)
    lists = [[] for _ in range(nty * ntx)]
    for k in range(idx.size):
        if clo[k] > chi[k] or rlo[k] > rhi[k]:
            continue
        tx0 = max(0, (clo[k] - apron) // tile_w)
        tx1 = min(ntx - 1, (chi[k] + apron) // tile_w)
        ty0 = max(0, (rlo[k] - apron) // tile_h)
        ty1 = min(nty - 1, (rhi[k] + apron) // tile_h)
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                lists[ty * ntx + tx].append(int(idx[k]))
    counts = np.array([len(l) for l in lists], dtype=np.int64)
    offsets = np.zeros(counts.size + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    entries = np.array([i for l in lists for i in l], dtype=np.int64)
    return counts, offsets, entries


def bin_frame_bruteforce(x, y, d, I0, H: int, W: int, tile_h: int, tile_w: int, apron: int):
    """Same membership by enumerating every (particle, pixel) pair: particle i is
    in tile t iff some in-image pixel of its support lies within ``apron`` px
    (Chebyshev distance) of a pixel of t.  Slow; for tiny images only."""
    nty, ntx = tile_grid(H, W, tile_h, tile_w)
    x = np.asarray(x, dtype=f32)
    y = np.asarray(y, dtype=f32)
    d = np.asarray(d, dtype=f32)
    ok = valid_mask(x, y, d, I0)
    cols = np.arange(W, dtype=f32) + f32(0.5)
    rows = np.arange(H, dtype=f32) + f32(0.5)
    members = [set() for _ in range(nty * ntx)]
    for i in np.nonzero(ok)[0]:
        R = f32(1.5) * d[i]
        cin = np.nonzero(np.abs(cols - x[i]) <= R)[0]
        rin = np.nonzero(np.abs(rows - y[i]) <= R)[0]
        if cin.size == 0 or rin.size == 0:
            continue
        for ty in range(nty):
            for tx in range(ntx):
                c0, c1 = tx * tile_w - apron, min(W, (tx + 1) * tile_w) - 1 + apron
                r0, r1 = ty * tile_h - apron, min(H, (ty + 1) * tile_h) - 1 + apron
                if ((cin >= c0) & (cin <= c1)).any() and ((rin >= r0) & (rin <= r1)).any():
                    members[ty * ntx + tx].add(int(i))
    return members
