"""Particle image rendering, float64 definition (oracle).

Single particle (Eq. 1 with rho = 0 and sigma_x = sigma_y = d/4, i.e. the
classical e^-2 particle-image diameter d of the model the paper cites):

    A * exp(-8 ((x - x0)^2 + (y - y0)^2) / d^2),

evaluated at pixel centres (point sampling: Remark 2 says no fill factor is
modelled).  The peak A is the particle's intensity I0 times the laser-sheet
profile exp(-z^2 / (2 s^2)) at its out-of-plane position z (Remark 1 defers
the paper's own sheet law to future work; a Gaussian sheet of width s is the
reading used here).  The image is the plain sum of all particle contributions
(Section 2, "Considerations on the aggregation"), each restricted to its
square patch abs(dx), abs(dy) <= 1.5 d (Section 2, "Efficient rasterization":
patches of side 3 d + 1).  Pixel (r, c) is centred at (c + 1/2, r + 1/2).
"""

from __future__ import annotations

import numpy as np


def sheet_factor(z, s: float):
    z = np.asarray(z, dtype=np.float64)
    return np.exp(-(z * z) / (2.0 * float(s) ** 2))


def peak_amplitude(I0, z, s: float):
    return np.asarray(I0, dtype=np.float64) * sheet_factor(z, s)


def render_frame(x, y, z, d, I0, H: int, W: int, sheet_sigma: float, cutoff: bool = True,
                 chunk: int = 4096):
    """float64 image [H, W] of one exposure."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    A = peak_amplitude(I0, z, sheet_sigma)
    ok = (np.asarray(I0) > 0) & (d > 0) & np.isfinite(x) & np.isfinite(y)
    img = np.zeros((H, W), dtype=np.float64)
    idx = np.nonzero(ok)[0]
    if not cutoff:
        return render_frame_bruteforce(x[idx], y[idx], d[idx], A[idx], H, W)
    if idx.size == 0:
        return img
    K = int(np.floor(3.0 * d[idx].max())) + 4
    off = np.arange(K, dtype=np.int64)
    for s0 in range(0, idx.size, chunk):
        sel = idx[s0:s0 + chunk]
        R = 1.5 * d[sel]
        c0 = np.floor(x[sel] - R - 0.5).astype(np.int64)
        r0 = np.floor(y[sel] - R - 0.5).astype(np.int64)
        cc = c0[:, None] + off[None, :]                     # [n, K]
        rr = r0[:, None] + off[None, :]
        dx = cc + 0.5 - x[sel, None]
        dy = rr + 0.5 - y[sel, None]
        kap = 8.0 / (d[sel] ** 2)
        gx = np.exp(-kap[:, None] * dx * dx) * ((np.abs(dx) <= R[:, None]) & (cc >= 0) & (cc < W))
        gy = np.exp(-kap[:, None] * dy * dy) * ((np.abs(dy) <= R[:, None]) & (rr >= 0) & (rr < H))
        contrib = A[sel, None, None] * gy[:, :, None] * gx[:, None, :]   # [n, K(rows), K(cols)]
        R_idx = np.clip(rr, 0, H - 1)[:, :, None]
        C_idx = np.clip(cc, 0, W - 1)[:, None, :]
        np.add.at(img, (np.broadcast_to(R_idx, contrib.shape), np.broadcast_to(C_idx, contrib.shape)),
                  contrib)
    return img


def render_frame_bruteforce(x, y, d, A, H: int, W: int):
    """Every particle summed into every pixel with no patch cutoff (tiny images)."""
    cx = np.arange(W, dtype=np.float64) + 0.5
    cy = np.arange(H, dtype=np.float64) + 0.5
    img = np.zeros((H, W), dtype=np.float64)
    for i in range(len(x)):
        kap = 8.0 / (d[i] * d[i])
        gx = np.exp(-kap * (cx - x[i]) ** 2)
        gy = np.exp(-kap * (cy - y[i]) ** 2)
        img += A[i] * np.outer(gy, gx)
    return img


def render_pixel_direct(x, y, z, d, I0, r: int, c: int, sheet_sigma: float, cutoff: bool = True):
    """Single pixel value straight from the definition (sampled parity checks)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    A = peak_amplitude(I0, z, sheet_sigma)
    ok = (np.asarray(I0) > 0) & (d > 0)
    dx = (c + 0.5) - x
    dy = (r + 0.5) - y
    g = A * np.exp(-8.0 * (dx * dx + dy * dy) / np.where(d > 0, d * d, 1.0))
    if cutoff:
        ok = ok & (np.abs(dx) <= 1.5 * d) & (np.abs(dy) <= 1.5 * d)
    return float(np.sum(np.where(ok, g, 0.0)))
