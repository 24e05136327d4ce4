"""Procedural flow grids (the paper's "flow supplied by a function" provider).

Every grid is returned as float32 ``[Gh, Gw, 2]`` with the (u, v) displacement
rate in pixels per frame interleaved per node.  Nodes are cell centred: node
(i, j) sits at image position ((j + 0.5) * W / Gw, (i + 0.5) * H / Gh).  All
synthesis is done in float64 and rounded once at the end.

The flows are inputs, not part of the generator: the paper leaves the flow
source to the user (Section 2, "Data loaders and pre-fetching": analytic or
randomly generated flows supplied procedurally).
"""

from __future__ import annotations

import numpy as np


def _node_positions(H: int, W: int, Gh: int, Gw: int):
    xs = (np.arange(Gw, dtype=np.float64) + 0.5) * (W / Gw)
    ys = (np.arange(Gh, dtype=np.float64) + 0.5) * (H / Gh)
    return np.meshgrid(xs, ys)  # X[i, j], Y[i, j]


def _scale_to_max_displacement(u: np.ndarray, v: np.ndarray, max_disp: float, dt: float):
    speed = np.sqrt(u * u + v * v)
    peak = float(speed.max())
    if peak <= 0.0:
        return u, v
    s = max_disp / (dt * peak)
    return u * s, v * s


def uniform_grid(Gh: int, Gw: int, u: float, v: float) -> np.ndarray:
    """Constant displacement (u, v) px/frame at every node."""
    g = np.empty((Gh, Gw, 2), dtype=np.float32)
    g[..., 0] = u
    g[..., 1] = v
    return g


def lamb_oseen_grid(rng: np.random.Generator, H: int, W: int, Gh: int, Gw: int,
                    n_vortices: int = 8, rc_range=(20.0, 80.0), max_disp: float = 8.0,
                    dt: float = 1.0) -> np.ndarray:
    """Superposition of Lamb-Oseen vortices.

    Each vortex has azimuthal speed Gamma / (2 pi r) * (1 - exp(-r^2 / rc^2)),
    centre uniform over the image, core radius rc ~ U[rc_range] px and
    circulation Gamma = +-U[0.5, 1] with a random sign.  All circulations are
    then scaled together so that the largest node speed times dt equals
    ``max_disp`` pixels.
    """
    X, Y = _node_positions(H, W, Gh, Gw)
    u = np.zeros_like(X)
    v = np.zeros_like(X)
    cx = rng.uniform(0.0, W, n_vortices)
    cy = rng.uniform(0.0, H, n_vortices)
    rc = rng.uniform(rc_range[0], rc_range[1], n_vortices)
    gam = rng.uniform(0.5, 1.0, n_vortices) * rng.choice([-1.0, 1.0], n_vortices)
    for k in range(n_vortices):
        dx = X - cx[k]
        dy = Y - cy[k]
        r2 = dx * dx + dy * dy
        r2 = np.maximum(r2, 1e-12)
        # u_theta / r = Gamma / (2 pi r^2) * (1 - exp(-r^2/rc^2))
        f = gam[k] / (2.0 * np.pi * r2) * (-np.expm1(-r2 / (rc[k] * rc[k])))
        u += -f * dy
        v += f * dx
    u, v = _scale_to_max_displacement(u, v, max_disp, dt)
    return np.stack([u, v], axis=-1).astype(np.float32)


def fourier_grid(rng: np.random.Generator, H: int, W: int, Gh: int, Gw: int,
                 max_disp: float = 6.0, dt: float = 1.0, kmax: int | None = None) -> np.ndarray:
    """Divergence-free random Fourier-mode flow with a k^(-5/3) energy spectrum.

    Stream function psi = sum_k A(k) cos(2 pi (kx x / W + ky y / H) + phi_k) over
    integer wave vectors 1 <= |k| <= kmax (default min(Gh, Gw) // 8), one mode
    per +-k pair, A(k) ~ |k|^(-7/3) (so the shell energy goes as |k|^(-5/3) in
    2-D), phases uniform; u = d psi / dy, v = -d psi / dx.  Evaluated exactly
    at the nodes with an inverse FFT (no aliasing since kmax < G / 2), then
    scaled to the requested peak node displacement.
    """
    if kmax is None:
        kmax = max(1, min(Gh, Gw) // 8)
    ky = np.fft.fftfreq(Gh, d=1.0 / Gh)  # integer wave numbers
    kx = np.fft.fftfreq(Gw, d=1.0 / Gw)
    KX, KY = np.meshgrid(kx, ky)
    kk = np.sqrt(KX * KX + KY * KY)
    # half plane: (ky > 0) or (ky == 0 and kx > 0)
    half = (KY > 0) | ((KY == 0) & (KX > 0))
    sel = half & (kk >= 1.0) & (kk <= kmax)
    amp = np.zeros_like(kk)
    amp[sel] = kk[sel] ** (-7.0 / 3.0)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=kk.shape)
    # cell-centre offset: node j at (j + 0.5) / Gw of a period
    shift = np.pi * (KX / Gw + KY / Gh)
    C = amp * np.exp(1j * (phase + shift))
    # d/dy -> i 2 pi ky / H, d/dx -> i 2 pi kx / W ; psi = Re(sum C e^{i theta})
    Cu = C * (1j * 2.0 * np.pi * KY / H)
    Cv = -C * (1j * 2.0 * np.pi * KX / W)
    n = Gh * Gw
    u = np.real(np.fft.ifft2(Cu)) * n
    v = np.real(np.fft.ifft2(Cv)) * n
    u, v = _scale_to_max_displacement(u, v, max_disp, dt)
    return np.stack([u, v], axis=-1).astype(np.float32)


def make_flows(kind: str, seed: int, sizes, grid_div: int = 4, max_disp: float = 8.0,
               dt: float = 1.0, uniform_uv=(2.5, -1.25)):
    """One flow grid per pair.

    ``sizes`` is a list of (H, W); each pair's grid is (H // grid_div, W // grid_div).
    Each pair draws from its own stream ``SeedSequence([seed, pair])`` so a pair's
    flow does not depend on the batch it is in.
    """
    out = []
    for p, (H, W) in enumerate(sizes):
        Gh, Gw = H // grid_div, W // grid_div
        rng = np.random.default_rng(np.random.SeedSequence([seed, p, 0xF10]))
        if kind == "uniform":
            out.append(uniform_grid(Gh, Gw, *uniform_uv))
        elif kind == "lamb_oseen":
            out.append(lamb_oseen_grid(rng, H, W, Gh, Gw, max_disp=max_disp, dt=dt))
        elif kind == "fourier":
            out.append(fourier_grid(rng, H, W, Gh, Gw, max_disp=max_disp, dt=dt))
        elif kind == "zero":
            out.append(uniform_grid(Gh, Gw, 0.0, 0.0))
        else:
            raise ValueError(f"unknown flow kind {kind!r}")
    return out
