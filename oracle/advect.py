"""Flow mapping between the two exposures, float64 definition (oracle).

Section 2, "Sampling the particles": the second image's particles are the
first image's moved by (x, y) -> (x + u(x, y), y + v(x, y)).  Reading: this is
one explicit Euler step of dx/dt = u(x) over the inter-frame time dt = 1; the
generalisation integrates the frozen field over dt with n equal substeps of
either explicit Euler or classical fourth-order Runge-Kutta.  Euler, dt = 1,
n = 1 is exactly the paper's mapping.

The field is sampled bilinearly from a cell-centred grid: node (i, j) sits at
((j + 1/2) W / Gw, (i + 1/2) H / Gh); outside the node hull the grid is clamped
to its edge.
"""

from __future__ import annotations

import numpy as np


def sample(flow: np.ndarray, H: int, W: int, px, py):
    """Bilinear sample of flow[Gh, Gw, 2] at image positions (px, py)."""
    Gh, Gw = flow.shape[0], flow.shape[1]
    F = np.asarray(flow, dtype=np.float64)
    gx = np.asarray(px, dtype=np.float64) * (Gw / W) - 0.5
    gy = np.asarray(py, dtype=np.float64) * (Gh / H) - 0.5
    gx = np.clip(gx, 0.0, Gw - 1.0)
    gy = np.clip(gy, 0.0, Gh - 1.0)
    j0 = np.minimum(np.floor(gx).astype(np.int64), Gw - 2)
    i0 = np.minimum(np.floor(gy).astype(np.int64), Gh - 2)
    fx = (gx - j0)[..., None]
    fy = (gy - i0)[..., None]
    a = F[i0, j0]
    b = F[i0, j0 + 1]
    c = F[i0 + 1, j0]
    d = F[i0 + 1, j0 + 1]
    val = (1 - fy) * ((1 - fx) * a + fx * b) + fy * ((1 - fx) * c + fx * d)
    return val[..., 0], val[..., 1]


def advect(flow, H: int, W: int, x, y, dt: float = 1.0, substeps: int = 1,
           integrator: str = "euler"):
    """Position after dt under the frozen field; returns float64 (x2, y2)."""
    px = np.array(x, dtype=np.float64)
    py = np.array(y, dtype=np.float64)
    h = float(dt) / int(substeps)
    for _ in range(int(substeps)):
        if integrator == "euler":
            u, v = sample(flow, H, W, px, py)
            px, py = px + h * u, py + h * v
        elif integrator == "rk4":
            k1u, k1v = sample(flow, H, W, px, py)
            k2u, k2v = sample(flow, H, W, px + 0.5 * h * k1u, py + 0.5 * h * k1v)
            k3u, k3v = sample(flow, H, W, px + 0.5 * h * k2u, py + 0.5 * h * k2v)
            k4u, k4v = sample(flow, H, W, px + h * k3u, py + h * k3v)
            px = px + h * (k1u + 2 * k2u + 2 * k3u + k4u) / 6.0
            py = py + h * (k1v + 2 * k2v + 2 * k3v + k4v) / 6.0
        else:
            raise ValueError(integrator)
    return px, py


def flow_field(flow, H: int, W: int):
    """Ground-truth flow [H, W, 2]: the field sampled at every pixel centre
    (the flow_fields a sampler returns next to the images, Section 2 "Usage")."""
    cx = np.arange(W, dtype=np.float64) + 0.5
    cy = np.arange(H, dtype=np.float64) + 0.5
    px, py = np.meshgrid(cx, cy)
    u, v = sample(flow, H, W, px, py)
    return np.stack([u, v], axis=-1)
