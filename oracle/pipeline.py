"""End-to-end float64 generation of image pairs (oracle).

Composes the steps in the paper's order (Fig. 1 pipeline, Section 2):
seed particles -> move them by the flow -> render both exposures (sum of
Gaussian particle images) -> acquisition effects (blur, noise, storage).
"""

from __future__ import annotations

import numpy as np

from . import advect as adv
from . import epilogue as ep
from . import render as rd
from . import seed as sd


def generate_pair(wl, pair_index: int, flow: np.ndarray, H: int, W: int, cutoff: bool = True,
                  pair_id: int | None = None):
    """One pair of a workload ``wl`` (a ``workloads.Workload``) in float64.

    Returns the particles, the frame-2 positions, the rendered exposures I
    [2, H, W], the blurred J, the noisy K and (for bits > 0) the integer codes.
    """
    pid = pair_index if pair_id is None else pair_id
    P = sd.seed_pair(H, W, pid, wl.seed, ppp=wl.ppp, d_dist=wl.d_dist, d_params=wl.d_params,
                     I0=wl.I0, z=wl.z)
    x2, y2 = adv.advect(flow, H, W, P["x"], P["y"], wl.dt, wl.substeps, wl.integrator)
    I = np.stack([
        rd.render_frame(P["x"], P["y"], P["z"], P["d"], P["I0"], H, W, wl.sheet_sigma, cutoff),
        rd.render_frame(x2, y2, P["z"], P["d"], P["I0"], H, W, wl.sheet_sigma, cutoff),
    ])
    if wl.blur_radius > 0:
        w = ep.blur_weights(wl.blur_radius, wl.blur_sigma)
        J = np.stack([ep.blur(I[0], w), ep.blur(I[1], w)])
    else:
        J = I.copy()
    K = J.copy()
    if wl.noise_sigma > 0:
        for f in range(2):
            K[f] = J[f] + wl.noise_sigma * ep.noise_normals(H, W, f, pid, wl.seed)
    out = {"particles": P, "x2": x2, "y2": y2, "I": I, "J": J, "K": K}
    if wl.bits > 0:
        out["codes"] = ep.quantise(K, wl.bits)
    return out
