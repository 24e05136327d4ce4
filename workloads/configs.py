"""Workload descriptions: the synthetic batches the generator is measured on.

A workload fixes image sizes, the acquisition/seeding parameter ranges and the
flow family.  Parameter names follow the paper's acquisition parameters
(seeding density in particles per pixel, particle image diameter, peak
intensity, laser-sheet thickness, inter-frame time, noise, blur).

The shapes mirror the paper's throughput and ablation setups (Section 3,
"Throughput" and "Ablations": synthetic 512x512 pairs, ppp around 0.06,
batched generation) scaled to the sizes this implementation is measured at.
"""

from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Tuple

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    sizes: Tuple[Tuple[int, int], ...]          # (H, W) per pair
    ppp: Tuple[float, float]                    # seeding density range [lo, hi]
    d_dist: str                                 # "uniform" or "normal"
    d_params: Tuple[float, ...]                 # (a, b) or (mu, sigma, lo, hi)
    I0: Tuple[float, float] = (0.8, 1.0)        # peak intensity range, full-scale units
    z: Tuple[float, float] = (-1.0, 1.0)        # out-of-plane position, sheet units
    sheet_sigma: float = 0.5                    # laser-sheet Gaussian sigma, sheet units
    flow: str = "uniform"                       # uniform | lamb_oseen | fourier | zero
    grid_div: int = 4                           # flow grid = image / grid_div per axis
    max_disp: float = 8.0                       # peak node displacement [px] (scaled flows)
    dt: float = 1.0                             # inter-frame time [frames]
    integrator: str = "euler"                   # euler | rk4
    substeps: int = 1
    blur_radius: int = 0                        # 0: no blur; 1: 3x3; 2: 5x5
    blur_sigma: float = 0.7
    noise_sigma: float = 0.0                    # additive Gaussian, full-scale units
    bits: int = 0                               # 0: float32 output; 1..16: uint16 codes
    seed: int = 0
    uniform_uv: Tuple[float, float] = (2.5, -1.25)

    @property
    def n_pairs(self) -> int:
        return len(self.sizes)

    @property
    def d_max(self) -> float:
        if self.d_dist == "uniform":
            return float(self.d_params[1])
        return float(self.d_params[3])

    def pixels(self) -> int:
        """Output pixels of both frames of every pair."""
        return int(sum(2 * h * w for h, w in self.sizes))

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def _uneven_sizes(n: int, seed: int) -> Tuple[Tuple[int, int], ...]:
    menu = [(256, 256), (512, 512), (768, 1024), (1024, 1280), (2048, 2048)]
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5E5]))
    idx = rng.integers(0, len(menu), size=n)
    return tuple(menu[i] for i in idx)


WORKLOADS = {
    # one 256x256 pair, fp32, uniform flow, Euler, no blur/noise
    "plain_256": Workload(
        name="plain_256", sizes=((256, 256),), ppp=(0.02, 0.02),
        d_dist="uniform", d_params=(1.5, 3.0), flow="uniform", integrator="euler",
        substeps=1, bits=0),
    # 64 pairs 1024x1024: Lamb-Oseen, RK4x4, 3x3 blur, noise 0.01, 12-bit codes
    "scale_1024": Workload(
        name="scale_1024", sizes=((1024, 1024),) * 64, ppp=(0.05, 0.05),
        d_dist="normal", d_params=(2.5, 0.5, 1.0, 5.0), flow="lamb_oseen", max_disp=8.0,
        integrator="rk4", substeps=4, blur_radius=1, blur_sigma=0.7, noise_sigma=0.01,
        bits=12),
    # 256 pairs of uneven size, ppp ~ U[0.005, 0.1], d ~ U[1, 5]
    "uneven_256": Workload(
        name="uneven_256", sizes=_uneven_sizes(256, 0), ppp=(0.005, 0.1),
        d_dist="uniform", d_params=(1.0, 5.0), flow="lamb_oseen", max_disp=8.0,
        integrator="rk4", substeps=4, blur_radius=1, blur_sigma=0.7, noise_sigma=0.01,
        bits=12),
    # 64 pairs 512x512 fp32 for the differentiable path
    "grad_512": Workload(
        name="grad_512", sizes=((512, 512),) * 64, ppp=(0.05, 0.05),
        d_dist="normal", d_params=(2.5, 0.5, 1.0, 5.0), flow="fourier", max_disp=6.0,
        integrator="rk4", substeps=4, blur_radius=1, blur_sigma=0.7, noise_sigma=0.0,
        bits=0),
    # 32 pairs 2048x2048 dense stress
    "dense_2048": Workload(
        name="dense_2048", sizes=((2048, 2048),) * 32, ppp=(0.1, 0.1),
        d_dist="uniform", d_params=(2.0, 6.0), flow="fourier", max_disp=12.0,
        integrator="rk4", substeps=8, blur_radius=2, blur_sigma=1.0, noise_sigma=0.02,
        bits=12),
    # the paper's own ablation defaults (512^2, ppp 0.06, d ~ U[0.8, 1.2]); context only
    "paper_512": Workload(
        name="paper_512", sizes=((512, 512),) * 64, ppp=(0.06, 0.06),
        d_dist="uniform", d_params=(0.8, 1.2), flow="lamb_oseen", grid_div=4, max_disp=8.0,
        integrator="euler", substeps=1, bits=0),
}


def get_workload(name: str, n_pairs: int | None = None, size: Tuple[int, int] | None = None,
                 **overrides) -> Workload:
    """A named workload, optionally cut to ``n_pairs`` pairs or resized."""
    w = WORKLOADS[name]
    sizes = list(w.sizes)
    if size is not None:
        sizes = [tuple(size)] * len(sizes)
    if n_pairs is not None:
        sizes = (sizes * ((n_pairs + len(sizes) - 1) // len(sizes)))[:n_pairs]
    return replace(w, sizes=tuple(sizes), **overrides)
