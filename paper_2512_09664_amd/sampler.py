"""Sampler front end: ``make(config)`` and ``next(sampler)``.

The paper's user-facing interface (Section 2, "Usage", Listing 1): a sampler
built from a configuration returns, batch after batch, the first and second
images, the ground-truth flow fields and the sampled parameters.  The
configuration names the image shape, the batch size B, the number F of flow
fields per batch (B / F pairs per flow field) and for how many consecutive
batches a loaded flow field is reused (Section 2, "Configuration file"); flow
fields come from a provider and are moved to the device ahead of use, with
pre-fetching overlapping generation and consumption (Section 2, "Data loaders
and pre-fetching").  Optional steps: the full particle model, histogram
adjustment (Section 2, after Remark 2) and particle reuse across batches
(Conclusions: the next batch's first positions are this batch's second
positions moved by the flow over a second time dt').

Everything here is argument marshalling and scheduling: every step of a batch
runs in the library's kernels (seed, shape, advect, render, flow field,
histogram) or, for isotropic configurations without particle reuse, in one
captured plan replayed per batch.  Batches are generated on a side stream of
default priority; the consumer's stream waits on an event before it reads a
batch.
"""

from __future__ import annotations

import math
import os
from dataclasses import dataclass, field
from typing import Callable, Dict, Optional

import numpy as np
import torch

from . import api

__all__ = ["SamplerConfig", "Batch", "Sampler", "make"]


@dataclass
class SamplerConfig:
    image_shape: tuple = (512, 512)             # (H, W)
    batch_size: int = 64                        # B
    flows_per_batch: int = 1                    # F (B / F pairs per flow field)
    batches_per_flow: int = 1                   # consecutive batches that reuse the loaded flow fields
    seeding_density: tuple = (0.06, 0.06)       # ppp range
    diameter: dict = field(default_factory=lambda: {"dist": "uniform", "range": [0.8, 1.2]})
    intensity: tuple = (0.8, 1.0)
    z: tuple = (-1.0, 1.0)
    sheet: dict = field(default_factory=lambda: {"law": "gauss", "sigma": 0.5})
    dt: float = 1.0
    integrator: str = "euler"
    substeps: int = 1
    blur: dict = field(default_factory=lambda: {"radius": 0, "sigma": 0.7})
    noise_sigma: float = 0.0
    bits: int = 0                               # 0: float images; 1..16: uint16 codes
    rho: Optional[tuple] = None                 # anisotropic particle images: rho range (d_y from the diameter law)
    jitter: tuple = (0.0, 0.0, 0.0)             # frame-2 variation std of (diameters, rho, I0)
    hide_p: float = 0.0
    histogram: Optional[object] = None          # target counts [2^bits] (list or .npy path)
    flow: dict = field(default_factory=lambda: {"kind": "lamb_oseen", "grid_div": 4, "max_disp": 8.0})
    particle_reuse: Optional[dict] = None       # {"dt": dt', "batches": n}: reuse for n batches, then re-seed
    device: str = "cuda:0"
    seed: int = 0
    prefetch: bool = True
    use_graph: bool = True                      # replay a captured plan when the configuration allows it

    @staticmethod
    def from_any(cfg) -> "SamplerConfig":
        if isinstance(cfg, SamplerConfig):
            return cfg
        if isinstance(cfg, (str, os.PathLike)):
            import yaml
            with open(cfg) as f:
                cfg = yaml.safe_load(f)
        known = set(SamplerConfig.__dataclass_fields__)
        unknown = set(cfg) - known
        if unknown:
            raise ValueError(f"unknown configuration keys: {sorted(unknown)}")
        c = SamplerConfig(**cfg)
        c.validate()
        return c

    def validate(self):
        H, W = self.image_shape
        if self.batch_size < 1 or self.flows_per_batch < 1 or self.batch_size % self.flows_per_batch:
            raise ValueError("batch_size must be a positive multiple of flows_per_batch")
        if self.batches_per_flow < 1:
            raise ValueError("batches_per_flow must be >= 1")
        if H < 1 or W < 1:
            raise ValueError("image_shape must be positive")
        if self.particle_reuse is not None and self.batches_per_flow < 2:
            raise ValueError("particle reuse moves particles through the same flow field: batches_per_flow >= 2")
        if self.histogram is not None and not (1 <= self.bits <= 14):
            raise ValueError("histogram adjustment needs integer codes of 1..14 bits")

    @property
    def d_dist(self):
        return "normal" if self.diameter.get("dist", "uniform") == "normal" else "uniform"

    @property
    def d_params(self):
        if self.d_dist == "uniform":
            return tuple(float(v) for v in self.diameter["range"])
        lo, hi = self.diameter["clip"]
        return (float(self.diameter["mean"]), float(self.diameter["std"]), float(lo), float(hi))

    @property
    def d_max(self):
        return self.d_params[1] if self.d_dist == "uniform" else self.d_params[3]

    @property
    def isotropic(self):
        return (self.rho is None and not any(self.jitter) and self.hide_p == 0.0
                and self.sheet.get("law", "gauss") == "gauss" and not self.flow.get("w_scale"))


@dataclass
class Batch:
    images1: torch.Tensor            # [B, H, W] (uint16 codes or float32)
    images2: torch.Tensor
    flow_fields: torch.Tensor        # [B, H, W, 2] float32, pixels per frame at the pixel centres
    params: Dict[str, object]        # seeding_densities [B], n_active [B], pair_ids [B], flow_index [B]
    event: Optional[torch.cuda.Event] = None


class FlowProvider:
    """F flow grids per flow epoch: procedural (the synthetic families of the
    input generators), from a .npy stack [N, Gh, Gw, 2], or a callable
    (epoch, F, H, W) -> array [F, Gh, Gw, 2].  Returns host float32 arrays."""

    def __init__(self, spec: dict, H: int, W: int, F: int, seed: int):
        self.spec, self.H, self.W, self.F, self.seed = dict(spec), H, W, F, seed
        self._stack = None
        if self.spec.get("kind") == "npy":
            self._stack = np.load(self.spec["path"], mmap_mode="r", allow_pickle=False)
            if self._stack.ndim != 4 or self._stack.shape[-1] != 2:
                raise ValueError("a .npy flow stack must be [N, Gh, Gw, 2]")

    def grids(self, epoch: int):
        kind = self.spec.get("kind", "lamb_oseen")
        if callable(self.spec.get("fn")):
            out = np.asarray(self.spec["fn"](epoch, self.F, self.H, self.W), dtype=np.float32)
        elif kind == "npy":
            n = self._stack.shape[0]
            out = np.stack([np.asarray(self._stack[(epoch * self.F + f) % n], dtype=np.float32)
                            for f in range(self.F)])
        else:
            from workloads import flows as wf
            g = int(self.spec.get("grid_div", 4))
            Gh, Gw = max(self.H // g, 2), max(self.W // g, 2)
            out = []
            for f in range(self.F):
                rng = np.random.default_rng(np.random.SeedSequence([self.seed, epoch, f, 0xF10]))
                if kind == "lamb_oseen":
                    out.append(wf.lamb_oseen_grid(rng, self.H, self.W, Gh, Gw,
                                                  max_disp=float(self.spec.get("max_disp", 8.0)), dt=1.0))
                elif kind == "fourier":
                    out.append(wf.fourier_grid(rng, self.H, self.W, Gh, Gw,
                                               max_disp=float(self.spec.get("max_disp", 6.0)), dt=1.0))
                elif kind == "uniform":
                    u, v = self.spec.get("uv", (2.5, -1.25))
                    out.append(wf.uniform_grid(Gh, Gw, float(u), float(v)))
                else:
                    raise ValueError(f"unknown flow kind {kind!r}")
            out = np.stack(out).astype(np.float32)
        if out.shape[0] != self.F or out.shape[-1] != 2 or min(out.shape[1:3]) < 2:
            raise ValueError("a flow provider must return [F, Gh, Gw, 2] with Gh, Gw >= 2")
        return np.ascontiguousarray(out)

    def w_grids(self, epoch: int, shape):
        """Out-of-plane velocity grids [F, Gh, Gw] (sheet units per frame) when
        the provider asks for three-dimensional motion (``w_scale``)."""
        s = float(self.spec.get("w_scale", 0.0))
        if not s:
            return None
        rng = np.random.default_rng(np.random.SeedSequence([self.seed, epoch, 0x3D]))
        return (s * rng.standard_normal((self.F,) + tuple(shape))).astype(np.float32)


class Sampler:
    """Iterator over batches of image pairs (``next(sampler)``)."""

    def __init__(self, cfg: SamplerConfig):
        self.cfg = cfg
        c = cfg
        self.dev = torch.device(c.device)
        H, W = c.image_shape
        self.H, self.W, self.B, self.F = H, W, c.batch_size, c.flows_per_batch
        self.flows = FlowProvider(c.flow, H, W, self.F, c.seed)
        g0 = self.flows.grids(0)
        self.Gh, self.Gw = g0.shape[1], g0.shape[2]
        self.n_max = api.particle_count(H, W, c.seeding_density[1])
        self.sprm = api.seed_params(c.seeding_density, c.d_dist, c.d_params, c.intensity, c.z)
        self.aprm = api.advect_params(c.dt, c.substeps, c.integrator)
        law = c.sheet.get("law", "gauss")
        self.rprm = api.render_params(c.sheet.get("sigma", 0.5), c.d_max, c.blur.get("radius", 0),
                                      c.blur.get("sigma", 0.7), c.noise_sigma, c.bits, c.seed, c.dt, c.substeps,
                                      c.integrator, hide_p=c.hide_p, jitter=c.jitter, sheet_law=law,
                                      sheet_dz0=c.sheet.get("dz0", 0.0), sheet_shape=c.sheet.get("shape", 0.0))
        self.stream = torch.cuda.Stream(device=self.dev)       # default priority
        self.k = 0
        self._pending = None
        self._flow_epoch = -1
        self._flow_dev = None
        self._w_dev = None
        self._state = None
        self._plan = None
        self._target = None
        with torch.cuda.stream(self.stream):
            if c.histogram is not None:
                t = np.load(c.histogram, allow_pickle=False) if isinstance(c.histogram, str) else c.histogram
                t = np.asarray(t, dtype=np.int64).reshape(-1)
                if t.size != (1 << c.bits) or t.min() < 0 or not (0 < t.sum() < (1 << 32)):
                    raise ValueError("histogram target: 2^bits non-negative counts with a total in [1, 2^32)")
                self._target = torch.from_numpy(t.astype(np.int32)).to(self.dev)
            n = max(self.B * self.n_max, 1)
            self._buf = {k: torch.empty(n, dtype=torch.float32, device=self.dev)
                         for k in ("x1", "y1", "x2", "y2", "z", "d", "I0", "dy", "rho", "z2")}
            self._buf["n_active"] = torch.empty(self.B, dtype=torch.int32, device=self.dev)
            self._buf["ppp"] = torch.empty(self.B, dtype=torch.float64, device=self.dev)
            base = self._pairs(0)
            self._ws = api.alloc_workspace(base, self.rprm)
            self._hws = None
        self._graph = c.use_graph and c.isotropic and c.particle_reuse is None

    # ---------------------------------------------------------------- helpers

    def _pairs(self, k: int):
        """The batch's pair table: pair i uses flow field i // (B / F); pair ids
        continue across batches so every batch draws new particles and noise."""
        per = self.B // self.F
        return api.PairBatch.build([(self.H, self.W)] * self.B, [(self.Gh, self.Gw)] * self.B, [self.n_max] * self.B,
                                   [k * self.B + i for i in range(self.B)], device=self.dev,
                                   flow_index=[i // per for i in range(self.B)], non_blocking=True)

    def _load_flows(self, k: int):
        epoch = k // self.cfg.batches_per_flow
        if epoch == self._flow_epoch:
            return
        g = self.flows.grids(epoch)
        if g.shape[1:3] != (self.Gh, self.Gw):
            raise ValueError("every flow epoch must keep the grid shape")
        self._flow_dev = torch.from_numpy(g.reshape(-1)).pin_memory().to(self.dev, non_blocking=True)
        w = self.flows.w_grids(epoch, (self.Gh, self.Gw))
        self._w_dev = torch.from_numpy(w.reshape(-1)).pin_memory().to(self.dev, non_blocking=True) \
            if w is not None else None
        self._flow_epoch = epoch

    def _io(self, images):
        b = self._buf
        return {"flow": self._flow_dev, "x1": b["x1"], "y1": b["y1"], "x2": b["x2"], "y2": b["y2"], "z": b["z"],
                "d": b["d"], "I0": b["I0"], "images": images, "n_active": b["n_active"], "ppp": b["ppp"]}

    # ---------------------------------------------------------------- one batch

    def _enqueue(self, k: int) -> Batch:
        c = self.cfg
        b = self._buf
        with torch.cuda.stream(self.stream):
            self._load_flows(k)
            pairs = self._pairs(k)
            dtype = api.U16 if c.bits else torch.float32
            images = torch.empty(pairs.n_pixels, dtype=dtype, device=self.dev)
            if self._graph:
                if self._plan is None:
                    self._plan = api.Plan(pairs, self.sprm, c.seed, self.aprm, self.rprm, self._io(images))
                self._plan.launch(self._io(images), c.seed, k * self.B)
            else:
                reuse = c.particle_reuse
                fresh = (reuse is None or self._state is None
                         or (k - self._state) >= int(reuse.get("batches", 1 << 30)))
                if fresh:
                    api.seed(pairs, self.sprm, c.seed, out={"x": b["x1"], "y": b["y1"], "z": b["z"], "d": b["d"],
                                                            "I0": b["I0"], "n_active": b["n_active"], "ppp": b["ppp"]})
                    if c.rho is not None:
                        api.seed_shape(pairs, self.sprm, c.rho, c.seed, out=(b["dy"], b["rho"]))
                    self._state = k
                else:
                    # particle reuse: last batch's second positions moved on by dt'
                    ap2 = api.advect_params(float(reuse["dt"]), c.substeps, c.integrator)
                    if self._w_dev is not None:
                        api.advect(pairs, self._flow_dev, ap2, b["x2"], b["y2"], b["x1"], b["y1"],
                                   wflow=self._w_dev, z1=b["z2"], z2=b["z"])
                    else:
                        api.advect(pairs, self._flow_dev, ap2, b["x2"], b["y2"], b["x1"], b["y1"], self._ws)
                z2 = None
                if self._w_dev is not None:
                    api.advect(pairs, self._flow_dev, self.aprm, b["x1"], b["y1"], b["x2"], b["y2"],
                               wflow=self._w_dev, z1=b["z"], z2=b["z2"])
                    z2 = b["z2"]
                else:
                    api.advect(pairs, self._flow_dev, self.aprm, b["x1"], b["y1"], b["x2"], b["y2"], self._ws)
                rp = api.L.RenderParams.from_buffer_copy(self.rprm)
                rp.seed = c.seed
                api.render_pair(pairs, b["x1"], b["y1"], b["x2"], b["y2"], b["z"], b["d"], b["I0"], rp, None,
                                images, self._ws, dy=b["dy"] if c.rho is not None else None,
                                rho=b["rho"] if c.rho is not None else None, z2=z2)
            if self._target is not None:
                if self._hws is None:
                    self._hws = api.histogram_match(pairs, images, self._target, c.bits)
                else:
                    api.histogram_match(pairs, images, self._target, c.bits, self._hws)
            flows = api.flow_field(pairs, self._flow_dev)
            ppp = b["ppp"].clone()
            n_active = b["n_active"].clone()
            ev = torch.cuda.Event()
            ev.record(self.stream)
        per = self.B // self.F
        im = images.view(self.B, 2, self.H, self.W)
        return Batch(im[:, 0], im[:, 1], flows.view(self.B, self.H, self.W, 2),
                     {"seeding_densities": ppp, "n_active": n_active,
                      "pair_ids": np.arange(k * self.B, (k + 1) * self.B, dtype=np.int64),
                      "flow_index": np.arange(self.B) // per, "flow_epoch": k // self.cfg.batches_per_flow},
                     ev)

    # ---------------------------------------------------------------- iterator

    def __iter__(self):
        return self

    def __next__(self) -> Batch:
        if self._pending is None:
            self._pending = self._enqueue(self.k)
        out = self._pending
        self.k += 1
        self._pending = self._enqueue(self.k) if self.cfg.prefetch else None
        cur = torch.cuda.current_stream(self.dev)
        cur.wait_event(out.event)
        for t in (out.images1, out.flow_fields, out.params["seeding_densities"], out.params["n_active"]):
            t.record_stream(cur)
        return out

    def close(self):
        if self._plan is not None:
            self._plan.close()
            self._plan = None


def make(config) -> Sampler:
    """A sampler from a configuration (a ``SamplerConfig``, a dict of its
    fields, or the path of a YAML file holding them)."""
    return Sampler(SamplerConfig.from_any(config))
