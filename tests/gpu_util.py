"""Helpers shared by the GPU parity tests: build pair batches, move arrays,
and run the HIP path through the C ABI binding."""

from __future__ import annotations

import numpy as np
import torch

import paper_2512_09664_amd as sp
from workloads import make_flows

DEV = torch.device("cuda:0")


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def to_np(t):
    if t.dtype == sp.api.U16:
        return t.cpu().view(torch.int16).numpy().view(np.uint16)
    return t.cpu().numpy()


def batch_for(sizes, grids, n_max, pair_ids=None):
    return sp.PairBatch.build(sizes, grids, n_max, pair_ids, device=DEV)


def workload_inputs(wl):
    """Flows and pair batch of a workload (flows are host float32 grids)."""
    flows = make_flows(wl.flow, wl.seed, wl.sizes, wl.grid_div, wl.max_disp, wl.dt, wl.uniform_uv)
    n_max = [sp.particle_count(H, W, wl.ppp[1]) for (H, W) in wl.sizes]
    batch = batch_for(wl.sizes, [f.shape[:2] for f in flows], n_max)
    flow_dev = to_dev(np.concatenate([f.reshape(-1) for f in flows]))
    return flows, batch, flow_dev


def params_of(wl, bits=None, noise=None):
    return (sp.seed_params(wl.ppp, wl.d_dist, wl.d_params, wl.I0, wl.z),
            sp.advect_params(wl.dt, wl.substeps, wl.integrator),
            sp.render_params(wl.sheet_sigma, wl.d_max, wl.blur_radius, wl.blur_sigma,
                             wl.noise_sigma if noise is None else noise, wl.bits if bits is None else bits,
                             wl.seed, wl.dt, wl.substeps, wl.integrator))


def run_pipeline(wl, bits=None, noise=None, tile=None):
    """seed -> advect -> render on the GPU; returns (batch, flows, particles, x2, y2, images).
    The device status word must come back clear (no diameter above d_max, no
    row whose peaks could leave the fixed-point range)."""
    flows, batch, flow_dev = workload_inputs(wl)
    sprm, aprm, rprm = params_of(wl, bits, noise)
    P = sp.seed(batch, sprm, wl.seed)
    x2, y2 = sp.advect(batch, flow_dev, aprm, P["x"], P["y"])
    ws = sp.alloc_workspace(batch, rprm, tile)
    img = sp.render_pair(batch, P["x"], P["y"], x2, y2, P["z"], P["d"], P["I0"], rprm, tile, workspace=ws)
    torch.cuda.synchronize()
    flags = sp.read_status(ws)
    assert flags == 0, f"device status {flags:#x} on {wl.name}"
    return batch, flows, P, x2, y2, img


def pair_slices(batch):
    out = []
    for p in range(batch.n_pairs):
        po = batch.host[p].particle_offset
        out.append(slice(po, po + batch.host[p].n_max))
    return out
