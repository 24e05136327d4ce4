#!/usr/bin/env python
"""Throughput of the generator's hot path on one MI355X.

One step = one batch through the whole path: seed particles -> advect them
through each pair's flow -> bin -> render both exposures -> blur, noise and
integer codes, all inputs resident in HBM.  Default workload: 64 pairs of
1024x1024 at 0.05 ppp (Lamb-Oseen flows, RK4 x4, 3x3 blur, noise 0.01,
12-bit codes).  Prints ONE JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "image pairs/s & Gpx/s at 1024²,0.05 ppp; % HBM roofline; batched vs plain"
HBM_PEAK_GBS = 8000.0
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4   # CUs x SIMDs x GHz / 4 cycles per wave64 instruction = 614.4
RENDER_SRC = os.path.join(ROOT, "paper_2512_09664_amd", "csrc", "bin_render.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "render_tile_scale_1024_traffic.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def describe(wl):
    H, W = wl.sizes[0]
    d = (f"U[{wl.d_params[0]}, {wl.d_params[1]}]" if wl.d_dist == "uniform"
         else f"N({wl.d_params[0]}, {wl.d_params[1]}) clip [{wl.d_params[2]}, {wl.d_params[3]}]")
    return {"workload": wl.name, "pairs": wl.n_pairs,
            "sizes": "x".join(map(str, (H, W))) if len(set(wl.sizes)) == 1 else "uneven",
            "ppp": list(wl.ppp), "d": d, "flow": f"{wl.flow} grid image/{wl.grid_div}",
            "integrator": f"{wl.integrator}x{wl.substeps}", "blur_radius": wl.blur_radius,
            "blur_sigma": wl.blur_sigma, "noise_sigma": wl.noise_sigma, "bits": wl.bits}


def _inputs(sp, torch, np, dev, wl):
    from workloads import make_flows
    flows = make_flows(wl.flow, wl.seed, wl.sizes, wl.grid_div, wl.max_disp, wl.dt, wl.uniform_uv)
    n_max = [sp.particle_count(H, W, wl.ppp[1]) for (H, W) in wl.sizes]
    batch = sp.PairBatch.build(wl.sizes, [f.shape[:2] for f in flows], n_max, device=dev)
    flow = torch.from_numpy(np.concatenate([f.reshape(-1) for f in flows])).to(dev)
    sprm = sp.seed_params(wl.ppp, wl.d_dist, wl.d_params, wl.I0, wl.z)
    aprm = sp.advect_params(wl.dt, wl.substeps, wl.integrator)
    rprm = sp.render_params(wl.sheet_sigma, wl.d_max, wl.blur_radius, wl.blur_sigma, wl.noise_sigma, wl.bits,
                            wl.seed, wl.dt, wl.substeps, wl.integrator)
    return flows, n_max, batch, flow, sprm, aprm, rprm


def _plan_io(sp, torch, batch, flow, bits, dev):
    n = max(batch.n_particles, 1)
    io = {k: torch.empty(n, dtype=torch.float32, device=dev) for k in ("x1", "y1", "x2", "y2", "z", "d", "I0")}
    io["flow"] = flow
    io["images"] = torch.empty(batch.n_pixels, dtype=sp.api.U16 if bits else torch.float32, device=dev)
    return io


def _time_plan(torch, plan, steps):
    plan.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.launch()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def plan_throughput(sp, torch, np, dev, wl, flows, flow, batch, sprm, aprm, rprm, steps=20):
    """The same workload as one autotuned, graph-captured plan (fresh pair ids every launch)."""
    io = _plan_io(sp, torch, batch, flow, wl.bits, dev)
    plan = sp.Plan(batch, sprm, wl.seed, aprm, rprm, io, autotune=True, advance_pair_ids=True)
    t = plan.tiling
    dt = _time_plan(torch, plan, steps)
    plan.close()
    return {"pairs_per_s": round(wl.n_pairs / dt, 1), "ms_per_step": round(1000 * dt, 4),
            "tiling": [t.tile_w, t.tile_h, t.chunk, t.cap, t.persistent]}


def dense_throughput(sp, torch, np, dev, steps=10):
    """dense_2048 (32 pairs of 2048^2, 0.1 ppp, d ~ U[2, 6], RK4 x 8, 5x5 blur,
    noise 0.02, 12-bit) as one autotuned graph-captured plan."""
    from workloads import get_workload
    wl = get_workload("dense_2048")
    flows, n_max, batch, flow, sprm, aprm, rprm = _inputs(sp, torch, np, dev, wl)
    io = _plan_io(sp, torch, batch, flow, wl.bits, dev)
    plan = sp.Plan(batch, sprm, wl.seed, aprm, rprm, io, autotune=True, advance_pair_ids=True)
    t = plan.tiling
    dt = _time_plan(torch, plan, steps)
    plan.close()
    del io
    torch.cuda.empty_cache()
    return {"pairs_per_s": round(wl.n_pairs / dt, 1), "gpx_per_s": round(wl.pixels() / dt / 1e9, 2),
            "ms_per_step": round(1000 * dt, 4), "tiling": [t.tile_w, t.tile_h, t.chunk, t.cap, t.persistent]}


def uneven_batched_vs_per_pair(sp, torch, np, dev, steps=5):
    """256 uneven pairs (256^2 .. 2048^2, ppp U[0.005, 0.1]): one graph-captured
    batch vs one launch sequence per pair."""
    from workloads import get_workload
    wl = get_workload("uneven_256")
    flows, n_max, batch, flow, sprm, aprm, rprm = _inputs(sp, torch, np, dev, wl)
    io = _plan_io(sp, torch, batch, flow, wl.bits, dev)
    plan = sp.Plan(batch, sprm, wl.seed, aprm, rprm, io, autotune=True, advance_pair_ids=True)
    t_batched = _time_plan(torch, plan, steps)
    plan.close()
    singles = []
    for p in range(wl.n_pairs):
        H, W = wl.sizes[p]
        hp = batch.host[p]
        b1 = sp.PairBatch.build([wl.sizes[p]], [flows[p].shape[:2]], [n_max[p]], [p], device=dev)
        sl = slice(hp.particle_offset, hp.particle_offset + n_max[p])
        P1 = {"x": io["x1"][sl], "y": io["y1"][sl], "z": io["z"][sl], "d": io["d"][sl], "I0": io["I0"][sl],
              "n_active": torch.empty(1, dtype=torch.int32, device=dev),
              "ppp": torch.empty(1, dtype=torch.float64, device=dev)}
        singles.append((b1, flow[hp.flow_offset:hp.flow_offset + flows[p].size], P1, io["x2"][sl], io["y2"][sl],
                        io["images"][hp.image_offset:hp.image_offset + 2 * H * W],
                        sp.alloc_workspace(b1, rprm)))

    def per_pair_step(k):
        for b1, fl1, P1, x21, y21, im1, ws1 in singles:
            sp.seed(b1, sprm, wl.seed + k, out=P1)
            sp.advect(b1, fl1, aprm, P1["x"], P1["y"], x21, y21, ws1)
            sp.render_pair(b1, P1["x"], P1["y"], x21, y21, P1["z"], P1["d"], P1["I0"], rprm, None, im1, ws1)

    per_pair_step(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        per_pair_step(k + 1)
    torch.cuda.synchronize()
    t_single = (time.perf_counter() - t0) / steps
    out = {"pairs": wl.n_pairs, "gpx_per_step": round(wl.pixels() / 1e9, 4),
           "batched_pairs_per_s": round(wl.n_pairs / t_batched, 1),
           "per_pair_pairs_per_s": round(wl.n_pairs / t_single, 1),
           "batched_vs_per_pair": round(t_single / t_batched, 3)}
    del singles, io, plan
    torch.cuda.empty_cache()
    return out


def measured_peaks(sp, torch, dev):
    """Ceilings measured on this device by the library's probe kernels: HBM
    store and copy rates over 1 GiB, and the wave64 instruction issue rates of
    float32 FMA chains, v_sin chains and 32x32->64 multiply chains at eight
    waves per SIMD."""
    out = {}
    big = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    small = torch.empty(4096, dtype=torch.uint8, device=dev)
    for kind, buf, iters, unit in (("store", big, 0, "GB/s"), ("store_nt", big, 0, "GB/s"), ("copy", big, 0, "GB/s"),
                                   ("fma", small, 4096, "G wave64 instructions/s"),
                                   ("trans", small, 1024, "G wave64 instructions/s"),
                                   ("mul64", small, 2048, "G wave64 instructions/s"),
                                   ("mix", small, 1024, "G wave64 instructions/s"),
                                   ("int", small, 4096, "G wave64 instructions/s")):
        sp.probe(kind, buf, iters)                    # warm-up
        torch.cuda.synchronize()
        sp.timing_read(None)
        sp.timing_enable(True)
        work = 0.0
        for _ in range(5):
            work = sp.probe(kind, buf, iters)
        torch.cuda.synchronize()
        sp.timing_enable(False)
        ms, n = sp.timing_read("probe_" + kind)
        out[kind] = {"rate": round(work * n / (ms * 1e-3) / 1e9, 1), "unit": unit}
    del big, small
    torch.cuda.empty_cache()
    return out


def render_only_us(sp, torch, batch, P, x2, y2, rprm, images, ws, reps=20):
    """Average render_tile launch time (us) of `reps` renders of the same particles."""
    sp.render_pair(batch, P["x"], P["y"], x2, y2, P["z"], P["d"], P["I0"], rprm, None, images, ws)
    torch.cuda.synchronize()
    sp.timing_read(None)
    sp.timing_enable(True)
    for _ in range(reps):
        sp.render_pair(batch, P["x"], P["y"], x2, y2, P["z"], P["d"], P["I0"], rprm, None, images, ws)
    torch.cuda.synchronize()
    sp.timing_enable(False)
    ms, n = sp.timing_read("render_tile")
    sp.timing_read(None)
    return 1000.0 * ms / n


def latency_plain_256(sp, torch, np, dev, reps=200):
    """One 256x256 pair (0.02 ppp, Euler, fp32 images): microseconds per pair for
    eager seed -> advect -> render calls and for a graph-captured plan replay."""
    from workloads import get_workload
    wl = get_workload("plain_256")
    flows, n_max, batch, flow, sprm, aprm, rprm = _inputs(sp, torch, np, dev, wl)
    P = sp.seed(batch, sprm, wl.seed)
    x2 = torch.empty_like(P["x"])
    y2 = torch.empty_like(P["y"])
    images = torch.empty(batch.n_pixels, dtype=torch.float32, device=dev)
    ws = sp.alloc_workspace(batch, rprm)

    def step():
        sp.seed(batch, sprm, wl.seed, out=P)
        sp.advect(batch, flow, aprm, P["x"], P["y"], x2, y2, ws)
        sp.render_pair(batch, P["x"], P["y"], x2, y2, P["z"], P["d"], P["I0"], rprm, None, images, ws)

    for _ in range(10):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    eager = (time.perf_counter() - t0) / reps
    io = _plan_io(sp, torch, batch, flow, wl.bits, dev)
    plan = sp.Plan(batch, sprm, wl.seed, aprm, rprm, io, autotune=False, advance_pair_ids=True)
    for _ in range(10):
        plan.launch()
    graph = _time_plan(torch, plan, reps)
    plan.close()
    return {"eager_us_per_pair": round(1e6 * eager, 1), "graph_us_per_pair": round(1e6 * graph, 1)}


def fp64_error(sp, torch, np, dev):
    """Error of the float images (noise off, no integer codes) against the
    all-float64 oracle pipeline (float64 seed, advection, render and blur),
    relative to each image's peak: max and mean over two pairs each of
    plain_256, scale_1024 and dense_2048."""
    from oracle import pipeline as opipe
    from workloads import get_workload
    out = {}
    for name in ("plain_256", "scale_1024", "dense_2048"):
        wl = get_workload(name).with_(bits=0, noise_sigma=0.0)
        wl = wl.with_(sizes=wl.sizes[:2])
        flows, n_max, batch, flow, sprm, aprm, rprm = _inputs(sp, torch, np, dev, wl)
        P = sp.seed(batch, sprm, wl.seed)
        x2, y2 = sp.advect(batch, flow, aprm, P["x"], P["y"])
        img = sp.render_pair(batch, P["x"], P["y"], x2, y2, P["z"], P["d"], P["I0"], rprm)
        torch.cuda.synchronize()
        got = img.cpu().numpy()
        mx, sm, cnt = 0.0, 0.0, 0
        for p in range(wl.n_pairs):
            H, W = wl.sizes[p]
            o = batch.host[p].image_offset
            ref = opipe.generate_pair(wl, p, flows[p], H, W)["J"]
            e = np.abs(got[o:o + 2 * H * W].astype(np.float64) - ref.reshape(-1)) / float(ref.max())
            mx = max(mx, float(e.max()))
            sm += float(e.sum())
            cnt += e.size
        out[name] = {"pairs": wl.n_pairs, "max_rel_peak": float(f"{mx:.3e}"), "mean_rel_peak": float(f"{sm / cnt:.3e}")}
    return out


def model_throughput(sp, torch, np, dev, steps=10):
    """scale_1024 under the full particle model (anisotropic particles with
    rho ~ U[-0.5, 0.5], frame-2 variation (0.1 px, 0.05, 0.02), hiding 0.1, the
    Remark 1 sheet law with DZ0 = 1, shape 2, out-of-plane motion), eager calls,
    against the isotropic path on the same batch."""
    from workloads import get_workload
    wl = get_workload("scale_1024")
    flows, n_max, batch, flow, sprm, aprm, rprm = _inputs(sp, torch, np, dev, wl)
    rpm = sp.render_params(wl.sheet_sigma, wl.d_max, wl.blur_radius, wl.blur_sigma, wl.noise_sigma, wl.bits,
                           wl.seed, wl.dt, wl.substeps, wl.integrator, hide_p=0.1, jitter=(0.1, 0.05, 0.02),
                           sheet_law="remark1", sheet_dz0=1.0, sheet_shape=2.0)
    wflow = 0.02 * torch.randn(flow.numel() // 2, device=dev, generator=torch.Generator(device=dev).manual_seed(2))
    P = sp.seed(batch, sprm, wl.seed)
    dy, rho = sp.seed_shape(batch, sprm, (-0.5, 0.5), wl.seed)
    x2 = torch.empty_like(P["x"])
    y2 = torch.empty_like(P["x"])
    z2 = torch.empty_like(P["x"])
    img = torch.empty(batch.n_pixels, dtype=sp.api.U16, device=dev)
    ws = sp.alloc_workspace(batch, rpm)

    def step(k):
        sp.seed(batch, sprm, wl.seed + k, out=P)
        sp.seed_shape(batch, sprm, (-0.5, 0.5), wl.seed + k, out=(dy, rho))
        sp.advect(batch, flow, aprm, P["x"], P["y"], x2, y2, wflow=wflow, z1=P["z"], z2=z2)
        sp.render_pair(batch, P["x"], P["y"], x2, y2, P["z"], P["d"], P["I0"], rpm, None, img, ws, dy=dy, rho=rho,
                       z2=z2)

    step(0)
    torch.cuda.synchronize()
    sp.timing_read(None)
    sp.timing_enable(True)
    t0 = time.perf_counter()
    for k in range(steps):
        step(k + 1)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    sp.timing_enable(False)
    ms, n = sp.timing_read("render_tile")
    sp.timing_read(None)
    flags = sp.read_status(ws)
    del ws, img, P, dy, rho, x2, y2, z2, wflow
    torch.cuda.empty_cache()
    return {"pairs_per_s": round(wl.n_pairs / dt, 1), "ms_per_step": round(1000 * dt, 4),
            "render_tile_us": round(1000 * ms / max(n, 1), 2), "status": flags}


def sampler_throughput(sp, torch, np, dev, batches=30):
    """The sampler front end (make / next) on the paper's ablation setting:
    512x512, ppp 0.06, d ~ U[0.8, 1.2], B = 64, F = 1, one flow field kept for
    all batches, Euler dt = 1, float images; batches consumed back to back with
    pre-fetching.  Also the same with the full model and 12-bit codes adjusted
    to a flat histogram."""
    from paper_2512_09664_amd import sampler as smp
    out = {}
    base = dict(image_shape=(512, 512), batch_size=64, flows_per_batch=1, batches_per_flow=1 << 20,
                seeding_density=(0.06, 0.06), diameter={"dist": "uniform", "range": [0.8, 1.2]},
                flow={"kind": "lamb_oseen", "grid_div": 4, "max_disp": 8.0}, seed=0)
    full = dict(base, rho=(-0.5, 0.5), jitter=(0.05, 0.05, 0.02), hide_p=0.05, bits=12, noise_sigma=0.01,
                blur={"radius": 1, "sigma": 0.7}, histogram=[1] * 4096,
                sheet={"law": "remark1", "dz0": 1.0, "shape": 2.0})
    for name, cfg in (("ablation_512", base), ("full_model_512", full)):
        s = smp.make(cfg)
        for _ in range(3):
            next(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(batches):
            b = next(s)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / batches
        s.close()
        out[name] = {"pairs_per_s": round(64 / dt, 1), "ms_per_batch": round(1000 * dt, 4),
                     "graph": bool(s._graph)}
        del s, b
        torch.cuda.empty_cache()
    return out


def histogram_cost(sp, torch, np, dev, batch, images, reps=10):
    """Histogram adjustment of scale_1024's 12-bit images to a flat target:
    microseconds per batch and the rate over its algorithmic bytes (the codes
    read twice and written once)."""
    target = torch.ones(4096, dtype=torch.int32, device=dev)
    ws = sp.histogram_match(batch, images, target, 12)
    torch.cuda.synchronize()
    sp.timing_read(None)
    sp.timing_enable(True)
    for _ in range(reps):
        sp.histogram_match(batch, images, target, 12, ws)
    torch.cuda.synchronize()
    sp.timing_enable(False)
    ms, n = sp.timing_read("histogram_match")
    sp.timing_read(None)
    us = 1000.0 * ms / n
    return {"us_per_batch": round(us, 2), "gb_per_s": round(3 * images.numel() * 2 / (us * 1e-6) / 1e9, 1)}


def _one_thread():
    """Pool initializer: one BLAS/OpenMP thread per worker process."""
    os.environ["OMP_NUM_THREADS"] = "1"


def _oracle_pair(args):
    """Worker of the all-core CPU baseline: one pair through the float64 oracle."""
    name, p, flow = args
    from oracle import pipeline as opipe
    from workloads import get_workload
    wl = get_workload(name)
    H, W = wl.sizes[p]
    opipe.generate_pair(wl, p, flow, H, W)
    return p


def gradient_cost(sp, torch, np, dev, name="grad_512", steps=10):
    """Advect + render forward vs the backward of an image loss, on float
    images: grad_512 (64 pairs of 512^2, RK4 x4, 3x3 blur) or dense_2048 (32
    pairs of 2048^2, 0.1 ppp, d ~ U[2, 6], RK4 x8, 5x5 blur; the differentiable
    form renders float images, so noise and codes are off).  The loss is the
    mean squared difference to a target pair rendered from the same particles
    moved by a perturbed flow (the grid plus Gaussian noise of 5% of its rms,
    seed 1): every step renders J and runs the loss-fused backward
    (synthpix_render_pair_backward_mse: dL/dJ = 2 (J - T) / M formed inside
    the backward's per-pixel pass).  Timed eagerly and as HIP graph replays of
    each half (a training loop's form; ``graph``); ``two_step`` is the same
    backward with dL/dJ stored first (synthpix_mse_grad, then
    synthpix_render_pair_backward)."""
    from workloads import get_workload
    wl = get_workload(name).with_(bits=0, noise_sigma=0.0)
    flows, n_max, batch, flow, sprm, aprm, rprm = _inputs(sp, torch, np, dev, wl)
    P = sp.seed(batch, sprm, wl.seed)
    x2 = torch.empty_like(P["x"])
    y2 = torch.empty_like(P["y"])
    img = torch.empty(batch.n_pixels, dtype=torch.float32, device=dev)
    wsf = sp.alloc_workspace(batch, rprm)
    wsb = sp.alloc_workspace(batch, rprm, backward=True)
    wsm = sp.alloc_workspace(batch, rprm, backward="mse")
    g = torch.Generator(device=dev).manual_seed(1)
    flow_t = flow + 0.05 * flow.pow(2).mean().sqrt() * torch.randn(flow.shape, device=dev, generator=g)
    sp.advect(batch, flow_t, aprm, P["x"], P["y"], x2, y2, wsf)
    target = sp.render_pair(batch, P["x"], P["y"], x2, y2, P["z"], P["d"], P["I0"], rprm, None, None, wsf)
    gJ = torch.empty_like(img)
    scale = 2.0 / img.numel()

    def fwd():
        sp.advect(batch, flow, aprm, P["x"], P["y"], x2, y2, wsf)
        sp.render_pair(batch, P["x"], P["y"], x2, y2, P["z"], P["d"], P["I0"], rprm, None, img, wsf)

    def bwd():   # the forward's frame-2 positions are reused, as the autograd wrapper does
        sp.render_pair_backward_mse(batch, flow, P["x"], P["y"], P["z"], P["d"], P["I0"], rprm, img, target, scale,
                                    workspace=wsm, x2=x2, y2=y2)

    def bwd_two_step():
        sp.mse_grad(img, target, scale, out=gJ)                   # the loss's own gradient, one pass
        sp.render_pair_backward(batch, flow, P["x"], P["y"], P["z"], P["d"], P["I0"], rprm, gJ, None, wsb, x2=x2, y2=y2)

    fwd()
    bwd()
    bwd_two_step()
    torch.cuda.synchronize()

    def timed(fn):
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    eager = {"fwd": timed(fwd), "bwd": timed(bwd), "bwd_two_step": timed(bwd_two_step)}
    # a training loop's form: each half captured once as a HIP graph and replayed
    # (no per-launch host work; the same kernels and buffers)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fwd()
        bwd()
    torch.cuda.current_stream().wait_stream(side)
    graphs = {}
    for name, fn in (("fwd", fwd), ("bwd", bwd)):
        graphs[name] = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graphs[name]):
            fn()
    graph = {name: timed(graphs[name].replay) for name in ("fwd", "bwd")}
    loss = float(sp.render_pair_backward_mse(batch, flow, P["x"], P["y"], P["z"], P["d"], P["I0"], rprm, img, target,
                                             scale, loss=True, workspace=wsm, x2=x2, y2=y2)["loss"])
    del graphs, wsb, wsf, wsm, gJ, img, target, flow_t
    torch.cuda.empty_cache()
    return {"loss": "mse_vs_perturbed_flow_target", "loss_value": float(f"{loss:.6e}"),
            "fwd_ms": round(1000 * eager["fwd"], 4), "bwd_ms": round(1000 * eager["bwd"], 4),
            "fwd_bwd_over_fwd": round((eager["fwd"] + eager["bwd"]) / eager["fwd"], 3),
            "graph": {"fwd_ms": round(1000 * graph["fwd"], 4), "bwd_ms": round(1000 * graph["bwd"], 4),
                      "fwd_bwd_over_fwd": round((graph["fwd"] + graph["bwd"]) / graph["fwd"], 3)},
            "two_step": {"bwd_ms": round(1000 * eager["bwd_two_step"], 4),
                         "fwd_bwd_over_fwd": round((eager["fwd"] + eager["bwd_two_step"]) / eager["fwd"], 3)}}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="scale_1024")
    ap.add_argument("--plain-steps", type=int, default=3, help="steps of the per-pair-launch comparison")
    ap.add_argument("--cpu-sample-pairs", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the uneven-batch (graph plan vs per-pair launches) and gradient measurements")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="also run a plain device copy of MB megabytes (counter calibration under a profiler)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(pairs are independent: each GPU would run this same batch on its own share)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2512_09664_amd as sp
    from workloads import get_workload, make_flows

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    wl = get_workload(args.workload)
    log(f"[bench] workload {wl.name}: {wl.n_pairs} pairs, building inputs")
    flows = make_flows(wl.flow, wl.seed, wl.sizes, wl.grid_div, wl.max_disp, wl.dt, wl.uniform_uv)
    n_max = [sp.particle_count(H, W, wl.ppp[1]) for (H, W) in wl.sizes]
    batch = sp.PairBatch.build(wl.sizes, [f.shape[:2] for f in flows], n_max, device=dev)
    flow = torch.from_numpy(np.concatenate([f.reshape(-1) for f in flows])).to(dev)
    sprm = sp.seed_params(wl.ppp, wl.d_dist, wl.d_params, wl.I0, wl.z)
    aprm = sp.advect_params(wl.dt, wl.substeps, wl.integrator)
    rprm = sp.render_params(wl.sheet_sigma, wl.d_max, wl.blur_radius, wl.blur_sigma, wl.noise_sigma, wl.bits,
                            wl.seed, wl.dt, wl.substeps, wl.integrator)
    P = sp.seed(batch, sprm, wl.seed)
    x2 = torch.empty_like(P["x"])
    y2 = torch.empty_like(P["y"])
    images = torch.empty(batch.n_pixels, dtype=sp.api.U16 if wl.bits else torch.float32, device=dev)
    ws = sp.alloc_workspace(batch, rprm)

    def step(k):
        rprm.seed = wl.seed + k                       # a fresh batch of particles and noise per step
        sp.seed(batch, sprm, wl.seed + k, out=P)
        sp.advect(batch, flow, aprm, P["x"], P["y"], x2, y2, ws)
        sp.render_pair(batch, P["x"], P["y"], x2, y2, P["z"], P["d"], P["I0"], rprm, None, images, ws)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    flags = sp.read_status(ws)
    if flags:
        raise RuntimeError(f"device status flags {flags:#x}")
    sp.timing_read(None)                              # drop anything recorded so far
    sp.timing_enable(True)
    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sp.timing_enable(False)
    kernels = {}
    for name in ("seed", "order", "advect", "bin_layout", "prep", "bin_count", "bin_scan", "bin_scatter",
                 "render_tile"):
        ms, n = sp.timing_read(name)
        if n:
            kernels[name] = {"avg_us": 1000.0 * ms / n, "launches": n}
    elapsed = t1 - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    pairs_per_s = wl.n_pairs * args.steps / elapsed
    px = wl.pixels()
    gpx_per_s = px * args.steps / elapsed / 1e9
    out_bytes = px * (2 if wl.bits else 4)
    flow_bytes = int(flow.numel()) * 4
    step_hbm_frac = (out_bytes + flow_bytes) / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9)

    # dominant kernel: the fused tile renderer; its algorithmic bytes are the stored codes
    rt = kernels.get("render_tile", {"avg_us": float("nan")})
    achieved = out_bytes / (rt["avg_us"] * 1e-6) / 1e9
    traffic = None
    valu = None
    prof = {}
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = dict(ln.strip().split("=", 1) for ln in f if "=" in ln and not ln.startswith("#"))
        if tr.get("source_sha") == source_sha(RENDER_SRC) and tr.get("workload") == wl.name:
            prof = tr
            traffic = int(tr["bytes_per_launch"])
            if "valu_insts_per_launch" in tr:
                # VALU issue of the same kernel: wave64 instructions counted by rocprofv3 per
                # launch over this run's launch time, against one per 4 cycles per SIMD
                insts = int(tr["valu_insts_per_launch"])
                rate = insts / (rt["avg_us"] * 1e-6) / 1e9
                valu = {"insts_per_launch": insts, "achieved": round(rate, 1), "peak": VALU_PEAK_GINST,
                        "unit": "G wave64 instructions/s", "frac": round(rate / VALU_PEAK_GINST, 4)}
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic}

    # batched launch vs one launch sequence per pair, same GPU, same work
    plain = None
    if args.plain_steps > 0:
        singles = []
        for p in range(wl.n_pairs):
            H, W = wl.sizes[p]
            po = batch.host[p].particle_offset
            fo = batch.host[p].flow_offset
            io = batch.host[p].image_offset
            b1 = sp.PairBatch.build([wl.sizes[p]], [flows[p].shape[:2]], [n_max[p]], [p], device=dev)
            sl = slice(po, po + n_max[p])
            singles.append((b1, flow[fo:fo + flows[p].size], {k: P[k][sl] for k in ("x", "y", "z", "d", "I0")},
                            x2[sl], y2[sl], images[io:io + 2 * H * W]))
        for b1, fl1, P1, x21, y21, im1 in singles:
            P1["n_active"] = P["n_active"][:1]
            P1["ppp"] = P["ppp"][:1]

        def plain_step(k):
            rprm.seed = wl.seed + k
            for b1, fl1, P1, x21, y21, im1 in singles:
                sp.seed(b1, sprm, wl.seed + k, out=P1)
                sp.advect(b1, fl1, aprm, P1["x"], P1["y"], x21, y21, ws)
                sp.render_pair(b1, P1["x"], P1["y"], x21, y21, P1["z"], P1["d"], P1["I0"], rprm, None, im1, ws)

        plain_step(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.plain_steps):
            plain_step(k)
        torch.cuda.synchronize()
        plain_pairs_per_s = wl.n_pairs * args.plain_steps / (time.perf_counter() - t0)
        plain = {"pairs_per_s": round(plain_pairs_per_s, 1), "batched_vs_plain": round(pairs_per_s / plain_pairs_per_s, 3)}

    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 copies of {nbytes} bytes")

    # the same renders with the noise off: the noise's share of the renderer
    rt_noise_on = render_only_us(sp, torch, batch, P, x2, y2, rprm, images, ws)
    rprm_quiet = sp.render_params(wl.sheet_sigma, wl.d_max, wl.blur_radius, wl.blur_sigma, 0.0, wl.bits,
                                  wl.seed, wl.dt, wl.substeps, wl.integrator)
    rt_noise_off = render_only_us(sp, torch, batch, P, x2, y2, rprm_quiet, images, ws)
    flags = sp.read_status(ws)
    if flags:
        raise RuntimeError(f"device status flags {flags:#x}")

    extras = {}
    if not args.no_extras:
        extras["histogram_match"] = histogram_cost(sp, torch, np, dev, batch, images)
        log(f"[bench] histogram_match: {extras['histogram_match']}")
        extras["graph_plan"] = plan_throughput(sp, torch, np, dev, wl, flows, flow, batch, sprm, aprm, rprm)
        log(f"[bench] graph plan on {wl.name}: {extras['graph_plan']}")
        del images, ws, P, x2, y2
        torch.cuda.empty_cache()
        extras["uneven_256"] = uneven_batched_vs_per_pair(sp, torch, np, dev)
        log(f"[bench] uneven_256: {extras['uneven_256']}")
        extras["grad_512"] = gradient_cost(sp, torch, np, dev)
        log(f"[bench] grad_512: {extras['grad_512']}")
        extras["dense_2048"] = dense_throughput(sp, torch, np, dev)
        log(f"[bench] dense_2048: {extras['dense_2048']}")
        extras["dense_2048_grad"] = gradient_cost(sp, torch, np, dev, "dense_2048", steps=5)
        log(f"[bench] dense_2048_grad: {extras['dense_2048_grad']}")
        extras["full_model"] = model_throughput(sp, torch, np, dev)
        log(f"[bench] full_model: {extras['full_model']}")
        extras["sampler"] = sampler_throughput(sp, torch, np, dev)
        log(f"[bench] sampler: {extras['sampler']}")
        extras["plain_256_latency"] = latency_plain_256(sp, torch, np, dev)
        log(f"[bench] plain_256 latency: {extras['plain_256_latency']}")
        extras["fp64_err"] = fp64_error(sp, torch, np, dev)
        log(f"[bench] fp64_err: {extras['fp64_err']}")
    peaks = measured_peaks(sp, torch, dev)
    log(f"[bench] measured peaks: {peaks}")
    store_peak = max(peaks["store"]["rate"], peaks["store_nt"]["rate"])
    roofline["measured_peak"] = store_peak
    roofline["frac_of_measured"] = round(achieved / store_peak, 4)
    noise = {"render_tile_us_noise_on": round(rt_noise_on, 2), "render_tile_us_noise_off": round(rt_noise_off, 2),
             "hbm_frac_noise_on": round(out_bytes / (rt_noise_on * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
             "hbm_frac_noise_off": round(out_bytes / (rt_noise_off * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    if valu is not None:
        # against the issue rate a probe of the renderer's instruction mix (float
        # FMA, multiplies and conversions interleaved with integer add, shift and bit
        # operations) sustains on this device: gfx950 issues such a mix well above
        # one wave64 instruction per four cycles per SIMD, while float-only or
        # integer-only chains stay at about that rate (fma_peak, int_peak); the
        # nominal one-per-four-cycles figure is kept beside it
        valu["nominal_peak"] = valu["peak"]
        valu["frac_of_nominal"] = valu["frac"]
        valu["fma_peak"] = peaks["fma"]["rate"]
        valu["int_peak"] = peaks["int"]["rate"]
        valu["peak"] = peaks["mix"]["rate"]
        valu["frac"] = round(valu["achieved"] / peaks["mix"]["rate"], 4)
        if prof.get("valu_busy_pct"):
            valu["valu_busy"] = round(float(prof["valu_busy_pct"]) / 100.0, 4)
    trans = None
    if prof.get("trans_insts_per_launch"):
        tr_n = int(prof["trans_insts_per_launch"])
        tr_rate = tr_n / (rt["avg_us"] * 1e-6) / 1e9
        trans = {"insts_per_launch": tr_n, "achieved": round(tr_rate, 1), "peak": peaks["trans"]["rate"],
                 "unit": "G wave64 instructions/s", "frac": round(tr_rate / peaks["trans"]["rate"], 4),
                 "share_of_valu": round(tr_n / valu["insts_per_launch"], 4) if valu else None}

    cpu = None
    if not args.no_cpu_baseline:
        import multiprocessing as mp
        from oracle import pipeline as opipe
        n = min(args.cpu_sample_pairs, wl.n_pairs)
        host_cpus = os.cpu_count() or 1
        log(f"[bench] timing the float64 CPU oracle on {n} pairs, one process")
        t0 = time.perf_counter()
        for p in range(n):
            H, W = wl.sizes[p]
            opipe.generate_pair(wl, p, flows[p], H, W)
        dt1 = time.perf_counter() - t0
        # all cores: one process per core (at most 16, the host share of one GPU), pairs spread over them
        workers = max(1, min(host_cpus, 16))
        n_pool = min(wl.n_pairs, 2 * workers)
        log(f"[bench] timing the float64 CPU oracle on {n_pool} pairs, {workers} processes")
        ctx = mp.get_context("spawn")
        with ctx.Pool(workers, initializer=_one_thread) as pool:
            pool.map(_oracle_pair, [(wl.name, 0, flows[0])] * workers)          # start-up and imports
            t0 = time.perf_counter()
            pool.map(_oracle_pair, [(wl.name, p, flows[p]) for p in range(n_pool)], chunksize=1)
            dtp = time.perf_counter() - t0
        cpu = {"value": round(n_pool / dtp, 4), "unit": "pairs/s", "cores": workers, "kind": "oracle",
               "host_cpus": host_cpus, "per_core": round(n / dt1, 4),
               "sample": f"{n_pool} of {wl.n_pairs} pairs of {wl.name} over {workers} processes ({dtp:.1f} s); "
                         f"per_core: {n} pairs in one process ({dt1:.1f} s); full path (seed, RK4 advect, render, "
                         f"blur, noise, codes) in float64 NumPy"}

    line = {"metric": METRIC, "value": round(pairs_per_s, 1), "unit": "pairs/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic", "config": describe(wl), "gpx_per_s": round(gpx_per_s, 2),
            "step_hbm_frac": round(step_hbm_frac, 4), "kernels_us": {k: round(v["avg_us"], 2) for k, v in
                                                                      kernels.items()},
            "plain": plain, **extras, "noise_split": noise, "measured_peaks": peaks, "roofline": roofline,
            "valu_issue": valu, "transcendental": trans, "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
