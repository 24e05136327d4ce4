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
            "tiling": [t.tile_w, t.tile_h, t.chunk, t.cap]}


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
            "ms_per_step": round(1000 * dt, 4), "tiling": [t.tile_w, t.tile_h, t.chunk, t.cap]}


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


def gradient_cost(sp, torch, np, dev, name="grad_512", steps=10):
    """Advect + render forward vs the backward from dL/dJ, on float images:
    grad_512 (64 pairs of 512^2, RK4 x4, 3x3 blur) or dense_2048 (32 pairs of
    2048^2, 0.1 ppp, d ~ U[2, 6], RK4 x8, 5x5 blur; the differentiable form
    renders float images, so noise and codes are off)."""
    from workloads import get_workload
    wl = get_workload(name).with_(bits=0, noise_sigma=0.0)
    flows, n_max, batch, flow, sprm, aprm, rprm = _inputs(sp, torch, np, dev, wl)
    P = sp.seed(batch, sprm, wl.seed)
    x2 = torch.empty_like(P["x"])
    y2 = torch.empty_like(P["y"])
    img = torch.empty(batch.n_pixels, dtype=torch.float32, device=dev)
    gJ = torch.randn(batch.n_pixels, device=dev, generator=torch.Generator(device=dev).manual_seed(1))
    wsf = sp.alloc_workspace(batch, rprm)
    wsb = sp.alloc_workspace(batch, rprm, backward=True)

    def fwd():
        sp.advect(batch, flow, aprm, P["x"], P["y"], x2, y2, wsf)
        sp.render_pair(batch, P["x"], P["y"], x2, y2, P["z"], P["d"], P["I0"], rprm, None, img, wsf)

    def bwd():   # as the autograd wrapper calls it: the forward's frame-2 positions are reused
        sp.render_pair_backward(batch, flow, P["x"], P["y"], P["z"], P["d"], P["I0"], rprm, gJ, None, wsb, x2=x2, y2=y2)

    fwd()
    bwd()
    torch.cuda.synchronize()
    res = {}
    for name, fn in (("fwd", fwd), ("bwd", bwd)):
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) / steps
    del wsb, wsf, gJ, img
    torch.cuda.empty_cache()
    return {"fwd_ms": round(1000 * res["fwd"], 4), "bwd_ms": round(1000 * res["bwd"], 4),
            "fwd_bwd_over_fwd": round((res["fwd"] + res["bwd"]) / res["fwd"], 3)}


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
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = dict(ln.strip().split("=", 1) for ln in f if "=" in ln and not ln.startswith("#"))
        if tr.get("source_sha") == source_sha(RENDER_SRC) and tr.get("workload") == wl.name:
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

    extras = {}
    if not args.no_extras:
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

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import pipeline as opipe
        n = min(args.cpu_sample_pairs, wl.n_pairs)
        log(f"[bench] timing the float64 CPU oracle on {n} pairs")
        t0 = time.perf_counter()
        for p in range(n):
            H, W = wl.sizes[p]
            opipe.generate_pair(wl, p, flows[p], H, W)
        dt = time.perf_counter() - t0
        cpu = {"value": round(n / dt, 4), "unit": "pairs/s", "cores": 1, "kind": "oracle",
               "sample": f"{n} of {wl.n_pairs} pairs of {wl.name}, full path (seed, RK4 advect, render, blur, "
                         f"noise, codes) in float64 NumPy, one process, {dt:.1f} s"}

    line = {"metric": METRIC, "value": round(pairs_per_s, 1), "unit": "pairs/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic", "config": describe(wl), "gpx_per_s": round(gpx_per_s, 2),
            "step_hbm_frac": round(step_hbm_frac, 4), "kernels_us": {k: round(v["avg_us"], 2) for k, v in
                                                                      kernels.items()},
            "plain": plain, **extras, "roofline": roofline, "valu_issue": valu, "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
