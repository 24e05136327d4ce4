"""GPU backward (``synthpix_render_pair_backward``) against the float64 oracle
gradient and float64 central differences.

Inputs (particles, flows, dL/dJ) are seeded host draws shared by both sides;
the oracle's frame-2 positions are its own float64 advection, except where a
test names the binary32 mirror's.
"""

import numpy as np
import pytest
import torch

from oracle import advect as oadv
from oracle import epilogue as oep
from oracle import grad as ogr
from workloads import get_workload, make_flows, particles

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2512_09664_amd as sp
    import gpu_util as gu

TOL = 1e-4   # of each quantity's largest magnitude


def _batch(sizes, grids, n_per_pair, seed, zero_frac=0.15, d_range=(1.0, 4.5)):
    """Host particles and flows of a small uneven batch, plus its device copies."""
    rng = np.random.default_rng(seed)
    P = {k: [] for k in ("x", "y", "z", "d", "I0")}
    flows = []
    for p, ((H, W), (Gh, Gw)) in enumerate(zip(sizes, grids)):
        q = particles.random_particles(seed * 100 + p, n_per_pair, H, W, d_range=d_range, pad=3.0,
                                       zero_frac=zero_frac)
        for k in P:
            P[k].append(q[k])
        flows.append(rng.normal(0.0, 1.2, size=(Gh, Gw, 2)).astype(np.float32))
    batch = gu.batch_for(sizes, grids, [n_per_pair] * len(sizes))
    dev = {k: gu.to_dev(np.concatenate(v)) for k, v in P.items()}
    flow_dev = gu.to_dev(np.concatenate([f.reshape(-1) for f in flows]))
    return P, flows, batch, dev, flow_dev


def _grad_images(batch, seed):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(batch.n_pixels).astype(np.float32)
    return g, gu.to_dev(g)


def _oracle_pair(P, p, flows, H, W, gJ, off, rp, blur, frame2=None):
    w = oep.blur_weights(blur, rp.blur_sigma) if blur else None
    integ = "rk4" if rp.advect.integrator == 1 else "euler"
    return ogr.backward_pair(P["x"][p], P["y"][p], P["z"][p], P["d"][p], P["I0"][p], float(np.float32(rp.sheet_sigma)),
                             flows[p], H, W, gJ[off:off + 2 * H * W].reshape(2, H, W), dt=rp.advect.dt,
                             substeps=rp.advect.substeps, integrator=integ, w_blur=w, cutoff=True, frame2=frame2)


def _kinks(flow, H, W, x1, y1, dt, substeps, integrator, eps=2e-4):
    """Particles whose float64 trajectory has a bilinear sample within ``eps``
    grid units (several times the binary32 trajectory's rounding) of a cell
    edge or of the clamp boundary.  The velocity's
    derivative jumps there, so either one-sided derivative is a correct
    gradient and binary32 and float64 trajectories may take different sides.
    Returns the per-particle flag and a mask of the grid nodes those
    particles' samples touch."""
    Gh, Gw = flow.shape[:2]
    px = np.asarray(x1, np.float64)
    py = np.asarray(y1, np.float64)
    h = dt / substeps
    stages = []
    for _ in range(substeps):
        if integrator == "euler":
            stages.append((px, py))
            u, v = oadv.sample(flow, H, W, px, py)
            px, py = px + h * u, py + h * v
            continue
        k1 = oadv.sample(flow, H, W, px, py)
        p2 = (px + 0.5 * h * k1[0], py + 0.5 * h * k1[1])
        k2 = oadv.sample(flow, H, W, *p2)
        p3 = (px + 0.5 * h * k2[0], py + 0.5 * h * k2[1])
        k3 = oadv.sample(flow, H, W, *p3)
        p4 = (px + h * k3[0], py + h * k3[1])
        k4 = oadv.sample(flow, H, W, *p4)
        stages += [(px, py), p2, p3, p4]
        px = px + h * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0]) / 6.0
        py = py + h * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1]) / 6.0
    flag = np.zeros(len(px), dtype=bool)
    cells = []
    for sx, sy in stages:
        gx = sx * (Gw / W) - 0.5
        gy = sy * (Gh / H) - 0.5
        flag |= (np.abs(gx - np.rint(gx)) < eps) | (np.abs(gy - np.rint(gy)) < eps)
        j0 = np.minimum(np.floor(np.clip(gx, 0, Gw - 1)).astype(int), Gw - 2)
        i0 = np.minimum(np.floor(np.clip(gy, 0, Gh - 1)).astype(int), Gh - 2)
        cells.append((i0, j0))
    nodes = np.zeros((Gh, Gw), dtype=bool)
    for i0, j0 in cells:
        for di in (0, 1):
            for dj in (0, 1):
                nodes[i0[flag] + di, j0[flag] + dj] = True
    return flag, nodes


def _close(got, ref, what, tol=TOL):
    scale = float(np.max(np.abs(ref))) if np.size(ref) else 0.0
    err = float(np.max(np.abs(np.asarray(got, np.float64) - ref))) if np.size(ref) else 0.0
    assert err <= tol * scale + 1e-30, f"{what}: max error {err:.3e} vs scale {scale:.3e}"


# (integrator, substeps, blur radius, sheet width, diameter range, d_max): the last
# two cases are the dense stress shape (d up to 6, 5x5 blur, RK4 x 8) and
# diameters wide enough for the 64-slot factor tables
CASES = [("euler", 1, 0, 0.5, (1.0, 4.5), 5.0), ("rk4", 2, 1, 0.5, (1.0, 4.5), 5.0),
         ("rk4", 4, 2, 0.8, (1.0, 4.5), 5.0), ("euler", 3, 3, 0.45, (1.0, 4.5), 5.0),
         ("rk4", 8, 2, 0.5, (2.0, 6.0), 6.0), ("rk4", 2, 1, 0.6, (5.0, 9.5), 10.0)]


@pytest.mark.parametrize("integ,n_sub,blur,sheet,d_range,d_max", CASES)
def test_backward_matches_oracle_gradient(integ, n_sub, blur, sheet, d_range, d_max):
    sizes = [(16, 16), (24, 20), (40, 48), (33, 17)]
    grids = [(6, 6), (8, 7), (10, 12), (9, 5)]
    P, flows, batch, dev, flow_dev = _batch(sizes, grids, 14, 3 + n_sub + 10 * blur, d_range=d_range)
    rp = sp.render_params(sheet, d_max, blur, 0.8, 0.0, 0, 0, 1.0, n_sub, integ)
    gJ, gJ_dev = _grad_images(batch, 99 + blur)
    ws = sp.alloc_workspace(batch, rp, backward=True)
    g = sp.render_pair_backward(batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"], rp, gJ_dev,
                                workspace=ws)
    torch.cuda.synchronize()
    assert sp.read_status(ws) == 0
    G = {k: gu.to_np(v) for k, v in g.items()}
    fo = 0
    for p, (H, W) in enumerate(sizes):
        ref = _oracle_pair(P, p, flows, H, W, gJ, batch.host[p].image_offset, rp, blur)
        sl = slice(batch.host[p].particle_offset, batch.host[p].particle_offset + 14)
        for key in ("x1", "y1", "z", "d", "I0"):
            _close(G[key][sl], ref[key], f"pair {p} {key}")
        n_f = flows[p].size
        _close(G["flow"][fo:fo + n_f].reshape(flows[p].shape), ref["flow"], f"pair {p} flow")
        fo += n_f
        term_scale = np.sum(np.abs(ref["z"] * P["z"][p])) / np.float32(rp.sheet_sigma)
        assert abs(G["sheet"][p] - ref["s"]) <= TOL * term_scale + 1e-30, (p, G["sheet"][p], ref["s"])
        # masked particles get exactly zero
        dead = P["I0"][p] == 0
        for key in ("x1", "y1", "z", "d", "I0"):
            assert np.all(G[key][sl][dead] == 0.0)


@pytest.mark.parametrize("blur,fused", [(2, False), (3, False), (0, True), (1, True), (2, True), (3, True)])
def test_backward_wide_blur_across_strips(ra, blur, fused):
    """Pairs wider than one strip of the per-pixel pass (256 columns; the last
    strip of each row ragged) and with ragged row counts (not multiples of the
    strip's 24 or 16 rows): every gradient against the oracle, frame-2
    positions from the binary32 mirror.  fused: the loss-fused backward, whose
    per-pixel pass runs at every blur radius, with dL/dJ = scale (J - T) of
    seeded images and targets (the product formed in binary32 on the host for
    the oracle), and its loss against the float64 mean over the pairs' pixels."""
    sizes = [(70, 530), (45, 300)]
    grids = [(18, 133), (12, 75)]
    n = 40
    P, flows, batch, dev, flow_dev = _batch(sizes, grids, n, 60 + blur, d_range=(1.0, 4.5))
    rp = sp.render_params(0.5, 5.0, blur, 0.9, 0.0, 0, 0, 1.0, 2, "rk4")
    args = (batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"], rp)
    if fused:
        rng = np.random.default_rng(400 + blur)
        J = rng.standard_normal(batch.n_pixels, dtype=np.float32)
        T = rng.standard_normal(batch.n_pixels, dtype=np.float32)
        scale = np.float32(2.0 / sum(2 * H * W for (H, W) in sizes))
        gJ = scale * (J - T)
        ws = sp.alloc_workspace(batch, rp, backward="mse")
        g = sp.render_pair_backward_mse(*args, gu.to_dev(J), gu.to_dev(T), float(scale), loss=True, workspace=ws)
        torch.cuda.synchronize()
        ref_loss = float(np.mean((J.astype(np.float64) - T) ** 2))
        assert abs(float(g.pop("loss")) - ref_loss) <= 1e-12 * ref_loss
    else:
        gJ, gJ_dev = _grad_images(batch, 300 + blur)
        ws = sp.alloc_workspace(batch, rp, backward=True)
        g = sp.render_pair_backward(*args, gJ_dev, workspace=ws)
        torch.cuda.synchronize()
    assert sp.read_status(ws) == 0
    G = {k: gu.to_np(v) for k, v in g.items()}
    for p, (H, W) in enumerate(sizes):
        x2, y2 = ra.advect(flows[p], H, W, P["x"][p], P["y"][p], 1.0, 2, "rk4")
        ref = _oracle_pair(P, p, flows, H, W, gJ, batch.host[p].image_offset, rp, blur, (x2, y2))
        sl = slice(batch.host[p].particle_offset, batch.host[p].particle_offset + n)
        kink, kink_nodes = _kinks(flows[p], H, W, P["x"][p], P["y"][p], 1.0, 2, "rk4")
        for key in ("z", "d", "I0"):
            _close(G[key][sl], ref[key], f"pair {p} {key}")
        for key in ("x1", "y1"):
            _close(G[key][sl][~kink], ref[key][~kink], f"pair {p} {key}")
        fo = batch.host[p].flow_offset
        gf = G["flow"][fo:fo + flows[p].size].reshape(flows[p].shape)
        assert np.max(np.abs(gf - ref["flow"])[~kink_nodes]) <= TOL * np.max(np.abs(ref["flow"])), f"pair {p} flow"
        term_scale = np.sum(np.abs(ref["z"] * P["z"][p])) / np.float32(rp.sheet_sigma)
        assert abs(G["sheet"][p] - ref["s"]) <= TOL * term_scale, p


def test_backward_matches_central_differences():
    """16x16 pair: every per-particle gradient, the sheet width and a set of flow
    nodes against float64 central differences (h = 1e-4) of the smooth forward."""
    H = W = 16
    P, flows, batch, dev, flow_dev = _batch([(H, W)], [(6, 6)], 6, 41, zero_frac=0.0)
    rp = sp.render_params(0.6, 5.0, 1, 0.7, 0.0, 0, 0, 1.0, 2, "rk4")
    gJ, gJ_dev = _grad_images(batch, 5)
    g = sp.render_pair_backward(batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"], rp, gJ_dev)
    G = {k: gu.to_np(v) for k, v in g.items()}
    w = oep.blur_weights(1, rp.blur_sigma)
    s = float(np.float32(rp.sheet_sigma))
    base = {k: P[k][0].astype(np.float64) for k in P}
    flow = flows[0].astype(np.float64)
    target = gJ.astype(np.float64).reshape(2, H, W)

    def L(x=base["x"], y=base["y"], z=base["z"], d=base["d"], I0=base["I0"], s=s, flow=flow):
        J = ogr.forward_pair(x, y, z, d, I0, s, flow, H, W, dt=1.0, substeps=2, integrator="rk4", w_blur=w,
                             cutoff=False)
        return float(np.sum(J * target))

    h = 1e-4

    def fd(name, arr, idx):
        a = arr.copy()
        a[idx] += h
        lp = L(**{name: a})
        a[idx] -= 2 * h
        lm = L(**{name: a})
        return (lp - lm) / (2 * h)

    for name, key in (("x", "x1"), ("y", "y1"), ("z", "z"), ("d", "d"), ("I0", "I0")):
        num = np.array([fd(name, base[name], i) for i in range(6)])
        _close(G[key], num, key, tol=1e-3)
    num_s = (L(s=s + h) - L(s=s - h)) / (2 * h)
    assert abs(G["sheet"][0] - num_s) <= 1e-3 * abs(num_s)
    rng = np.random.default_rng(0)
    nodes = [tuple(rng.integers(0, n) for n in flow.shape) for _ in range(24)]
    num_f = np.array([fd("flow", flow, idx) for idx in nodes])
    got_f = np.array([G["flow"].reshape(flow.shape)[idx] for idx in nodes])
    full_scale = np.max(np.abs(G["flow"]))
    assert full_scale > 0
    assert np.max(np.abs(got_f - num_f)) <= 1e-3 * full_scale


def test_backward_is_deterministic_and_autograd_agrees():
    sizes = [(40, 48), (24, 20)]
    P, flows, batch, dev, flow_dev = _batch(sizes, [(10, 12), (8, 7)], 30, 7)
    rp = sp.render_params(0.5, 5.0, 1, 0.7, 0.0, 0, 0, 1.0, 4, "rk4")
    gJ, gJ_dev = _grad_images(batch, 11)
    runs = [sp.render_pair_backward(batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"], rp, gJ_dev)
            for _ in range(2)]
    x2, y2 = sp.advect(batch, flow_dev, rp.advect, dev["x"], dev["y"])
    given = sp.render_pair_backward(batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"], rp, gJ_dev,
                                    x2=x2, y2=y2)
    torch.cuda.synchronize()
    for k in runs[0]:
        assert torch.equal(runs[0][k], runs[1][k]), k
        assert torch.equal(runs[0][k], given[k]), k   # the forward's x2, y2 instead of recomputing them
    inp = {k: v.clone().requires_grad_(True) for k, v in dev.items()}
    fl = flow_dev.clone().requires_grad_(True)
    sheet = torch.tensor(0.5, device=gu.DEV, requires_grad=True)
    img = sp.render_images(batch, fl, inp["x"], inp["y"], inp["z"], inp["d"], inp["I0"], sheet, rp)
    ref_img = sp.render_pair(batch, dev["x"], dev["y"], *sp.advect(batch, flow_dev, rp.advect, dev["x"], dev["y"]),
                             dev["z"], dev["d"], dev["I0"], rp)
    assert torch.equal(img.detach(), ref_img)
    (img * gJ_dev).sum().backward()
    g = runs[0]
    for name, key in (("x", "x1"), ("y", "y1"), ("z", "z"), ("d", "d"), ("I0", "I0")):
        assert torch.equal(inp[name].grad, g[key]), key
    assert torch.equal(fl.grad, g["flow"])
    # the shared-sheet gradient is summed by the library (float64, fixed order)
    assert torch.equal(sheet.grad, g["sheet_total"])
    assert abs(float(g["sheet_total"]) - float(g["sheet"].double().sum())) <= 1e-6 * float(g["sheet"].abs().sum())


@pytest.mark.parametrize("blur", [1, 2])
def test_backward_with_gaps_matches_packed(blur):
    """A batch whose particle, image and flow arrays leave unused gaps before
    every pair: the in-pair gradients equal those of the packed batch bit for
    bit, and every gap slot below the particle span comes back 0 (the output
    memory is filled with NaN first, so unwritten slots would show).  Blur 1
    takes the particle-major gather, blur 2 the tile-major one."""
    sizes, grids, m = [(40, 48), (24, 20), (31, 17)], [(10, 12), (8, 7), (6, 5)], 30
    P, flows, batch, dev, flow_dev = _batch(sizes, grids, m, 13)
    rp = sp.render_params(0.5, 5.0, blur, 0.7, 0.0, 0, 0, 1.0, 2, "rk4")
    gJ, gJ_dev = _grad_images(batch, 17)
    ref = sp.render_pair_backward(batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"], rp, gJ_dev)
    gaps = (5, 12, 4)
    gb = sp.PairBatch.build(sizes, grids, [m] * 3, device=gu.DEV, gaps=gaps)

    def spread(a, n_total, gap, sizes_):
        out = np.full(n_total, np.nan, np.float32)
        o = 0
        for p, k in enumerate(sizes_):
            o += gap
            out[o:o + k] = a[sum(sizes_[:p]):sum(sizes_[:p]) + k]
            o += k
        return out

    n_sizes = [m] * 3
    gdev = {k: gu.to_dev(np.nan_to_num(spread(np.concatenate(P[k]), gb.n_particles, gaps[0], n_sizes), nan=0.0))
            for k in P}
    pix = [2 * H * W for (H, W) in sizes]
    gJg = gu.to_dev(np.nan_to_num(spread(gJ, gb.n_pixels, gaps[1], pix), nan=0.0))
    fl = [2 * a * b for (a, b) in grids]
    gflow = gu.to_dev(np.nan_to_num(spread(np.concatenate([f.reshape(-1) for f in flows]), gb.n_flow, gaps[2], fl),
                                    nan=0.0))
    for _ in range(3):     # NaN-filled blocks for the caching allocator to hand out next
        junk = torch.full((gb.n_particles,), float("nan"), device=gu.DEV)
        del junk
    got = sp.render_pair_backward(gb, gflow, gdev["x"], gdev["y"], gdev["z"], gdev["d"], gdev["I0"], rp, gJg)
    torch.cuda.synchronize()
    for key in ("x1", "y1", "z", "d", "I0"):
        g = gu.to_np(got[key])
        r = gu.to_np(ref[key])
        o = 0
        for p in range(3):
            assert np.all(g[o:o + gaps[0]] == 0.0), (key, p)
            o += gaps[0]
            assert np.array_equal(g[o:o + m], r[p * m:(p + 1) * m]), (key, p)
            o += m
    assert torch.equal(got["sheet"], ref["sheet"]) and torch.equal(got["sheet_total"], ref["sheet_total"])
    gf, rf = gu.to_np(got["flow"]), gu.to_np(ref["flow"])
    o = ro = 0
    for p in range(3):
        assert np.all(gf[o:o + gaps[2]] == 0.0)
        o += gaps[2]
        assert np.array_equal(gf[o:o + fl[p]], rf[ro:ro + fl[p]]), p
        o += fl[p]
        ro += fl[p]
    # forward on the gapped layout: pairs' images equal the packed ones, gaps stay 0
    img_g = gu.to_np(sp.render_images(gb, gflow, gdev["x"], gdev["y"], gdev["z"], gdev["d"], gdev["I0"], 0.5, rp))
    img_r = gu.to_np(sp.render_images(batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"], 0.5, rp))
    o = ro = 0
    for p in range(3):
        assert np.all(img_g[o:o + gaps[1]] == 0.0)
        o += gaps[1]
        assert np.array_equal(img_g[o:o + pix[p]], img_r[ro:ro + pix[p]]), p
        o += pix[p]
        ro += pix[p]


def test_backward_full_size_pairs(ra):
    """grad_512 at full size (64 pairs of 512x512, RK4 x4, 3x3 blur): every
    gradient of two sampled pairs against the oracle."""
    wl = get_workload("grad_512")
    flows = make_flows(wl.flow, wl.seed, wl.sizes, wl.grid_div, wl.max_disp, wl.dt, wl.uniform_uv)
    n_max = [sp.particle_count(H, W, wl.ppp[1]) for (H, W) in wl.sizes]
    batch = gu.batch_for(wl.sizes, [f.shape[:2] for f in flows], n_max)
    P = {k: [] for k in ("x", "y", "z", "d", "I0")}
    for p, (H, W) in enumerate(wl.sizes):
        q = ra.seed_pair(H, W, n_max[p], wl.ppp, p, wl.seed, wl.d_dist, wl.d_params, wl.I0, wl.z)
        for k in P:
            P[k].append(q[k])
    dev = {k: gu.to_dev(np.concatenate(v)) for k, v in P.items()}
    flow_dev = gu.to_dev(np.concatenate([f.reshape(-1) for f in flows]))
    rp = sp.render_params(wl.sheet_sigma, wl.d_max, wl.blur_radius, wl.blur_sigma, 0.0, 0, wl.seed, wl.dt,
                          wl.substeps, wl.integrator)
    gJ, gJ_dev = _grad_images(batch, 2024)
    ws = sp.alloc_workspace(batch, rp, backward=True)
    g = sp.render_pair_backward(batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"], rp, gJ_dev,
                                workspace=ws)
    torch.cuda.synchronize()
    assert sp.read_status(ws) == 0
    G = {k: gu.to_np(v) for k, v in g.items()}
    for p in (0, 37):
        H, W = wl.sizes[p]
        # frame-2 positions of the binary32 mirror (the kernels' own rounding of the
        # trajectory), so the comparison measures the gradient arithmetic; against
        # the float64 trajectory the position rounding (~1e-4 px at 512 px) moves the
        # frame-2 gradients by up to a few 1e-4 of their scale
        x2, y2 = ra.advect(flows[p], H, W, P["x"][p], P["y"][p], wl.dt, wl.substeps, wl.integrator)
        ref = _oracle_pair(P, p, flows, H, W, gJ, batch.host[p].image_offset, rp, wl.blur_radius, (x2, y2))
        ref64 = _oracle_pair(P, p, flows, H, W, gJ, batch.host[p].image_offset, rp, wl.blur_radius)
        po = batch.host[p].particle_offset
        sl = slice(po, po + n_max[p])
        kink, kink_nodes = _kinks(flows[p], H, W, P["x"][p], P["y"][p], wl.dt, wl.substeps, wl.integrator)
        assert kink.sum() < 0.05 * len(kink)
        for key in ("z", "d", "I0"):
            _close(G[key][sl], ref[key], f"pair {p} {key}")
            _close(G[key][sl], ref64[key], f"pair {p} {key} (float64 trajectory)", tol=2e-3)
        for key in ("x1", "y1"):
            # exact where the trajectory's velocity is differentiable; at a kink
            # the two one-sided derivatives differ by O(h) of the flow's jump
            scale = np.max(np.abs(ref[key]))
            _close(G[key][sl][~kink], ref[key][~kink], f"pair {p} {key}")
            assert np.max(np.abs(G[key][sl] - ref[key])) <= 5e-3 * scale, key
        fo = batch.host[p].flow_offset
        gf = G["flow"][fo:fo + flows[p].size].reshape(flows[p].shape)
        scale = np.max(np.abs(ref["flow"]))
        assert np.max(np.abs(gf - ref["flow"])[~kink_nodes]) <= TOL * scale, f"pair {p} flow"
        assert np.max(np.abs(gf - ref["flow"])) <= 5e-3 * scale, f"pair {p} flow near kinks"
        term_scale = np.sum(np.abs(ref["z"] * P["z"][p])) / np.float32(rp.sheet_sigma)
        assert abs(G["sheet"][p] - ref["s"]) <= TOL * term_scale


def test_backward_dense_2048_sampled(ra):
    """dense_2048 at full size (32 pairs of 2048^2, 0.1 ppp, d ~ U[2, 6], RK4 x 8,
    5x5 blur).  A particle's own gradients depend only on dL/dJ, its parameters
    and the flow, so a sample of particles is checked against the oracle run on
    that sample alone; the flow and sheet gradients, sums over particles, are
    checked on a second launch in which only the sample is lit."""
    wl = get_workload("dense_2048")
    flows = make_flows(wl.flow, wl.seed, wl.sizes, wl.grid_div, wl.max_disp, wl.dt, wl.uniform_uv)
    n_max = [sp.particle_count(H, W, wl.ppp[1]) for (H, W) in wl.sizes]
    batch = gu.batch_for(wl.sizes, [f.shape[:2] for f in flows], n_max)
    P = {k: [] for k in ("x", "y", "z", "d", "I0")}
    for p, (H, W) in enumerate(wl.sizes):
        q = ra.seed_pair(H, W, n_max[p], wl.ppp, p, wl.seed, wl.d_dist, wl.d_params, wl.I0, wl.z)
        for k in P:
            P[k].append(q[k])
    dev = {k: gu.to_dev(np.concatenate(v)) for k, v in P.items()}
    flow_dev = gu.to_dev(np.concatenate([f.reshape(-1) for f in flows]))
    rp = sp.render_params(wl.sheet_sigma, wl.d_max, wl.blur_radius, wl.blur_sigma, 0.0, 0, wl.seed, wl.dt,
                          wl.substeps, wl.integrator)
    gJ, gJ_dev = _grad_images(batch, 2048)
    ws = sp.alloc_workspace(batch, rp, backward=True)
    print("[case] dense_2048 backward, all particles", flush=True)
    g = sp.render_pair_backward(batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"], rp, gJ_dev,
                                workspace=ws)
    torch.cuda.synchronize()
    assert sp.read_status(ws) == 0
    G = {k: gu.to_np(v) for k, v in g.items()}
    pairs = (0, 31)
    sel = {p: np.arange(p % 7, n_max[p], 211) for p in pairs}
    lit = np.concatenate(P["I0"]).copy()
    keep = np.zeros(lit.size, dtype=bool)
    for p in pairs:
        keep[batch.host[p].particle_offset + sel[p]] = True
    lit[~keep] = 0.0
    print("[case] dense_2048 backward, sampled particles lit", flush=True)
    gs = sp.render_pair_backward(batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], gu.to_dev(lit), rp,
                                 gJ_dev, workspace=ws)
    torch.cuda.synchronize()
    assert sp.read_status(ws) == 0
    GS = {k: gu.to_np(v) for k, v in gs.items()}
    for p in pairs:
        H, W = wl.sizes[p]
        s = sel[p]
        Q = {k: [P[k][p][s]] for k in P}
        x2, y2 = ra.advect(flows[p], H, W, Q["x"][0], Q["y"][0], wl.dt, wl.substeps, wl.integrator)
        ref = _oracle_pair(Q, 0, [flows[p]], H, W, gJ, batch.host[p].image_offset, rp, wl.blur_radius, (x2, y2))
        sl = batch.host[p].particle_offset + s
        kink, kink_nodes = _kinks(flows[p], H, W, Q["x"][0], Q["y"][0], wl.dt, wl.substeps, wl.integrator)
        assert kink.sum() < 0.05 * len(kink)
        for key in ("z", "d", "I0"):
            _close(G[key][sl], ref[key], f"pair {p} {key}")
            _close(GS[key][sl], ref[key], f"pair {p} {key} (sample lit)")
        for key in ("x1", "y1"):
            scale = np.max(np.abs(ref[key]))
            _close(G[key][sl][~kink], ref[key][~kink], f"pair {p} {key}")
            assert np.max(np.abs(G[key][sl] - ref[key])) <= 5e-3 * scale, key
        fo = batch.host[p].flow_offset
        gf = GS["flow"][fo:fo + flows[p].size].reshape(flows[p].shape)
        scale = np.max(np.abs(ref["flow"]))
        assert np.max(np.abs(gf - ref["flow"])[~kink_nodes]) <= TOL * scale, f"pair {p} flow"
        assert np.max(np.abs(gf - ref["flow"])) <= 5e-3 * scale, f"pair {p} flow near kinks"
        term_scale = np.sum(np.abs(ref["z"] * Q["z"][0])) / np.float32(rp.sheet_sigma)
        assert abs(GS["sheet"][p] - ref["s"]) <= TOL * term_scale, p
    # pairs with no lit particle get a zero flow gradient in the masked launch
    fo = batch.host[5].flow_offset
    assert not np.any(GS["flow"][fo:fo + flows[5].size])


def test_mse_loss_against_perturbed_flow_target():
    """The differentiable workload's loss: the mean squared difference between
    the rendered pair and a target pair rendered from the same particles under a
    perturbed flow (the grid plus Gaussian noise of 5% of its rms).  The
    autograd gradient of every input equals the float64 oracle gradient of the
    same loss (its dL/dJ formed from the oracle's own images)."""
    sizes = [(40, 48), (24, 20)]
    grids = [(10, 12), (8, 7)]
    P, flows, batch, dev, flow_dev = _batch(sizes, grids, 24, 21)
    rng = np.random.default_rng(1)
    flows_t = [(f + 0.05 * np.sqrt(np.mean(f.astype(np.float64) ** 2)) * rng.standard_normal(f.shape))
               .astype(np.float32) for f in flows]
    flow_t_dev = gu.to_dev(np.concatenate([f.reshape(-1) for f in flows_t]))
    rp = sp.render_params(0.5, 5.0, 1, 0.7, 0.0, 0, 0, 1.0, 2, "rk4")
    inp = {k: v.clone().requires_grad_(True) for k, v in dev.items()}
    fl = flow_dev.clone().requires_grad_(True)
    img = sp.render_images(batch, fl, inp["x"], inp["y"], inp["z"], inp["d"], inp["I0"], 0.5, rp)
    with torch.no_grad():
        x2t, y2t = sp.advect(batch, flow_t_dev, rp.advect, dev["x"], dev["y"])
        target = sp.render_pair(batch, dev["x"], dev["y"], x2t, y2t, dev["z"], dev["d"], dev["I0"], rp)
    loss = ((img - target) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    w = oep.blur_weights(1, rp.blur_sigma)
    M = batch.n_pixels
    fo = 0
    for p, (H, W) in enumerate(sizes):
        args = (P["x"][p], P["y"][p], P["z"][p], P["d"][p], P["I0"][p], 0.5)
        J = ogr.forward_pair(*args, flows[p], H, W, 1.0, 2, "rk4", w, cutoff=True)
        T = ogr.forward_pair(*args, flows_t[p], H, W, 1.0, 2, "rk4", w, cutoff=True)
        gJ = 2.0 * (J - T) / M
        ref = ogr.backward_pair(*args, flows[p], H, W, gJ, dt=1.0, substeps=2, integrator="rk4", w_blur=w,
                                cutoff=True)
        sl = slice(batch.host[p].particle_offset, batch.host[p].particle_offset + 24)
        for name, key in (("x", "x1"), ("y", "y1"), ("z", "z"), ("d", "d"), ("I0", "I0")):
            _close(gu.to_np(inp[name].grad)[sl], ref[key], f"pair {p} {key}", tol=1e-3)
        n_f = flows[p].size
        _close(gu.to_np(fl.grad)[fo:fo + n_f].reshape(flows[p].shape), ref["flow"], f"pair {p} flow", tol=1e-3)
        fo += n_f


@pytest.mark.parametrize("blur", [2, 3])
def test_tile_gather_matches_particle_gather(blur):
    """The two adjoint gathers on one batch: the tile-major one (particles grouped
    by the home block of each frame's position, the block plus its halo staged in
    LDS; taken for blur radius >= 2 and d_max <= 9) and the particle-major one
    (global reads; taken here by raising d_max to 10, which changes no
    footprint).  Pairs span many 32-pixel home blocks with ragged edges;
    particles lie inside, on block and image edges and up to 3 px outside the
    image; frame 2 is both recomputed and passed in.  Both gathers read the same
    B^T dL/dJ, so every gradient agrees bit for bit."""
    sizes = [(70, 97), (33, 130), (128, 64)]
    grids = [(18, 25), (9, 33), (32, 16)]
    P, flows, batch, dev, flow_dev = _batch(sizes, grids, 90, 500 + blur, d_range=(1.0, 6.0))
    out = []
    for d_max in (6.0, 10.0):
        rp = sp.render_params(0.5, d_max, blur, 0.8, 0.0, 0, 0, 1.0, 3, "rk4")
        gJ, gJ_dev = _grad_images(batch, 700 + blur)
        ws = sp.alloc_workspace(batch, rp, backward=True)
        g = sp.render_pair_backward(batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"], rp, gJ_dev,
                                    workspace=ws)
        x2, y2 = sp.advect(batch, flow_dev, rp.advect, dev["x"], dev["y"])
        g2 = sp.render_pair_backward(batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"], rp, gJ_dev,
                                     x2=x2, y2=y2)
        torch.cuda.synchronize()
        assert sp.read_status(ws) == 0
        for k in g:
            assert torch.equal(g[k], g2[k]), (d_max, k)
        out.append({k: gu.to_np(v) for k, v in g.items()})
    tile, part = out
    for k in ("x1", "y1", "z", "d", "I0", "sheet", "flow"):
        assert np.array_equal(tile[k], part[k]), k


@pytest.mark.parametrize("n", [0, 3, 4096, 1_000_003])
def test_mse_grad_matches_definition(n):
    """dL/dJ = scale (J - T) equals the same binary32 operations on the host bit
    for bit (a ragged tail included, and in place over J); the loss equals the
    float64 mean of (J - T)^2 to rounding, and repeats bit for bit."""
    rng = np.random.default_rng(n)
    J = rng.standard_normal(n).astype(np.float32)
    T = rng.standard_normal(n).astype(np.float32)
    Jd, Td = gu.to_dev(J), gu.to_dev(T)
    scale = np.float32(2.0 / max(n, 1))
    g, loss = sp.mse_grad(Jd, Td, float(scale), loss=True)
    g2, loss2 = sp.mse_grad(Jd, Td, float(scale), loss=True)
    torch.cuda.synchronize()
    assert np.array_equal(gu.to_np(g), scale * (J - T))
    ref = float(np.mean((J.astype(np.float64) - T) ** 2)) if n else 0.0
    assert abs(float(loss) - ref) <= 1e-12 * max(ref, 1.0)
    assert float(loss) == float(loss2) and torch.equal(g, g2)
    if n:
        sp.mse_grad(Jd, Td, float(scale), out=Jd)             # in place over J
        torch.cuda.synchronize()
        assert np.array_equal(gu.to_np(Jd), scale * (J - T))


def _far_batch(n, seed, speed):
    """One 48 x 160 pair on a grid of one node per 1.25 px, its n particles in a
    3 x 3-pixel cluster near the left edge, and a smooth flow carrying them
    about ``speed`` px to the right: their later samples leave the node window
    of their workgroup (the box of the starting cells grown to fill the window)."""
    H, W, Gh, Gw = 48, 160, 38, 128
    rng = np.random.default_rng(seed)
    P = {"x": (10.0 + 3.0 * rng.random(n)).astype(np.float32), "y": (22.0 + 3.0 * rng.random(n)).astype(np.float32),
         "z": rng.uniform(-0.5, 0.5, n).astype(np.float32), "d": rng.uniform(2.0, 3.0, n).astype(np.float32),
         "I0": rng.uniform(0.8, 1.0, n).astype(np.float32)}
    yy, xx = np.meshgrid(np.arange(Gh), np.arange(Gw), indexing="ij")
    flow = np.stack([speed * (1.0 + 0.1 * np.sin(xx / 9.0)), 0.8 * np.cos(yy / 5.0)], -1).astype(np.float32)
    batch = gu.batch_for([(H, W)], [(Gh, Gw)], [n])
    dev = {k: gu.to_dev(v) for k, v in P.items()}
    return (H, W), P, flow, batch, dev, gu.to_dev(flow.reshape(-1))


def test_flow_gradient_outside_the_window():
    """Particles that travel ~60 nodes, beyond their workgroup's node window:
    the contributions outside it travel as records and the flow gradient (and
    every other gradient) still matches the float64 oracle; no overflow."""
    (H, W), P, flow, batch, dev, flow_dev = _far_batch(4, 3, 75.0)
    rp = sp.render_params(0.5, 5.0, 0, 0.8, 0.0, 0, 0, 1.0, 4, "rk4")
    gJ, gJ_dev = _grad_images(batch, 17)
    ws = sp.alloc_workspace(batch, rp, backward=True)
    g = sp.render_pair_backward(batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"], rp, gJ_dev,
                                workspace=ws)
    torch.cuda.synchronize()
    assert sp.read_status(ws) == 0
    G = {k: gu.to_np(v) for k, v in g.items()}
    x2, _ = sp.advect(batch, flow_dev, rp.advect, dev["x"], dev["y"])
    assert float(gu.to_np(x2).min()) > 10.0 + 55.0                  # they did travel
    ref = _oracle_pair({k: [v] for k, v in P.items()}, 0, [flow], H, W, gJ, 0, rp, 0)
    kink, kink_nodes = _kinks(flow, H, W, P["x"], P["y"], 1.0, 4, "rk4")
    for key in ("z", "d", "I0"):
        _close(G[key], ref[key], key)
    for key in ("x1", "y1"):
        _close(G[key][~kink], ref[key][~kink], key)
    gf = G["flow"].reshape(flow.shape)
    assert np.max(np.abs(gf)[:, 50:]) > 0                            # far nodes got their share
    assert np.max(np.abs(gf - ref["flow"])[~kink_nodes]) <= TOL * np.max(np.abs(ref["flow"]))


def test_flow_gradient_overflow_is_flagged():
    """Far more far-travelling contributions than a workgroup keeps: the status
    word says the flow gradient is incomplete."""
    (H, W), P, flow, batch, dev, flow_dev = _far_batch(256, 4, 75.0)
    rp = sp.render_params(0.5, 5.0, 0, 0.8, 0.0, 0, 0, 1.0, 4, "rk4")
    gJ, gJ_dev = _grad_images(batch, 18)
    ws = sp.alloc_workspace(batch, rp, backward=True)
    sp.render_pair_backward(batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"], rp, gJ_dev,
                            workspace=ws)
    torch.cuda.synchronize()
    assert sp.read_status(ws) & 0x20


@pytest.mark.parametrize("fused", [False, True])
def test_forward_backward_replay_from_a_graph(fused):
    """Advect + render and the loss's backward (loss gradient + backward, or the
    loss-fused backward with its loss value) captured as HIP graphs and
    replayed three times, with eager work in between: every replay's images,
    gradients and loss equal the eager call's bit for bit."""
    sizes = [(64, 80), (48, 48)]
    grids = [(16, 20), (12, 12)]
    P, flows, batch, dev, flow_dev = _batch(sizes, grids, 60, 77)
    for blur in (1, 2):
        rp = sp.render_params(0.5, 5.0, blur, 0.8, 0.0, 0, 0, 1.0, 2, "rk4")
        wsf = sp.alloc_workspace(batch, rp)
        wsb = sp.alloc_workspace(batch, rp, backward="mse" if fused else True)
        x2 = torch.empty_like(dev["x"])
        y2 = torch.empty_like(dev["y"])
        img = torch.empty(batch.n_pixels, dtype=torch.float32, device=gu.DEV)
        target = torch.from_numpy(np.random.default_rng(blur).random(batch.n_pixels, dtype=np.float32)).to(gu.DEV)
        gJ = torch.empty_like(img)
        out = {}

        def step():
            sp.advect(batch, flow_dev, rp.advect, dev["x"], dev["y"], x2, y2, wsf)
            sp.render_pair(batch, dev["x"], dev["y"], x2, y2, dev["z"], dev["d"], dev["I0"], rp, None, img, wsf)
            if fused:
                out["g"] = sp.render_pair_backward_mse(batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"],
                                                       dev["I0"], rp, img, target, 2.0 / batch.n_pixels, loss=True,
                                                       workspace=wsb, x2=x2, y2=y2)
                return
            sp.mse_grad(img, target, out=gJ)
            out["g"] = sp.render_pair_backward(batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"],
                                               rp, gJ, None, wsb, x2=x2, y2=y2)

        step()
        torch.cuda.synchronize()
        ref_img = img.clone()
        ref = {k: v.clone() for k, v in out["g"].items()}
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        g_graph = out["g"]
        for k in range(3):
            img.fill_(-1.0)
            for v in g_graph.values():
                v.fill_(float("nan"))
            sp.render_pair(batch, dev["x"], dev["y"], x2, y2, dev["z"], dev["d"], dev["I0"], rp)   # eager work
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(img, ref_img), (blur, k)
            for key in ref:
                assert torch.equal(g_graph[key], ref[key]), (blur, k, key)
        del graph


@pytest.mark.parametrize("integ,n_sub,blur,sheet,d_range,d_max", CASES)
def test_backward_mse_matches_oracle_and_two_step(integ, n_sub, blur, sheet, d_range, d_max):
    """The loss-fused backward (``synthpix_render_pair_backward_mse``) on seeded
    float images J and a target T: its gradients equal the float64 oracle
    gradient for dL/dJ = scale (J - T) (that product formed in binary32 on the
    host, as the loss defines it); they equal ``mse_grad`` followed by
    ``render_pair_backward`` bit for bit where both run the same per-pixel pass
    (no blur, radius >= 2) and to float32 rounding where the two-step form folds
    a radius-1 blur into its factor tables; the loss is the float64 mean of
    (J - T)^2 over the pairs' pixels and repeats bit for bit."""
    sizes = [(16, 16), (24, 20), (40, 48), (33, 17)]
    grids = [(6, 6), (8, 7), (10, 12), (9, 5)]
    P, flows, batch, dev, flow_dev = _batch(sizes, grids, 14, 3 + n_sub + 10 * blur, d_range=d_range)
    rp = sp.render_params(sheet, d_max, blur, 0.8, 0.0, 0, 0, 1.0, n_sub, integ)
    rng = np.random.default_rng(31 + blur)
    J = rng.standard_normal(batch.n_pixels).astype(np.float32)
    T = rng.standard_normal(batch.n_pixels).astype(np.float32)
    Jd, Td = gu.to_dev(J), gu.to_dev(T)
    M = sum(2 * H * W for (H, W) in sizes)
    scale = np.float32(2.0 / M)
    gJ = scale * (J - T)
    ws = sp.alloc_workspace(batch, rp, backward="mse")
    args = (batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"], rp)
    g = sp.render_pair_backward_mse(*args, Jd, Td, float(scale), loss=True, workspace=ws)
    g_again = sp.render_pair_backward_mse(*args, Jd, Td, float(scale), loss=True)
    gJ_dev, _ = sp.mse_grad(Jd, Td, float(scale))
    two = sp.render_pair_backward(*args, gJ_dev)
    torch.cuda.synchronize()
    assert sp.read_status(ws) == 0
    ref_loss = float(np.mean((J.astype(np.float64) - T) ** 2))
    assert abs(float(g["loss"]) - ref_loss) <= 1e-12 * ref_loss
    for k in g:
        assert torch.equal(g[k], g_again[k]), k
    for k in two:
        if blur == 1:
            _close(gu.to_np(g[k]), gu.to_np(two[k]).astype(np.float64), f"two-step {k}", tol=1e-5)
        else:
            assert torch.equal(g[k], two[k]), k
    G = {k: gu.to_np(v) for k, v in g.items()}
    fo = 0
    for p, (H, W) in enumerate(sizes):
        ref = _oracle_pair(P, p, flows, H, W, gJ, batch.host[p].image_offset, rp, blur)
        sl = slice(batch.host[p].particle_offset, batch.host[p].particle_offset + 14)
        for key in ("x1", "y1", "z", "d", "I0"):
            _close(G[key][sl], ref[key], f"pair {p} {key}")
        n_f = flows[p].size
        _close(G["flow"][fo:fo + n_f].reshape(flows[p].shape), ref["flow"], f"pair {p} flow")
        fo += n_f


def test_backward_mse_loss_without_particles():
    """With no particle in any pair the loss-fused backward still reports the
    loss of the images (and zero gradients)."""
    sizes = [(20, 300), (37, 5)]
    batch = gu.batch_for(sizes, [(4, 4), (4, 4)], [0, 0])
    rp = sp.render_params(0.5, 5.0, 2, 0.8, 0.0, 0, 0, 1.0, 2, "rk4")
    rng = np.random.default_rng(5)
    J = rng.standard_normal(batch.n_pixels).astype(np.float32)
    T = rng.standard_normal(batch.n_pixels).astype(np.float32)
    e = torch.zeros(1, dtype=torch.float32, device="cuda")
    flow = torch.zeros(2 * 2 * 16, dtype=torch.float32, device="cuda")
    g = sp.render_pair_backward_mse(batch, flow, e, e, e, e, e, rp, gu.to_dev(J), gu.to_dev(T), 1.0, loss=True)
    torch.cuda.synchronize()
    ref = float(np.mean((J.astype(np.float64) - T) ** 2))
    assert abs(float(g["loss"]) - ref) <= 1e-12 * ref
    assert float(g["flow"].abs().max()) == 0.0 and float(g["sheet"].abs().max()) == 0.0


@pytest.mark.parametrize("name", ["grad_512", "dense_2048"])
def test_backward_mse_full_size(ra, name):
    """The loss-fused backward at the bench's full sizes (grad_512: 3x3 blur,
    particle-major gather; dense_2048: 5x5 blur, tile-major gather) against the
    two-step form whose gradients the tests above check against the oracle:
    the same values with the 5x5 blur (both run the same per-pixel pass), to
    1e-5 of each output's largest magnitude with the 3x3 blur (folded into the
    two-step gather's tables); the loss is the float64 mean of (J - T)^2 to
    1e-12, and the device status word stays clear."""
    wl = get_workload(name)
    flows = make_flows(wl.flow, wl.seed, wl.sizes, wl.grid_div, wl.max_disp, wl.dt, wl.uniform_uv)
    n_max = [sp.particle_count(H, W, wl.ppp[1]) for (H, W) in wl.sizes]
    batch = gu.batch_for(wl.sizes, [f.shape[:2] for f in flows], n_max)
    P = {k: [] for k in ("x", "y", "z", "d", "I0")}
    for p, (H, W) in enumerate(wl.sizes):
        q = ra.seed_pair(H, W, n_max[p], wl.ppp, p, wl.seed, wl.d_dist, wl.d_params, wl.I0, wl.z)
        for k in P:
            P[k].append(q[k])
    dev = {k: gu.to_dev(np.concatenate(v)) for k, v in P.items()}
    flow_dev = gu.to_dev(np.concatenate([f.reshape(-1) for f in flows]))
    rp = sp.render_params(wl.sheet_sigma, wl.d_max, wl.blur_radius, wl.blur_sigma, 0.0, 0, wl.seed, wl.dt,
                          wl.substeps, wl.integrator)
    rng = np.random.default_rng(77)
    J = rng.standard_normal(batch.n_pixels, dtype=np.float32)
    T = rng.standard_normal(batch.n_pixels, dtype=np.float32)
    Jd, Td = gu.to_dev(J), gu.to_dev(T)
    scale = np.float32(2.0 / batch.n_pixels)
    args = (batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"], rp)
    print(f"[case] {name} loss-fused backward", flush=True)
    ws = sp.alloc_workspace(batch, rp, backward="mse")
    g = sp.render_pair_backward_mse(*args, Jd, Td, float(scale), loss=True, workspace=ws)
    torch.cuda.synchronize()
    assert sp.read_status(ws) == 0
    print(f"[case] {name} two-step backward", flush=True)
    gJ_dev, _ = sp.mse_grad(Jd, Td, float(scale))
    two = sp.render_pair_backward(*args, gJ_dev)
    torch.cuda.synchronize()
    ref_loss = float(np.mean((J.astype(np.float64) - T) ** 2))
    assert abs(float(g["loss"]) - ref_loss) <= 1e-12 * ref_loss
    for k in two:
        if wl.blur_radius == 1:
            _close(gu.to_np(g[k]), gu.to_np(two[k]).astype(np.float64), f"{name} {k}", tol=1e-5)
        else:
            assert torch.equal(g[k], two[k]), k


@pytest.mark.parametrize("blur", [1, 2])
def test_backward_mse_with_gaps_matches_packed(blur):
    """The loss-fused backward on a batch whose particle, image and flow arrays
    leave gaps before every pair, the images' and the target's gaps holding NaN:
    gradients and loss equal those of the packed batch bit for bit (so no gap
    pixel is read), gap slots come back 0."""
    sizes, grids, m = [(40, 48), (24, 20), (31, 17)], [(10, 12), (8, 7), (6, 5)], 30
    P, flows, batch, dev, flow_dev = _batch(sizes, grids, m, 23)
    rp = sp.render_params(0.5, 5.0, blur, 0.7, 0.0, 0, 0, 1.0, 2, "rk4")
    rng = np.random.default_rng(29)
    J = rng.standard_normal(batch.n_pixels).astype(np.float32)
    T = rng.standard_normal(batch.n_pixels).astype(np.float32)
    scale = 0.125
    ref = sp.render_pair_backward_mse(batch, flow_dev, dev["x"], dev["y"], dev["z"], dev["d"], dev["I0"], rp,
                                      gu.to_dev(J), gu.to_dev(T), scale, loss=True)
    gaps = (5, 12, 4)
    gb = sp.PairBatch.build(sizes, grids, [m] * 3, device=gu.DEV, gaps=gaps)

    def spread(a, n_total, gap, sizes_):
        out = np.full(n_total, np.nan, np.float32)
        o = 0
        for p, k in enumerate(sizes_):
            o += gap
            out[o:o + k] = a[sum(sizes_[:p]):sum(sizes_[:p]) + k]
            o += k
        return out

    gdev = {k: gu.to_dev(np.nan_to_num(spread(np.concatenate(P[k]), gb.n_particles, gaps[0], [m] * 3), nan=0.0))
            for k in P}
    pix = [2 * H * W for (H, W) in sizes]
    Jg, Tg = gu.to_dev(spread(J, gb.n_pixels, gaps[1], pix)), gu.to_dev(spread(T, gb.n_pixels, gaps[1], pix))
    fl = [2 * a * b for (a, b) in grids]
    gflow = gu.to_dev(np.nan_to_num(spread(np.concatenate([f.reshape(-1) for f in flows]), gb.n_flow, gaps[2], fl),
                                    nan=0.0))
    got = sp.render_pair_backward_mse(gb, gflow, gdev["x"], gdev["y"], gdev["z"], gdev["d"], gdev["I0"], rp, Jg, Tg,
                                      scale, loss=True)
    torch.cuda.synchronize()
    assert float(got["loss"]) == float(ref["loss"])
    for key in ("x1", "y1", "z", "d", "I0"):
        g, r = gu.to_np(got[key]), gu.to_np(ref[key])
        o = 0
        for p in range(3):
            assert np.all(g[o:o + gaps[0]] == 0.0), (key, p)
            o += gaps[0]
            assert np.array_equal(g[o:o + m], r[p * m:(p + 1) * m]), (key, p)
            o += m
    assert torch.equal(got["sheet"], ref["sheet"]) and torch.equal(got["sheet_total"], ref["sheet_total"])
    gf, rf = gu.to_np(got["flow"]), gu.to_np(ref["flow"])
    o = ro = 0
    for p in range(3):
        assert np.all(gf[o:o + gaps[2]] == 0.0)
        o += gaps[2]
        assert np.array_equal(gf[o:o + fl[p]], rf[ro:ro + fl[p]]), p
        o += fl[p]
        ro += fl[p]
