"""Batch layouts the C ABI accepts but the packed workloads never produce:
unused gaps between pairs' particle, image and flow ranges, pairs without
particles, and the largest image a tiling can render."""

import numpy as np
import pytest
import torch

from oracle import epilogue as oep
from workloads import get_workload, make_flows, particles

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2512_09664_amd as sp
    import gpu_util as gu

    from test_gpu_parity import _e2e, _say


def _run(batch, flow, wl, seed):
    sprm, aprm, rprm = gu.params_of(wl)
    n = max(batch.n_particles, 1)
    P = {k: torch.full((n,), float("nan"), device=gu.DEV) for k in ("x", "y", "z", "d", "I0")}
    P["n_active"] = torch.full((batch.n_pairs,), -7, dtype=torch.int32, device=gu.DEV)
    P["ppp"] = torch.full((batch.n_pairs,), -7.0, dtype=torch.float64, device=gu.DEV)
    sp.seed(batch, sprm, seed, out=P)
    x2 = torch.full_like(P["x"], float("nan"))
    y2 = torch.full_like(P["y"], float("nan"))
    sp.advect(batch, flow, aprm, P["x"], P["y"], x2, y2)
    img = torch.full((batch.n_pixels,), 0x5A5A, dtype=torch.int16, device=gu.DEV).view(sp.api.U16)
    sp.render_pair(batch, P["x"], P["y"], x2, y2, P["z"], P["d"], P["I0"], rprm, None, img)
    torch.cuda.synchronize()
    return P, x2, y2, img


def test_gaps_between_pairs_are_untouched():
    wl = get_workload("uneven_256").with_(sizes=((40, 48), (64, 33), (17, 90)), ppp=(0.05, 0.08), blur_radius=1,
                                          noise_sigma=0.01, bits=12)
    flows = make_flows(wl.flow, wl.seed, wl.sizes, wl.grid_div, wl.max_disp, wl.dt, wl.uniform_uv)
    n_max = [sp.particle_count(H, W, wl.ppp[1]) for (H, W) in wl.sizes]
    grids = [f.shape[:2] for f in flows]
    gaps = (37, 101, 6)
    packed = gu.batch_for(wl.sizes, grids, n_max)
    gapped = sp.PairBatch.build(wl.sizes, grids, n_max, device=gu.DEV, gaps=gaps)
    fp = gu.to_dev(np.concatenate([f.reshape(-1) for f in flows]))
    fg = torch.zeros(gapped.n_flow, device=gu.DEV)
    for p in range(3):
        o = gapped.host[p].flow_offset
        fg[o:o + flows[p].size] = fp[packed.host[p].flow_offset:packed.host[p].flow_offset + flows[p].size]
    Pp, x2p, y2p, ip = _run(packed, fp, wl, 3)
    Pg, x2g, y2g, ig = _run(gapped, fg, wl, 3)
    assert torch.equal(Pp["n_active"], Pg["n_active"]) and torch.equal(Pp["ppp"], Pg["ppp"])
    iv = gu.to_np(ig).astype(np.int64)
    used_p = np.zeros(gapped.n_particles, bool)
    used_i = np.zeros(gapped.n_pixels, bool)
    for p, (H, W) in enumerate(wl.sizes):
        a, b = packed.host[p].particle_offset, gapped.host[p].particle_offset
        for k in ("x", "y", "z", "d", "I0"):
            assert torch.equal(Pp[k][a:a + n_max[p]], Pg[k][b:b + n_max[p]]), (p, k)
        assert torch.equal(x2p[a:a + n_max[p]], x2g[b:b + n_max[p]])
        assert torch.equal(y2p[a:a + n_max[p]], y2g[b:b + n_max[p]])
        used_p[b:b + n_max[p]] = True
        ia, ib = packed.host[p].image_offset, gapped.host[p].image_offset
        assert torch.equal(ip[ia:ia + 2 * H * W], ig[ib:ib + 2 * H * W]), p
        used_i[ib:ib + 2 * H * W] = True
    # nothing is written outside the pairs' ranges
    for k in ("x", "y", "z", "d", "I0"):
        assert torch.isnan(Pg[k][torch.from_numpy(~used_p).to(gu.DEV)]).all(), k
    assert torch.isnan(x2g[torch.from_numpy(~used_p).to(gu.DEV)]).all()
    assert np.all(iv[~used_i] == 0x5A5A)


def test_edge_pairs_without_particles(ra):
    """A 2x2 pair at 0.1 ppp has floor(0.4 + 1/2) = 0 particles: its images are
    noise-free zeros and its neighbours are unaffected."""
    wl = get_workload("plain_256").with_(sizes=((2, 2), (5, 3), (16, 16), (3, 3)), ppp=(0.1, 0.1), grid_div=1)
    assert sp.particle_count(2, 2, 0.1) == 0
    _e2e(ra, wl)


def test_largest_tiled_image(ra):
    """An 8192 x 8192 pair (128 x 32 tiles: 16384 tiles, the per-pair limit) next to
    a small one, float images, against the binary32 mirror bit for bit."""
    sizes = [(8192, 8192), (40, 24)]
    n = [3000, 60]
    parts = [particles.random_particles(70 + p, n[p], H, W, d_range=(1.0, 5.0), pad=4) for p, (H, W) in
             enumerate(sizes)]
    rng = np.random.default_rng(3)
    x2s = [(q["x"] + rng.uniform(-3, 3, q["x"].size)).astype(np.float32) for q in parts]
    y2s = [(q["y"] + rng.uniform(-3, 3, q["y"].size)).astype(np.float32) for q in parts]
    b = gu.batch_for(sizes, [(8, 8), (4, 4)], n)
    cat = lambda L: gu.to_dev(np.concatenate(L))
    rp = sp.render_params(0.5, 5.0, 0, 0.7, 0.0, 0)
    _say("largest tiled image")
    img = sp.render_pair(b, cat([q["x"] for q in parts]), cat([q["y"] for q in parts]), cat(x2s), cat(y2s),
                         cat([q["z"] for q in parts]), cat([q["d"] for q in parts]), cat([q["I0"] for q in parts]),
                         rp, sp.tiling(128, 32, 4096, 64))
    torch.cuda.synchronize()
    got = gu.to_np(img)
    o = 0
    for p, (H, W) in enumerate(sizes):
        q = parts[p]
        for f, (xx, yy) in enumerate(((q["x"], q["y"]), (x2s[p], y2s[p]))):
            ref = ra.render(xx, yy, q["z"], q["d"], q["I0"], H, W, 0.5)
            assert np.array_equal(got[o:o + H * W].reshape(H, W), ref), (p, f)
            o += H * W
    # one tile more than the per-pair limit is refused before anything runs
    with pytest.raises(sp._lib.SynthPixError):
        sp.render_pair(b, cat([q["x"] for q in parts]), cat([q["y"] for q in parts]), cat(x2s), cat(y2s),
                       cat([q["z"] for q in parts]), cat([q["d"] for q in parts]), cat([q["I0"] for q in parts]),
                       rp, sp.tiling(64, 32, 4096, 64))
