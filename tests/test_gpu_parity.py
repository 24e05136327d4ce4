"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bit-exact against the binary32 mirror (Philox words, uniforms, positions, tile
membership, fixed-point render, blur, integer codes with noise off); within
1e-5 of the peak against the float64 oracle for every float image.
"""

import math

import numpy as np
import pytest
import torch

from oracle import advect as oadv
from oracle import bins as obins
from oracle import epilogue as oep
from oracle import pipeline as opipe
from oracle import render as orend
from oracle import seed as oseed
from workloads import flows as wflows
from workloads import get_workload, particles

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2512_09664_amd as sp
    import gpu_util as gu

TOL = 1e-5   # of the peak, float64 comparison


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    sp._lib.load()


def _say(*a):
    print("[case]", *a, flush=True)


# ----------------------------------------------------------------------------- seed

@pytest.mark.parametrize("d_dist,d_params", [("uniform", (1.5, 3.0)), ("normal", (2.5, 0.5, 1.0, 5.0))])
def test_seed_matches_oracle(ra, d_dist, d_params):
    sizes = [(256, 256), (96, 1280), (37, 53), (1, 1), (300, 7)]
    pids = [0, 7, (1 << 33) + 5, 11, 3]
    ppp = (0.02, 0.06)
    seed = 0xDEADBEEF12345
    n_max = [sp.particle_count(H, W, ppp[1]) for H, W in sizes]
    _say("seed", d_dist, sizes, n_max)
    b = gu.batch_for(sizes, [(4, 4)] * len(sizes), n_max, pids)
    P = sp.seed(b, sp.seed_params(ppp, d_dist, d_params), seed)
    torch.cuda.synchronize()
    got = {k: gu.to_np(P[k]) for k in ("x", "y", "z", "d", "I0")}
    na = gu.to_np(P["n_active"])
    pp = gu.to_np(P["ppp"])
    for p, sl in enumerate(gu.pair_slices(b)):
        H, W = sizes[p]
        R = ra.seed_pair(H, W, n_max[p], ppp, pids[p], seed, d_dist, d_params)
        O = oseed.seed_pair(H, W, pids[p], seed, ppp, d_dist, d_params)
        assert na[p] == R["n_active"] == O["n_active"]
        assert pp[p] == O["ppp"]
        for k in ("x", "y", "z", "d", "I0"):
            assert np.array_equal(got[k][sl], R[k]), (p, k)
            ref = O[k]
            if ref.size:
                assert np.max(np.abs(got[k][sl] - ref)) <= 2e-6 * max(1.0, np.abs(ref).max()), (p, k)


# ----------------------------------------------------------------------------- advect

@pytest.mark.parametrize("integ,n,dt", [("euler", 1, 1.0), ("rk4", 4, 1.0), ("rk4", 8, 0.7), ("euler", 3, -1.5)])
def test_advect_matches_oracle(ra, integ, n, dt):
    sizes = [(256, 384), (64, 64), (100, 36)]
    rng = np.random.default_rng(5)
    fl = [wflows.lamb_oseen_grid(rng, 256, 384, 64, 96, max_disp=8.0),
          wflows.fourier_grid(rng, 64, 64, 16, 16, max_disp=6.0),
          wflows.uniform_grid(25, 9, 2.5, -1.25)]
    parts = [particles.random_particles(10 + p, 3000, H, W, pad=12) for p, (H, W) in enumerate(sizes)]
    _say("advect", integ, n, dt)
    b = gu.batch_for(sizes, [f.shape[:2] for f in fl], [3000] * 3)
    flow = gu.to_dev(np.concatenate([f.reshape(-1) for f in fl]))
    x1 = gu.to_dev(np.concatenate([q["x"] for q in parts]))
    y1 = gu.to_dev(np.concatenate([q["y"] for q in parts]))
    x2, y2 = sp.advect(b, flow, sp.advect_params(dt, n, integ), x1, y1)
    ux2, uy2 = sp.advect(b, flow, sp.advect_params(dt, n, integ), x1, y1, ordered=False)
    torch.cuda.synchronize()
    # the home-block order changes which thread moves which particle, nothing else
    assert torch.equal(x2, ux2) and torch.equal(y2, uy2)
    gx, gy = gu.to_np(x2), gu.to_np(y2)
    for p, sl in enumerate(gu.pair_slices(b)):
        H, W = sizes[p]
        rx, ry = ra.advect(fl[p], H, W, parts[p]["x"], parts[p]["y"], dt, n, integ)
        assert np.array_equal(gx[sl], rx) and np.array_equal(gy[sl], ry), p
        ox, oy = oadv.advect(fl[p], H, W, parts[p]["x"], parts[p]["y"], dt, n, integ)
        # binary32 drift: about two roundings of the position per substep plus the
        # start value's own spacing
        tol = (4 + 2 * n) * float(np.spacing(np.float32(max(np.abs(ox).max(), np.abs(oy).max()))))
        assert np.max(np.abs(gx[sl] - ox)) <= tol and np.max(np.abs(gy[sl] - oy)) <= tol


def test_advect_order_with_large_pairs(ra):
    """Pairs large enough that the home blocks grow past 32 px (8192^2 and
    16384 x 1024), between small ones;
    ordered and index-order launches agree with the mirror bit for bit."""
    sizes = [(33, 17), (8192, 8192), (16384, 1024), (64, 64)]
    rng = np.random.default_rng(9)
    fl = [wflows.fourier_grid(rng, H, W, 9, 7, max_disp=5.0) for (H, W) in sizes]
    n = [200, 6000, 3000, 500]
    parts = [particles.random_particles(40 + p, n[p], H, W, pad=6) for p, (H, W) in enumerate(sizes)]
    _say("advect order, large pairs")
    b = gu.batch_for(sizes, [f.shape[:2] for f in fl], n)
    flow = gu.to_dev(np.concatenate([f.reshape(-1) for f in fl]))
    x1 = gu.to_dev(np.concatenate([q["x"] for q in parts]))
    y1 = gu.to_dev(np.concatenate([q["y"] for q in parts]))
    ap = sp.advect_params(1.0, 2, "rk4")
    x2, y2 = sp.advect(b, flow, ap, x1, y1)
    ux2, uy2 = sp.advect(b, flow, ap, x1, y1, ordered=False)
    torch.cuda.synchronize()
    assert torch.equal(x2, ux2) and torch.equal(y2, uy2)
    gx, gy = gu.to_np(x2), gu.to_np(y2)
    for p, sl in enumerate(gu.pair_slices(b)):
        H, W = sizes[p]
        rx, ry = ra.advect(fl[p], H, W, parts[p]["x"], parts[p]["y"], 1.0, 2, "rk4")
        assert np.array_equal(gx[sl], rx) and np.array_equal(gy[sl], ry), p


def test_advect_order_with_many_particles(ra):
    """A pair with 1.2 M particles (more than 512 blocks of 2048, so the order
    takes larger blocks of particles) beside a small one, with the grid nodes
    of most workgroups in their LDS window and a flow strong enough to carry
    some samples out of it: ordered and index-order launches agree with the
    mirror bit for bit."""
    sizes = [(4096, 4096), (40, 56)]
    rng = np.random.default_rng(11)
    fl = [wflows.lamb_oseen_grid(rng, H, W, H // 4, W // 4, max_disp=30.0) for (H, W) in sizes]
    n = [1_200_000, 300]
    parts = [particles.random_particles(70 + p, n[p], H, W, pad=6) for p, (H, W) in enumerate(sizes)]
    _say("advect order, 1.2 M particles in one pair")
    b = gu.batch_for(sizes, [f.shape[:2] for f in fl], n)
    flow = gu.to_dev(np.concatenate([f.reshape(-1) for f in fl]))
    x1 = gu.to_dev(np.concatenate([q["x"] for q in parts]))
    y1 = gu.to_dev(np.concatenate([q["y"] for q in parts]))
    ap = sp.advect_params(1.0, 4, "rk4")
    x2, y2 = sp.advect(b, flow, ap, x1, y1)
    ux2, uy2 = sp.advect(b, flow, ap, x1, y1, ordered=False)
    torch.cuda.synchronize()
    assert torch.equal(x2, ux2) and torch.equal(y2, uy2)
    gx, gy = gu.to_np(x2), gu.to_np(y2)
    for p, sl in enumerate(gu.pair_slices(b)):
        H, W = sizes[p]
        rx, ry = ra.advect(fl[p], H, W, parts[p]["x"], parts[p]["y"], 1.0, 4, "rk4")
        assert np.array_equal(gx[sl], rx) and np.array_equal(gy[sl], ry), p


# ----------------------------------------------------------------------------- render

def _render_case(seed, sizes, n_per, d_range=(1.0, 5.0), zero_frac=0.1, edge=True):
    xs, ys, zs, ds, Is, x2s, y2s = [], [], [], [], [], [], []
    for p, (H, W) in enumerate(sizes):
        q = particles.random_particles(seed + p, n_per, H, W, d_range=d_range, pad=8, zero_frac=zero_frac)
        if edge:
            e = particles.edge_case_particles(H, W, tile=32, d=float(np.mean(d_range)))
            q = {k: np.concatenate([q[k], e[k]]) for k in q}
        rng = np.random.default_rng(seed + 100 + p)
        xs.append(q["x"]); ys.append(q["y"]); zs.append(q["z"]); ds.append(q["d"]); Is.append(q["I0"])
        x2s.append((q["x"] + rng.uniform(-3, 3, q["x"].size)).astype(np.float32))
        y2s.append((q["y"] + rng.uniform(-3, 3, q["y"].size)).astype(np.float32))
    n_max = [len(a) for a in xs]
    cat = lambda L: np.concatenate(L)
    return dict(x1=cat(xs), y1=cat(ys), x2=cat(x2s), y2=cat(y2s), z=cat(zs), d=cat(ds), I0=cat(Is)), n_max


def _render_gpu(b, arrs, rp, tile=None, workspace=None):
    t = {k: gu.to_dev(v) for k, v in arrs.items()}
    img = sp.render_pair(b, t["x1"], t["y1"], t["x2"], t["y2"], t["z"], t["d"], t["I0"], rp, tile,
                         workspace=workspace)
    torch.cuda.synchronize()
    return gu.to_np(img)


TILINGS = [None, (8, 8, 256, 32), (64, 32, 256, 64), (128, 32, 16384, 128), (32, 16, 512, 96),
           (64, 32, 2048, 64, 1), (8, 8, 256, 32, 1)]


@pytest.mark.parametrize("tile", TILINGS)
@pytest.mark.parametrize("blur", [0, 1, 2])
def test_render_matches_oracle(ra, tile, blur):
    sizes = [(64, 96), (37, 53), (128, 128), (8, 4)]
    arrs, n_max = _render_case(21, sizes, 400)
    _say("render", tile, blur, sizes)
    b = gu.batch_for(sizes, [(4, 4)] * len(sizes), n_max)
    rp = sp.render_params(0.5, 5.0, blur, 0.8, 0.0, 0)
    tl = sp.tiling(*tile) if tile else None
    img = _render_gpu(b, arrs, rp, tl)
    w = oep.blur_weights(blur, 0.8) if blur else None
    o = 0
    po = 0
    for p, (H, W) in enumerate(sizes):
        sl = slice(po, po + n_max[p])
        po += n_max[p]
        for f, (xk, yk) in enumerate((("x1", "y1"), ("x2", "y2"))):
            got = img[o:o + H * W].reshape(H, W)
            o += H * W
            args = (arrs[xk][sl], arrs[yk][sl], arrs["z"][sl], arrs["d"][sl], arrs["I0"][sl])
            mirror = ra.render(*args, H, W, 0.5)
            ref = orend.render_frame(*args, H, W, 0.5)
            if blur:
                mirror = ra.blur(mirror, w)
                ref = oep.blur(ref, w)
            assert np.array_equal(got, mirror), (p, f)
            assert np.max(np.abs(got - ref)) <= TOL * max(ref.max(), 1e-30), (p, f)


def test_tiling_and_batching_do_not_change_bits():
    sizes = [(200, 136), (64, 64), (33, 99)]
    arrs, n_max = _render_case(31, sizes, 900, d_range=(0.8, 6.0))
    b = gu.batch_for(sizes, [(4, 4)] * 3, n_max)
    rp = sp.render_params(0.5, 6.0, 1, 0.7, 0.0, 12)
    imgs = [_render_gpu(b, arrs, rp, sp.tiling(*t) if t else None) for t in TILINGS]
    for im in imgs[1:]:
        assert np.array_equal(im, imgs[0])
    # each pair alone (same pair_id) gives the same bits as inside the batch
    o = po = 0
    for p, (H, W) in enumerate(sizes):
        sl = slice(po, po + n_max[p])
        po += n_max[p]
        b1 = gu.batch_for([sizes[p]], [(4, 4)], [n_max[p]], [p])
        one = _render_gpu(b1, {k: v[sl] for k, v in arrs.items()}, rp)
        assert np.array_equal(one, imgs[0][o:o + 2 * H * W])
        o += 2 * H * W


@pytest.mark.parametrize("tile", [None, (8, 8, 256, 32), (128, 32, 16384, 128), (64, 64, 2048, 128, 1)])
def test_large_diameters_match_oracle(ra, tile):
    """Diameters up to 15 px under d_max = 16 (the largest accepted) with the
    widest blur: patches far wider than small tiles, the widest factor tables."""
    sizes = [(72, 90), (41, 23)]
    arrs, n_max = _render_case(61, sizes, 60, d_range=(5.0, 15.0), edge=False)
    _say("large diameters", tile, sizes)
    b = gu.batch_for(sizes, [(4, 4)] * 2, n_max)
    rp = sp.render_params(0.5, 16.0, 3, 1.3, 0.0, 0)
    tl = sp.tiling(*tile) if tile else None
    ws = sp.alloc_workspace(b, rp, tl)
    img = _render_gpu(b, arrs, rp, tl, workspace=ws)
    assert sp.read_status(ws) == 0
    w = oep.blur_weights(3, 1.3)
    o = po = 0
    for p, (H, W) in enumerate(sizes):
        sl = slice(po, po + n_max[p])
        po += n_max[p]
        for xk, yk in (("x1", "y1"), ("x2", "y2")):
            got = img[o:o + H * W].reshape(H, W)
            o += H * W
            args = (arrs[xk][sl], arrs[yk][sl], arrs["z"][sl], arrs["d"][sl], arrs["I0"][sl])
            assert np.array_equal(got, ra.blur(ra.render(*args, H, W, 0.5), w)), p
            ref = oep.blur(orend.render_frame(*args, H, W, 0.5), w)
            assert np.max(np.abs(got - ref)) <= TOL * ref.max(), p


@pytest.mark.parametrize("tile", [None, (16, 16, 256, 32)])
def test_bins_match_oracle(tile):
    sizes = [(64, 96), (37, 53)]
    arrs, n_max = _render_case(41, sizes, 300)
    b = gu.batch_for(sizes, [(4, 4)] * 2, n_max)
    rp = sp.render_params(0.5, 5.0, 2, 1.0, 0.0, 12)
    tl = sp.tiling(*tile) if tile else None
    ws = sp.alloc_workspace(b, rp, tl)
    _render_gpu(b, arrs, rp, tl, workspace=ws)
    count, offset, entries = (gu.to_np(t) for t in sp.bin_views(b, rp, tl, ws))
    dt_ = sp.default_tiling(b, rp)
    tw, th = (tile[0], tile[1]) if tile else (dt_.tile_w, dt_.tile_h)
    tbase = 0
    po = 0
    for p, (H, W) in enumerate(sizes):
        sl = slice(po, po + n_max[p])
        po += n_max[p]
        nty, ntx = obins.tile_grid(H, W, th, tw)
        nt = nty * ntx
        for f, (xk, yk) in enumerate((("x1", "y1"), ("x2", "y2"))):
            c, off, ent = obins.bin_frame(arrs[xk][sl], arrs[yk][sl], arrs["d"][sl], arrs["I0"][sl], H, W, th, tw, 2)
            gc = count[f, tbase:tbase + nt]
            go = offset[f, tbase:tbase + nt]
            assert np.array_equal(gc, c), (p, f)
            assert np.array_equal(go - go[0], off[:-1]), (p, f)      # exclusive scan inside the pair-frame
            for t in range(nt):
                g = np.sort(entries[go[t]:go[t] + gc[t]])
                assert np.array_equal(g, ent[off[t]:off[t + 1]]), (p, f, t)
        tbase += nt


@pytest.mark.parametrize("bits", [8, 12, 16])
def test_codes_bit_exact_noise_off(ra, bits):
    sizes = [(96, 128), (45, 61)]
    arrs, n_max = _render_case(51, sizes, 800, d_range=(1.0, 4.0), zero_frac=0.0)
    arrs["I0"] = (arrs["I0"] * 1.3).astype(np.float32)          # some pixels saturate
    b = gu.batch_for(sizes, [(4, 4)] * 2, n_max)
    rp = sp.render_params(0.5, 4.0, 1, 0.7, 0.0, bits)
    img = _render_gpu(b, arrs, rp)
    w = oep.blur_weights(1, 0.7)
    o = po = 0
    for p, (H, W) in enumerate(sizes):
        sl = slice(po, po + n_max[p])
        po += n_max[p]
        for f, (xk, yk) in enumerate((("x1", "y1"), ("x2", "y2"))):
            J = ra.blur(ra.render(arrs[xk][sl], arrs[yk][sl], arrs["z"][sl], arrs["d"][sl], arrs["I0"][sl],
                                  H, W, 0.5), w)
            q = ra.quantise(J, bits)
            got = img[o:o + H * W].reshape(H, W)
            o += H * W
            assert np.array_equal(got, q), (p, f)
            assert got.max() == (1 << bits) - 1                 # saturation reached


def test_noise_matches_oracle():
    """Noise uses the GPU's fast log/sqrt/sin/cos, so it is compared within
    tolerance: float images within 1e-5 of the peak; integer codes equal except
    where the float64 value K * L lies within L * eps of a rounding boundary,
    eps being the largest float difference measured on the same draws."""
    sizes = [(64, 130), (32, 32)]
    arrs, n_max = _render_case(61, sizes, 300, zero_frac=0.0)
    pids = [4, 9]
    b = gu.batch_for(sizes, [(4, 4)] * 2, n_max, pids)
    sigma = 0.02
    w = oep.blur_weights(1, 0.7)
    refs = []
    o = po = 0
    for p, (H, W) in enumerate(sizes):
        sl = slice(po, po + n_max[p])
        po += n_max[p]
        for f, (xk, yk) in enumerate((("x1", "y1"), ("x2", "y2"))):
            J = oep.blur(orend.render_frame(arrs[xk][sl], arrs[yk][sl], arrs["z"][sl], arrs["d"][sl],
                                            arrs["I0"][sl], H, W, 0.5), w)
            refs.append((o, H, W, J, J + np.float32(sigma) * oep.noise_normals(H, W, f, pids[p], 77)))
            o += H * W
    img = _render_gpu(b, arrs, sp.render_params(0.5, 5.0, 1, 0.7, sigma, 0, seed=77), None)
    eps = 0.0
    for (o, H, W, J, K) in refs:
        got = img[o:o + H * W].reshape(H, W)
        err = np.max(np.abs(got - K))
        assert err <= TOL * max(1.0, J.max())
        eps = max(eps, err)
    L = 4095
    codes = _render_gpu(b, arrs, sp.render_params(0.5, 5.0, 1, 0.7, sigma, 12, seed=77), None)
    for (o, H, W, J, K) in refs:
        got = codes[o:o + H * W].reshape(H, W).astype(np.int64)
        q = oep.quantise(K, 12).astype(np.int64)
        diff = np.abs(got - q)
        assert diff.max() <= 1
        dist = np.abs((K * L) % 1.0 - 0.5)            # distance to the nearest rounding boundary
        assert np.all(dist[diff > 0] <= L * eps * 1.01 + 1e-9), (dist[diff > 0], eps)


# ----------------------------------------------------------------------------- end to end

def _e2e(ra, wl, n_check=None):
    """Whole path, noise off.  (1) GPU output bit-exact with the binary32 mirror
    (codes or floats).  (2) GPU float images within 1e-5 of the peak of the
    float64 render+blur of the mirror's binary32 positions: the render and blur
    arithmetic against the definition.  (3) The error against the all-float64
    pipeline (positions integrated in float64 too) is reported; it adds the
    binary32 spacing of the positions times the image gradient, and is only
    held to 1e-3 of the peak."""
    _, flows, _, _, _, img = gu.run_pipeline(wl, noise=0.0)
    _, _, _, _, _, fimg = gu.run_pipeline(wl, noise=0.0, bits=0)
    im, fim = gu.to_np(img), gu.to_np(fimg)
    w = oep.blur_weights(wl.blur_radius, wl.blur_sigma) if wl.blur_radius else None
    o = 0
    for p, (H, W) in enumerate(wl.sizes):
        n = 2 * H * W
        if n_check is None or p in n_check:
            _say("e2e", wl.name, p, H, W)
            mir = ra.generate_pair_noiseless(wl, p, flows[p], H, W)
            key = "codes" if wl.bits > 0 else "J"
            assert np.array_equal(im[o:o + n].reshape(2, H, W), mir[key]), (wl.name, p)
            got = fim[o:o + n].reshape(2, H, W)
            assert np.array_equal(got, ra.generate_pair_noiseless(wl.with_(bits=0), p, flows[p], H, W)["J"])
            Pm = mir["particles"]
            ref = np.stack([orend.render_frame(xx, yy, Pm["z"], Pm["d"], Pm["I0"], H, W, wl.sheet_sigma)
                            for (xx, yy) in ((Pm["x"], Pm["y"]), (mir["x2"], mir["y2"]))])
            if w is not None:
                ref = np.stack([oep.blur(ref[0], w), oep.blur(ref[1], w)])
            peak = max(ref.max(), 1e-30)
            assert np.max(np.abs(got - ref)) <= TOL * peak, (wl.name, p)
            full = opipe.generate_pair(wl.with_(noise_sigma=0.0), p, flows[p], H, W)["J"]
            err64 = float(np.max(np.abs(got - full)))
            print(f"[e2e] {wl.name} pair {p}: max |GPU - float64 pipeline| = {err64:.3e} "
                  f"({err64 / peak:.2e} of peak)", flush=True)
            assert err64 <= 1e-3 * peak
        o += n


def test_end_to_end_plain_256(ra):
    _e2e(ra, get_workload("plain_256"))


def test_end_to_end_scale_1024_pairs(ra):
    _e2e(ra, get_workload("scale_1024", n_pairs=2))


def test_end_to_end_uneven(ra):
    wl = get_workload("uneven_256").with_(sizes=((256, 256), (768, 1024), (512, 512), (256, 256)))
    _e2e(ra, wl)


def test_end_to_end_grad_workload_float(ra):
    _e2e(ra, get_workload("grad_512", n_pairs=2))


def test_edge_empty_and_tiny_pairs(ra):
    wl = get_workload("plain_256").with_(sizes=((2, 2), (3, 5), (8, 8), (2, 130)), ppp=(0.3, 0.3), grid_div=1)
    _e2e(ra, wl)


def test_diameter_above_max_is_flagged():
    sizes = [(32, 32)]
    arrs = dict(x1=np.array([10.5, 20.5], np.float32), y1=np.array([10.5, 20.5], np.float32),
                x2=np.array([10.5, 20.5], np.float32), y2=np.array([10.5, 20.5], np.float32),
                z=np.zeros(2, np.float32), d=np.array([2.0, 9.0], np.float32), I0=np.ones(2, np.float32))
    b = gu.batch_for(sizes, [(4, 4)], [2])
    rp = sp.render_params(0.5, 4.0, 0, 0.7, 0.0, 0)
    ws = sp.alloc_workspace(b, rp)
    img = _render_gpu(b, arrs, rp, workspace=ws).reshape(2, 32, 32)
    assert sp.read_status(ws) & sp._lib.SP_STATUS_D_ABOVE_MAX
    assert img[0, 10, 10] == 1.0 and img[0, 20, 20] == 0.0


def test_fixed_point_range_is_flagged():
    """The integer pixel sums hold up to 256 full-scale units; a tile whose staged
    peaks could reach that raises SP_STATUS_FIXED_RANGE, ordinary tiles do not."""
    n = 300
    arrs = dict(x1=np.full(n, 10.5, np.float32), y1=np.full(n, 10.5, np.float32),
                x2=np.full(n, 40.5, np.float32), y2=np.full(n, 40.5, np.float32),
                z=np.zeros(n, np.float32), d=np.full(n, 2.0, np.float32), I0=np.ones(n, np.float32))
    b = gu.batch_for([(64, 64)], [(4, 4)], [n])
    rp = sp.render_params(0.5, 4.0, 0, 0.7, 0.0, 0)
    ws = sp.alloc_workspace(b, rp)
    _render_gpu(b, arrs, rp, workspace=ws)
    assert sp.read_status(ws) & sp._lib.SP_STATUS_FIXED_RANGE
    arrs["I0"][:] = 0.5                      # 150 full-scale units: in range
    _render_gpu(b, arrs, rp, workspace=ws)
    assert sp.read_status(ws) == 0


# ----------------------------------------------------------------------------- full size, sampled

def _full_size_sampled(ra, wl, pairs, exact_pairs, per_frame=24, seed=0):
    """A whole workload launched as the benchmark launches it (noise on, integer
    codes): sampled pixels against the float64 oracle computed one by one, and
    whole pairs bit-exact against the binary32 mirror with noise off."""
    batch, flows, P, x2, y2, img = gu.run_pipeline(wl)
    im = gu.to_np(img)
    rng = np.random.default_rng(seed)
    b = wl.blur_radius
    w = oep.blur_weights(b, wl.blur_sigma).astype(np.float64)
    H, W = wl.sizes[0]
    plane = H * W
    L = (1 << wl.bits) - 1
    reach = 1.5 * wl.d_max + b + 2
    checked = 0
    for p in pairs:
        _say("full-size sampled pair", p)
        O = oseed.seed_pair(H, W, p, wl.seed, wl.ppp, wl.d_dist, wl.d_params, wl.I0, wl.z)
        ox2, oy2 = oadv.advect(flows[p], H, W, O["x"], O["y"], wl.dt, wl.substeps, wl.integrator)
        for f, (xx, yy) in enumerate(((O["x"], O["y"]), (ox2, oy2))):
            noise = oep.noise_normals(H, W, f, p, wl.seed)
            for _ in range(per_frame):
                r, c = int(rng.integers(0, H)), int(rng.integers(0, W))
                sel = (np.abs(xx - c) < reach) & (np.abs(yy - r) < reach)
                J = 0.0
                for i in range(-b, b + 1):
                    for j in range(-b, b + 1):
                        rr, cc = r + i, c + j
                        if 0 <= rr < H and 0 <= cc < W:
                            J += w[i + b] * w[j + b] * orend.render_pixel_direct(
                                xx[sel], yy[sel], O["z"][sel], O["d"][sel], O["I0"][sel], rr, cc, wl.sheet_sigma)
                K = J + wl.noise_sigma * noise[r, c]
                q = int(oep.quantise(np.array([K]), wl.bits)[0])
                g = int(im[p * 2 * plane + f * plane + r * W + c])
                assert abs(g - q) <= 1, (p, f, r, c, g, q, K)
                if abs(g - q) == 1:
                    # only next to a rounding boundary: float error budget 1e-5 of the
                    # noise term plus the render's 1e-6 of full scale
                    bound = L * (1e-5 * wl.noise_sigma * abs(noise[r, c]) + 1e-6)
                    assert abs((K * L) % 1.0 - 0.5) <= bound, (p, f, r, c)
                checked += 1
    assert checked == len(pairs) * 2 * per_frame
    # noise off: whole pairs bit-exact against the mirror
    batch, flows, P, x2, y2, img = gu.run_pipeline(wl, noise=0.0)
    im = gu.to_np(img)
    for p in exact_pairs:
        _say("full-size bit-exact pair", p)
        mir = ra.generate_pair_noiseless(wl, p, flows[p], H, W)
        assert np.array_equal(im[p * 2 * plane:(p + 1) * 2 * plane].reshape(2, H, W), mir["codes"]), p


def test_full_size_scale_1024_sampled(ra):
    """64 pairs of 1024x1024, 0.05 ppp, 3x3 blur, noise 0.01, 12-bit codes."""
    _full_size_sampled(ra, get_workload("scale_1024"), (0, 17, 63), (0, 63))


def test_full_size_dense_2048_sampled(ra):
    """32 pairs of 2048x2048, 0.1 ppp, d ~ U[2, 6], RK4 x 8, 5x5 blur, noise 0.02,
    12-bit codes: the dense stress configuration."""
    _full_size_sampled(ra, get_workload("dense_2048"), (0, 31), (5,), per_frame=16, seed=1)
