"""The captured, autotuned batch (plan) path against the CPU oracle on a batch
shaped like the uneven workload: pairs of 2048x2048, 1024x1280 (1280 wide),
1024x768 (1024 wide), 512x512 and 256x256 plus a ragged one, ppp drawn per
pair from U[0.005, 0.1], d ~ U[1, 5], Lamb-Oseen flows on image/4 grids, RK4
with 4 substeps, 3x3 blur.

Integer codes with noise off are bit-exact against the binary32 mirror for the
autotuned plan and for every tiling the autotuner may choose; float images are
bit-exact against the mirror and within 1e-5 of the peak of the float64 render
and blur of the mirror's positions; with noise on, float images are within
1e-5 of the peak of the float64 value plus the float64 Box-Muller noise."""

import numpy as np
import pytest
import torch

from oracle import epilogue as oep
from oracle import render as orend
from workloads import get_workload

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2512_09664_amd as sp
    from gpu_util import DEV, params_of, to_np, workload_inputs

SIZES = ((2048, 2048), (1024, 1280), (768, 1024), (512, 512), (256, 256), (97, 131))
TOL = 1e-5


def _say(*a):
    print("[case]", *a, flush=True)


def _wl(bits, noise):
    return get_workload("uneven_256").with_(sizes=SIZES, bits=bits, noise_sigma=noise)


def _io(batch, flow_dev, bits):
    n = batch.n_particles
    io = {k: torch.empty(n, dtype=torch.float32, device=DEV) for k in ("x1", "y1", "x2", "y2", "z", "d", "I0")}
    io["flow"] = flow_dev
    io["images"] = torch.zeros(batch.n_pixels, dtype=sp.api.U16 if bits else torch.float32, device=DEV)
    io["n_active"] = torch.empty(batch.n_pairs, dtype=torch.int32, device=DEV)
    io["ppp"] = torch.empty(batch.n_pairs, dtype=torch.float64, device=DEV)
    return io


def _plan_run(wl, autotune=True):
    flows, batch, flow_dev = workload_inputs(wl)
    sprm, aprm, rprm = params_of(wl)
    io = _io(batch, flow_dev, wl.bits)
    plan = sp.Plan(batch, sprm, wl.seed, aprm, rprm, io, autotune=autotune)
    plan.launch()
    torch.cuda.synchronize()
    t = plan.tiling
    status = plan.read_status()
    plan.close()
    return flows, batch, io, (t.tile_w, t.tile_h, t.chunk, t.cap, t.persistent), status


@pytest.fixture(scope="module")
def mirrors(ra):
    """The binary32 mirror of every pair, noise off (codes and float images)."""
    wl = _wl(12, 0.0)
    flows, _, _ = workload_inputs(wl)
    out = []
    for p, (H, W) in enumerate(SIZES):
        out.append(ra.generate_pair_noiseless(wl, p, flows[p], H, W))
    return out


def test_autotuned_plan_codes_match_mirror(mirrors):
    flows, batch, io, tiling, status = _plan_run(_wl(12, 0.0))
    _say("autotuned plan tiling", tiling)
    assert status == 0
    im = to_np(io["images"])
    na = to_np(io["n_active"])
    o = 0
    for p, (H, W) in enumerate(SIZES):
        assert na[p] == int(np.count_nonzero(mirrors[p]["particles"]["I0"] > 0))
        got = im[o:o + 2 * H * W].reshape(2, H, W)
        o += 2 * H * W
        assert np.array_equal(got, mirrors[p]["codes"]), (p, H, W, tiling)


def test_autotuned_plan_float_images_match_oracle(ra, mirrors):
    wl = _wl(0, 0.0)
    flows, batch, io, tiling, status = _plan_run(wl)
    assert status == 0
    im = to_np(io["images"])
    w = oep.blur_weights(wl.blur_radius, wl.blur_sigma)
    o = 0
    for p, (H, W) in enumerate(SIZES):
        got = im[o:o + 2 * H * W].reshape(2, H, W)
        o += 2 * H * W
        mir = ra.generate_pair_noiseless(wl, p, flows[p], H, W)
        assert np.array_equal(got, mir["J"]), (p, tiling)
        Pm = mir["particles"]
        ref = np.stack([oep.blur(orend.render_frame(xx, yy, Pm["z"], Pm["d"], Pm["I0"], H, W, wl.sheet_sigma), w)
                        for (xx, yy) in ((Pm["x"], Pm["y"]), (mir["x2"], mir["y2"]))])
        err = float(np.max(np.abs(got - ref)))
        _say("plan float pair", p, H, W, "max err / peak", err / ref.max())
        assert err <= TOL * ref.max(), (p, err)


def test_every_tiling_candidate_matches_mirror(mirrors):
    """Seed and advect once, then render with every tiling the autotuner may
    pick: codes bit-exact against the mirror each time, status word clear."""
    wl = _wl(12, 0.0)
    flows, batch, flow_dev = workload_inputs(wl)
    sprm, aprm, rprm = params_of(wl)
    P = sp.seed(batch, sprm, wl.seed)
    x2, y2 = sp.advect(batch, flow_dev, aprm, P["x"], P["y"])
    cands = sp.tiling_candidates(rprm)
    assert len(cands) >= 10
    for t in cands:
        ws = sp.alloc_workspace(batch, rprm, t)
        img = sp.render_pair(batch, P["x"], P["y"], x2, y2, P["z"], P["d"], P["I0"], rprm, t, workspace=ws)
        torch.cuda.synchronize()
        assert sp.read_status(ws) == 0
        im = to_np(img)
        o = 0
        for p, (H, W) in enumerate(SIZES):
            got = im[o:o + 2 * H * W].reshape(2, H, W)
            o += 2 * H * W
            assert np.array_equal(got, mirrors[p]["codes"]), (p, t.tile_w, t.tile_h, t.chunk, t.cap, t.persistent)
        del ws, img


def test_autotuned_plan_with_noise_matches_oracle(mirrors):
    """Noise on, float images: within 1e-5 of the peak of the mirror's float
    image plus sigma times the float64 Box-Muller normals of the same Philox
    words (the mirror's float image is itself within 1e-5 of float64)."""
    wl = _wl(0, 0.01)
    flows, batch, io, tiling, status = _plan_run(wl)
    assert status == 0
    im = to_np(io["images"])
    o = 0
    for p, (H, W) in enumerate(SIZES):
        got = im[o:o + 2 * H * W].reshape(2, H, W)
        o += 2 * H * W
        mir = _mirror_float(wl, flows, p, H, W)
        for f in range(2):
            K = mir[f].astype(np.float64) + wl.noise_sigma * oep.noise_normals(H, W, f, p, wl.seed)
            err = float(np.max(np.abs(got[f] - K)))
            assert err <= TOL * max(1.0, float(mir[f].max())), (p, f, err)


def _mirror_float(wl, flows, p, H, W):
    from oracle import ra32
    return ra32.generate_pair_noiseless(wl.with_(noise_sigma=0.0, bits=0), p, flows[p], H, W)["J"]
