"""Captured batch plans on the GPU: a plan's graph replay gives exactly what the
eager calls give, the autotuner only changes speed, and pair-id advance draws
the next batch of pairs."""

import numpy as np
import pytest
import torch

from workloads import get_workload

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2512_09664_amd as sp
    from gpu_util import DEV, batch_for, params_of, to_np, workload_inputs

# uneven pair sizes, a ragged mix with odd edges
SIZES = ((64, 96), (128, 128), (33, 200), (256, 64), (97, 31), (160, 144), (48, 48), (200, 120))


def _workload(bits=12, noise=0.01):
    return get_workload("uneven_256").with_(sizes=SIZES, bits=bits, noise_sigma=noise, blur_radius=1,
                                            integrator="rk4", substeps=2, flow="lamb_oseen")


def _io(batch, flow_dev, bits):
    n = batch.n_particles
    io = {k: torch.empty(n, dtype=torch.float32, device=DEV) for k in ("x1", "y1", "x2", "y2", "z", "d", "I0")}
    io["flow"] = flow_dev
    io["images"] = torch.empty(batch.n_pixels, dtype=sp.api.U16 if bits else torch.float32, device=DEV)
    io["n_active"] = torch.empty(batch.n_pairs, dtype=torch.int32, device=DEV)
    io["ppp"] = torch.empty(batch.n_pairs, dtype=torch.float64, device=DEV)
    return io


def _eager(batch, flow_dev, sprm, aprm, rprm, seed, tile=None):
    rprm = type(rprm).from_buffer_copy(rprm)
    rprm.seed = seed                        # a plan keys particles and noise with one seed
    P = sp.seed(batch, sprm, seed)
    x2, y2 = sp.advect(batch, flow_dev, aprm, P["x"], P["y"])
    img = sp.render_pair(batch, P["x"], P["y"], x2, y2, P["z"], P["d"], P["I0"], rprm, tile)
    torch.cuda.synchronize()
    return P, x2, y2, img


def _same(a, b):
    return np.array_equal(to_np(a), to_np(b))


def _plan_x2(batch, P, x1, x2):
    """The frame-2 positions a plan produces: the eager advection's for active
    particles, the frame-1 position for masked candidates (a plan does not
    advect them; their I0 is 0 and they add nothing to the images)."""
    out = to_np(x2).copy()
    xs = to_np(x1)
    na = to_np(P["n_active"])
    for p, hp in enumerate(batch.host):
        o = hp.particle_offset
        out[o + int(na[p]):o + hp.n_max] = xs[o + int(na[p]):o + hp.n_max]
    return out


@pytest.mark.parametrize("bits,noise", [(12, 0.01), (0, 0.0)])
def test_plan_replays_match_eager(bits, noise):
    wl = _workload(bits, noise)
    flows, batch, flow_dev = workload_inputs(wl)
    sprm, aprm, rprm = params_of(wl)
    P, x2, y2, img = _eager(batch, flow_dev, sprm, aprm, rprm, wl.seed)
    io = _io(batch, flow_dev, bits)
    plan = sp.Plan(batch, sprm, wl.seed, aprm, rprm, io)
    for r in range(3):
        io["images"].zero_()
        io["x2"].fill_(-7.0)
        plan.launch()
        torch.cuda.synchronize()
        assert _same(io["images"], img), f"replay {r}"
        assert _same(io["x1"], P["x"])
        assert np.array_equal(to_np(io["x2"]), _plan_x2(batch, P, P["x"], x2))
        assert np.array_equal(to_np(io["y2"]), _plan_x2(batch, P, P["y"], y2))
        assert np.all(to_np(P["I0"])[to_np(io["x2"]) != to_np(x2)] == 0.0)   # only masked candidates differ
        assert _same(io["n_active"], P["n_active"])
        # unrelated eager work between replays
        _ = (io["x1"] * 2).sum().item()
    plan.close()


def test_autotuned_plan_is_bitwise_identical():
    wl = _workload()
    flows, batch, flow_dev = workload_inputs(wl)
    sprm, aprm, rprm = params_of(wl)
    _, _, _, img = _eager(batch, flow_dev, sprm, aprm, rprm, wl.seed)
    io = _io(batch, flow_dev, wl.bits)
    plan = sp.Plan(batch, sprm, wl.seed, aprm, rprm, io, autotune=True)
    t = plan.tiling
    assert t.tile_w in (32, 64, 128) and t.tile_h in (16, 32, 64) and t.cap in (32, 64, 128)
    for _ in range(2):
        io["images"].zero_()
        plan.launch()
        torch.cuda.synchronize()
        assert _same(io["images"], img)
    plan.close()


def test_plan_advances_pair_ids():
    wl = _workload()
    flows, batch, flow_dev = workload_inputs(wl)
    sprm, aprm, rprm = params_of(wl)
    n = batch.n_pairs
    io = _io(batch, flow_dev, wl.bits)
    plan = sp.Plan(batch, sprm, wl.seed, aprm, rprm, io, advance_pair_ids=True)
    for k in range(3):
        plan.launch()
        torch.cuda.synchronize()
        ids = [k * n + p for p in range(n)]
        bk = batch_for(wl.sizes, [f.shape[:2] for f in flows], batch.n_max, ids)
        _, _, _, img = _eager(bk, flow_dev, sprm, aprm, rprm, wl.seed)
        assert _same(io["images"], img), f"launch {k}"
    plan.close()


def test_plan_launch_into_new_buffers():
    """One captured plan replayed into a second set of tensors with another key
    and pair-id offset, then back into the first: every launch equals the eager
    calls on the same buffers, ids and key, and leaves the other set untouched."""
    wl = _workload()
    flows, batch, flow_dev = workload_inputs(wl)
    sprm, aprm, rprm = params_of(wl)
    io1 = _io(batch, flow_dev, wl.bits)
    io2 = _io(batch, flow_dev, wl.bits)
    plan = sp.Plan(batch, sprm, wl.seed, aprm, rprm, io1)
    n = batch.n_pairs
    for k in range(2):
        io1["images"].zero_()
        io2["images"].zero_()
        plan.launch(io2, seed_value=5 + k, pair_id_base=100 * (k + 1))
        torch.cuda.synchronize()
        bk = batch_for(wl.sizes, [f.shape[:2] for f in flows], batch.n_max, [100 * (k + 1) + p for p in range(n)])
        P, x2, _, img = _eager(bk, flow_dev, sprm, aprm, rprm, 5 + k)
        assert _same(io2["images"], img) and _same(io2["x1"], P["x"]), k
        assert np.array_equal(to_np(io2["x2"]), _plan_x2(bk, P, P["x"], x2)), k
        assert _same(io2["n_active"], P["n_active"])
        assert not io1["images"].view(torch.int16).any()
        assert plan.read_status() == 0
    # a launch without io replays the last descriptor
    io2["images"].zero_()
    plan.launch()
    torch.cuda.synchronize()
    assert _same(io2["images"], img)
    plan.launch(io1, seed_value=wl.seed, pair_id_base=0)
    torch.cuda.synchronize()
    _, _, _, img1 = _eager(batch, flow_dev, sprm, aprm, rprm, wl.seed)
    assert _same(io1["images"], img1)
    plan.close()
