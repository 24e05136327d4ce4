"""Allocation-free render: ``synthpix_render_pair_noalloc`` uses the library's
static device scratch as its workspace and must give the images that
``synthpix_render_pair`` gives with a caller workspace, bit for bit, on two
calls in a row (the second batch smaller than the first, so it runs on what the
first left in the scratch); a batch whose workspace exceeds the scratch is
refused on the host before anything is enqueued."""

import numpy as np
import pytest
import torch

from workloads import get_workload

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2512_09664_amd as sp
    from paper_2512_09664_amd import _lib
    from gpu_util import DEV, params_of, to_np, workload_inputs


def _render_both(sizes, seed, bits, noise, tile=None):
    wl = get_workload("uneven_256").with_(sizes=sizes, bits=bits, noise_sigma=noise, blur_radius=1,
                                          integrator="rk4", substeps=2, flow="lamb_oseen", seed=seed)
    flows, batch, flow_dev = workload_inputs(wl)
    sprm, aprm, rprm = params_of(wl)
    P = sp.seed(batch, sprm, wl.seed)
    x2, y2 = sp.advect(batch, flow_dev, aprm, P["x"], P["y"])
    ws = sp.alloc_workspace(batch, rprm, tile)
    ref = sp.render_pair(batch, P["x"], P["y"], x2, y2, P["z"], P["d"], P["I0"], rprm, tile, None, ws)
    out = torch.empty_like(ref)
    out.view(torch.int16 if bits else torch.int32).fill_(0x7777)      # every pixel must be overwritten
    status = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    sp.render_pair_noalloc(batch, P["x"], P["y"], x2, y2, P["z"], P["d"], P["I0"], rprm, out, tile, status)
    torch.cuda.synchronize()
    assert sp.read_status(ws) == 0
    assert int(status.item()) == 0, f"device status {int(status.item()):#x}"
    return ref, out


def test_noalloc_matches_workspace_render_two_calls():
    print("[noalloc] call 1: 3 pairs up to 512x512, 12-bit codes with noise", flush=True)
    ref1, out1 = _render_both(((512, 512), (300, 200), (256, 384)), 3, 12, 0.01)
    assert np.array_equal(to_np(ref1), to_np(out1))
    print("[noalloc] call 2: 1 pair 128x160, float images", flush=True)
    ref2, out2 = _render_both(((128, 160),), 4, 0, 0.0)
    assert np.array_equal(to_np(ref2), to_np(out2))
    print("[noalloc] call 3: 2 pairs, 64x64 tiles, 8-bit codes", flush=True)
    ref3, out3 = _render_both(((200, 120), (97, 31)), 5, 8, 0.02, sp.tiling(64, 64, 1024, 128))
    assert np.array_equal(to_np(ref3), to_np(out3))


def test_noalloc_refuses_batch_larger_than_scratch():
    wl = get_workload("scale_1024")
    n_max = [sp.particle_count(H, W, wl.ppp[1]) for (H, W) in wl.sizes]
    batch = sp.PairBatch.build(wl.sizes, [(H // 4, W // 4) for (H, W) in wl.sizes], n_max, device=DEV)
    sprm, aprm, rprm = params_of(wl)
    need = sp.workspace_size(batch, rprm)
    assert need > (64 << 20)
    dummy = torch.zeros(4, dtype=torch.float32, device=DEV)
    images = torch.zeros(4, dtype=sp.api.U16, device=DEV)
    with pytest.raises(_lib.SynthPixError) as ei:
        sp.render_pair_noalloc(batch, dummy, dummy, dummy, dummy, dummy, dummy, dummy, rprm, images)
    assert ei.value.status == _lib.SP_ERR_WORKSPACE
    torch.cuda.synchronize()
