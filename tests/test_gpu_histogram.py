"""Histogram adjustment on the GPU against the oracle: every frame's codes
mapped onto a target histogram, bit for bit equal to ``oracle.histogram``."""

import numpy as np
import pytest
import torch

from oracle import histogram as oh
from workloads import get_workload

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2512_09664_amd as sp
    from gpu_util import DEV, run_pipeline, to_dev, to_np


def _frames(batch, img):
    a = to_np(img)
    for p in range(batch.n_pairs):
        H, W = batch.host[p].H, batch.host[p].W
        o = batch.host[p].image_offset
        for f in range(2):
            yield p, f, a[o + f * H * W:o + (f + 1) * H * W].reshape(H, W)


def _render(bits, sizes=((160, 224), (97, 131), (256, 256)), noise=0.02):
    wl = get_workload("uneven_256").with_(sizes=sizes, bits=bits, noise_sigma=noise, blur_radius=1,
                                          integrator="rk4", substeps=2, flow="lamb_oseen", seed=3)
    batch, flows, P, x2, y2, img = run_pipeline(wl)
    return batch, img


@pytest.mark.parametrize("bits", [3, 8, 12, 14])
def test_histogram_match_equals_oracle(bits):
    batch, img = _render(bits)
    before = [f.copy() for _, _, f in _frames(batch, img)]
    rng = np.random.default_rng(bits)
    target = rng.integers(0, 1000, 1 << bits).astype(np.uint32)
    target[rng.integers(0, 1 << bits)] += 1
    ws = sp.histogram_match(batch, img, to_dev(target), bits)
    torch.cuda.synchronize()
    assert sp.read_status(ws) == 0
    for (p, f, got), src in zip(_frames(batch, img), before):
        ref = oh.match(src, target, bits)
        assert np.array_equal(got, ref), f"pair {p} frame {f}: {(got != ref).sum()} codes differ"


def test_own_histogram_is_identity_and_bad_target_is_flagged():
    bits = 12
    batch, img = _render(bits, sizes=((128, 192),))
    frames = list(_frames(batch, img))
    own = np.bincount(frames[0][2].reshape(-1), minlength=1 << bits).astype(np.uint32)
    keep = to_np(img).copy()
    ws = sp.histogram_match(batch, img, to_dev(own), bits)
    torch.cuda.synchronize()
    assert sp.read_status(ws) == 0
    got = to_np(img)
    H, W = 128, 192
    assert np.array_equal(got[:H * W], keep[:H * W])           # frame 1: its own histogram
    ref2 = oh.match(keep[H * W:2 * H * W].reshape(H, W), own, bits)
    assert np.array_equal(got[H * W:2 * H * W].reshape(H, W), ref2)
    # an all-zero target leaves the images as they are and raises the flag
    keep = to_np(img).copy()
    ws = sp.histogram_match(batch, img, torch.zeros(1 << bits, dtype=torch.int32, device=DEV), bits)
    torch.cuda.synchronize()
    assert sp.read_status(ws) == 8
    assert np.array_equal(to_np(img), keep)


def test_histogram_match_full_size():
    # four 1024x1024 pairs of the scale workload, 12-bit codes, a flat target
    wl = get_workload("scale_1024").with_(sizes=((1024, 1024),) * 4)
    batch, flows, P, x2, y2, img = run_pipeline(wl)
    before = [f.copy() for _, _, f in _frames(batch, img)]
    target = np.ones(4096, dtype=np.uint32)
    ws = sp.histogram_match(batch, img, to_dev(target), 12)
    torch.cuda.synchronize()
    assert sp.read_status(ws) == 0
    for (p, f, got), src in zip(_frames(batch, img), before):
        assert np.array_equal(got, oh.match(src, target, 12))
