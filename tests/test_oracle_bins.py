"""Pins of the oracle's tile membership (patch support of Section 2,
"Efficient rasterization", grown by the blur apron)."""

import numpy as np
import pytest

from oracle import bins as bn
from workloads import particles


@pytest.mark.parametrize("H,W,th,tw,apron", [(20, 28, 8, 8, 0), (20, 28, 8, 8, 1),
                                             (33, 17, 16, 8, 2), (16, 16, 16, 16, 1)])
def test_bins_match_bruteforce(H, W, th, tw, apron):
    P = particles.random_particles(11, 80, H, W, d_range=(0.7, 6.0), pad=7, zero_frac=0.1)
    E = particles.edge_case_particles(H, W, tile=th)
    x = np.concatenate([P["x"], E["x"]])
    y = np.concatenate([P["y"], E["y"]])
    d = np.concatenate([P["d"], E["d"]])
    I0 = np.concatenate([P["I0"], E["I0"]])
    counts, offsets, entries = bn.bin_frame(x, y, d, I0, H, W, th, tw, apron)
    ref = bn.bin_frame_bruteforce(x, y, d, I0, H, W, th, tw, apron)
    assert counts.sum() == entries.size == offsets[-1]
    for t, members in enumerate(ref):
        seg = entries[offsets[t]:offsets[t + 1]]
        assert list(seg) == sorted(members)
    assert counts.sum() > len(x) // 2          # the fixture does produce members


def test_support_range_is_the_float32_predicate(ra):
    rng = np.random.default_rng(3)
    for _ in range(3000):
        p = np.float32(rng.uniform(-10, 60))
        R = np.float32(rng.uniform(0.1, 9))
        if rng.random() < 0.2:                               # land exactly on a boundary
            p = np.float32(np.floor(p) + 0.5 + R) if rng.random() < 0.5 else np.float32(np.floor(p) + 0.5 - R)
        lo, hi = bn.support_range_f32(np.array([p]), np.array([R]), 50)
        k = np.arange(50)
        inside = np.abs((k.astype(np.float32) + np.float32(0.5)) - p) <= R
        got = ra.support_range(p, R, 50)
        if inside.any():
            assert (lo[0], hi[0]) == (k[inside][0], k[inside][-1])
            assert got == (lo[0], hi[0])
            assert inside[lo[0]:hi[0] + 1].all()
        else:
            assert lo[0] > hi[0] and got is None


def test_masked_particles_are_not_binned():
    x = np.array([5.5, 5.5], dtype=np.float32)
    y = np.array([5.5, 5.5], dtype=np.float32)
    d = np.array([2.0, 2.0], dtype=np.float32)
    I0 = np.array([0.0, 0.5], dtype=np.float32)
    counts, offsets, entries = bn.bin_frame(x, y, d, I0, 16, 16, 8, 8, 1)
    assert set(entries.tolist()) == {1} and counts.tolist() == [1, 1, 1, 1]
