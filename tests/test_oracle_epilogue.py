"""Pins of the oracle's acquisition effects: blur, noise, integer codes."""

import math

import numpy as np
import pytest
from scipy import stats

from oracle import epilogue as ep
from oracle import philox as ph


@pytest.mark.parametrize("b,s", [(1, 0.7), (2, 1.0), (3, 1.3)])
def test_blur_impulse_response_is_outer_product(ra, b, s):
    w = ep.blur_weights(b, s)
    k = np.arange(-b, b + 1)
    g = np.exp(-k * k / (2 * s * s))
    assert np.allclose(w, g / g.sum(), rtol=1e-7)
    assert abs(float(w.astype(np.float64).sum()) - 1) < 1e-6
    img = np.zeros((15, 17))
    img[7, 8] = 1.0
    out = ep.blur(img, w)
    ref = np.zeros_like(img)
    ref[7 - b:8 + b, 8 - b:9 + b] = np.outer(w.astype(np.float64), w.astype(np.float64))
    assert np.allclose(out, ref, atol=1e-16)
    r = ra.blur(img.astype(np.float32), w)
    assert np.max(np.abs(r - ref)) < 1e-7


def test_blur_preserves_constant_in_interior_and_zero_pads():
    w = ep.blur_weights(2, 1.0)
    img = np.full((12, 12), 0.37)
    out = ep.blur(img, w)
    wsum = float(w.astype(np.float64).sum())
    assert np.allclose(out[2:-2, 2:-2], 0.37 * wsum ** 2, rtol=1e-14)
    assert out[0, 0] == pytest.approx(0.37 * float(w[2:].astype(np.float64).sum()) ** 2, rel=1e-14)


def test_blur_adjoint_dot_product():
    rng = np.random.default_rng(0)
    w = np.array([0.1, 0.25, 0.3, 0.2, 0.15], dtype=np.float32)     # deliberately asymmetric
    x = rng.normal(size=(13, 9))
    yv = rng.normal(size=(13, 9))
    lhs = np.sum(ep.blur(x, w) * yv)
    rhs = np.sum(x * ep.blur_adjoint(yv, w))
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


def test_noise_statistics_and_box_muller_structure():
    H, W = 128, 130                                      # W not a multiple of 4
    n0 = ep.noise_normals(H, W, 0, pair_id=3, seed=9)
    n1 = ep.noise_normals(H, W, 1, pair_id=3, seed=9)
    for n in (n0, n1):
        assert abs(n.mean()) < 5 / math.sqrt(n.size)
        assert abs(n.var() - 1) < 0.03
        assert stats.kstest(n.reshape(-1), "norm").pvalue > 1e-3
    assert abs(np.corrcoef(n0.reshape(-1), n1.reshape(-1))[0, 1]) < 5 / math.sqrt(n0.size)
    assert abs(np.corrcoef(n0[:, :-1].reshape(-1), n0[:, 1:].reshape(-1))[0, 1]) < 0.02
    # columns 4k, 4k+1 share one (u1, u2): their squares sum to -2 ln u1
    Wq = (W + 3) // 4
    w = ph.draw(np.uint64(5 * Wq + 7), ph.STREAM_NOISE0, 3, 9)
    u1 = float(ph.uniform24_open0(w[0]))
    assert n0[5, 28] ** 2 + n0[5, 29] ** 2 == pytest.approx(-2 * math.log(u1), rel=1e-12)
    u1b = float(ph.uniform24_open0(w[2]))
    assert n0[5, 30] ** 2 + n0[5, 31] ** 2 == pytest.approx(-2 * math.log(u1b), rel=1e-12)
    # frames use different streams; pairs and seeds differ
    assert not np.any(n0 == n1)
    assert not np.any(ep.noise_normals(8, 8, 0, 4, 9) == ep.noise_normals(8, 8, 0, 3, 9))


@pytest.mark.parametrize("bits", [8, 12, 16])
def test_quantiser_codes(ra, bits):
    L = (1 << bits) - 1
    k = np.arange(L + 1)
    exact = (k / L).astype(np.float32)                   # nearest float to each code's value
    assert np.array_equal(ra.quantise(exact, bits).astype(np.int64), k)
    assert np.array_equal(ep.quantise(exact, bits).astype(np.int64), k)
    v = np.array([-1.0, -1e-9, 0.0, 1.0, 1.5, 1e9, np.nan], dtype=np.float32)
    assert list(ra.quantise(v, bits)) == [0, 0, 0, L, L, L, 0]
    # monotone and within half a code everywhere in range
    rng = np.random.default_rng(bits)
    v = np.sort(rng.uniform(-0.01, 1.01, 200000).astype(np.float32))
    q = ra.quantise(v, bits).astype(np.int64)
    assert np.all(np.diff(q) >= 0)
    inr = (v >= 0) & (v <= 1)
    assert np.all(np.abs(q[inr] - v[inr].astype(np.float64) * L) <= 0.5 + 1e-6 * L)


def test_quantiser_ties_go_to_even(ra):
    # v * L lands exactly on k + 1/2 when v = (k + 1/2) / L is representable and
    # the product rounds back exactly: search binary32 values with that property.
    L = 4095
    hits = 0
    for k in range(0, L, 7):
        v = np.float32((k + 0.5) / L)
        for cand in (np.nextafter(v, np.float32(0)), v, np.nextafter(v, np.float32(2))):
            p = np.float32(cand) * np.float32(L)
            if float(p) == k + 0.5:
                q = int(ra.quantise(np.array([cand], dtype=np.float32), 12)[0])
                assert q == (k if k % 2 == 0 else k + 1)
                hits += 1
    assert hits > 10
