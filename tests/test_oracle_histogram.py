"""Pins of the histogram-adjustment oracle (``oracle/histogram.py``): the
identity for an image's own histogram, a single-bin target, equalisation to a
flat target, the exact-rational definition by brute force, scale invariance,
and NumPy's CDF search where every ratio is exact in binary."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import histogram as oh


def _img(rng, bits, n, skew=2.0):
    B = 1 << bits
    return np.minimum((rng.random(n) ** skew * B).astype(np.int64), B - 1).astype(np.uint16)


@pytest.mark.parametrize("bits", [4, 8, 12])
def test_own_histogram_is_identity(bits):
    rng = np.random.default_rng(bits)
    img = _img(rng, bits, 5000)
    h = np.bincount(img, minlength=1 << bits)
    assert np.array_equal(oh.match(img, h, bits), img)


def test_single_bin_target_and_monotone_lut():
    rng = np.random.default_rng(1)
    img = _img(rng, 8, 3000)
    t = np.zeros(256, dtype=np.int64)
    t[77] = 5
    assert np.all(oh.match(img, t, 8) == 77)
    lut = oh.mapping(img, rng.integers(0, 9, 256), 8)
    assert np.all(np.diff(lut.astype(np.int64)) >= 0)


def test_flat_target_equalises():
    rng = np.random.default_rng(2)
    bits = 8
    img = _img(rng, bits, 1 << 16, skew=3.0)
    out = oh.match(img, np.ones(256, dtype=np.int64), bits)
    h = np.bincount(out, minlength=256)
    hs = np.bincount(img, minlength=256)
    # every output bin holds N / 256 pixels up to one source bin's worth
    assert np.all(np.abs(h[h > 0] - (1 << 16) / 256) <= hs.max())


def test_matches_exact_rational_definition():
    rng = np.random.default_rng(3)
    for bits in (3, 5):
        B = 1 << bits
        for _ in range(20):
            img = rng.integers(0, B, size=int(rng.integers(1, 60))).astype(np.uint16)
            t = rng.integers(0, 4, B)
            t[rng.integers(0, B)] += 1
            h = np.bincount(img, minlength=B)
            N, T_tot = img.size, int(t.sum())
            ref = []
            for k in range(B):
                Sk = Fraction(int(h[:k + 1].sum()), N)
                ref.append(next(m for m in range(B) if Fraction(int(t[:m + 1].sum()), T_tot) >= Sk))
            assert np.array_equal(oh.mapping(img, t, bits), np.array(ref, dtype=np.uint16))


def test_scale_invariance_and_numpy_cdf_search():
    rng = np.random.default_rng(4)
    bits = 10
    img = _img(rng, bits, 1 << 14)                             # N a power of two
    for t in (np.where(np.arange(1 << bits) < 512, 8, 0),
              rng.multinomial(1 << 12, rng.dirichlet(np.ones(1 << bits)))):   # totals powers of two
        lut = oh.mapping(img, t, bits)
        assert np.array_equal(lut, oh.mapping(img, 7 * t, bits))
        # every CDF value is a dyadic rational, exact in float64
        Scdf = np.cumsum(np.bincount(img, minlength=1 << bits)) / img.size
        Tcdf = np.cumsum(t) / t.sum()
        assert np.array_equal(lut, np.searchsorted(Tcdf, Scdf, side="left").astype(np.uint16))
