"""Pins of the oracle's rendering: Eq. 1 (rho = 0, sigma = d/4) summed over
particles (Section 2, "Considerations on the aggregation"), each on its patch
(Section 2, "Efficient rasterization")."""

import math

import numpy as np
import pytest

from oracle import advect as adv
from oracle import render as rd
from workloads import flows, particles


def _one(x, y, d=2.5, I0=0.9, z=0.0):
    a = lambda v: np.array([v], dtype=np.float64)
    return a(x), a(y), a(z), a(d), a(I0)


@pytest.mark.parametrize("z", [0.0, 0.3, -0.8])
def test_particle_on_pixel_centre_peak_and_neighbours(ra, z):
    H, W, d, I0, s = 12, 20, 2.5, 0.9, 0.5
    x, y, zz, dd, II = _one(10.5, 3.5, d, I0, z)           # pixel (row 3, col 10)
    img = rd.render_frame(x, y, zz, dd, II, H, W, s)
    A = I0 * math.exp(-z * z / (2 * s * s))
    assert img[3, 10] == pytest.approx(A, rel=1e-15)
    assert np.unravel_index(np.argmax(img), img.shape) == (3, 10)
    assert img[3, 11] == pytest.approx(A * math.exp(-8 / d ** 2), rel=1e-14)
    assert img[4, 10] == pytest.approx(A * math.exp(-8 / d ** 2), rel=1e-14)
    assert img[4, 11] == pytest.approx(A * math.exp(-16 / d ** 2), rel=1e-14)
    assert img[3, 12] == pytest.approx(A * math.exp(-32 / d ** 2), rel=1e-14)
    # support: |dx| <= 1.5 d = 3.75 -> columns 7..13 only
    assert img[3, 14] == 0.0 and img[3, 6] == 0.0 and img[3, 13] > 0 and img[3, 7] > 0
    r = ra.render(x.astype(np.float32), y.astype(np.float32), zz.astype(np.float32),
                  dd.astype(np.float32), II.astype(np.float32), H, W, s)
    assert abs(r[3, 10] - A) < 2e-7 and np.max(np.abs(r - img)) < 2e-7


def _lattice_sum(p, sigma):
    """sum_k exp(-(k + 1/2 - p)^2 / (2 sigma^2)) over all integers k, by Poisson
    summation: sqrt(2 pi) sigma [1 + 2 sum_m exp(-2 pi^2 m^2 sigma^2) cos(2 pi m (p - 1/2))]."""
    m = np.arange(1, 40)
    return math.sqrt(2 * math.pi) * sigma * (1 + 2 * np.sum(np.exp(-2 * math.pi ** 2 * m ** 2 * sigma ** 2)
                                                            * np.cos(2 * math.pi * m * (p - 0.5))))


@pytest.mark.parametrize("d,x,y", [(1.0, 20.3, 17.9), (1.5, 20.0, 20.0), (2.7, 19.71, 21.13),
                                   (4.0, 20.25, 18.6), (6.0, 21.0, 19.5)])
def test_isolated_particle_mass(d, x, y):
    """Sum over pixels = A * Lx * Ly with the exact lattice sums per axis; for
    d >= 4 this is A pi d^2 / 8 to 1e-6 (the continuous Gaussian mass)."""
    H = W = 40
    img = rd.render_frame(*_one(x, y, d, 1.0, 0.0), H, W, 0.5, cutoff=False)
    s = d / 4.0
    ref = _lattice_sum(x, s) * _lattice_sum(y, s)
    assert img.sum() == pytest.approx(ref, rel=1e-12)
    cut = rd.render_frame(*_one(x, y, d, 1.0, 0.0), H, W, 0.5, cutoff=True)
    assert abs(cut.sum() - ref) < 1e-7 * ref * d ** 2        # patch tail: erfc(6/sqrt 2) per axis
    if d >= 4:
        assert img.sum() == pytest.approx(math.pi * d * d / 8, rel=1e-6)


def test_cutoff_matches_bruteforce_sum():
    H, W = 32, 24
    P = particles.random_particles(4, 60, H, W, d_range=(1.0, 5.0), pad=6)
    cut = rd.render_frame(P["x"], P["y"], P["z"], P["d"], P["I0"], H, W, 0.5, cutoff=True)
    full = rd.render_frame(P["x"], P["y"], P["z"], P["d"], P["I0"], H, W, 0.5, cutoff=False)
    # values beyond 1.5 d are below A e^-18 per particle
    assert np.max(np.abs(cut - full)) < 60 * math.exp(-18) * 4
    assert np.max(np.abs(cut - full)) <= 1e-5 * full.max()
    # per-pixel definition agrees with the vectorised render
    for (r, c) in ((0, 0), (5, 7), (31, 23), (16, 12)):
        assert rd.render_pixel_direct(P["x"], P["y"], P["z"], P["d"], P["I0"], r, c, 0.5) == \
            pytest.approx(cut[r, c], rel=1e-12, abs=1e-300)


def test_masked_and_outside_particles():
    H, W = 16, 16
    x, y, z, d, I0 = (np.array(v, dtype=np.float64) for v in
                      ([8.5, 8.5, -30.0, 17.0], [8.5, 8.5, 5.0, 8.5], [0, 0, 0, 0], [2, 2, 2, 2],
                       [0.0, 0.7, 1.0, 1.0]))
    img = rd.render_frame(x, y, z, d, I0, H, W, 0.5)
    assert img[8, 8] == pytest.approx(0.7, rel=1e-15)      # masked one adds nothing
    assert img[:, :10].sum() > 0 and img[8, 15] > 0          # half-outside particle (x = 17) reaches col 15
    # the far-outside particle contributes nothing
    img2 = rd.render_frame(x[:2], y[:2], z[:2], d[:2], I0[:2], H, W, 0.5)
    img3 = rd.render_frame(x[[0, 1, 3]], y[[0, 1, 3]], z[[0, 1, 3]], d[[0, 1, 3]], I0[[0, 1, 3]], H, W, 0.5)
    assert np.array_equal(img, img3) and not np.array_equal(img, img2)


def test_linearity_and_mirror_symmetry():
    H, W = 20, 28
    P = particles.random_particles(5, 40, H, W)
    a = rd.render_frame(P["x"], P["y"], P["z"], P["d"], P["I0"], H, W, 0.5)
    b = rd.render_frame(P["x"], P["y"], P["z"], P["d"], 2 * P["I0"].astype(np.float64), H, W, 0.5)
    assert np.allclose(b, 2 * a, rtol=1e-14, atol=0)
    m = rd.render_frame(W - P["x"].astype(np.float64), P["y"], P["z"], P["d"], P["I0"], H, W, 0.5)
    assert np.allclose(m, a[:, ::-1], rtol=1e-12, atol=1e-300)
    zf = rd.render_frame(P["x"], P["y"], -P["z"].astype(np.float64), P["d"], P["I0"], H, W, 0.5)
    assert np.array_equal(zf, a)                                # sheet profile is even in z


def test_zero_flow_gives_identical_frames(ra):
    H, W = 48, 64
    P = particles.random_particles(6, 200, H, W)
    F = flows.uniform_grid(12, 16, 0.0, 0.0)
    x2, y2 = adv.advect(F, H, W, P["x"], P["y"], 1.0, 4, "rk4")
    f1 = rd.render_frame(P["x"], P["y"], P["z"], P["d"], P["I0"], H, W, 0.5)
    f2 = rd.render_frame(x2, y2, P["z"], P["d"], P["I0"], H, W, 0.5)
    assert np.array_equal(f1, f2)
    rx, ry = ra.advect(F, H, W, P["x"], P["y"], 1.0, 4, "rk4")
    r1 = ra.render(P["x"], P["y"], P["z"], P["d"], P["I0"], H, W, 0.5)
    r2 = ra.render(rx, ry, P["z"], P["d"], P["I0"], H, W, 0.5)
    assert np.array_equal(r1, r2)


@pytest.mark.parametrize("du,dv", [(3, -2), (-5, 4), (0, 7)])
def test_integer_flow_shifts_frame(ra, du, dv):
    """Frame 2 under a uniform integer flow is frame 1 moved by whole pixels:
    exact in float64, and exact in binary32 for positions on a dyadic grid
    (so x + du is representable)."""
    H, W = 40, 48
    rng = np.random.default_rng(7)
    n = 120
    x = (rng.integers(-256, (W + 4) * 64, n) / 64.0).astype(np.float32)
    y = (rng.integers(-256, (H + 4) * 64, n) / 64.0).astype(np.float32)
    d = (rng.integers(64, 320, n) / 64.0).astype(np.float32)
    z = (rng.uniform(-1, 1, n)).astype(np.float32)
    I0 = rng.uniform(0.8, 1, n).astype(np.float32)
    F = flows.uniform_grid(10, 12, float(du), float(dv))
    x2, y2 = adv.advect(F, H, W, x, y, 1.0, 1, "euler")
    f1 = rd.render_frame(x, y, z, d, I0, H, W, 0.5)
    f2 = rd.render_frame(x2, y2, z, d, I0, H, W, 0.5)
    r0, r1 = max(0, dv), H + min(0, dv)
    c0, c1 = max(0, du), W + min(0, du)
    assert np.array_equal(f2[r0:r1, c0:c1], f1[r0 - dv:r1 - dv, c0 - du:c1 - du])
    rx, ry = ra.advect(F, H, W, x, y, 1.0, 1, "euler")
    assert np.array_equal(rx, x + np.float32(du)) and np.array_equal(ry, y + np.float32(dv))
    g1 = ra.render(x, y, z, d, I0, H, W, 0.5)
    g2 = ra.render(rx, ry, z, d, I0, H, W, 0.5)
    assert np.array_equal(g2[r0:r1, c0:c1], g1[r0 - dv:r1 - dv, c0 - du:c1 - du])


def test_binary32_mirror_tracks_float64(ra):
    H, W = 96, 80
    P = particles.random_particles(8, 600, H, W, d_range=(1.0, 6.0), pad=8, zero_frac=0.1)
    ref = rd.render_frame(P["x"], P["y"], P["z"], P["d"], P["I0"], H, W, 0.5)
    got = ra.render(P["x"], P["y"], P["z"], P["d"], P["I0"], H, W, 0.5)
    err = np.max(np.abs(got.astype(np.float64) - ref))
    assert err <= 1e-6 * ref.max(), err
