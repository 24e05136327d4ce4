"""Pins of the full-model oracle (``oracle/model.py``) and its binary32 mirror:
Eq. 1 against its covariance-matrix form and its closed-form mass, the patch
against the untruncated sum, the isotropic reduction, mirror and transpose
symmetries, the statistics of the shape, jitter and hiding draws, the
Remark 1 law at its closed-form points, and the out-of-plane motion under
fields the integrators reproduce exactly."""

import math

import numpy as np
import pytest
from scipy import stats

from oracle import model as om
from oracle import ra32
from oracle import render as rd


def _cov_form(dx, dy, d, dyd, rho):
    """exp(-v^T S^-1 v / 2) with S the covariance of Eq. 1 (independent of the expanded form)."""
    sx, sy = d / 4.0, dyd / 4.0
    S = np.array([[sx * sx, rho * sx * sy], [rho * sx * sy, sy * sy]])
    Si = np.linalg.inv(S)
    v = np.stack([dx, dy], axis=-1)
    return np.exp(-0.5 * np.einsum("...i,ij,...j->...", v, Si, v))


def test_footprint_matches_covariance_form():
    rng = np.random.default_rng(1)
    for _ in range(50):
        d, dyd = rng.uniform(1.0, 8.0, 2)
        rho = rng.uniform(-0.95, 0.95)
        dx = rng.uniform(-10, 10, 64)
        dy = rng.uniform(-10, 10, 64)
        a = om.footprint(dx, dy, d, dyd, rho)
        b = _cov_form(dx, dy, d, dyd, rho)
        assert np.max(np.abs(a - b)) <= 1e-12


def test_rho_sign_orientation():
    # positive rho elongates the particle along x = y (image coordinates, y down)
    a = om.footprint(np.array([1.0]), np.array([1.0]), 3.0, 3.0, 0.5)[0]
    b = om.footprint(np.array([1.0]), np.array([-1.0]), 3.0, 3.0, 0.5)[0]
    assert a > b


@pytest.mark.parametrize("d,dyd,rho", [(4.0, 4.0, 0.0), (4.0, 6.0, 0.5), (6.0, 4.5, -0.8), (8.0, 8.0, 0.9)])
def test_mass_closed_form(d, dyd, rho):
    # Poisson summation: the lattice sum of a Gaussian of covariance S differs from
    # its integral by terms exp(-2 pi^2 k^T S k), k != 0 integer; every case here
    # has k^T S k >= 0.8 (< 2e-7 relative).  The integral of Eq. 1 is
    # 2 pi sx sy sqrt(1 - rho^2).
    H = W = 96
    img = om.render_frame([47.3], [48.6], [0.9], [d], [dyd], [rho], H, W)
    mass = 0.9 * 2.0 * math.pi * (d / 4) * (dyd / 4) * math.sqrt(1 - rho * rho)
    assert abs(img.sum() - mass) <= 1e-6 * mass


def test_patch_truncation_is_negligible():
    rng = np.random.default_rng(2)
    H, W, n = 40, 44, 12
    x, y = rng.uniform(0, W, n), rng.uniform(0, H, n)
    d, dyd = rng.uniform(1.5, 6, n), rng.uniform(1.5, 6, n)
    rho = rng.uniform(-0.95, 0.95, n)
    A = rng.uniform(0.5, 1.0, n)
    a = om.render_frame(x, y, A, d, dyd, rho, H, W, cutoff=True)
    b = om.render_frame(x, y, A, d, dyd, rho, H, W, cutoff=False)
    # outside the box the exponent exceeds 18: every dropped term is below e^-18 A
    assert np.max(np.abs(a - b)) <= n * math.exp(-18.0)


def test_isotropic_reduction_matches_isotropic_oracle():
    rng = np.random.default_rng(3)
    H, W, n = 48, 40, 30
    x, y = rng.uniform(-3, W + 3, n), rng.uniform(-3, H + 3, n)
    d = rng.uniform(1.0, 5.0, n)
    z = rng.uniform(-1, 1, n)
    I0 = rng.uniform(0.8, 1.0, n)
    iso = rd.render_frame(x, y, z, d, I0, H, W, 0.5)
    A = om.peaks(I0, z, "gauss", 0.5)
    full = om.render_frame(x, y, A, d, d, np.zeros(n), H, W)
    assert np.max(np.abs(iso - full)) <= 1e-12


def test_mirror_and_transpose_symmetry():
    rng = np.random.default_rng(4)
    H, W, n = 32, 36, 10
    x, y = rng.uniform(0, W, n), rng.uniform(0, H, n)
    d, dyd = rng.uniform(1.5, 5, n), rng.uniform(1.5, 5, n)
    rho = rng.uniform(-0.9, 0.9, n)
    A = rng.uniform(0.5, 1.0, n)
    img = om.render_frame(x, y, A, d, dyd, rho, H, W, cutoff=False)
    # x -> W - x mirrors the columns and flips the sign of rho
    mir = om.render_frame(W - x, y, A, d, dyd, -rho, H, W, cutoff=False)
    assert np.max(np.abs(img[:, ::-1] - mir)) <= 1e-12
    # swapping the axes swaps the diameters and keeps rho
    tr = om.render_frame(y, x, A, dyd, d, rho, W, H, cutoff=False)
    assert np.max(np.abs(img.T - tr)) <= 1e-12


def test_seed_shape_statistics():
    n = 200000
    dy, rho = om.seed_shape(n, 7, 11, "uniform", (1.0, 5.0), (-0.5, 0.8))
    assert stats.kstest(dy, stats.uniform(1.0, 4.0).cdf).pvalue > 1e-3
    assert stats.kstest(rho, stats.uniform(-0.5, 1.3).cdf).pvalue > 1e-3
    dyn, _ = om.seed_shape(n, 7, 11, "normal", (2.5, 0.5, 1.0, 5.0), (0.0, 0.0))
    assert abs(dyn.mean() - 2.5) < 0.01 and abs(dyn.std() - 0.5) < 0.01
    # the shape stream is independent of the geometry stream's diameter
    from oracle import seed as sd
    P = sd.seed_pair(400, 500, 7, 11, ppp=(1.0, 1.0), d_dist="uniform", d_params=(1.0, 5.0))
    dy2, _ = om.seed_shape(P["n_max"], 7, 11, "uniform", (1.0, 5.0), (0.0, 0.0))
    assert abs(np.corrcoef(P["d"], dy2)[0, 1]) < 0.01


def test_jitter_statistics_and_identity():
    n = 200000
    rng = np.random.default_rng(5)
    d = rng.uniform(3.0, 4.0, n)
    dyd = rng.uniform(3.0, 4.0, n)
    rho = rng.uniform(-0.3, 0.3, n)
    I0 = np.where(np.arange(n) < n - 1000, rng.uniform(0.8, 1.0, n), 0.0)
    f1, f2 = om.frame_params(d, dyd, rho, I0, 3, 9)
    for a, b in zip(f1, f2):
        assert np.array_equal(a, b)
    f1, f2 = om.frame_params(d, dyd, rho, I0, 3, 9, jitter=(0.1, 0.05, 0.02), d_max=6.0)
    assert np.array_equal(f1[0], d) and np.array_equal(f1[3], I0)
    nd = (f2[0] - d) / 0.1
    assert stats.kstest(nd, "norm").pvalue > 1e-3
    nr = (f2[2] - rho) / 0.05
    assert stats.kstest(nr, "norm").pvalue > 1e-3
    act = I0 > 0
    ni = (f2[3][act] - I0[act]) / 0.02
    assert stats.kstest(ni, "norm").pvalue > 1e-3
    assert np.all(f2[3][~act] == 0.0)
    c = np.corrcoef(np.stack([nd, (f2[1] - dyd) / 0.1, nr, (f2[3] - I0)]))
    assert np.max(np.abs(c - np.diag(np.diag(c)))) < 0.01


def test_jitter_clips_to_valid_ranges():
    n = 50000
    d = np.full(n, 0.5)
    rho = np.full(n, 0.98)
    I0 = np.full(n, 0.01)
    f1, f2 = om.frame_params(d, d, rho, I0, 1, 2, jitter=(1.0, 0.5, 0.5), d_max=1.0)
    assert f2[0].min() == 0.0 and f2[0].max() == 1.0
    assert f2[2].max() == om.RHO_MAX and f2[2].min() >= -om.RHO_MAX
    assert f2[3].min() == 0.0


@pytest.mark.parametrize("p", [0.0, 0.2, 1.0])
def test_hiding_statistics(p):
    n = 100000
    I0 = np.full(n, 0.9)
    d = np.full(n, 3.0)
    f1, f2 = om.frame_params(d, d, np.zeros(n), I0, 4, 8, hide_p=p)
    h1, h2 = f1[3] == 0, f2[3] == 0
    if p == 0.0:
        assert not h1.any() and not h2.any()
        return
    if p == 1.0:
        assert h1.all() and h2.all()
        return
    sd = math.sqrt(n * p * (1 - p))
    assert abs(h1.sum() - n * p) < 5 * sd and abs(h2.sum() - n * p) < 5 * sd
    both = (h1 & h2).sum()
    assert abs(both - n * p * p) < 5 * math.sqrt(n * p * p * (1 - p * p))


def test_remark1_law_closed_forms():
    dz0 = 0.7
    for s in (0.5, 1.0, 2.0, 3.3):
        assert om.sheet_remark1(0.0, dz0, s) == 1.0
        # |2 z^2 / DZ0^2| = 1 at z = DZ0 / sqrt(2): the law is exp(-1/sqrt(2 pi)) for every shape
        assert abs(om.sheet_remark1(dz0 / math.sqrt(2.0), dz0, s) - math.exp(-1.0 / math.sqrt(2 * math.pi))) < 1e-15
    # shape 1 is a Gaussian in z of variance DZ0^2 sqrt(2 pi) / 4
    z = np.linspace(-2, 2, 101)
    var = dz0 ** 2 * math.sqrt(2 * math.pi) / 4.0
    assert np.max(np.abs(om.sheet_remark1(z, dz0, 1.0) - np.exp(-z * z / (2 * var)))) < 1e-15
    # larger shape factors are flatter inside |2 z^2 / DZ0^2| < 1 and steeper outside
    zi, zo = 0.3 * dz0, 1.2 * dz0
    assert om.sheet_remark1(zi, dz0, 3.0) > om.sheet_remark1(zi, dz0, 1.0)
    assert om.sheet_remark1(zo, dz0, 3.0) < om.sheet_remark1(zo, dz0, 1.0)


@pytest.mark.parametrize("integrator,substeps", [("euler", 1), ("euler", 4), ("rk4", 2)])
def test_out_of_plane_motion_exact_cases(integrator, substeps):
    H, W, Gh, Gw = 64, 80, 16, 20
    rng = np.random.default_rng(6)
    n = 500
    x, y, z = rng.uniform(0, W, n), rng.uniform(0, H, n), rng.uniform(-1, 1, n)
    flow = np.zeros((Gh, Gw, 2))
    flow[..., 0], flow[..., 1] = 1.5, -0.75
    # zero w: z unchanged bitwise
    _, _, z2 = om.advect3(flow, np.zeros((Gh, Gw)), H, W, x, y, z, 1.0, substeps, integrator)
    assert np.array_equal(z2, z)
    # uniform dyadic w: z2 = z + w dt
    _, _, z2 = om.advect3(flow, np.full((Gh, Gw), 0.125), H, W, x, y, z, 1.0, substeps, integrator)
    assert np.max(np.abs(z2 - (z + 0.125))) < 1e-15
    # w affine in x inside the node hull, uniform (u, v): w along the path is
    # linear in t, so Euler with n steps gives the left Riemann sum and RK4 the integral
    a, b = 0.01, -0.2
    jx = (np.arange(Gw) + 0.5) * W / Gw
    wg = np.broadcast_to(a * jx + b, (Gh, Gw)).copy()
    xi = rng.uniform(20, 50, n)
    yi = rng.uniform(10, 50, n)
    _, _, z2 = om.advect3(flow, wg, H, W, xi, yi, z, 1.0, substeps, integrator)
    if integrator == "rk4":
        expect = z + a * (xi + 0.75) + b
    else:
        h = 1.0 / substeps
        expect = z + sum(h * (a * (xi + 1.5 * k * h) + b) for k in range(substeps))
    assert np.max(np.abs(z2 - expect)) < 1e-12


# ------------------------------------------------------------------ binary32 mirror

def test_mirror_sin2pi_accuracy():
    u = np.arange(0, 1, 1.0 / 4099)
    got = np.array([ra32.sin2pi(float(np.float32(v))) for v in u])
    ref = np.sin(2 * np.pi * u.astype(np.float32).astype(np.float64))
    assert np.max(np.abs(got - ref)) < 2e-6


def test_mirror_isotropic_reduction_bitwise():
    # rho = 0 and d_y = d through the full-model mirror gives the isotropic mirror's bits
    rng = np.random.default_rng(7)
    H, W, n = 64, 72, 300
    x = rng.uniform(-4, W + 4, n).astype(np.float32)
    y = rng.uniform(-4, H + 4, n).astype(np.float32)
    d = rng.uniform(1.0, 6.0, n).astype(np.float32)
    z = rng.uniform(-1, 1, n).astype(np.float32)
    I0 = rng.uniform(0.8, 1.0, n).astype(np.float32)
    iso = ra32.render_fixed(x, y, z, d, I0, H, W, 0.5)
    A = ra32.peaks(I0, z, "gauss", 0.5)
    acc = np.zeros(H * W, dtype=np.uint32)
    ra32.load().ra_render_model_fixed(H, W, n, x, y, A, d, d, np.zeros(n, np.float32), acc)
    assert np.array_equal(iso, acc.reshape(H, W))


def test_mirror_model_matches_float64():
    rng = np.random.default_rng(8)
    H, W, n = 56, 60, 80
    x = rng.uniform(0, W, n).astype(np.float32)
    y = rng.uniform(0, H, n).astype(np.float32)
    d = rng.uniform(1.5, 6.0, n).astype(np.float32)
    dyd = rng.uniform(1.5, 6.0, n).astype(np.float32)
    rho = rng.uniform(-0.95, 0.95, n).astype(np.float32)
    rho[:10] = 0.0
    z = rng.uniform(-1, 1, n).astype(np.float32)
    I0 = rng.uniform(0.8, 1.0, n).astype(np.float32)
    for law in ("gauss", "remark1"):
        A32 = ra32.peaks(I0, z, law, 0.5, 0.8, 2.5)
        A64 = om.peaks(I0, z, law, 0.5, 0.8, 2.5)
        assert np.max(np.abs(A32 - A64)) <= 2e-6
        got = ra32.render_model(x, y, A32, d, dyd, rho, H, W)
        ref = om.render_frame(x, y, A64, d, dyd, rho, H, W)
        assert np.max(np.abs(got - ref)) <= 1e-5 * ref.max()


def test_mirror_frame_params_match_float64():
    n = 20000
    rng = np.random.default_rng(9)
    d = rng.uniform(2.0, 5.0, n).astype(np.float32)
    dyd = rng.uniform(2.0, 5.0, n).astype(np.float32)
    rho = rng.uniform(-0.5, 0.5, n).astype(np.float32)
    I0 = rng.uniform(0.8, 1.0, n).astype(np.float32)
    a1, a2 = ra32.frame_params(d, dyd, rho, I0, 5, 6, (0.2, 0.1, 0.05), 0.3, 6.0)
    b1, b2 = om.frame_params(d, dyd, rho, I0, 5, 6, (0.2, 0.1, 0.05), 0.3, 6.0)
    assert np.array_equal(a1[3] == 0, b1[3] == 0) and np.array_equal(a2[3] == 0, b2[3] == 0)
    for a, b in zip(a2, b2):
        assert np.max(np.abs(a.astype(np.float64) - b)) <= 1e-5


def test_mirror_out_of_plane_motion_matches_float64():
    H, W, Gh, Gw = 96, 128, 24, 32
    rng = np.random.default_rng(10)
    flow = rng.normal(0, 2.0, (Gh, Gw, 2)).astype(np.float32)
    wg = rng.normal(0, 0.1, (Gh, Gw)).astype(np.float32)
    n = 2000
    x = rng.uniform(0, W, n).astype(np.float32)
    y = rng.uniform(0, H, n).astype(np.float32)
    z = rng.uniform(-1, 1, n).astype(np.float32)
    for integ, ns in (("euler", 1), ("rk4", 4)):
        got = ra32.advect_z(flow, wg, H, W, x, y, z, 1.0, ns, integ)
        _, _, ref = om.advect3(flow, wg, H, W, x, y, z, 1.0, ns, integ)
        assert np.max(np.abs(got - ref)) <= 1e-5
