"""Pins of the oracle's flow mapping (Section 2, "Sampling the particles":
frame-2 particles are frame-1 particles moved by the flow)."""

import numpy as np
import pytest

from oracle import advect as adv
from workloads import flows, particles


def _linear_grid(H, W, Gh, Gw, fu, fv):
    xs = (np.arange(Gw) + 0.5) * W / Gw
    ys = (np.arange(Gh) + 0.5) * H / Gh
    X, Y = np.meshgrid(xs, ys)
    return np.stack([fu(X, Y), fv(X, Y)], axis=-1)


@pytest.mark.parametrize("integrator,n", [("euler", 1), ("euler", 3), ("rk4", 1), ("rk4", 4)])
def test_zero_flow_is_identity(ra, integrator, n):
    P = particles.random_particles(1, 500, 64, 80)
    F = flows.uniform_grid(16, 20, 0.0, 0.0)
    x2, y2 = adv.advect(F, 64, 80, P["x"], P["y"], 1.0, n, integrator)
    assert np.array_equal(x2, P["x"].astype(np.float64)) and np.array_equal(y2, P["y"].astype(np.float64))
    r2 = ra.advect(F, 64, 80, P["x"], P["y"], 1.0, n, integrator)
    assert np.array_equal(r2[0], P["x"]) and np.array_equal(r2[1], P["y"])


@pytest.mark.parametrize("integrator,n", [("euler", 1), ("rk4", 1), ("rk4", 4), ("rk4", 8)])
def test_uniform_flow_is_exact_shift(ra, integrator, n):
    H, W = 256, 256
    F = flows.uniform_grid(64, 64, 2.5, -1.25)
    P = particles.random_particles(2, 2000, H, W)
    x2, y2 = adv.advect(F, H, W, P["x"], P["y"], 1.0, n, integrator)
    x64, y64 = P["x"].astype(np.float64), P["y"].astype(np.float64)
    assert np.array_equal(x2, x64 + 2.5) and np.array_equal(y2, y64 - 1.25)
    # binary32: each substep adds the exact step h*u with one rounding
    rx, ry = ra.advect(F, H, W, P["x"], P["y"], 1.0, n, integrator)
    ex, ey = P["x"].copy(), P["y"].copy()
    for _ in range(n):
        ex = ex + np.float32(2.5 / n)
        ey = ey + np.float32(-1.25 / n)
    assert np.array_equal(rx, ex) and np.array_equal(ry, ey)


def test_bilinear_reproduces_affine_field_inside_hull():
    H, W, Gh, Gw = 96, 128, 12, 16
    F = _linear_grid(H, W, Gh, Gw, lambda X, Y: 0.3 + 0.02 * X - 0.05 * Y, lambda X, Y: -1 + 0.01 * X * 1 + 0.03 * Y)
    rng = np.random.default_rng(0)
    x = rng.uniform(W / Gw / 2, W - W / Gw / 2, 1000)
    y = rng.uniform(H / Gh / 2, H - H / Gh / 2, 1000)
    u, v = adv.sample(F, H, W, x, y)
    assert np.allclose(u, 0.3 + 0.02 * x - 0.05 * y, atol=1e-12, rtol=0)
    assert np.allclose(v, -1 + 0.01 * x + 0.03 * y, atol=1e-12, rtol=0)


def test_clamp_to_edge_outside_hull():
    H, W, Gh, Gw = 64, 64, 8, 8
    rng = np.random.default_rng(1)
    F = rng.normal(size=(Gh, Gw, 2))
    u, v = adv.sample(F, H, W, np.array([-5.0, 100.0, 2.0, 62.5]), np.array([-5.0, -3.0, 70.0, 1.0]))
    assert u[0] == F[0, 0, 0] and v[0] == F[0, 0, 1]
    assert u[1] == F[0, Gw - 1, 0]
    assert u[2] == F[Gh - 1, 0, 0]
    assert u[3] == F[0, Gw - 1, 0]


def test_node_values_are_interpolated_exactly():
    H, W, Gh, Gw = 40, 60, 10, 15
    F = np.random.default_rng(2).normal(size=(Gh, Gw, 2))
    i, j = np.meshgrid(np.arange(Gh), np.arange(Gw), indexing="ij")
    u, v = adv.sample(F, H, W, (j + 0.5) * W / Gw, (i + 0.5) * H / Gh)
    assert np.allclose(u, F[..., 0], atol=1e-13) and np.allclose(v, F[..., 1], atol=1e-13)


@pytest.mark.parametrize("integrator,n", [("euler", 1), ("euler", 5), ("rk4", 1), ("rk4", 3)])
def test_rotation_matches_stability_polynomial(integrator, n):
    """u = -w (y - c), v = w (x - c) is linear, so bilinear sampling is exact in
    the hull and one substep multiplies (x - c) + i (y - c) by the method's
    stability polynomial R(i w h): 1 + z (Euler), 1 + z + z^2/2 + z^3/6 + z^4/24
    (classical RK4)."""
    H = W = 128
    G = 32
    c = 64.0
    w = 0.05
    F = _linear_grid(H, W, G, G, lambda X, Y: -w * (Y - c), lambda X, Y: w * (X - c))
    rng = np.random.default_rng(3)
    r = rng.uniform(5, 30, 200)
    th = rng.uniform(0, 2 * np.pi, 200)
    x = c + r * np.cos(th)
    y = c + r * np.sin(th)
    dt = 2.0
    x2, y2 = adv.advect(F, H, W, x, y, dt, n, integrator)
    z = 1j * w * dt / n
    Rz = 1 + z if integrator == "euler" else 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    ref = ((x - c) + 1j * (y - c)) * Rz ** n
    assert np.allclose(x2 - c, ref.real, atol=1e-10) and np.allclose(y2 - c, ref.imag, atol=1e-10)


def test_rk4_global_error_is_fourth_order():
    H = W = 128
    G = 32
    c = 64.0
    w = 0.2
    F = _linear_grid(H, W, G, G, lambda X, Y: -w * (Y - c), lambda X, Y: w * (X - c))
    x, y = np.array([c + 20.0]), np.array([c])
    errs = []
    for n in (2, 4, 8):
        x2, y2 = adv.advect(F, H, W, x, y, 3.0, n, "rk4")
        ex = c + 20 * np.cos(w * 3.0)
        ey = c + 20 * np.sin(w * 3.0)
        errs.append(np.hypot(x2[0] - ex, y2[0] - ey))
    assert 12 < errs[0] / errs[1] < 20 and 12 < errs[1] / errs[2] < 20


@pytest.mark.parametrize("integrator,n", [("euler", 1), ("rk4", 4)])
def test_binary32_mirror_tracks_float64(ra, integrator, n):
    H, W = 256, 384
    F = flows.lamb_oseen_grid(np.random.default_rng(5), H, W, 64, 96, max_disp=8.0)
    P = particles.random_particles(3, 5000, H, W, pad=10)
    x2, y2 = adv.advect(F, H, W, P["x"], P["y"], 1.0, n, integrator)
    rx, ry = ra.advect(F, H, W, P["x"], P["y"], 1.0, n, integrator)
    assert np.max(np.abs(rx - x2)) < 1e-4 and np.max(np.abs(ry - y2)) < 1e-4
    assert np.max(np.hypot(x2 - P["x"], y2 - P["y"])) > 1.0   # the flow actually moved them


def test_flow_field_pins():
    from oracle import ra32
    H, W, Gh, Gw = 48, 64, 12, 16
    # uniform grid: every pixel carries the grid's value exactly
    flow = np.zeros((Gh, Gw, 2))
    flow[..., 0], flow[..., 1] = 2.5, -1.25
    f = adv.flow_field(flow, H, W)
    assert np.all(f[..., 0] == 2.5) and np.all(f[..., 1] == -1.25)
    assert np.array_equal(ra32.flow_field(flow, H, W), f.astype(np.float32))
    # affine field: reproduced exactly inside the node hull; pixel centres that
    # coincide with nodes carry the node values
    jx = (np.arange(Gw) + 0.5) * W / Gw
    iy = (np.arange(Gh) + 0.5) * H / Gh
    flow[..., 0] = 0.03 * jx[None, :] - 0.02 * iy[:, None] + 0.5
    flow[..., 1] = -0.01 * jx[None, :] + 0.04 * iy[:, None]
    f = adv.flow_field(flow, H, W)
    px, py = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    inside = (px >= jx[0]) & (px <= jx[-1]) & (py >= iy[0]) & (py <= iy[-1])
    assert np.max(np.abs(f[..., 0] - (0.03 * px - 0.02 * py + 0.5))[inside]) < 1e-12
    assert np.max(np.abs(f[..., 1] - (-0.01 * px + 0.04 * py))[inside]) < 1e-12
    # the binary32 mirror within rounding of the definition
    rng = np.random.default_rng(0)
    flow = rng.normal(0, 3, (Gh, Gw, 2))
    assert np.max(np.abs(ra32.flow_field(flow, H, W) - adv.flow_field(flow.astype(np.float32), H, W))) < 1e-5
