"""Pins of the oracle's analytic gradients: float64 central finite differences
(h = 1e-4) on 16x16 cases, a single-particle closed form, and adjoint
dot-product tests of the bilinear scatter."""

import math

import numpy as np
import pytest

from oracle import advect as adv
from oracle import epilogue as ep
from oracle import grad as gr
from oracle import render as rd

H = W = 16
G = 4


def _stage_points(flow, x, y, dt, n, integ):
    """All positions at which the field is sampled (to keep FD cases away from
    bilinear cell lines and clamp edges)."""
    pts = []
    h = dt / n
    px, py = np.array(x, float), np.array(y, float)
    for _ in range(n):
        if integ == "euler":
            pts.append((px.copy(), py.copy()))
            u, v = adv.sample(flow, H, W, px, py)
            px, py = px + h * u, py + h * v
        else:
            k1 = adv.sample(flow, H, W, px, py)
            p2 = (px + 0.5 * h * k1[0], py + 0.5 * h * k1[1])
            k2 = adv.sample(flow, H, W, *p2)
            p3 = (px + 0.5 * h * k2[0], py + 0.5 * h * k2[1])
            k3 = adv.sample(flow, H, W, *p3)
            p4 = (px + h * k3[0], py + h * k3[1])
            k4 = adv.sample(flow, H, W, *p4)
            pts += [(px.copy(), py.copy()), p2, p3, p4]
            px = px + h * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0]) / 6
            py = py + h * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1]) / 6
    return pts


def _case(seed, integ, n_sub):
    rng = np.random.default_rng(seed)
    flow = rng.normal(scale=0.6, size=(G, G, 2))
    for _ in range(200):
        n = 5
        x = rng.uniform(3.0, 13.0, n)
        y = rng.uniform(3.0, 13.0, n)
        ok = True
        for (px, py) in _stage_points(flow, x, y, 1.0, n_sub, integ):
            for q in (px, py):
                g = q * (G / W) - 0.5
                if np.any(np.abs(g - np.round(g)) < 0.02) or np.any(g < 0.05) or np.any(g > G - 1.05):
                    ok = False
        if ok:
            break
    assert ok
    z = rng.uniform(-0.9, 0.9, n)
    d = rng.uniform(1.5, 4.0, n)
    I0 = rng.uniform(0.8, 1.0, n)
    s = 0.55
    T = rng.uniform(0, 0.5, size=(2, H, W))
    return x, y, z, d, I0, s, flow, T


def _loss(J, T):
    return float(np.mean((J - T) ** 2))


@pytest.mark.parametrize("integ,n_sub,blur", [("euler", 1, False), ("rk4", 2, True), ("rk4", 4, True)])
def test_gradients_match_central_differences(integ, n_sub, blur):
    x, y, z, d, I0, s, flow, T = _case(17 + n_sub, integ, n_sub)
    w = ep.blur_weights(1, 0.7) if blur else None
    kw = dict(dt=1.0, substeps=n_sub, integrator=integ, w_blur=w, cutoff=False)

    def L(x=x, y=y, z=z, d=d, I0=I0, s=s, flow=flow):
        return _loss(gr.forward_pair(x, y, z, d, I0, s, flow, H, W, **kw), T)

    J = gr.forward_pair(x, y, z, d, I0, s, flow, H, W, **kw)
    gJ = 2 * (J - T) / J.size
    g = gr.backward_pair(x, y, z, d, I0, s, flow, H, W, gJ, **kw)
    h = 1e-4

    def fd(name, arr, idx):
        a = arr.copy()
        a[idx] += h
        lp = L(**{name: a})
        a[idx] -= 2 * h
        lm = L(**{name: a})
        return (lp - lm) / (2 * h)

    for name, arr, key in (("x", x, "x1"), ("y", y, "y1"), ("z", z, "z"), ("d", d, "d"), ("I0", I0, "I0")):
        num = np.array([fd(name, arr, i) for i in range(len(arr))])
        scale = np.max(np.abs(num)) + 1e-30
        assert np.max(np.abs(num - g[key])) <= 1e-6 * scale, (key, num, g[key])
    num_s = (L(s=s + h) - L(s=s - h)) / (2 * h)
    assert abs(num_s - g["s"]) <= 1e-6 * abs(num_s)
    num_f = np.zeros_like(flow)
    for idx in np.ndindex(flow.shape):
        num_f[idx] = fd("flow", flow, idx)
    scale = np.max(np.abs(num_f))
    assert scale > 0
    assert np.max(np.abs(num_f - g["flow"])) <= 1e-6 * scale


def test_single_particle_intensity_gradient_is_patch_mass():
    """For dL/dI = 1 everywhere, dL/dI0 = S(z) * sum of the unit-peak patch, which
    for a particle far from the borders is the lattice mass (pi d^2 / 8 for d >= 4)."""
    d, z, s = 5.0, 0.4, 0.5
    x = np.array([32.3]); y = np.array([31.8])
    gJ = np.ones((2, 64, 64))
    flow = np.zeros((16, 16, 2))
    g = gr.backward_pair(x, y, np.array([z]), np.array([d]), np.array([1.0]), s, flow, 64, 64, gJ)
    S = math.exp(-z * z / (2 * s * s))
    assert g["I0"][0] == pytest.approx(2 * S * math.pi * d * d / 8, rel=1e-6)
    # translating the particle does not change its mass: position gradients vanish
    assert abs(g["x1"][0]) < 1e-6 and abs(g["y1"][0]) < 1e-6
    # mass ~ d^2 -> dL/dd = 2 * 2 A pi d / 8
    assert g["d"][0] == pytest.approx(2 * S * 2 * math.pi * d / 8, rel=1e-5)
    # dA/dz = -A z / s^2
    assert g["z"][0] == pytest.approx(-2 * S * math.pi * d * d / 8 * z / s ** 2, rel=1e-6)


def test_bilinear_scatter_is_adjoint_of_sampling():
    rng = np.random.default_rng(4)
    flow = rng.normal(size=(6, 7, 2))
    dF = rng.normal(size=flow.shape)
    px = rng.uniform(-3, 30, 50)
    py = rng.uniform(-3, 26, 50)
    gu = rng.normal(size=50)
    gv = rng.normal(size=50)
    u1, v1 = adv.sample(flow + dF, 24, 28, px, py)
    u0, v0 = adv.sample(flow, 24, 28, px, py)
    lhs = np.sum((u1 - u0) * gu + (v1 - v0) * gv)            # sampling is linear in the grid
    gF = np.zeros_like(flow)
    _, _, _, nodes = gr._sample_with_jac(flow, 24, 28, px, py)
    gr._scatter_flow(gF, nodes, gu, gv)
    assert abs(lhs - np.sum(gF * dF)) < 1e-12 * (1 + abs(lhs))


def test_masked_particles_get_zero_gradient():
    x = np.array([8.0, 8.3]); y = np.array([8.0, 7.7])
    g = gr.backward_pair(x, y, np.zeros(2), np.array([2.0, 2.0]), np.array([0.0, 1.0]), 0.5,
                         np.zeros((4, 4, 2)), 16, 16, np.ones((2, 16, 16)))
    assert g["x1"][0] == 0 and g["d"][0] == 0 and g["I0"][0] == 0 and g["I0"][1] > 0


@pytest.mark.parametrize("integ,n_sub", [("euler", 1), ("rk4", 4)])
def test_cutoff_gradient_matches_smooth_gradient(integ, n_sub):
    """The patch cutoff at |dx|, |dy| <= 1.5 d drops terms of at most exp(-18)
    of the peak, so the windowed (cut-off) gradient equals the full-support one
    to ~1e-7 of its scale; this also pins the windowed sums to the FD-checked
    full ones."""
    x, y, z, d, I0, s, flow, T = _case(5 + n_sub, integ, n_sub)
    kw = dict(dt=1.0, substeps=n_sub, integrator=integ, w_blur=ep.blur_weights(1, 0.7))
    J = gr.forward_pair(x, y, z, d, I0, s, flow, H, W, cutoff=False, **kw)
    gJ = 2 * (J - T) / J.size
    g_full = gr.backward_pair(x, y, z, d, I0, s, flow, H, W, gJ, cutoff=False, **kw)
    g_cut = gr.backward_pair(x, y, z, d, I0, s, flow, H, W, gJ, cutoff=True, **kw)
    for key in ("x1", "y1", "z", "d", "I0", "flow"):
        scale = np.max(np.abs(g_full[key]))
        assert scale > 0
        assert np.max(np.abs(g_cut[key] - g_full[key])) <= 1e-6 * scale, key
    assert abs(g_cut["s"] - g_full["s"]) <= 1e-6 * abs(g_full["s"])
