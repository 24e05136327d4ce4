"""Gradients of an image loss with respect to the generator's inputs (oracle).

The paper motivates generating images inside closed loops such as
acquisition/parameter co-design (Abstract).  This module differentiates the
float64 forward (seed positions -> flow mapping -> render -> blur) analytically:

* render (Eq. 1 with rho = 0, sigma = d/4, peak A = I0 exp(-z^2 / (2 s^2))):
  with t = A exp(-8 (dx^2 + dy^2) / d^2) and dx = (c + 1/2) - x,
  dt/dx = t 16 dx / d^2, dt/dy = t 16 dy / d^2, dt/dd = t 16 (dx^2 + dy^2) / d^3,
  dt/dA = t / A, dA/dI0 = A / I0, dA/dz = -A z / s^2, dA/ds = A z^2 / s^3;
* blur: its transpose is the zero-padded correlation with mirrored taps;
* flow mapping: reverse sweep through each Euler / RK4 substep, with the
  bilinear sample's Jacobian in position (zero along clamped axes) and its
  weights as the derivative with respect to the four grid nodes.

``forward_pair`` and ``loss_fd`` give the float64 forward used for central
finite differences.
"""

from __future__ import annotations

import numpy as np

from . import advect as adv
from . import epilogue as ep
from . import render as rd


# ----------------------------------------------------------------------------- forward

def forward_pair(x1, y1, z, d, I0, s, flow, H, W, dt=1.0, substeps=1, integrator="euler",
                 w_blur=None, cutoff=False):
    x2, y2 = adv.advect(flow, H, W, x1, y1, dt, substeps, integrator)
    out = []
    for (xf, yf) in ((x1, y1), (x2, y2)):
        img = rd.render_frame(xf, yf, z, d, I0, H, W, s, cutoff=cutoff)
        if w_blur is not None and len(w_blur) > 1:
            img = ep.blur(img, w_blur)
        out.append(img)
    return np.stack(out)


# ----------------------------------------------------------------------------- render adjoint

def _particle_sums(x, y, d, A, e, cutoff):
    """Per particle: S0 = sum e G, Sx = sum e G dx, Sy = sum e G dy,
    Sr = sum e G (dx^2 + dy^2) over its (cut-off) support, G unscaled.

    With the cutoff, G vanishes outside the particle's square patch of half
    side 1.5 d (Section 2, "Efficient rasterization"), so only the image
    window around the patch is visited."""
    H, W = e.shape
    n = len(x)
    S = np.zeros((4, n))
    for i in range(n):
        if not (A[i] != 0 and d[i] > 0):
            continue
        c_lo, c_hi, r_lo, r_hi = 0, W, 0, H
        if cutoff:
            R = 1.5 * d[i]
            c_lo = max(int(np.floor(x[i] - R - 0.5)), 0)
            c_hi = min(int(np.ceil(x[i] + R - 0.5)) + 1, W)
            r_lo = max(int(np.floor(y[i] - R - 0.5)), 0)
            r_hi = min(int(np.ceil(y[i] + R - 0.5)) + 1, H)
            if c_lo >= c_hi or r_lo >= r_hi:
                continue
        dx = np.arange(c_lo, c_hi, dtype=np.float64) + 0.5 - x[i]
        dy = np.arange(r_lo, r_hi, dtype=np.float64) + 0.5 - y[i]
        kap = 8.0 / (d[i] * d[i])
        gx = np.exp(-kap * dx * dx)
        gy = np.exp(-kap * dy * dy)
        if cutoff:
            gx = gx * (np.abs(dx) <= R)
            gy = gy * (np.abs(dy) <= R)
        G = np.outer(gy, gx)
        eG = e[r_lo:r_hi, c_lo:c_hi] * G
        S[0, i] = eG.sum()
        S[1, i] = (eG * dx[None, :]).sum()
        S[2, i] = (eG * dy[:, None]).sum()
        S[3, i] = (eG * (dx[None, :] ** 2 + dy[:, None] ** 2)).sum()
    return S


# ----------------------------------------------------------------------------- advect adjoint

def _sample_with_jac(flow, H, W, px, py):
    Gh, Gw = flow.shape[0], flow.shape[1]
    F = np.asarray(flow, dtype=np.float64)
    sx, sy = Gw / W, Gh / H
    gx_raw = px * sx - 0.5
    gy_raw = py * sy - 0.5
    gx = np.clip(gx_raw, 0.0, Gw - 1.0)
    gy = np.clip(gy_raw, 0.0, Gh - 1.0)
    inx = (gx_raw > 0.0) & (gx_raw < Gw - 1.0)
    iny = (gy_raw > 0.0) & (gy_raw < Gh - 1.0)
    j0 = np.minimum(np.floor(gx).astype(np.int64), Gw - 2)
    i0 = np.minimum(np.floor(gy).astype(np.int64), Gh - 2)
    fx = gx - j0
    fy = gy - i0
    a = F[i0, j0]
    b = F[i0, j0 + 1]
    c = F[i0 + 1, j0]
    dd = F[i0 + 1, j0 + 1]
    fx_ = fx[..., None]
    fy_ = fy[..., None]
    val = (1 - fy_) * ((1 - fx_) * a + fx_ * b) + fy_ * ((1 - fx_) * c + fx_ * dd)
    dval_dx = ((1 - fy_) * (b - a) + fy_ * (dd - c)) * (sx * inx)[..., None]
    dval_dy = ((1 - fx_) * (c - a) + fx_ * (dd - b)) * (sy * iny)[..., None]
    wts = np.stack([(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy], axis=-1)
    return val, dval_dx, dval_dy, (i0, j0, wts)


def _scatter_flow(gF, nodes, gu, gv):
    i0, j0, wts = nodes
    for k, (di, dj) in enumerate(((0, 0), (0, 1), (1, 0), (1, 1))):
        np.add.at(gF[..., 0], (i0 + di, j0 + dj), wts[:, k] * gu)
        np.add.at(gF[..., 1], (i0 + di, j0 + dj), wts[:, k] * gv)


def advect_adjoint(flow, H, W, x1, y1, gx2, gy2, dt=1.0, substeps=1, integrator="euler"):
    """Given dL/d(x2, y2), return dL/d(x1, y1) and dL/dflow by a reverse sweep
    through the recomputed substeps."""
    h = float(dt) / int(substeps)
    px = np.array(x1, dtype=np.float64)
    py = np.array(y1, dtype=np.float64)
    traj = []
    for _ in range(int(substeps)):
        traj.append((px.copy(), py.copy()))
        if integrator == "euler":
            u, _, _, _ = _sample_with_jac(flow, H, W, px, py)
            px, py = px + h * u[:, 0], py + h * u[:, 1]
        else:
            k1, _, _, _ = _sample_with_jac(flow, H, W, px, py)
            k2, _, _, _ = _sample_with_jac(flow, H, W, px + 0.5 * h * k1[:, 0], py + 0.5 * h * k1[:, 1])
            k3, _, _, _ = _sample_with_jac(flow, H, W, px + 0.5 * h * k2[:, 0], py + 0.5 * h * k2[:, 1])
            k4, _, _, _ = _sample_with_jac(flow, H, W, px + h * k3[:, 0], py + h * k3[:, 1])
            px = px + h * (k1[:, 0] + 2 * k2[:, 0] + 2 * k3[:, 0] + k4[:, 0]) / 6.0
            py = py + h * (k1[:, 1] + 2 * k2[:, 1] + 2 * k3[:, 1] + k4[:, 1]) / 6.0
    gF = np.zeros(np.asarray(flow).shape, dtype=np.float64)
    gpx = np.array(gx2, dtype=np.float64)
    gpy = np.array(gy2, dtype=np.float64)

    def stage_back(sx, sy, kbar_u, kbar_v):
        """Backprop a velocity sample U(sx, sy) with upstream (kbar_u, kbar_v):
        returns the gradient w.r.t. the sample position, scatters into gF."""
        _, jx, jy, nodes = _sample_with_jac(flow, H, W, sx, sy)
        _scatter_flow(gF, nodes, kbar_u, kbar_v)
        return (jx[:, 0] * kbar_u + jx[:, 1] * kbar_v, jy[:, 0] * kbar_u + jy[:, 1] * kbar_v)

    for (px, py) in reversed(traj):
        if integrator == "euler":
            bx, by = stage_back(px, py, h * gpx, h * gpy)
            gpx, gpy = gpx + bx, gpy + by
            continue
        k1, _, _, _ = _sample_with_jac(flow, H, W, px, py)
        p2 = (px + 0.5 * h * k1[:, 0], py + 0.5 * h * k1[:, 1])
        k2, _, _, _ = _sample_with_jac(flow, H, W, *p2)
        p3 = (px + 0.5 * h * k2[:, 0], py + 0.5 * h * k2[:, 1])
        k3, _, _, _ = _sample_with_jac(flow, H, W, *p3)
        p4 = (px + h * k3[:, 0], py + h * k3[:, 1])
        c = h / 6.0
        b4x, b4y = stage_back(*p4, c * gpx, c * gpy)               # k4 bar = c g
        k3u, k3v = 2 * c * gpx + h * b4x, 2 * c * gpy + h * b4y
        b3x, b3y = stage_back(*p3, k3u, k3v)
        k2u, k2v = 2 * c * gpx + 0.5 * h * b3x, 2 * c * gpy + 0.5 * h * b3y
        b2x, b2y = stage_back(*p2, k2u, k2v)
        k1u, k1v = c * gpx + 0.5 * h * b2x, c * gpy + 0.5 * h * b2y
        b1x, b1y = stage_back(px, py, k1u, k1v)
        gpx = gpx + b4x + b3x + b2x + b1x
        gpy = gpy + b4y + b3y + b2y + b1y
    return gpx, gpy, gF


# ----------------------------------------------------------------------------- full backward

def backward_pair(x1, y1, z, d, I0, s, flow, H, W, gJ, dt=1.0, substeps=1,
                  integrator="euler", w_blur=None, cutoff=False, frame2=None):
    """dL/d{x1, y1, z, d, I0, s, flow} given dL/dJ [2, H, W] for one pair.

    ``frame2`` optionally gives the frame-2 positions (x2, y2) the render adjoint
    is evaluated at (default: this module's float64 advection of (x1, y1)); the
    flow adjoint always follows the float64 trajectory.  It lets a comparison
    with a binary32 implementation separate position rounding from the
    gradient arithmetic."""
    x1 = np.asarray(x1, dtype=np.float64)
    y1 = np.asarray(y1, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    I0 = np.asarray(I0, dtype=np.float64)
    x2, y2 = adv.advect(flow, H, W, x1, y1, dt, substeps, integrator)
    if frame2 is not None:
        x2 = np.asarray(frame2[0], dtype=np.float64)
        y2 = np.asarray(frame2[1], dtype=np.float64)
    Sz = rd.sheet_factor(z, s)
    A = I0 * Sz
    g = {k: np.zeros_like(x1) for k in ("x1", "y1", "z", "d", "I0")}
    g_x2 = np.zeros_like(x1)
    g_y2 = np.zeros_like(x1)
    gA = np.zeros_like(x1)
    for f, (xf, yf) in enumerate(((x1, y1), (x2, y2))):
        e = np.asarray(gJ[f], dtype=np.float64)
        if w_blur is not None and len(w_blur) > 1:
            e = ep.blur_adjoint(e, w_blur)
        S0, Sx, Sy, Sr = _particle_sums(xf, yf, d, A, e, cutoff)
        live = (I0 > 0) & (d > 0)
        dd = np.where(d > 0, d, 1.0)
        gxf = np.where(live, A * 16.0 * Sx / dd ** 2, 0.0)
        gyf = np.where(live, A * 16.0 * Sy / dd ** 2, 0.0)
        g["d"] += np.where(live, A * 16.0 * Sr / dd ** 3, 0.0)
        gA += np.where(live, S0, 0.0)
        if f == 0:
            g["x1"] += gxf
            g["y1"] += gyf
        else:
            g_x2 += gxf
            g_y2 += gyf
    g["I0"] = gA * Sz
    g["z"] = gA * A * (-z / s ** 2)
    g_s = float(np.sum(gA * A * z * z / s ** 3))
    bx, by, gF = advect_adjoint(flow, H, W, x1, y1, g_x2, g_y2, dt, substeps, integrator)
    g["x1"] += bx
    g["y1"] += by
    g["s"] = g_s
    g["flow"] = gF
    return g
