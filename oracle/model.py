"""The full per-particle model, float64 definition (oracle, test infrastructure).

Extends the isotropic path (``seed``, ``render``) to everything the paper's
particle model allows:

* Eq. 1 with its own parameters: sigma_x, sigma_y and the correlation rho.
  As for the isotropic path the widths are read from e^-2 particle-image
  diameters, sigma_x = d / 4 and sigma_y = d_y / 4; rho is drawn uniformly
  from a configured interval (the sentence after Eq. 1 draws every parameter
  uniformly per particle) and read as |rho| < 1 (the text says rho > 0, which
  would exclude the axis-aligned case it generalises).
* Frame-2 parameter variation (the sentence after Eq. 1): every parameter of
  a frame-2 particle is its frame-1 value plus a zero-mean Gaussian of a
  configured standard deviation, clipped to the parameter's valid range.
* Hiding (Section 2, "Considerations on the aggregation"): in each frame a
  particle is hidden, i.e. its intensity is zero, with a configured
  probability, independently per frame.
* The out-of-focus law of Remark 1: the peak is
  I0(z) = q exp(-(1/sqrt(2 pi)) |2 Z^2 / DZ0^2|^s), with the particle's drawn
  intensity as its scattering efficiency q, the sheet thickness DZ0 and the
  shape factor s; and a three-dimensional flow: the out-of-plane velocity w
  moves z between the exposures (Remark 1 pairs the law with 3-D particles
  and flow; the Conclusions list it as the next extension).

Draw layout (Philox4x32-10 as in ``philox``): stream 6 (SHAPE) at the
particle index gives d_y (word 0 uniform; words 1, 2 Box-Muller for a normal
distribution) and rho (word 3); stream 2 (JITTER) gives four normals (words
0, 1 and 2, 3 as Box-Muller pairs: cosine then sine) for d, d_y, rho and I0 of
frame 2; stream 7 (HIDE) gives the hiding uniforms of frame 1 (word 0) and
frame 2 (word 1).
"""

from __future__ import annotations

import math

import numpy as np

from . import philox as ph
from . import seed as sd

STREAM_JITTER = 2
STREAM_SHAPE = 6
STREAM_HIDE = 7
RHO_MAX = 0.99          # |rho| bound of the drawn and the varied correlation


# ---------------------------------------------------------------- seeding

def seed_shape(n_max: int, pair_id: int, seed: int, d_dist: str = "uniform", d_params=(1.0, 5.0),
               rho=(0.0, 0.0)):
    """Second diameter d_y (same distribution as d) and correlation rho of each
    candidate particle (stream 6)."""
    i = np.arange(int(n_max), dtype=np.uint64)
    w = ph.draw(i, STREAM_SHAPE, pair_id, seed)
    if d_dist == "uniform":
        dy = d_params[0] + (d_params[1] - d_params[0]) * ph.uniform24(w[0])
    elif d_dist == "normal":
        mu, sigma, lo, hi = d_params
        dy = np.clip(mu + sigma * sd.box_muller_cos(w[1], w[2]), lo, hi)
    else:
        raise ValueError(d_dist)
    r = rho[0] + (rho[1] - rho[0]) * ph.uniform24(w[3])
    return dy, r


def jitter_normals(n: int, pair_id: int, seed: int):
    """Four standard normals per particle (stream 2): rows n0..n3."""
    i = np.arange(int(n), dtype=np.uint64)
    w = ph.draw(i, STREAM_JITTER, pair_id, seed)
    out = []
    for (wa, wb) in ((w[0], w[1]), (w[2], w[3])):
        R = np.sqrt(-2.0 * np.log(ph.uniform24_open0(wa)))
        th = 2.0 * np.pi * ph.uniform24(wb)
        out += [R * np.cos(th), R * np.sin(th)]
    return np.stack(out)


def hidden(n: int, pair_id: int, seed: int, p: float):
    """Boolean [2, n]: particle hidden in frame 1 / frame 2 (stream 7)."""
    i = np.arange(int(n), dtype=np.uint64)
    w = ph.draw(i, STREAM_HIDE, pair_id, seed)
    return np.stack([ph.uniform24(w[0]) < p, ph.uniform24(w[1]) < p])


def frame_params(d, dy, rho, I0, pair_id: int, seed: int, jitter=(0.0, 0.0, 0.0), hide_p: float = 0.0,
                 d_max: float = 16.0):
    """Per-frame particle parameters (d, d_y, rho, I0) of frame 1 and frame 2.

    Frame 2 varies each parameter by a zero-mean Gaussian: diameters by
    jitter[0] (clipped to [0, d_max]; a zero diameter renders nothing), rho by
    jitter[1] (clipped to [-RHO_MAX, RHO_MAX]), the intensity by jitter[2]
    (clipped at 0).  Masked particles (I0 = 0) stay dark.  A zero standard
    deviation leaves the parameter unchanged.  Hidden particles get I0 = 0 in
    that frame."""
    d = np.asarray(d, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    I0 = np.asarray(I0, dtype=np.float64)
    n = d.size
    f2 = [d.copy(), dy.copy(), rho.copy(), I0.copy()]
    if any(j > 0 for j in jitter):
        nrm = jitter_normals(n, pair_id, seed)
        if jitter[0] > 0:
            f2[0] = np.clip(d + jitter[0] * nrm[0], 0.0, d_max)
            f2[1] = np.clip(dy + jitter[0] * nrm[1], 0.0, d_max)
        if jitter[1] > 0:
            f2[2] = np.clip(rho + jitter[1] * nrm[2], -RHO_MAX, RHO_MAX)
        if jitter[2] > 0:
            f2[3] = np.where(I0 > 0, np.maximum(I0 + jitter[2] * nrm[3], 0.0), 0.0)
    f1 = [d.copy(), dy.copy(), rho.copy(), I0.copy()]
    if hide_p > 0:
        hid = hidden(n, pair_id, seed, hide_p)
        f1[3] = np.where(hid[0], 0.0, f1[3])
        f2[3] = np.where(hid[1], 0.0, f2[3])
    return f1, f2


# ---------------------------------------------------------------- sheet laws

def sheet_gauss(z, s: float):
    z = np.asarray(z, dtype=np.float64)
    return np.exp(-(z * z) / (2.0 * float(s) ** 2))


def sheet_remark1(z, dz0: float, shape: float):
    """exp(-(1/sqrt(2 pi)) |2 z^2 / DZ0^2|^s) (Remark 1 with q = 1)."""
    z = np.asarray(z, dtype=np.float64)
    v = np.abs(2.0 * z * z / (float(dz0) ** 2))
    return np.exp(-(1.0 / math.sqrt(2.0 * math.pi)) * v ** float(shape))


# ---------------------------------------------------------------- 3-D motion

def sample_scalar(grid, H: int, W: int, px, py):
    """Bilinear, clamped sample of a cell-centred scalar grid [Gh, Gw] (the
    registration of the (u, v) grid)."""
    Gh, Gw = grid.shape
    G = np.asarray(grid, dtype=np.float64)
    gx = np.clip(np.asarray(px, dtype=np.float64) * (Gw / W) - 0.5, 0.0, Gw - 1.0)
    gy = np.clip(np.asarray(py, dtype=np.float64) * (Gh / H) - 0.5, 0.0, Gh - 1.0)
    j0 = np.minimum(np.floor(gx).astype(np.int64), Gw - 2)
    i0 = np.minimum(np.floor(gy).astype(np.int64), Gh - 2)
    fx = gx - j0
    fy = gy - i0
    return ((1 - fy) * ((1 - fx) * G[i0, j0] + fx * G[i0, j0 + 1])
            + fy * ((1 - fx) * G[i0 + 1, j0] + fx * G[i0 + 1, j0 + 1]))


def advect3(flow, wgrid, H: int, W: int, x, y, z, dt: float = 1.0, substeps: int = 1, integrator: str = "euler"):
    """(x2, y2, z2) under the frozen 3-D field (u, v)(x, y), w(x, y): the
    in-plane motion is that of ``advect.advect``; z integrates w along the
    in-plane trajectory with the same stages."""
    from . import advect as adv
    px = np.array(x, dtype=np.float64)
    py = np.array(y, dtype=np.float64)
    pz = np.array(z, dtype=np.float64)
    h = float(dt) / int(substeps)
    for _ in range(int(substeps)):
        if integrator == "euler":
            u, v = adv.sample(flow, H, W, px, py)
            wz = sample_scalar(wgrid, H, W, px, py)
            px, py, pz = px + h * u, py + h * v, pz + h * wz
        elif integrator == "rk4":
            k1u, k1v = adv.sample(flow, H, W, px, py)
            k1w = sample_scalar(wgrid, H, W, px, py)
            q2x, q2y = px + 0.5 * h * k1u, py + 0.5 * h * k1v
            k2u, k2v = adv.sample(flow, H, W, q2x, q2y)
            k2w = sample_scalar(wgrid, H, W, q2x, q2y)
            q3x, q3y = px + 0.5 * h * k2u, py + 0.5 * h * k2v
            k3u, k3v = adv.sample(flow, H, W, q3x, q3y)
            k3w = sample_scalar(wgrid, H, W, q3x, q3y)
            q4x, q4y = px + h * k3u, py + h * k3v
            k4u, k4v = adv.sample(flow, H, W, q4x, q4y)
            k4w = sample_scalar(wgrid, H, W, q4x, q4y)
            px = px + h * (k1u + 2 * k2u + 2 * k3u + k4u) / 6.0
            py = py + h * (k1v + 2 * k2v + 2 * k3v + k4v) / 6.0
            pz = pz + h * (k1w + 2 * k2w + 2 * k3w + k4w) / 6.0
        else:
            raise ValueError(integrator)
    return px, py, pz


# ---------------------------------------------------------------- rendering

def footprint(dx, dy, d, dyd, rho):
    """Eq. 1 without its peak: exp(-(dx^2/sx^2 - 2 rho dx dy/(sx sy) + dy^2/sy^2) / (2 (1 - rho^2))),
    sx = d / 4, sy = d_y / 4."""
    sx = np.asarray(d, dtype=np.float64) / 4.0
    sy = np.asarray(dyd, dtype=np.float64) / 4.0
    r = np.asarray(rho, dtype=np.float64)
    q = (dx * dx) / (sx * sx) - 2.0 * r * dx * dy / (sx * sy) + (dy * dy) / (sy * sy)
    return np.exp(-q / (2.0 * (1.0 - r * r)))


def render_frame(x, y, A, d, dyd, rho, H: int, W: int, cutoff: bool = True):
    """float64 exposure [H, W]: sum over particles of A * Eq. 1 at pixel
    centres, each on its patch |dx| <= 1.5 d, |dy| <= 1.5 d_y (the bounding
    box of the ellipse where the exponent reaches 18, for any rho: its
    half-widths are sqrt(18 / 8) d and sqrt(18 / 8) d_y).  Particles with
    A <= 0, a non-positive diameter or a non-finite position add nothing."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    dyd = np.asarray(dyd, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    img = np.zeros((H, W))
    ok = (A > 0) & (d > 0) & (dyd > 0) & np.isfinite(x) & np.isfinite(y)
    cx = np.arange(W) + 0.5
    cy = np.arange(H) + 0.5
    for i in np.nonzero(ok)[0]:
        if cutoff:
            c0 = max(int(math.floor(x[i] - 1.5 * d[i] - 0.5)), 0)
            c1 = min(int(math.ceil(x[i] + 1.5 * d[i] + 0.5)), W - 1)
            r0 = max(int(math.floor(y[i] - 1.5 * dyd[i] - 0.5)), 0)
            r1 = min(int(math.ceil(y[i] + 1.5 * dyd[i] + 0.5)), H - 1)
            if c0 > c1 or r0 > r1:
                continue
        else:
            c0, c1, r0, r1 = 0, W - 1, 0, H - 1
        DX = (cx[c0:c1 + 1] - x[i])[None, :]
        DY = (cy[r0:r1 + 1] - y[i])[:, None]
        g = A[i] * footprint(DX, DY, d[i], dyd[i], rho[i])
        if cutoff:
            g = g * ((np.abs(DX) <= 1.5 * d[i]) & (np.abs(DY) <= 1.5 * dyd[i]))
        img[r0:r1 + 1, c0:c1 + 1] += g
    return img


def peaks(I0, z, law: str = "gauss", sheet_sigma: float = 0.5, dz0: float = 1.0, shape: float = 1.0):
    I0 = np.asarray(I0, dtype=np.float64)
    if law == "gauss":
        return I0 * sheet_gauss(z, sheet_sigma)
    if law == "remark1":
        return I0 * sheet_remark1(z, dz0, shape)
    raise ValueError(law)


def generate_pair(m, H: int, W: int, pair_id: int, seed: int, flow, wgrid=None, cutoff: bool = True):
    """One pair under the full model, float64: exposures I [2, H, W] (no blur,
    noise or codes: those are the isotropic path's ``epilogue``).  ``m`` is a
    dict of the model parameters: ppp, d_dist, d_params, I0, z, rho,
    anisotropic, jitter, hide_p, d_max, law, sheet_sigma, dz0, shape, dt,
    substeps, integrator."""
    from . import advect as adv
    P = sd.seed_pair(H, W, pair_id, seed, ppp=m["ppp"], d_dist=m["d_dist"], d_params=m["d_params"],
                     I0=m["I0"], z=m["z"])
    n = P["n_max"]
    if m.get("anisotropic"):
        dy, rho = seed_shape(n, pair_id, seed, m["d_dist"], m["d_params"], m["rho"])
    else:
        dy, rho = P["d"].copy(), np.zeros(n)
    if wgrid is not None:
        x2, y2, z2 = advect3(flow, wgrid, H, W, P["x"], P["y"], P["z"], m["dt"], m["substeps"], m["integrator"])
    else:
        x2, y2 = adv.advect(flow, H, W, P["x"], P["y"], m["dt"], m["substeps"], m["integrator"])
        z2 = P["z"].copy()
    f1, f2 = frame_params(P["d"], dy, rho, P["I0"], pair_id, seed, m.get("jitter", (0.0, 0.0, 0.0)),
                          m.get("hide_p", 0.0), m.get("d_max", 16.0))
    law = m.get("law", "gauss")
    out = []
    for (xf, yf, zf, f) in ((P["x"], P["y"], P["z"], f1), (x2, y2, z2, f2)):
        A = peaks(f[3], zf, law, m.get("sheet_sigma", 0.5), m.get("dz0", 1.0), m.get("shape", 1.0))
        out.append(render_frame(xf, yf, A, f[0], f[1], f[2], H, W, cutoff))
    return {"particles": P, "dy": dy, "rho": rho, "x2": x2, "y2": y2, "z2": z2, "frame1": f1, "frame2": f2,
            "I": np.stack(out)}
