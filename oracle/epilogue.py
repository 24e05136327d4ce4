"""Acquisition effects applied to a rendered exposure (oracle).

The paper names blur, noise and the storage format as configurable
acquisition parameters without fixing their models (Abstract; Section 1 on
noise, blur and uint8 storage).  Readings used here:

* blur: a normalised separable Gaussian of radius b (taps -b..b, weights
  g_k / sum g with g_k = exp(-k^2 / (2 sigma_b^2))), zero padding outside the
  image, horizontal pass then vertical pass;
* noise: additive, independent per pixel and per frame, N(0, sigma^2) in
  full-scale units, drawn after the blur, by Box-Muller on Philox words of
  stream 3 (frame 1) or 4 (frame 2): counter index r * ceil(W / 4) + c // 4,
  words (w0, w1) give the cosine / sine normals of pixels c = 4k, 4k+1 and
  (w2, w3) those of 4k+2, 4k+3;
* storage: integer codes q = clamp(rint(v * (2^bits - 1)), 0, 2^bits - 1) with
  round-half-to-even, full scale 1.0.
"""

from __future__ import annotations

import numpy as np

from . import philox as ph


def blur_weights(radius: int, sigma: float) -> np.ndarray:
    """float32 taps w[0..2b] (computed in float64, rounded once).  The blur width
    is an acquisition parameter carried in binary32, so it is taken at its
    binary32 value."""
    sigma = float(np.float32(sigma))
    k = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-(k * k) / (2.0 * float(sigma) ** 2))
    return (g / g.sum()).astype(np.float32)


def blur(img: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Zero-padded separable blur with taps ``w`` (float64 arithmetic)."""
    img = np.asarray(img, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    b = (w.size - 1) // 2
    H, W = img.shape
    pad = np.zeros((H + 2 * b, W + 2 * b))
    pad[b:b + H, b:b + W] = img
    h = np.zeros((H + 2 * b, W))
    for k in range(-b, b + 1):
        h += w[k + b] * pad[:, b + k:b + k + W]
    out = np.zeros((H, W))
    for k in range(-b, b + 1):
        out += w[k + b] * h[b + k:b + k + H, :]
    return out


def blur_adjoint(g: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Transpose of ``blur``: correlation with the mirrored taps, zero padded."""
    return blur(g, np.asarray(w)[::-1])


def noise_normals(H: int, W: int, frame: int, pair_id: int, seed: int) -> np.ndarray:
    """float64 N(0, 1) field [H, W] of one frame (frame 0 or 1)."""
    Wq = (W + 3) // 4
    r = np.arange(H, dtype=np.uint64)[:, None]
    q = np.arange(Wq, dtype=np.uint64)[None, :]
    w0, w1, w2, w3 = ph.draw(r * np.uint64(Wq) + q, ph.STREAM_NOISE0 + frame, pair_id, seed)
    out = np.empty((H, Wq * 4))
    for (wa, wb, col) in ((w0, w1, 0), (w2, w3, 2)):
        u1 = ph.uniform24_open0(wa)
        u2 = ph.uniform24(wb)
        R = np.sqrt(-2.0 * np.log(u1))
        out[:, col::4] = R * np.cos(2.0 * np.pi * u2)
        out[:, col + 1::4] = R * np.sin(2.0 * np.pi * u2)
    return out[:, :W]


def quantise(v: np.ndarray, bits: int) -> np.ndarray:
    L = float((1 << bits) - 1)
    q = np.rint(np.asarray(v, dtype=np.float64) * L)     # numpy rint: half to even
    return np.clip(q, 0.0, L).astype(np.uint16)
