"""Histogram adjustment of the stored images, definition (oracle, test infrastructure).

Section 2 (after Remark 2): the output may be remapped so that its
intensities follow a histogram the user chooses.  Reading: classical histogram
specification of each stored image (each frame of each pair, its integer
codes 0 .. 2^bits - 1) to one target histogram t[0 .. 2^bits - 1] of
non-negative counts.  With the image's cumulative counts S(k) (pixels with a
code <= k, N pixels in all) and the target's T(m) (total T_tot), code k maps
to the smallest m with T(m) / T_tot >= S(k) / N, i.e. T(m) N >= S(k) T_tot, an
exact integer comparison (Python integers here, no rounding anywhere).

Particle reuse (Conclusions, third item) needs no arithmetic of its own: the
next batch's frame-1 positions are this batch's frame-2 positions moved by the
same flow over a second time dt' (``advect.advect``).
"""

from __future__ import annotations

import numpy as np


def mapping(codes: np.ndarray, target, bits: int) -> np.ndarray:
    """Look-up table [2^bits] (uint16) of one image's codes onto the target."""
    B = 1 << bits
    t = [int(v) for v in np.asarray(target).reshape(-1)]
    assert len(t) == B and min(t) >= 0 and sum(t) > 0
    h = np.bincount(np.asarray(codes, dtype=np.int64).reshape(-1), minlength=B)
    assert h.size == B
    N = int(codes.size)
    T_tot = sum(t)
    S = 0
    T = 0
    m = -1
    lut = np.zeros(B, dtype=np.uint16)
    for k in range(B):
        S += int(h[k])
        # the smallest m whose cumulative target reaches S(k) / N of the total
        # (non-decreasing in k, so the search resumes where it stopped)
        while m < B - 1 and (m < 0 or T * N < S * T_tot):
            m += 1
            T += t[m]
        lut[k] = m
    return lut


def match(codes: np.ndarray, target, bits: int) -> np.ndarray:
    """The image with every code replaced by its mapped code."""
    return mapping(codes, target, bits)[np.asarray(codes, dtype=np.int64)]
