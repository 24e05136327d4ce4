"""ctypes wrapper of the binary32 mirror ``ra32.c`` (oracle, test infrastructure).

``build()`` compiles the plain C file with gcc (host only, no fused operations
beyond the explicit fmaf calls).  ``load()`` builds it if no library is there.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ra32.c")
_LIB = os.path.join(_HERE, "libra32.so")
_lib = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u16p = np.ctypeslib.ndpointer(dtype=np.uint16, flags="C_CONTIGUOUS")


def build() -> str:
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-o", _LIB, _SRC, "-lm"]
    subprocess.check_call(cmd)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    L = ctypes.CDLL(_LIB)
    L.ra_philox.argtypes = [_u32p, _u32p, _u32p]
    L.ra_E.argtypes = [ctypes.c_float]
    L.ra_E.restype = ctypes.c_float
    L.ra_ln.argtypes = [ctypes.c_float]
    L.ra_ln.restype = ctypes.c_float
    L.ra_cos2pi.argtypes = [ctypes.c_float]
    L.ra_cos2pi.restype = ctypes.c_float
    L.ra_seed_pair.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                               ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                               _f32p, _f32p, _f32p, _f32p, _f32p, _f32p, _f32p, _f32p,
                               ctypes.POINTER(ctypes.c_double)]
    L.ra_seed_pair.restype = ctypes.c_int
    L.ra_advect.argtypes = [_f32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                            ctypes.c_int, _f32p, _f32p, ctypes.c_float, ctypes.c_int, ctypes.c_int,
                            _f32p, _f32p]
    L.ra_support_range.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.ra_support_range.restype = ctypes.c_int
    L.ra_render_fixed.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _f32p, _f32p, _f32p,
                                  _f32p, _f32p, ctypes.c_float, _u32p]
    L.ra_fixed_to_float.argtypes = [_u32p, ctypes.c_size_t, _f32p]
    L.ra_blur.argtypes = [_f32p, ctypes.c_int, ctypes.c_int, _f32p, ctypes.c_int, _f32p, _f32p]
    L.ra_quantise.argtypes = [_f32p, ctypes.c_size_t, ctypes.c_int, _u16p]
    L.ra_sin2pi.argtypes = [ctypes.c_float]
    L.ra_sin2pi.restype = ctypes.c_float
    L.ra_seed_shape.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, _f32p,
                                ctypes.c_float, ctypes.c_float, _f32p, _f32p]
    L.ra_frame_params.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, _f32p, ctypes.c_float,
                                  ctypes.c_float, _f32p, _f32p, _f32p, _f32p, _f32p, _f32p, _f32p, _f32p, _f32p]
    L.ra_peak.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                          ctypes.c_float]
    L.ra_peak.restype = ctypes.c_float
    L.ra_peaks.argtypes = [ctypes.c_int, _f32p, _f32p, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                           ctypes.c_float, _f32p]
    L.ra_render_model_fixed.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _f32p, _f32p, _f32p, _f32p,
                                        _f32p, _f32p, _u32p]
    L.ra_advect_z.argtypes = [_f32p, _f32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              _f32p, _f32p, _f32p, ctypes.c_float, ctypes.c_int, ctypes.c_int, _f32p]
    L.ra_flow_field.argtypes = [_f32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _f32p]
    _lib = L
    return L


def _f(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def philox(ctr, key):
    out = np.zeros(4, dtype=np.uint32)
    load().ra_philox(np.asarray(ctr, dtype=np.uint32), np.asarray(key, dtype=np.uint32), out)
    return out


def E(q: float) -> float:
    return float(load().ra_E(float(q)))


def ln(u: float) -> float:
    return float(load().ra_ln(float(u)))


def cos2pi(u: float) -> float:
    return float(load().ra_cos2pi(float(u)))


def seed_pair(H, W, n_max, ppp, pair_id, seed, d_dist, d_params, I0=(0.8, 1.0), z=(-1.0, 1.0)):
    n = int(n_max)
    out = {k: np.zeros(n, dtype=np.float32) for k in ("x", "y", "z", "d", "I0")}
    dp = np.zeros(4, dtype=np.float32)
    dp[:len(d_params)] = d_params
    ppp_out = ctypes.c_double(0.0)
    na = load().ra_seed_pair(int(H), int(W), n, float(ppp[0]), float(ppp[1]), int(pair_id), int(seed),
                             1 if d_dist == "normal" else 0, dp, _f(I0), _f(z),
                             out["x"], out["y"], out["z"], out["d"], out["I0"], ctypes.byref(ppp_out))
    out["n_active"] = int(na)
    out["ppp"] = ppp_out.value
    return out


def advect(flow, H, W, x1, y1, dt, substeps, integrator):
    flow = _f(flow)
    x1 = _f(x1)
    y1 = _f(y1)
    x2 = np.zeros_like(x1)
    y2 = np.zeros_like(y1)
    load().ra_advect(flow, flow.shape[0], flow.shape[1], int(H), int(W), x1.size, x1, y1,
                     float(dt), int(substeps), 1 if integrator == "rk4" else 0, x2, y2)
    return x2, y2


def support_range(p, R, n):
    lo = ctypes.c_int(0)
    hi = ctypes.c_int(0)
    ok = load().ra_support_range(float(p), float(R), int(n), ctypes.byref(lo), ctypes.byref(hi))
    return (lo.value, hi.value) if ok else None


def render_fixed(x, y, z, d, I0, H, W, sheet_sigma):
    acc = np.zeros(H * W, dtype=np.uint32)
    x = _f(x)
    load().ra_render_fixed(int(H), int(W), x.size, x, _f(y), _f(z), _f(d), _f(I0),
                           float(sheet_sigma), acc)
    return acc.reshape(H, W)


def fixed_to_float(acc):
    acc = np.ascontiguousarray(acc, dtype=np.uint32)
    out = np.zeros(acc.shape, dtype=np.float32)
    load().ra_fixed_to_float(acc.reshape(-1), acc.size, out.reshape(-1))
    return out


def render(x, y, z, d, I0, H, W, sheet_sigma):
    return fixed_to_float(render_fixed(x, y, z, d, I0, H, W, sheet_sigma))


def blur(img, w):
    img = _f(img)
    w = _f(w)
    H, W = img.shape
    tmp = np.zeros_like(img)
    out = np.zeros_like(img)
    load().ra_blur(img, H, W, w, (w.size - 1) // 2, tmp, out)
    return out


def quantise(v, bits):
    v = _f(v)
    q = np.zeros(v.shape, dtype=np.uint16)
    load().ra_quantise(v.reshape(-1), v.size, int(bits), q.reshape(-1))
    return q


def generate_pair_noiseless(wl, pair_index, flow, H, W, pair_id=None):
    """Binary32 end-to-end pair (no noise): float exposures J and, for bits > 0,
    the integer codes.  Blur taps are the float64-derived, float32-rounded
    weights of the float64 oracle."""
    from . import epilogue as ep
    from . import seed as sd
    pid = pair_index if pair_id is None else pair_id
    n_max = sd.particle_count(H, W, wl.ppp[1])
    P = seed_pair(H, W, n_max, wl.ppp, pid, wl.seed, wl.d_dist, wl.d_params, wl.I0, wl.z)
    x2, y2 = advect(flow, H, W, P["x"], P["y"], wl.dt, wl.substeps, wl.integrator)
    frames = []
    for (xf, yf) in ((P["x"], P["y"]), (x2, y2)):
        img = render(xf, yf, P["z"], P["d"], P["I0"], H, W, wl.sheet_sigma)
        if wl.blur_radius > 0:
            img = blur(img, ep.blur_weights(wl.blur_radius, wl.blur_sigma))
        frames.append(img)
    J = np.stack(frames)
    out = {"particles": P, "x2": x2, "y2": y2, "J": J}
    if wl.bits > 0:
        out["codes"] = quantise(J, wl.bits)
    return out


# ------------------------------------------------------------------ full model

LAWS = {"gauss": 0, "remark1": 1}


def sin2pi(u: float) -> float:
    return float(load().ra_sin2pi(float(u)))


def seed_shape(n_max, pair_id, seed, d_dist, d_params, rho):
    n = int(n_max)
    dp = np.zeros(4, dtype=np.float32)
    dp[:len(d_params)] = d_params
    dy = np.zeros(n, dtype=np.float32)
    r = np.zeros(n, dtype=np.float32)
    load().ra_seed_shape(n, int(pair_id), int(seed), 1 if d_dist == "normal" else 0, dp, float(rho[0]),
                         float(rho[1]), dy, r)
    return dy, r


def frame_params(d, dy, rho, I0, pair_id, seed, jitter=(0.0, 0.0, 0.0), hide_p=0.0, d_max=16.0):
    d, dy, rho, I0 = _f(d), _f(dy), _f(rho), _f(I0)
    n = d.size
    I1, d2, dy2, r2, I2 = (np.zeros(n, dtype=np.float32) for _ in range(5))
    load().ra_frame_params(n, int(pair_id), int(seed), _f(jitter), float(hide_p), float(d_max), d, dy, rho, I0,
                           I1, d2, dy2, r2, I2)
    return (d, dy, rho, I1), (d2, dy2, r2, I2)


def peaks(I0, z, law="gauss", sheet_sigma=0.5, dz0=1.0, shape=1.0):
    I0 = _f(I0)
    A = np.zeros_like(I0)
    load().ra_peaks(I0.size, I0, _f(z), LAWS[law], float(sheet_sigma), float(dz0), float(shape), A)
    return A


def render_model(x, y, A, d, dy, rho, H, W):
    acc = np.zeros(H * W, dtype=np.uint32)
    x = _f(x)
    load().ra_render_model_fixed(int(H), int(W), x.size, x, _f(y), _f(A), _f(d), _f(dy), _f(rho), acc)
    return fixed_to_float(acc.reshape(H, W))


def advect_z(flow, wgrid, H, W, x1, y1, z1, dt, substeps, integrator):
    flow = _f(flow)
    wgrid = _f(wgrid)
    x1 = _f(x1)
    z2 = np.zeros_like(x1)
    load().ra_advect_z(flow, wgrid, flow.shape[0], flow.shape[1], int(H), int(W), x1.size, x1, _f(y1), _f(z1),
                       float(dt), int(substeps), 1 if integrator == "rk4" else 0, z2)
    return z2


def generate_pair_model(m, H, W, pair_id, seed, flow, wgrid=None, blur_w=None, bits=0):
    """Binary32 pair under the full model (no noise): exposures J (blurred when
    blur_w is given) and, for bits > 0, the codes.  ``m`` as in
    ``oracle.model.generate_pair``."""
    from . import seed as sd
    n_max = sd.particle_count(H, W, m["ppp"][1])
    P = seed_pair(H, W, n_max, m["ppp"], pair_id, seed, m["d_dist"], m["d_params"], m["I0"], m["z"])
    if m.get("anisotropic"):
        dy, rho = seed_shape(n_max, pair_id, seed, m["d_dist"], m["d_params"], m["rho"])
    else:
        dy, rho = P["d"].copy(), np.zeros(n_max, dtype=np.float32)
    x2, y2 = advect(flow, H, W, P["x"], P["y"], m["dt"], m["substeps"], m["integrator"])
    z2 = advect_z(flow, wgrid, H, W, P["x"], P["y"], P["z"], m["dt"], m["substeps"], m["integrator"]) \
        if wgrid is not None else P["z"].copy()
    f1, f2 = frame_params(P["d"], dy, rho, P["I0"], pair_id, seed, m.get("jitter", (0.0, 0.0, 0.0)),
                          m.get("hide_p", 0.0), m.get("d_max", 16.0))
    law = m.get("law", "gauss")
    frames = []
    for (xf, yf, zf, f) in ((P["x"], P["y"], P["z"], f1), (x2, y2, z2, f2)):
        A = peaks(f[3], zf, law, m.get("sheet_sigma", 0.5), m.get("dz0", 1.0), m.get("shape", 1.0))
        img = render_model(xf, yf, A, f[0], f[1], f[2], H, W)
        if blur_w is not None:
            img = blur(img, blur_w)
        frames.append(img)
    J = np.stack(frames)
    out = {"particles": P, "dy": dy, "rho": rho, "x2": x2, "y2": y2, "z2": z2, "frame1": f1, "frame2": f2, "J": J}
    if bits > 0:
        out["codes"] = quantise(J, bits)
    return out


def flow_field(flow, H, W):
    """[H, W, 2] binary32 field at the pixel centres."""
    flow = _f(flow)
    out = np.zeros((H, W, 2), dtype=np.float32)
    load().ra_flow_field(flow, flow.shape[0], flow.shape[1], int(H), int(W), out.reshape(-1))
    return out
