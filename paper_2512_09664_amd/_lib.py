"""ctypes declarations of ``include/synthpix.h`` and the library loader.

Only argument marshalling lives here: every step of the generator runs in the
HIP kernels of ``libsynthpix.so``.  Loading fails loudly if the library has not
been built; there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsynthpix.so")

SP_OK = 0
SP_ERR_INVALID_ARG = -1
SP_ERR_WORKSPACE = -2
SP_ERR_UNSUPPORTED = -3
SP_ERR_HIP = -4
SP_ERR_DEVICE_STATUS = -5

SP_EULER = 0
SP_RK4 = 1
SP_DIST_UNIFORM = 0
SP_DIST_NORMAL_CLIPPED = 1
SP_SHEET_GAUSS = 0
SP_SHEET_REMARK1 = 1

SP_STATUS_D_ABOVE_MAX = 0x1
SP_STATUS_FIXED_RANGE = 0x2


class SynthPixError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"synthpix status {status}: {message}")
        self.status = status


class Pair(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("Gh", ctypes.c_int32), ("Gw", ctypes.c_int32),
                ("n_max", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("particle_offset", ctypes.c_int64), ("image_offset", ctypes.c_int64),
                ("flow_offset", ctypes.c_int64), ("pair_id", ctypes.c_uint64)]


class SeedParams(ctypes.Structure):
    _fields_ = [("ppp_lo", ctypes.c_double), ("ppp_hi", ctypes.c_double), ("d_dist", ctypes.c_int32),
                ("d_a", ctypes.c_float), ("d_b", ctypes.c_float), ("d_lo", ctypes.c_float),
                ("d_hi", ctypes.c_float), ("I0_lo", ctypes.c_float), ("I0_hi", ctypes.c_float),
                ("z_lo", ctypes.c_float), ("z_hi", ctypes.c_float)]


class AdvectParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_float), ("substeps", ctypes.c_int32), ("integrator", ctypes.c_int32)]


class RenderParams(ctypes.Structure):
    _fields_ = [("sheet_sigma", ctypes.c_float), ("d_max", ctypes.c_float), ("blur_radius", ctypes.c_int32),
                ("blur_sigma", ctypes.c_float), ("noise_sigma", ctypes.c_float), ("bits", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("advect", AdvectParams),
                ("hide_p", ctypes.c_float), ("jitter_d", ctypes.c_float), ("jitter_rho", ctypes.c_float),
                ("jitter_I0", ctypes.c_float), ("sheet_law", ctypes.c_int32), ("sheet_dz0", ctypes.c_float),
                ("sheet_shape", ctypes.c_float)]


class ParticleExtras(ctypes.Structure):
    _fields_ = [("dy", ctypes.c_void_p), ("rho", ctypes.c_void_p), ("z2", ctypes.c_void_p)]


class Tiling(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("cap", ctypes.c_int32), ("persistent", ctypes.c_int32)]


class BinViews(ctypes.Structure):
    _fields_ = [("tile_count", ctypes.c_size_t), ("tile_offset", ctypes.c_size_t), ("entries", ctypes.c_size_t),
                ("tiles", ctypes.c_int64)]


class BatchIO(ctypes.Structure):
    _fields_ = [("flow", ctypes.c_void_p), ("x1", ctypes.c_void_p), ("y1", ctypes.c_void_p),
                ("x2", ctypes.c_void_p), ("y2", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("d", ctypes.c_void_p), ("I0", ctypes.c_void_p), ("images", ctypes.c_void_p),
                ("n_active", ctypes.c_void_p), ("ppp", ctypes.c_void_p), ("seed", ctypes.c_uint64),
                ("pair_id_base", ctypes.c_uint64)]


assert ctypes.sizeof(Pair) == 56
assert ctypes.sizeof(RenderParams) == 72

_P = ctypes.c_void_p
_PP = ctypes.POINTER(Pair)
_ST = ctypes.c_int

# name -> argtypes (all return synthpix_status unless listed in _RESTYPES)
SIGNATURES = {
    "synthpix_version": [],
    "synthpix_last_error": [],
    "synthpix_particle_count": [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_int32)],
    "synthpix_default_tiling": [_PP, ctypes.c_int32, ctypes.POINTER(RenderParams), ctypes.POINTER(Tiling)],
    "synthpix_workspace_size": [_PP, ctypes.c_int32, ctypes.POINTER(RenderParams), ctypes.POINTER(Tiling),
                                ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
    "synthpix_read_status": [_P, _P, ctypes.POINTER(ctypes.c_uint32)],
    "synthpix_timing_enable": [ctypes.c_int32],
    "synthpix_timing_read": [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
    "synthpix_probe": [ctypes.c_int32, _P, ctypes.c_size_t, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_double)],
    "synthpix_bin_views_of": [_PP, ctypes.c_int32, ctypes.POINTER(RenderParams), ctypes.POINTER(Tiling),
                              ctypes.POINTER(BinViews)],
    "synthpix_seed": [_PP, _P, ctypes.c_int32, ctypes.POINTER(SeedParams), ctypes.c_uint64,
                      _P, _P, _P, _P, _P, _P, _P, _P],
    "synthpix_advect": [_PP, _P, ctypes.c_int32, _P, ctypes.POINTER(AdvectParams), _P, _P, _P, _P, _P, _P, _P, _P,
                        ctypes.c_size_t, _P],
    "synthpix_flow_field": [_PP, _P, ctypes.c_int32, _P, _P, _P],
    "synthpix_histogram_workspace_size": [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
    "synthpix_histogram_match": [_PP, _P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, ctypes.c_size_t, _P],
    "synthpix_mse_workspace_size": [ctypes.c_int64],
    "synthpix_mse_grad": [_P, _P, ctypes.c_int64, ctypes.c_float, _P, _P, _P, ctypes.c_size_t, _P],
    "synthpix_seed_shape": [_PP, _P, ctypes.c_int32, ctypes.POINTER(SeedParams), ctypes.c_float, ctypes.c_float,
                            ctypes.c_uint64, _P, _P, _P],
    "synthpix_advect_workspace_size": [_PP, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
    "synthpix_render_pair": [_PP, _P, ctypes.c_int32, ctypes.POINTER(Tiling), _P, _P, _P, _P, _P, _P, _P,
                             ctypes.POINTER(ParticleExtras), ctypes.POINTER(RenderParams), _P, _P, ctypes.c_size_t,
                             _P],
    "synthpix_render_pair_noalloc": [_PP, _P, ctypes.c_int32, ctypes.POINTER(Tiling), _P, _P, _P, _P, _P, _P, _P,
                                     ctypes.POINTER(ParticleExtras), ctypes.POINTER(RenderParams), _P, _P, _P],
    "synthpix_render_pair_backward": [_PP, _P, ctypes.c_int32, ctypes.POINTER(Tiling), _P, _P, _P, _P, _P, _P, _P,
                                      _P, ctypes.POINTER(RenderParams), _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                      ctypes.c_size_t, _P],
    "synthpix_render_pair_backward_mse": [_PP, _P, ctypes.c_int32, ctypes.POINTER(Tiling), _P, _P, _P, _P, _P, _P,
                                          _P, _P, ctypes.POINTER(RenderParams), _P, _P, ctypes.c_float, _P, _P, _P,
                                          _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P],
    "synthpix_tiling_candidates": [ctypes.POINTER(RenderParams), ctypes.POINTER(Tiling), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32)],
    "synthpix_plan_create": [_PP, ctypes.c_int32, ctypes.POINTER(SeedParams), ctypes.POINTER(AdvectParams),
                             ctypes.POINTER(RenderParams), ctypes.POINTER(BatchIO), ctypes.c_int32, ctypes.c_int32,
                             _P, ctypes.POINTER(ctypes.c_void_p)],
    "synthpix_plan_launch": [_P, ctypes.POINTER(BatchIO), _P],
    "synthpix_plan_read_status": [_P, _P, ctypes.POINTER(ctypes.c_uint32)],
    "synthpix_plan_tiling": [_P, ctypes.POINTER(Tiling)],
    "synthpix_plan_destroy": [_P],
}
_RESTYPES = {"synthpix_version": ctypes.c_int32, "synthpix_last_error": ctypes.c_char_p,
             "synthpix_mse_workspace_size": ctypes.c_size_t}

_lib = None


def load(path: str = LIB_PATH):
    """Load libsynthpix.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = _RESTYPES.get(name, _ST)
    _lib = L
    return L


def check(status: int):
    if status != SP_OK:
        msg = load().synthpix_last_error()
        raise SynthPixError(status, msg.decode() if msg else "")
