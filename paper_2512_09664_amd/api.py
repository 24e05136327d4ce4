"""PyTorch-facing binding of the C ABI (argument marshalling only).

Tensors provide device memory, ``torch.cuda.current_stream()`` provides the
stream; every computation runs in ``libsynthpix.so``.  Names follow the C
entry points: ``seed``, ``advect``, ``render_pair``, ``render_pair_backward``.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need_cuda(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("tensors must be contiguous CUDA (HIP) tensors")


U16 = getattr(torch, "uint16", torch.int16)


def particle_count(H: int, W: int, ppp: float) -> int:
    n = ctypes.c_int32(0)
    L.check(L.load().synthpix_particle_count(int(H), int(W), float(ppp), ctypes.byref(n)))
    return n.value


@dataclass
class PairBatch:
    """A batch of image pairs: the pair table on host and device plus the
    sizes of the packed particle, image and flow arrays."""
    host: ctypes.Array
    dev: torch.Tensor
    n_pairs: int
    n_particles: int
    n_pixels: int
    n_flow: int
    sizes: Tuple[Tuple[int, int], ...]
    grids: Tuple[Tuple[int, int], ...]
    n_max: Tuple[int, ...]

    @staticmethod
    def build(sizes: Sequence[Tuple[int, int]], grids: Sequence[Tuple[int, int]], n_max: Sequence[int],
              pair_ids: Optional[Sequence[int]] = None, device="cuda",
              gaps: Tuple[int, int, int] = (0, 0, 0), flow_index: Optional[Sequence[int]] = None,
              non_blocking: bool = False) -> "PairBatch":
        """Pairs packed in table order; ``gaps`` leaves that many unused particles,
        image elements and flow floats (even) before every pair's range.
        ``flow_index``: pairs that share a flow grid (pair p uses grid
        flow_index[p]; grids packed in index order, all of pair p's shape).
        ``non_blocking``: upload the table from pinned memory without waiting."""
        if gaps[2] % 2:
            raise ValueError("flow gaps must be even (one (u, v) node is two floats)")
        n = len(sizes)
        arr = (L.Pair * n)()
        po = io = fo = 0
        for p in range(n):
            H, W = sizes[p]
            Gh, Gw = grids[p]
            po, io, fo = po + gaps[0], io + gaps[1], fo + gaps[2]
            arr[p].H, arr[p].W, arr[p].Gh, arr[p].Gw = int(H), int(W), int(Gh), int(Gw)
            arr[p].n_max = int(n_max[p])
            arr[p].reserved = 0
            arr[p].particle_offset = po
            arr[p].image_offset = io
            arr[p].flow_offset = fo
            arr[p].pair_id = int(pair_ids[p]) if pair_ids is not None else p
            po += int(n_max[p])
            io += 2 * int(H) * int(W)
            fo += 2 * int(Gh) * int(Gw)
        if flow_index is not None:
            fo = 0
            for p in range(n):
                arr[p].flow_offset = 2 * int(grids[p][0]) * int(grids[p][1]) * int(flow_index[p])
                fo = max(fo, int(arr[p].flow_offset) + 2 * int(grids[p][0]) * int(grids[p][1]))
        raw = np.frombuffer(bytes(arr), dtype=np.uint8).copy()
        t = torch.from_numpy(raw)
        dev = t.pin_memory().to(device, non_blocking=True) if non_blocking else t.to(device)
        return PairBatch(arr, dev, n, po, io, fo, tuple(map(tuple, sizes)), tuple(map(tuple, grids)),
                         tuple(int(v) for v in n_max))

    @property
    def host_ptr(self):
        return ctypes.cast(self.host, ctypes.POINTER(L.Pair))

    @property
    def dev_ptr(self):
        return ctypes.c_void_p(self.dev.data_ptr())


def seed_params(ppp=(0.05, 0.05), d_dist="uniform", d_params=(1.0, 5.0), I0=(0.8, 1.0), z=(-1.0, 1.0)):
    sp = L.SeedParams()
    sp.ppp_lo, sp.ppp_hi = float(ppp[0]), float(ppp[1])
    if d_dist == "uniform":
        sp.d_dist = L.SP_DIST_UNIFORM
        sp.d_a, sp.d_b = float(d_params[0]), float(d_params[1])
        sp.d_lo, sp.d_hi = 0.0, 0.0
    elif d_dist == "normal":
        sp.d_dist = L.SP_DIST_NORMAL_CLIPPED
        sp.d_a, sp.d_b, sp.d_lo, sp.d_hi = (float(v) for v in d_params)
    else:
        raise ValueError(d_dist)
    sp.I0_lo, sp.I0_hi = float(I0[0]), float(I0[1])
    sp.z_lo, sp.z_hi = float(z[0]), float(z[1])
    return sp


def advect_params(dt=1.0, substeps=1, integrator="euler"):
    ap = L.AdvectParams()
    ap.dt = float(dt)
    ap.substeps = int(substeps)
    ap.integrator = {"euler": L.SP_EULER, "rk4": L.SP_RK4}[integrator]
    return ap


def render_params(sheet_sigma=0.5, d_max=5.0, blur_radius=0, blur_sigma=0.7, noise_sigma=0.0, bits=0, seed=0,
                  dt=1.0, substeps=1, integrator="euler", hide_p=0.0, jitter=(0.0, 0.0, 0.0), sheet_law="gauss",
                  sheet_dz0=0.0, sheet_shape=0.0):
    """Rendering parameters; ``jitter`` = standard deviations of the frame-2
    change of (diameters, rho, I0); ``sheet_law`` "gauss" or "remark1"."""
    rp = L.RenderParams()
    rp.hide_p = float(hide_p)
    rp.jitter_d, rp.jitter_rho, rp.jitter_I0 = (float(v) for v in jitter)
    rp.sheet_law = {"gauss": L.SP_SHEET_GAUSS, "remark1": L.SP_SHEET_REMARK1}[sheet_law]
    rp.sheet_dz0 = float(sheet_dz0)
    rp.sheet_shape = float(sheet_shape)
    rp.sheet_sigma = float(sheet_sigma)
    rp.d_max = float(d_max)
    rp.blur_radius = int(blur_radius)
    rp.blur_sigma = float(blur_sigma)
    rp.noise_sigma = float(noise_sigma)
    rp.bits = int(bits)
    rp.seed = int(seed)
    rp.advect = advect_params(dt, substeps, integrator)
    return rp


def tiling(tile_w=32, tile_h=32, chunk=4096, cap=128, persistent=0):
    t = L.Tiling()
    t.tile_w, t.tile_h, t.chunk, t.cap = int(tile_w), int(tile_h), int(chunk), int(cap)
    t.persistent = int(persistent)
    return t


def tiling_candidates(rp):
    """The tilings a plan's autotuner may try (``synthpix_tiling_candidates``)."""
    n = ctypes.c_int32(0)
    L.check(L.load().synthpix_tiling_candidates(ctypes.byref(rp), None, 0, ctypes.byref(n)))
    arr = (L.Tiling * max(n.value, 1))()
    L.check(L.load().synthpix_tiling_candidates(ctypes.byref(rp), arr, n.value, ctypes.byref(n)))
    return [arr[i] for i in range(n.value)]


def default_tiling(batch: PairBatch, rp):
    t = L.Tiling()
    L.check(L.load().synthpix_default_tiling(batch.host_ptr, batch.n_pairs, ctypes.byref(rp), ctypes.byref(t)))
    return t


def seed(batch: PairBatch, sp, seed_value: int, out=None):
    """Run ``synthpix_seed``; returns dict x, y, z, d, I0 (float32 [n_particles])
    plus n_active (int32 [n_pairs]) and ppp (float64 [n_pairs])."""
    dev = batch.dev.device
    n = max(batch.n_particles, 1)
    o = out or {k: torch.empty(n, dtype=torch.float32, device=dev) for k in ("x", "y", "z", "d", "I0")}
    if "n_active" not in o:
        o["n_active"] = torch.empty(batch.n_pairs, dtype=torch.int32, device=dev)
        o["ppp"] = torch.empty(batch.n_pairs, dtype=torch.float64, device=dev)
    L.check(L.load().synthpix_seed(batch.host_ptr, batch.dev_ptr, batch.n_pairs, ctypes.byref(sp),
                                   int(seed_value), _ptr(o["x"]), _ptr(o["y"]), _ptr(o["z"]), _ptr(o["d"]),
                                   _ptr(o["I0"]), _ptr(o["n_active"]), _ptr(o["ppp"]), _stream()))
    return o


def advect_workspace_size(batch: PairBatch) -> int:
    n = ctypes.c_size_t(0)
    L.check(L.load().synthpix_advect_workspace_size(batch.host_ptr, batch.n_pairs, ctypes.byref(n)))
    return n.value


def advect(batch: PairBatch, flow: torch.Tensor, ap, x1: torch.Tensor, y1: torch.Tensor, x2=None, y2=None,
           workspace: Optional[torch.Tensor] = None, ordered: bool = True, wflow=None, z1=None, z2=None):
    """Run ``synthpix_advect``.  ``ordered`` processes particles in home-block
    order (same results, faster); its scratch is ``workspace`` if given (e.g. a
    render workspace), else a temporary.  With ``wflow`` (each pair's w grid)
    and ``z1``, z is moved too and (x2, y2, z2) is returned."""
    _need_cuda(flow, x1, y1, wflow, z1, z2)
    if wflow is not None:
        x2 = torch.empty_like(x1) if x2 is None else x2
        y2 = torch.empty_like(y1) if y2 is None else y2
        z2 = torch.empty_like(z1) if z2 is None else z2
        L.check(L.load().synthpix_advect(batch.host_ptr, batch.dev_ptr, batch.n_pairs, _ptr(flow), ctypes.byref(ap),
                                         _ptr(x1), _ptr(y1), _ptr(x2), _ptr(y2), _ptr(wflow), _ptr(z1), _ptr(z2),
                                         None, 0, _stream()))
        return x2, y2, z2
    x2 = torch.empty_like(x1) if x2 is None else x2
    y2 = torch.empty_like(y1) if y2 is None else y2
    if ordered and workspace is None:
        workspace = torch.empty(max(advect_workspace_size(batch), 256), dtype=torch.uint8, device=x1.device)
    ws, nb = (_ptr(workspace), workspace.numel()) if ordered else (None, 0)
    L.check(L.load().synthpix_advect(batch.host_ptr, batch.dev_ptr, batch.n_pairs, _ptr(flow), ctypes.byref(ap),
                                     _ptr(x1), _ptr(y1), _ptr(x2), _ptr(y2), None, None, None, ws, nb, _stream()))
    return x2, y2


def seed_shape(batch: PairBatch, sp, rho, seed_value: int, out=None):
    """Run ``synthpix_seed_shape``: (dy, rho) float32 [n_particles]."""
    dev = batch.dev.device
    n = max(batch.n_particles, 1)
    dy, r = out if out is not None else (torch.empty(n, dtype=torch.float32, device=dev),
                                         torch.empty(n, dtype=torch.float32, device=dev))
    L.check(L.load().synthpix_seed_shape(batch.host_ptr, batch.dev_ptr, batch.n_pairs, ctypes.byref(sp),
                                         float(rho[0]), float(rho[1]), int(seed_value), _ptr(dy), _ptr(r), _stream()))
    return dy, r


def flow_field(batch: PairBatch, flow: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Run ``synthpix_flow_field``: each pair's (u, v) at its pixel centres,
    [H][W][2] at the pair's image offset of a float buffer of the images' size."""
    _need_cuda(flow, out)
    if out is None:
        out = torch.empty(batch.n_pixels, dtype=torch.float32, device=flow.device)
    L.check(L.load().synthpix_flow_field(batch.host_ptr, batch.dev_ptr, batch.n_pairs, _ptr(flow), _ptr(out),
                                         _stream()))
    return out


def histogram_match(batch: PairBatch, images: torch.Tensor, target: torch.Tensor, bits: int, workspace=None):
    """Run ``synthpix_histogram_match``: every frame's codes mapped in place onto
    the target histogram (uint32/int32 device counts [2^bits]).  Returns the
    workspace (its status word: ``read_status``)."""
    _need_cuda(images, target)
    n = ctypes.c_size_t(0)
    L.check(L.load().synthpix_histogram_workspace_size(batch.n_pairs, int(bits), ctypes.byref(n)))
    if workspace is None:
        workspace = torch.empty(max(n.value, 256), dtype=torch.uint8, device=images.device)
    L.check(L.load().synthpix_histogram_match(batch.host_ptr, batch.dev_ptr, batch.n_pairs, int(bits), _ptr(target),
                                              _ptr(images), _ptr(workspace), workspace.numel(), _stream()))
    return workspace


def mse_grad(J: torch.Tensor, T: torch.Tensor, scale: Optional[float] = None, out=None, loss: bool = False,
             workspace=None):
    """Run ``synthpix_mse_grad``: dL/dJ = scale (J - T) (scale 2 / n by default,
    the gradient of the mean squared difference) into ``out`` (new if None).
    With ``loss``, also the mean of (J - T)^2 as a float64 device scalar;
    returns (grad, loss or None)."""
    _need_cuda(J, T)
    n = J.numel()
    if T.numel() != n or J.dtype != torch.float32 or T.dtype != torch.float32:
        raise ValueError("J and T must be float32 tensors with the same number of elements")
    out = torch.empty_like(J) if out is None else out
    _need_cuda(out)
    lv = None
    ws_n = 0
    if loss:
        lv = torch.empty((), dtype=torch.float64, device=J.device)
        if workspace is None:
            workspace = torch.empty(max(L.load().synthpix_mse_workspace_size(n), 256), dtype=torch.uint8,
                                    device=J.device)
        ws_n = workspace.numel()
    L.check(L.load().synthpix_mse_grad(_ptr(J), _ptr(T), n, float(2.0 / max(n, 1) if scale is None else scale),
                                       _ptr(out), _ptr(lv), _ptr(workspace) if loss else None, ws_n, _stream()))
    return out, lv


def _extras(dy, rho, z2):
    if dy is None and rho is None and z2 is None:
        return None
    _need_cuda(dy, rho, z2)
    ex = L.ParticleExtras()
    ex.dy = dy.data_ptr() if dy is not None else None
    ex.rho = rho.data_ptr() if rho is not None else None
    ex.z2 = z2.data_ptr() if z2 is not None else None
    return ctypes.byref(ex)


def workspace_size(batch: PairBatch, rp, tile=None, backward=False) -> int:
    """Workspace bytes: the forward (backward False), ``render_pair_backward``
    (True) or ``render_pair_backward_mse`` (``"mse"``)."""
    n = ctypes.c_size_t(0)
    kind = 2 if backward == "mse" else 1 if backward else 0
    L.check(L.load().synthpix_workspace_size(batch.host_ptr, batch.n_pairs, ctypes.byref(rp),
                                             ctypes.byref(tile) if tile is not None else None,
                                             kind, ctypes.byref(n)))
    return n.value


def alloc_workspace(batch: PairBatch, rp, tile=None, backward=False) -> torch.Tensor:
    nbytes = workspace_size(batch, rp, tile, backward)
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=batch.dev.device)


def bin_views(batch: PairBatch, rp, tile=None, workspace: torch.Tensor = None):
    """Tile counts, offsets and member lists written into ``workspace`` by the
    last ``render_pair`` call with the same batch, parameters and tiling."""
    v = L.BinViews()
    L.check(L.load().synthpix_bin_views_of(batch.host_ptr, batch.n_pairs, ctypes.byref(rp),
                                           ctypes.byref(tile) if tile is not None else None, ctypes.byref(v)))
    T = int(v.tiles)
    ws = workspace
    count = ws[v.tile_count:v.tile_count + 8 * T].view(torch.int32).view(2, T)
    offset = ws[v.tile_offset:v.tile_offset + 16 * T].view(torch.int64).view(2, T)
    entries = ws[v.entries:].view(torch.int32)
    return count, offset, entries


def timing_enable(on: bool = True):
    L.check(L.load().synthpix_timing_enable(1 if on else 0))


def timing_read(name: Optional[str] = None):
    """(total milliseconds, launches) of the timed launches of kernel ``name``."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    L.check(L.load().synthpix_timing_read(name.encode() if name else None, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


PROBES = {"store": 0, "copy": 1, "fma": 2, "trans": 3, "mul64": 4, "store_nt": 5, "mix": 6, "int": 7}


def probe(kind: str, buf: torch.Tensor, iters: int = 0) -> float:
    """One ``synthpix_probe`` launch on the current stream; returns its unit
    count (bytes moved, or wave64 VALU instructions of the probe loop)."""
    _need_cuda(buf)
    work = ctypes.c_double(0.0)
    L.check(L.load().synthpix_probe(PROBES[kind], _ptr(buf), buf.numel() * buf.element_size(), iters, _stream(),
                                    ctypes.byref(work)))
    return work.value


def read_status(workspace: torch.Tensor) -> int:
    flags = ctypes.c_uint32(0)
    st = L.load().synthpix_read_status(_ptr(workspace), _stream(), ctypes.byref(flags))
    if st not in (L.SP_OK, L.SP_ERR_DEVICE_STATUS):
        L.check(st)
    return flags.value


def render_pair(batch: PairBatch, x1, y1, x2, y2, z, d, I0, rp, tile=None, images=None, workspace=None, dy=None,
                rho=None, z2=None):
    """Run ``synthpix_render_pair``; returns images [n_pixels] (float32 or uint16).
    dy, rho, z2: the full model's optional per-particle inputs."""
    _need_cuda(x1, y1, x2, y2, z, d, I0)
    dev = x1.device
    if images is None:
        # zero-filled: the library writes only the pairs' image ranges
        images = torch.zeros(batch.n_pixels, dtype=U16 if rp.bits > 0 else torch.float32, device=dev)
    if workspace is None:
        workspace = alloc_workspace(batch, rp, tile)
    L.check(L.load().synthpix_render_pair(batch.host_ptr, batch.dev_ptr, batch.n_pairs,
                                          ctypes.byref(tile) if tile is not None else None,
                                          _ptr(x1), _ptr(y1), _ptr(x2), _ptr(y2), _ptr(z), _ptr(d), _ptr(I0),
                                          _extras(dy, rho, z2), ctypes.byref(rp), _ptr(images), _ptr(workspace),
                                          workspace.numel(), _stream()))
    return images


def render_pair_noalloc(batch: PairBatch, x1, y1, x2, y2, z, d, I0, rp, images, tile=None, status=None, dy=None,
                        rho=None, z2=None):
    """Run ``synthpix_render_pair_noalloc`` into the caller's ``images`` (the
    library's static scratch is the workspace; nothing is allocated).
    ``status``: optional int32/uint32 device tensor of one element that receives
    the device status word."""
    _need_cuda(x1, y1, x2, y2, z, d, I0, images, status)
    L.check(L.load().synthpix_render_pair_noalloc(batch.host_ptr, batch.dev_ptr, batch.n_pairs,
                                                  ctypes.byref(tile) if tile is not None else None,
                                                  _ptr(x1), _ptr(y1), _ptr(x2), _ptr(y2), _ptr(z), _ptr(d),
                                                  _ptr(I0), _extras(dy, rho, z2), ctypes.byref(rp), _ptr(images),
                                                  _ptr(status), _stream()))
    return images


def render_pair_backward(batch: PairBatch, flow, x1, y1, z, d, I0, rp, grad_images, tile=None, workspace=None,
                         x2=None, y2=None):
    """Run ``synthpix_render_pair_backward``; returns dict of gradients.  Pass the
    forward's frame-2 positions as x2, y2 to skip their recomputation."""
    _need_cuda(flow, x1, y1, z, d, I0, grad_images, x2, y2)
    dev = x1.device
    g = {k: torch.empty_like(x1) for k in ("x1", "y1", "z", "d", "I0")}
    g["sheet"] = torch.empty(batch.n_pairs, dtype=torch.float32, device=dev)
    g["sheet_total"] = torch.empty((), dtype=torch.float32, device=dev)
    g["flow"] = torch.empty_like(flow)
    if workspace is None:
        workspace = alloc_workspace(batch, rp, tile, backward=True)
    L.check(L.load().synthpix_render_pair_backward(
        batch.host_ptr, batch.dev_ptr, batch.n_pairs, ctypes.byref(tile) if tile is not None else None,
        _ptr(flow), _ptr(x1), _ptr(y1), _ptr(x2), _ptr(y2), _ptr(z), _ptr(d), _ptr(I0), ctypes.byref(rp),
        _ptr(grad_images), _ptr(g["x1"]), _ptr(g["y1"]), _ptr(g["z"]), _ptr(g["d"]), _ptr(g["I0"]),
        _ptr(g["sheet"]), _ptr(g["sheet_total"]), _ptr(g["flow"]), _ptr(workspace), workspace.numel(), _stream()))
    return g


def render_pair_backward_mse(batch: PairBatch, flow, x1, y1, z, d, I0, rp, images, target, scale=None,
                             loss: bool = False, tile=None, workspace=None, x2=None, y2=None):
    """Run ``synthpix_render_pair_backward_mse``: the gradients of the mean
    squared difference of the float ``images`` to ``target`` (dL/dJ = scale
    (J - T), scale 2 / (number of the pairs' pixels) by default, formed inside
    the backward).  Returns the gradient dict of ``render_pair_backward``, with
    ``loss`` (a float64 device scalar) when asked for."""
    _need_cuda(flow, x1, y1, z, d, I0, images, target, x2, y2)
    if images.dtype != torch.float32 or target.dtype != torch.float32:
        raise ValueError("images and target must be float32")
    dev = x1.device
    g = {k: torch.empty_like(x1) for k in ("x1", "y1", "z", "d", "I0")}
    g["sheet"] = torch.empty(batch.n_pairs, dtype=torch.float32, device=dev)
    g["sheet_total"] = torch.empty((), dtype=torch.float32, device=dev)
    g["flow"] = torch.empty_like(flow)
    lv = torch.empty((), dtype=torch.float64, device=dev) if loss else None
    if scale is None:
        scale = 2.0 / max(sum(2 * H * W for (H, W) in batch.sizes), 1)
    if workspace is None:
        workspace = alloc_workspace(batch, rp, tile, backward="mse")
    L.check(L.load().synthpix_render_pair_backward_mse(
        batch.host_ptr, batch.dev_ptr, batch.n_pairs, ctypes.byref(tile) if tile is not None else None,
        _ptr(flow), _ptr(x1), _ptr(y1), _ptr(x2), _ptr(y2), _ptr(z), _ptr(d), _ptr(I0), ctypes.byref(rp),
        _ptr(images), _ptr(target), float(scale), _ptr(lv), _ptr(g["x1"]), _ptr(g["y1"]), _ptr(g["z"]),
        _ptr(g["d"]), _ptr(g["I0"]), _ptr(g["sheet"]), _ptr(g["sheet_total"]), _ptr(g["flow"]), _ptr(workspace),
        workspace.numel(), _stream()))
    if loss:
        g["loss"] = lv
    return g


def split_images(batch: PairBatch, images: torch.Tensor):
    """Views [2, H, W] of each pair's two frames in a packed image buffer."""
    out = []
    o = 0
    for (H, W) in batch.sizes:
        out.append(images[o:o + 2 * H * W].view(2, H, W))
        o += 2 * H * W
    return out


_IO_KEYS = ("flow", "x1", "y1", "x2", "y2", "z", "d", "I0", "images", "n_active", "ppp")


def _batch_io(io: dict, seed_value: int, pair_id_base: int):
    _need_cuda(*(io[k] for k in ("flow", "x1", "y1", "x2", "y2", "z", "d", "I0", "images")))
    b = L.BatchIO()
    for k in _IO_KEYS:
        t = io.get(k)
        setattr(b, k, t.data_ptr() if t is not None else None)
    b.seed = int(seed_value)
    b.pair_id_base = int(pair_id_base)
    return b


class Plan:
    """A batch signature captured once (``synthpix_plan_create``) and replayed
    as one HIP graph per call (``synthpix_plan_launch``).

    ``io`` holds the device tensors of the first launch: flow, x1, y1, x2, y2,
    z, d, I0, images and optionally n_active, ppp.  ``launch`` replays into the
    same tensors, or into new ones of the same sizes if given.  Every tensor a
    launch uses must stay alive until the stream has run it.
    """

    def __init__(self, batch: PairBatch, sp, seed_value: int, ap, rp, io: dict, autotune: bool = False,
                 advance_pair_ids: bool = False):
        self.io = dict(io)
        self.rp = rp
        self._b = _batch_io(io, seed_value, 0)
        h = ctypes.c_void_p(None)
        L.check(L.load().synthpix_plan_create(batch.host_ptr, batch.n_pairs, ctypes.byref(sp), ctypes.byref(ap),
                                              ctypes.byref(rp), ctypes.byref(self._b), 1 if autotune else 0,
                                              1 if advance_pair_ids else 0, _stream(), ctypes.byref(h)))
        self._h = h

    @property
    def tiling(self):
        t = L.Tiling()
        L.check(L.load().synthpix_plan_tiling(self._h, ctypes.byref(t)))
        return t

    def launch(self, io: Optional[dict] = None, seed_value: Optional[int] = None, pair_id_base: int = 0):
        """Replay the plan.  With ``io`` (and ``seed_value``), the launch reads and
        writes those tensors with that key and pair-id offset instead."""
        if io is None:
            L.check(L.load().synthpix_plan_launch(self._h, None, _stream()))
            return
        b = _batch_io(io, self._b.seed if seed_value is None else seed_value, pair_id_base)
        L.check(L.load().synthpix_plan_launch(self._h, ctypes.byref(b), _stream()))

    def read_status(self) -> int:
        flags = ctypes.c_uint32(0)
        st = L.load().synthpix_plan_read_status(self._h, _stream(), ctypes.byref(flags))
        if st not in (L.SP_OK, L.SP_ERR_DEVICE_STATUS):
            L.check(st)
        return flags.value

    def close(self):
        if self._h is not None and self._h.value:
            L.load().synthpix_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _RenderImages(torch.autograd.Function):
    """advect + render as one differentiable op: inputs flow, x1, y1, z, d, I0
    and the sheet width; output the float images.  The backward reuses the
    frame-2 positions and recomputes the rest (``synthpix_render_pair_backward``)."""

    @staticmethod
    def forward(ctx, flow, x1, y1, z, d, I0, sheet, batch, rp, tile):
        if rp.bits != 0:
            raise ValueError("differentiable rendering needs float images (bits = 0)")
        rp2 = L.RenderParams.from_buffer_copy(rp)
        rp2.sheet_sigma = float(sheet)
        x2, y2 = advect(batch, flow, rp2.advect, x1, y1)
        img = render_pair(batch, x1, y1, x2, y2, z, d, I0, rp2, tile)
        ctx.save_for_backward(flow, x1, y1, x2, y2, z, d, I0, sheet)
        ctx.batch, ctx.rp, ctx.tile = batch, rp2, tile
        return img

    @staticmethod
    def backward(ctx, grad):
        flow, x1, y1, x2, y2, z, d, I0, sheet = ctx.saved_tensors
        g = render_pair_backward(ctx.batch, flow, x1, y1, z, d, I0, ctx.rp, grad.contiguous(), ctx.tile,
                                 x2=x2, y2=y2)
        g_sheet = g["sheet_total"].to(sheet.dtype).reshape(sheet.shape)
        return g["flow"], g["x1"], g["y1"], g["z"], g["d"], g["I0"], g_sheet, None, None, None


def render_images(batch: PairBatch, flow, x1, y1, z, d, I0, sheet, rp, tile=None):
    """Differentiable float images of every pair (autograd through the HIP
    backward).  ``sheet`` is a 0-d tensor holding the sheet width; ``rp``
    supplies everything else (its advect member sets the integrator)."""
    if not torch.is_tensor(sheet):
        sheet = torch.tensor(float(sheet), dtype=torch.float32, device=x1.device)
    return _RenderImages.apply(flow, x1, y1, z, d, I0, sheet, batch, rp, tile)
