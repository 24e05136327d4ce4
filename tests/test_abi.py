"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point the header declares, and rejects invalid arguments before
enqueuing anything."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "synthpix.h")


@pytest.fixture(scope="module")
def L():
    from paper_2512_09664_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2512_09664_amd import build
        build.build()
    return _lib


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(synthpix_[a-z_]+)\s*\(", text)))


def test_header_declares_the_hot_path_calls():
    syms = declared_symbols()
    for name in ("synthpix_seed", "synthpix_advect", "synthpix_render_pair", "synthpix_render_pair_backward"):
        assert name in syms


def test_library_exports_every_declared_symbol(L):
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(declared_symbols()) <= set(L.SIGNATURES), "binding lacks a declared symbol"


def test_particle_count_and_errors(L):
    lib = L.load()
    n = ctypes.c_int32()
    assert lib.synthpix_particle_count(256, 256, 0.02, ctypes.byref(n)) == 0 and n.value == 1311
    assert lib.synthpix_particle_count(1024, 1024, 0.05, ctypes.byref(n)) == 0 and n.value == 52429
    assert lib.synthpix_particle_count(0, 5, 0.1, ctypes.byref(n)) == L.SP_ERR_INVALID_ARG
    assert lib.synthpix_particle_count(5, 5, 1.5, ctypes.byref(n)) == L.SP_ERR_INVALID_ARG
    assert b"ppp" in lib.synthpix_last_error()


def _pairs(L, specs):
    arr = (L.Pair * len(specs))()
    po = 0
    for p, (H, W, Gh, Gw, n) in enumerate(specs):
        arr[p].H, arr[p].W, arr[p].Gh, arr[p].Gw, arr[p].n_max = H, W, Gh, Gw, n
        arr[p].particle_offset = po
        po += n
    return arr


def _rp(L, **kw):
    rp = L.RenderParams()
    rp.sheet_sigma, rp.d_max, rp.blur_radius, rp.blur_sigma, rp.noise_sigma, rp.bits = 0.5, 5.0, 1, 0.7, 0.0, 12
    for k, v in kw.items():
        setattr(rp, k, v)
    return rp


def test_workspace_size_and_validation(L):
    lib = L.load()
    pairs = _pairs(L, [(1024, 1024, 256, 256, 52429), (256, 512, 64, 128, 6554)])
    n = ctypes.c_size_t()
    assert lib.synthpix_workspace_size(pairs, 2, ctypes.byref(_rp(L)), None, 0, ctypes.byref(n)) == 0
    fwd = n.value
    assert fwd > 0 and fwd % 256 == 0
    assert lib.synthpix_workspace_size(pairs, 2, ctypes.byref(_rp(L)), None, 1, ctypes.byref(n)) == 0
    # the backward is particle-major: five floats per particle plus 64-bit flow sums, no bins
    assert n.value >= 5 * 4 * (52429 + 6554) + 8 * 2 * 256 * 256   # both grids at flow_offset 0
    assert n.value % 256 == 0
    bad = [dict(sheet_sigma=0.0), dict(d_max=0.0), dict(d_max=17.0), dict(blur_radius=4),
           dict(blur_radius=1, blur_sigma=0.0), dict(noise_sigma=-1.0), dict(bits=17)]
    for kw in bad:
        assert lib.synthpix_workspace_size(pairs, 2, ctypes.byref(_rp(L, **kw)), None, 0,
                                           ctypes.byref(n)) == L.SP_ERR_INVALID_ARG, kw
    t = L.Tiling(24, 32, 4096, 128)
    assert lib.synthpix_workspace_size(pairs, 2, ctypes.byref(_rp(L)), ctypes.byref(t), 0,
                                       ctypes.byref(n)) == L.SP_ERR_INVALID_ARG
    big = _pairs(L, [(16384, 16384, 64, 64, 10)])
    assert lib.synthpix_workspace_size(big, 1, ctypes.byref(_rp(L)), None, 0,
                                       ctypes.byref(n)) == L.SP_ERR_UNSUPPORTED


@pytest.mark.parametrize("field,value", [("H", 0), ("W", 20000), ("Gh", 1), ("n_max", -1), ("reserved", 3)])
def test_pair_table_validation(L, field, value):
    lib = L.load()
    pairs = _pairs(L, [(64, 64, 16, 16, 100)])
    setattr(pairs[0], field, value)
    sp_ = L.SeedParams(0.02, 0.02, 0, 1.0, 2.0, 0, 0, 0.8, 1.0, -1, 1)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    st = lib.synthpix_seed(pairs, fake, 1, ctypes.byref(sp_), 0, fake, fake, fake, fake, fake, None, None, None)
    assert st == L.SP_ERR_INVALID_ARG
    assert lib.synthpix_last_error()


def test_seed_parameter_validation(L):
    lib = L.load()
    pairs = _pairs(L, [(64, 64, 16, 16, 82)])
    fake = ctypes.c_void_p(0x1000)
    cases = [L.SeedParams(0.0, 0.02, 0, 1.0, 2.0, 0, 0, 0.8, 1.0, -1, 1),     # ppp_lo = 0
             L.SeedParams(0.03, 0.02, 0, 1.0, 2.0, 0, 0, 0.8, 1.0, -1, 1),    # lo > hi
             L.SeedParams(0.02, 0.02, 5, 1.0, 2.0, 0, 0, 0.8, 1.0, -1, 1),    # unknown distribution
             L.SeedParams(0.02, 0.02, 0, -1.0, 2.0, 0, 0, 0.8, 1.0, -1, 1),   # d <= 0
             L.SeedParams(0.02, 0.02, 1, 2.5, 0.5, 0.0, 5.0, 0.8, 1.0, -1, 1),  # clip lo = 0
             L.SeedParams(0.02, 0.02, 0, 1.0, 2.0, 0, 0, 1.0, 0.8, -1, 1),    # I0 lo > hi
             L.SeedParams(0.02, 0.03, 0, 1.0, 2.0, 0, 0, 0.8, 1.0, -1, 1)]    # n_max != rule(ppp_hi)
    for c in cases:
        assert lib.synthpix_seed(pairs, fake, 1, ctypes.byref(c), 0, fake, fake, fake, fake, fake, None, None,
                                 None) == L.SP_ERR_INVALID_ARG
    good = L.SeedParams(0.02, 0.02, 0, 1.0, 2.0, 0, 0, 0.8, 1.0, -1, 1)
    assert lib.synthpix_seed(pairs, fake, 1, ctypes.byref(good), 0, None, fake, fake, fake, fake, None, None,
                             None) == L.SP_ERR_INVALID_ARG   # NULL output


def test_advect_and_render_validation(L):
    lib = L.load()
    pairs = _pairs(L, [(64, 64, 16, 16, 100)])
    fake = ctypes.c_void_p(0x1000)
    ap = L.AdvectParams(1.0, 0, 1)
    assert lib.synthpix_advect(pairs, fake, 1, fake, ctypes.byref(ap), fake, fake, ctypes.c_void_p(0x2000),
                               ctypes.c_void_p(0x3000), None, None, None, None, 0, None) == L.SP_ERR_INVALID_ARG
    ap = L.AdvectParams(1.0, 4, 7)
    assert lib.synthpix_advect(pairs, fake, 1, fake, ctypes.byref(ap), fake, fake, ctypes.c_void_p(0x2000),
                               ctypes.c_void_p(0x3000), None, None, None, None, 0, None) == L.SP_ERR_INVALID_ARG
    ap = L.AdvectParams(1.0, 4, 1)
    assert lib.synthpix_advect(pairs, fake, 1, fake, ctypes.byref(ap), fake, fake, fake, ctypes.c_void_p(0x3000),
                               None, None, None, None, 0, None) == L.SP_ERR_INVALID_ARG   # aliasing
    n = ctypes.c_size_t()
    assert lib.synthpix_advect_workspace_size(pairs, 1, ctypes.byref(n)) == 0 and n.value >= 4 * 100
    assert lib.synthpix_advect(pairs, fake, 1, fake, ctypes.byref(ap), fake, fake, ctypes.c_void_p(0x2000),
                               ctypes.c_void_p(0x3000), None, None, None, ctypes.c_void_p(0x10000), n.value - 1,
                               None) == L.SP_ERR_WORKSPACE
    assert lib.synthpix_advect(pairs, fake, 1, fake, ctypes.byref(ap), fake, fake, ctypes.c_void_p(0x2000),
                               ctypes.c_void_p(0x3000), None, None, None, ctypes.c_void_p(0x10010), n.value,
                               None) == L.SP_ERR_WORKSPACE
    wsz = ctypes.c_size_t()
    assert lib.synthpix_workspace_size(pairs, 1, ctypes.byref(_rp(L)), None, 0, ctypes.byref(wsz)) == 0
    assert wsz.value >= n.value
    # workspace too small / misaligned
    rp = _rp(L)
    st = lib.synthpix_render_pair(pairs, fake, 1, None, fake, fake, fake, fake, fake, fake, fake, None, ctypes.byref(rp),
                                  fake, ctypes.c_void_p(0x10000), 256, None)
    assert st == L.SP_ERR_WORKSPACE
    st = lib.synthpix_render_pair(pairs, fake, 1, None, fake, fake, fake, fake, fake, fake, fake, None, ctypes.byref(rp),
                                  fake, ctypes.c_void_p(0x10010), 1 << 30, None)
    assert st == L.SP_ERR_WORKSPACE
    # overlapping particle ranges
    two = _pairs(L, [(64, 64, 16, 16, 100), (64, 64, 16, 16, 100)])
    two[1].particle_offset = 50
    assert lib.synthpix_render_pair(two, fake, 2, None, fake, fake, fake, fake, fake, fake, fake, None,
                                    ctypes.byref(rp), fake, ctypes.c_void_p(0x10000), 1 << 30,
                                    None) == L.SP_ERR_INVALID_ARG


def test_plan_validation(L):
    """synthpix_plan_create refuses what the eager calls refuse (seed, advect and
    render parameters, io pointers) before touching the device."""
    lib = L.load()
    pairs = _pairs(L, [(64, 64, 16, 16, 82)])
    sp = L.SeedParams(0.02, 0.02, 0, 1.0, 5.0, 0.0, 0.0, 0.8, 1.0, -1.0, 1.0)
    ap = L.AdvectParams(1.0, 1, 0)
    rp = _rp(L)
    fake = [0x1000 * (k + 1) for k in range(9)]
    io = L.BatchIO(*fake)
    h = ctypes.c_void_p()

    def create(pairs_=pairs, n=1, sp_=sp, ap_=ap, rp_=rp, io_=io, out=ctypes.byref(h)):
        return lib.synthpix_plan_create(pairs_, n, ctypes.byref(sp_) if sp_ is not None else None,
                                        ctypes.byref(ap_) if ap_ is not None else None, ctypes.byref(rp_),
                                        ctypes.byref(io_) if io_ is not None else None, 0, 0, None, out)

    assert create(out=None) == L.SP_ERR_INVALID_ARG
    assert create(io_=None) == L.SP_ERR_INVALID_ARG
    assert create(n=0) == L.SP_ERR_INVALID_ARG
    assert create(sp_=None) == L.SP_ERR_INVALID_ARG
    assert create(ap_=None) == L.SP_ERR_INVALID_ARG
    bad_io = L.BatchIO(*fake)
    bad_io.flow = None
    assert create(io_=bad_io) == L.SP_ERR_INVALID_ARG
    bad_io = L.BatchIO(*fake)
    bad_io.flow = 0x1004                                # not 8-byte aligned
    assert create(io_=bad_io) == L.SP_ERR_INVALID_ARG
    assert b"flow" in lib.synthpix_last_error()
    bad_io = L.BatchIO(*fake)
    bad_io.x2 = bad_io.x1                               # aliasing
    assert create(io_=bad_io) == L.SP_ERR_INVALID_ARG
    bad_rp = _rp(L)
    bad_rp.bits = 17
    assert create(rp_=bad_rp) == L.SP_ERR_INVALID_ARG
    for bad_ap in (L.AdvectParams(1.0, 1, 7), L.AdvectParams(1.0, 0, 0), L.AdvectParams(float("nan"), 1, 0)):
        assert create(ap_=bad_ap) == L.SP_ERR_INVALID_ARG
    for bad_sp in (L.SeedParams(0.02, 0.03, 0, 1.0, 5.0, 0.0, 0.0, 0.8, 1.0, -1.0, 1.0),   # n_max rule
                   L.SeedParams(0.0, 0.02, 0, 1.0, 5.0, 0.0, 0.0, 0.8, 1.0, -1.0, 1.0),    # ppp_lo = 0
                   L.SeedParams(0.02, 0.02, 9, 1.0, 5.0, 0.0, 0.0, 0.8, 1.0, -1.0, 1.0)):  # distribution
        assert create(sp_=bad_sp) == L.SP_ERR_INVALID_ARG
    assert not h.value
    assert lib.synthpix_plan_launch(None, None, None) == L.SP_ERR_INVALID_ARG
    assert lib.synthpix_plan_tiling(None, None) == L.SP_ERR_INVALID_ARG
    flags = ctypes.c_uint32()
    assert lib.synthpix_plan_read_status(None, None, ctypes.byref(flags)) == L.SP_ERR_INVALID_ARG
    assert lib.synthpix_plan_destroy(None) == L.SP_OK


def test_tiling_candidates(L):
    """The autotuner's candidate list: the default first, every entry a valid,
    compiled tiling, the binning block sizes after the shapes."""
    lib = L.load()
    rp = _rp(L)
    n = ctypes.c_int32()
    assert lib.synthpix_tiling_candidates(ctypes.byref(rp), None, 0, ctypes.byref(n)) == 0
    assert n.value >= 10
    arr = (L.Tiling * n.value)()
    assert lib.synthpix_tiling_candidates(ctypes.byref(rp), arr, n.value, ctypes.byref(n)) == 0
    d = L.Tiling()
    assert lib.synthpix_default_tiling(None, 0, ctypes.byref(rp), ctypes.byref(d)) == 0
    assert (arr[0].tile_w, arr[0].tile_h, arr[0].chunk, arr[0].cap) == (d.tile_w, d.tile_h, d.chunk, d.cap)
    pairs = _pairs(L, [(256, 256, 64, 64, 1311)])
    chunks = set()
    for t in arr:
        size = ctypes.c_size_t()
        assert lib.synthpix_workspace_size(pairs, 1, ctypes.byref(rp), ctypes.byref(t), 0, ctypes.byref(size)) == 0
        chunks.add(t.chunk)
    assert chunks >= {1024, 2048, 4096, 8192}
    assert [t.persistent for t in arr].count(1) == 1 and arr[n.value - 1].persistent == 1
    bad = _rp(L, sheet_sigma=-1.0)
    assert lib.synthpix_tiling_candidates(ctypes.byref(bad), arr, n.value, ctypes.byref(n)) == L.SP_ERR_INVALID_ARG


def test_backward_validation(L):
    lib = L.load()
    pairs = _pairs(L, [(64, 64, 16, 16, 100)])
    fake = ctypes.c_void_p(0x1000)
    rp = _rp(L)
    n = ctypes.c_size_t()
    assert lib.synthpix_workspace_size(pairs, 1, ctypes.byref(rp), None, 1, ctypes.byref(n)) == 0
    # status + kmax + five per-particle float arrays + the fixed-point flow grid
    assert n.value >= 5 * 4 * 100 + 8 * 2 * 16 * 16
    args = [pairs, fake, 1, None, fake, fake, fake, None, None] + [fake] * 3

    def call(rp_, ws=ctypes.c_void_p(0x100000), nbytes=1 << 30, grad=fake, total=None):
        return lib.synthpix_render_pair_backward(*args, ctypes.byref(rp_), grad, fake, fake, fake, fake, fake,
                                                 fake, total, fake, ws, nbytes, None)

    rp.bits = 12
    assert call(rp) == L.SP_ERR_UNSUPPORTED
    rp.bits = 0
    rp.advect.substeps = 0
    assert call(rp) == L.SP_ERR_INVALID_ARG
    rp.advect.substeps = 2
    assert call(rp, grad=None) == L.SP_ERR_INVALID_ARG
    assert call(rp, nbytes=n.value - 1) == L.SP_ERR_WORKSPACE
    assert call(rp, ws=ctypes.c_void_p(0x100010)) == L.SP_ERR_WORKSPACE
    assert call(rp, total=ctypes.c_void_p(0x1002)) == L.SP_ERR_INVALID_ARG     # misaligned shared-sheet output
    half = [pairs, fake, 1, None, fake, fake, fake, fake, None] + [fake] * 3   # x2 without y2
    assert lib.synthpix_render_pair_backward(*half, ctypes.byref(rp), fake, fake, fake, fake, fake, fake, fake,
                                             None, fake, ctypes.c_void_p(0x100000), 1 << 30,
                                             None) == L.SP_ERR_INVALID_ARG


def test_backward_mse_validation(L):
    """The loss-fused backward checks its arguments and its own (larger)
    workspace size before enqueueing anything."""
    lib = L.load()
    pairs = _pairs(L, [(64, 64, 16, 16, 100)])
    fake = ctypes.c_void_p(0x1000)
    rp = _rp(L, bits=0)
    rp.advect.substeps = 2
    n1, n2 = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.synthpix_workspace_size(pairs, 1, ctypes.byref(rp), None, 1, ctypes.byref(n1)) == 0
    assert lib.synthpix_workspace_size(pairs, 1, ctypes.byref(rp), None, 2, ctypes.byref(n2)) == 0
    # the per-pixel pass's images (2 x 64 x 64 floats) and its loss partials
    assert n2.value >= n1.value + 4 * 2 * 64 * 64 and n2.value % 256 == 0
    for bad in (-1, 3):
        assert lib.synthpix_workspace_size(pairs, 1, ctypes.byref(rp), None, bad,
                                           ctypes.byref(n1)) == L.SP_ERR_INVALID_ARG
    args = [pairs, fake, 1, None, fake, fake, fake, None, None] + [fake] * 3

    def call(images=fake, target=fake, scale=1.0, loss=None, nbytes=n2.value, rp_=rp):
        return lib.synthpix_render_pair_backward_mse(*args, ctypes.byref(rp_), images, target, scale, loss, fake,
                                                     fake, fake, fake, fake, fake, None, fake,
                                                     ctypes.c_void_p(0x100000), nbytes, None)

    assert call(images=None) == L.SP_ERR_INVALID_ARG
    assert call(target=ctypes.c_void_p(0x1002)) == L.SP_ERR_INVALID_ARG
    assert call(scale=float("nan")) == L.SP_ERR_INVALID_ARG
    assert call(loss=ctypes.c_void_p(0x2004)) == L.SP_ERR_INVALID_ARG
    assert call(nbytes=n2.value - 1) == L.SP_ERR_WORKSPACE
    coded = _rp(L, bits=12)
    coded.advect.substeps = 2
    assert call(rp_=coded) == L.SP_ERR_UNSUPPORTED


def test_mse_grad_validation(L):
    """The loss-gradient call checks its arguments before enqueueing anything."""
    lib = L.load()
    fake = ctypes.c_void_p(0x1000)
    ws_n = lib.synthpix_mse_workspace_size(1 << 20)
    assert ws_n >= 8 * 1024 and ws_n % 256 == 0
    ws = ctypes.c_void_p(0x100000)
    assert lib.synthpix_mse_grad(fake, fake, -1, 1.0, fake, None, None, 0, None) == L.SP_ERR_INVALID_ARG
    assert lib.synthpix_mse_grad(None, fake, 8, 1.0, fake, None, None, 0, None) == L.SP_ERR_INVALID_ARG
    assert lib.synthpix_mse_grad(None, None, 0, 1.0, None, None, None, 0, None) == 0      # nothing to do
    assert lib.synthpix_mse_grad(fake, ctypes.c_void_p(0x1004), 8, 1.0, fake, None, None, 0,
                                 None) == L.SP_ERR_INVALID_ARG                        # misaligned target
    assert lib.synthpix_mse_grad(fake, fake, 8, float("inf"), fake, None, None, 0, None) == L.SP_ERR_INVALID_ARG
    assert lib.synthpix_mse_grad(fake, fake, 8, 1.0, fake, ctypes.c_void_p(0x2004), ws, ws_n,
                                 None) == L.SP_ERR_INVALID_ARG                        # misaligned loss
    assert lib.synthpix_mse_grad(fake, fake, 8, 1.0, fake, ctypes.c_void_p(0x2000), None, 0,
                                 None) == L.SP_ERR_WORKSPACE
    assert lib.synthpix_mse_grad(fake, fake, 8, 1.0, fake, ctypes.c_void_p(0x2000), ws, ws_n - 1,
                                 None) == L.SP_ERR_WORKSPACE


def test_model_validation(L):
    """The full model's parameters and inputs are checked on the host before
    anything is enqueued."""
    lib = L.load()
    pairs = _pairs(L, [(64, 64, 16, 16, 100)])
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x10000)

    def render(rp, ex=None):
        return lib.synthpix_render_pair(pairs, fake, 1, None, fake, fake, fake, fake, fake, fake, fake,
                                        ctypes.byref(ex) if ex is not None else None, ctypes.byref(rp), fake, ws,
                                        1 << 30, None)

    for field, value in (("hide_p", 1.5), ("hide_p", -0.1), ("jitter_d", -1.0), ("jitter_rho", float("nan")),
                         ("jitter_I0", float("inf")), ("sheet_law", 7)):
        rp = _rp(L)
        setattr(rp, field, value)
        assert render(rp) == L.SP_ERR_INVALID_ARG, field
    rp = _rp(L)
    rp.sheet_law = L.SP_SHEET_REMARK1
    rp.sheet_dz0, rp.sheet_shape = 0.0, 2.0
    assert render(rp) == L.SP_ERR_INVALID_ARG
    rp.sheet_dz0, rp.sheet_shape = 1.0, 0.0
    assert render(rp) == L.SP_ERR_INVALID_ARG
    ex = L.ParticleExtras(0x1002, None, None)           # misaligned d_y
    assert render(_rp(L), ex) == L.SP_ERR_INVALID_ARG
    # 3-D motion needs wflow, z1 and z2 together, z2 not aliasing z1
    ap = L.AdvectParams(1.0, 1, 0)
    a2, a3 = ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    assert lib.synthpix_advect(pairs, fake, 1, fake, ctypes.byref(ap), fake, fake, a2, a3, fake, None, None, None,
                               0, None) == L.SP_ERR_INVALID_ARG
    assert lib.synthpix_advect(pairs, fake, 1, fake, ctypes.byref(ap), fake, fake, a2, a3, fake,
                               ctypes.c_void_p(0x4000), ctypes.c_void_p(0x4000), None, 0,
                               None) == L.SP_ERR_INVALID_ARG
    # the shape draws' correlation range
    sp = L.SeedParams(0.02, 0.02, 0, 1.0, 2.0, 0, 0, 0.8, 1.0, -1, 1)
    pairs82 = _pairs(L, [(64, 64, 16, 16, 82)])
    for lo, hi in ((-1.0, 0.5), (0.2, 0.1), (0.0, 0.995)):
        assert lib.synthpix_seed_shape(pairs82, fake, 1, ctypes.byref(sp), lo, hi, 0, fake, a2,
                                       None) == L.SP_ERR_INVALID_ARG
    # the backward differentiates the isotropic model only
    rp = _rp(L)
    rp.hide_p = 0.1
    assert lib.synthpix_render_pair_backward(pairs, fake, 1, None, fake, fake, fake, None, None, fake, fake, fake,
                                             ctypes.byref(rp), fake, fake, fake, fake, fake, fake, fake, None, fake,
                                             ws, 1 << 30, None) == L.SP_ERR_UNSUPPORTED
