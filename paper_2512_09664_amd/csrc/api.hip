// C ABI of the generator: host-side validation, workspace sizing and kernel
// enqueueing.  See include/synthpix.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "launch.hpp"
#include "synthpix.h"

namespace {

thread_local std::string g_err;

synthpix_status fail(synthpix_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

synthpix_status hip_fail(hipError_t e, const char* what)
{
    return fail(SP_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Pair-table checks shared by every entry point.
synthpix_status check_pairs(const synthpix_pair* ph, const synthpix_pair* pd, int32_t n_pairs,
                            int64_t* n_span)
{
    if (n_pairs <= 0) return fail(SP_ERR_INVALID_ARG, "n_pairs must be positive (got %d)", n_pairs);
    if (!ph || !pd) return fail(SP_ERR_INVALID_ARG, "pairs_host and pairs_dev must be non-NULL");
    if (!aligned(pd, 8)) return fail(SP_ERR_INVALID_ARG, "pairs_dev must be 8-byte aligned");
    int64_t end_prev = 0, span = 0;
    for (int32_t p = 0; p < n_pairs; ++p) {
        const synthpix_pair& P = ph[p];
        if (P.H < 1 || P.W < 1 || P.H > 16384 || P.W > 16384)
            return fail(SP_ERR_INVALID_ARG, "pair %d: H, W must be in [1, 16384] (got %d x %d)", p, P.H, P.W);
        if (P.Gh < 2 || P.Gw < 2 || P.Gh > 8192 || P.Gw > 8192)
            return fail(SP_ERR_INVALID_ARG, "pair %d: flow grid must be in [2, 8192]^2 (got %d x %d)", p, P.Gh,
                        P.Gw);
        if (P.n_max < 0) return fail(SP_ERR_INVALID_ARG, "pair %d: n_max must be >= 0", p);
        if (P.reserved != 0) return fail(SP_ERR_INVALID_ARG, "pair %d: reserved field must be 0", p);
        if (P.particle_offset < end_prev)
            return fail(SP_ERR_INVALID_ARG,
                        "pair %d: particle ranges must be ascending and disjoint (offset %lld < %lld)", p,
                        (long long)P.particle_offset, (long long)end_prev);
        if (P.image_offset < 0 || P.flow_offset < 0 || (P.flow_offset & 1))
            return fail(SP_ERR_INVALID_ARG, "pair %d: offsets must be >= 0 and flow_offset even", p);
        end_prev = P.particle_offset + P.n_max;
        span = end_prev > span ? end_prev : span;
    }
    if (span >= ((int64_t)1 << 40)) return fail(SP_ERR_INVALID_ARG, "particle span too large");
    *n_span = span;
    return SP_OK;
}

bool dev_ptr_ok(const void* p) { return p && aligned(p, 4); }

synthpix_status check_render_params(const synthpix_render_params* rp)
{
    if (!rp) return fail(SP_ERR_INVALID_ARG, "render params must be non-NULL");
    if (!(rp->sheet_sigma > 0.0f) || !std::isfinite(rp->sheet_sigma))
        return fail(SP_ERR_INVALID_ARG, "sheet_sigma must be positive and finite");
    if (!(rp->d_max > 0.0f) || !(rp->d_max <= 16.0f))
        return fail(SP_ERR_INVALID_ARG, "d_max must be in (0, 16] (got %g)", (double)rp->d_max);
    if (rp->blur_radius < 0 || rp->blur_radius > 3)
        return fail(SP_ERR_INVALID_ARG, "blur_radius must be in [0, 3]");
    if (rp->blur_radius > 0 && !(rp->blur_sigma > 0.0f && std::isfinite(rp->blur_sigma)))
        return fail(SP_ERR_INVALID_ARG, "blur_sigma must be positive when blur is on");
    if (!(rp->noise_sigma >= 0.0f) || !std::isfinite(rp->noise_sigma))
        return fail(SP_ERR_INVALID_ARG, "noise_sigma must be >= 0 and finite");
    if (rp->bits < 0 || rp->bits > 16) return fail(SP_ERR_INVALID_ARG, "bits must be in [0, 16]");
    return SP_OK;
}

synthpix_status check_tiling(const synthpix_tiling& t)
{
    if (!sp::render_shape_supported(t.tile_w, t.tile_h))
        return fail(SP_ERR_INVALID_ARG, "tile %d x %d is not one of the compiled shapes (8x8, 16x16, 32x16, 32x32, "
                    "64x16, 64x32, 64x64, 128x32)", t.tile_w, t.tile_h);
    if (t.chunk < 256 || t.chunk > 16384 || (t.chunk & 255))
        return fail(SP_ERR_INVALID_ARG, "chunk must be a multiple of 256 in [256, 16384]");
    if (t.cap < 32 || t.cap > 256) return fail(SP_ERR_INVALID_ARG, "cap must be in [32, 256]");
    return SP_OK;
}

// Normalised Gaussian taps in float64, rounded to binary32 once.
void blur_taps(int b, float sigma, float* w)
{
    double g[7], s = 0.0;
    for (int k = -b; k <= b; ++k) {
        g[k + b] = std::exp(-(double)(k * k) / (2.0 * (double)sigma * (double)sigma));
        s += g[k + b];
    }
    for (int k = 0; k < 7; ++k) w[k] = k <= 2 * b ? (float)(g[k] / s) : 0.0f;
}

sp::RenderConfig make_config(const synthpix_render_params& rp, const synthpix_tiling& t)
{
    sp::RenderConfig c;
    c.tile_w = t.tile_w;
    c.tile_h = t.tile_h;
    c.chunk = t.chunk;
    c.cap = t.cap;
    c.apron = rp.blur_radius;
    c.d_max = rp.d_max;
    c.log_tw = 0;
    while ((1 << c.log_tw) < c.tile_w) ++c.log_tw;
    c.log_th = 0;
    while ((1 << c.log_th) < c.tile_h) ++c.log_th;
    const int span = (int)std::floor(3.0 * (double)rp.d_max) + 4;   // patch side bound incl. rounding
    const int RW = c.tile_w + 2 * c.apron, RH = c.tile_h + 2 * c.apron;
    c.wmax = span < (RW > RH ? RW : RH) ? span : (RW > RH ? RW : RH);
    c.wm4 = (c.wmax + 3) & ~3;
    c.kx = (span + 2 * c.apron) / c.tile_w + 2;
    c.ky = (span + 2 * c.apron) / c.tile_h + 2;
    return c;
}

synthpix_status batch_totals(const synthpix_pair* ph, int32_t n_pairs, const sp::RenderConfig& c,
                             sp::BatchTotals* tot)
{
    sp::BatchTotals T{};
    for (int32_t p = 0; p < n_pairs; ++p) {
        const synthpix_pair& P = ph[p];
        const int64_t n_chunks = (P.n_max + c.chunk - 1) / c.chunk;
        const int64_t nt = (int64_t)((P.W + c.tile_w - 1) / c.tile_w) * ((P.H + c.tile_h - 1) / c.tile_h);
        const int64_t cap = (int64_t)P.n_max * c.kx * c.ky;
        if (nt > 16384)
            return fail(SP_ERR_UNSUPPORTED, "pair %d has %lld tiles; at most 16384 per image (use larger tiles)", p,
                        (long long)nt);
        if (cap >= ((int64_t)1 << 31))
            return fail(SP_ERR_UNSUPPORTED, "pair %d: too many tile entries for 32-bit slots", p);
        T.n_span = std::max<int64_t>(T.n_span, P.particle_offset + P.n_max);
        T.chunks += n_chunks;
        T.tiles += nt;
        T.hist += 2 * n_chunks * nt;
        T.entries += 2 * cap;
        T.max_tiles = std::max<int64_t>(T.max_tiles, nt);
    }
    if (T.chunks >= 65536 * 32768LL || T.tiles * 2 >= ((int64_t)1 << 31))
        return fail(SP_ERR_UNSUPPORTED, "batch too large for one launch");
    *tot = T;
    return SP_OK;
}

sp::WorkspaceLayout workspace_layout(int32_t n_pairs, const sp::BatchTotals& T, int backward,
                                     const synthpix_pair* ph)
{
    sp::WorkspaceLayout w{};
    size_t o = 0;
    w.status = o; o = align256(o + 16);
    w.layout = o; o = align256(o + sizeof(sp::PairLayout) * (size_t)n_pairs);
    w.tile_count = o; o = align256(o + sizeof(uint32_t) * 2 * (size_t)T.tiles);
    w.tile_offset = o; o = align256(o + sizeof(int64_t) * 2 * (size_t)T.tiles);
    w.hist = o; o = align256(o + sizeof(uint32_t) * (size_t)T.hist);
    w.entries = o; o = align256(o + sizeof(int32_t) * (size_t)T.entries);
    w.records = o; o = align256(o + 2 * 16 * (size_t)T.n_span);
    if (backward) {
        size_t px = 0;
        for (int32_t p = 0; p < n_pairs; ++p) px += 2 * (size_t)ph[p].H * ph[p].W;
        w.grad_img = o; o = align256(o + sizeof(float) * px);
        w.x2 = o; o = align256(o + sizeof(float) * (size_t)T.n_span);
        w.y2 = o; o = align256(o + sizeof(float) * (size_t)T.n_span);
        w.gpart = o; o = align256(o + sizeof(float) * 8 * (size_t)T.n_span);
    }
    w.total = o;
    return w;
}

synthpix_tiling default_tiling()
{
    synthpix_tiling t;
    t.tile_w = 64;
    t.tile_h = 32;
    t.chunk = 4096;
    t.cap = 64;
    return t;
}

}  // namespace

extern "C" {

int32_t synthpix_version(void) { return SYNTHPIX_VERSION; }

const char* synthpix_last_error(void) { return g_err.c_str(); }

synthpix_status synthpix_particle_count(int32_t H, int32_t W, double ppp, int32_t* n_out)
{
    if (!n_out) return fail(SP_ERR_INVALID_ARG, "n_out must be non-NULL");
    if (H < 1 || W < 1) return fail(SP_ERR_INVALID_ARG, "H and W must be positive");
    if (!(ppp >= 0.0 && ppp <= 1.0)) return fail(SP_ERR_INVALID_ARG, "ppp must be in [0, 1]");
    *n_out = (int32_t)std::floor((double)H * (double)W * ppp + 0.5);
    return SP_OK;
}

synthpix_status synthpix_default_tiling(const synthpix_pair* pairs_host, int32_t n_pairs,
                                        const synthpix_render_params* rp, synthpix_tiling* out)
{
    if (!out) return fail(SP_ERR_INVALID_ARG, "out must be non-NULL");
    (void)pairs_host;
    (void)n_pairs;
    (void)rp;
    *out = default_tiling();
    return SP_OK;
}

synthpix_status synthpix_workspace_size(const synthpix_pair* pairs_host, int32_t n_pairs,
                                        const synthpix_render_params* rp, const synthpix_tiling* tiling,
                                        int32_t backward, size_t* bytes_out)
{
    if (!bytes_out) return fail(SP_ERR_INVALID_ARG, "bytes_out must be non-NULL");
    int64_t span;
    synthpix_status st = check_pairs(pairs_host, pairs_host, n_pairs, &span);
    if (st) return st;
    if ((st = check_render_params(rp))) return st;
    const synthpix_tiling t = tiling ? *tiling : default_tiling();
    if ((st = check_tiling(t))) return st;
    const sp::RenderConfig cfg = make_config(*rp, t);
    sp::BatchTotals T;
    if ((st = batch_totals(pairs_host, n_pairs, cfg, &T))) return st;
    *bytes_out = workspace_layout(n_pairs, T, backward ? 1 : 0, pairs_host).total;
    return SP_OK;
}

synthpix_status synthpix_timing_enable(int32_t on)
{
    sp::timing_enable(on != 0);
    return SP_OK;
}

synthpix_status synthpix_timing_read(const char* name, double* total_ms, int64_t* launches)
{
    if (!total_ms || !launches) return fail(SP_ERR_INVALID_ARG, "total_ms and launches must be non-NULL");
    if (sp::timing_read(name, total_ms, launches) != 0) return fail(SP_ERR_HIP, "reading timing events failed");
    return SP_OK;
}

synthpix_status synthpix_bin_views_of(const synthpix_pair* pairs_host, int32_t n_pairs,
                                      const synthpix_render_params* rp, const synthpix_tiling* tiling,
                                      synthpix_bin_views* out)
{
    if (!out) return fail(SP_ERR_INVALID_ARG, "out must be non-NULL");
    int64_t span;
    synthpix_status st = check_pairs(pairs_host, pairs_host, n_pairs, &span);
    if (st) return st;
    if ((st = check_render_params(rp))) return st;
    const synthpix_tiling t = tiling ? *tiling : default_tiling();
    if ((st = check_tiling(t))) return st;
    const sp::RenderConfig cfg = make_config(*rp, t);
    sp::BatchTotals T;
    if ((st = batch_totals(pairs_host, n_pairs, cfg, &T))) return st;
    const sp::WorkspaceLayout wl = workspace_layout(n_pairs, T, 0, pairs_host);
    out->tile_count = wl.tile_count;
    out->tile_offset = wl.tile_offset;
    out->entries = wl.entries;
    out->tiles = T.tiles;
    return SP_OK;
}

synthpix_status synthpix_read_status(const void* workspace_dev, void* stream, uint32_t* flags)
{
    if (!workspace_dev || !flags) return fail(SP_ERR_INVALID_ARG, "workspace and flags must be non-NULL");
    uint32_t w[4];
    hipError_t e = hipMemcpyAsync(w, workspace_dev, sizeof w, hipMemcpyDeviceToHost, as_stream(stream));
    if (e == hipSuccess) e = hipStreamSynchronize(as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "reading the status word");
    *flags = w[0];
    if (w[0]) return fail(SP_ERR_DEVICE_STATUS, "device status flags 0x%x", w[0]);
    return SP_OK;
}

synthpix_status synthpix_seed(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev, int32_t n_pairs,
                              const synthpix_seed_params* sp_, uint64_t seed, float* x, float* y, float* z,
                              float* d, float* I0, int32_t* n_active_dev, double* ppp_dev, void* stream)
{
    int64_t span;
    synthpix_status st = check_pairs(pairs_host, pairs_dev, n_pairs, &span);
    if (st) return st;
    if (!sp_) return fail(SP_ERR_INVALID_ARG, "seed params must be non-NULL");
    const synthpix_seed_params& q = *sp_;
    if (!(q.ppp_lo > 0.0 && q.ppp_lo <= q.ppp_hi && q.ppp_hi <= 1.0))
        return fail(SP_ERR_INVALID_ARG, "ppp range must satisfy 0 < lo <= hi <= 1");
    if (q.d_dist != SP_DIST_UNIFORM && q.d_dist != SP_DIST_NORMAL_CLIPPED)
        return fail(SP_ERR_INVALID_ARG, "unknown diameter distribution %d", q.d_dist);
    if (q.d_dist == SP_DIST_UNIFORM && !(q.d_a > 0.0f && q.d_a <= q.d_b && std::isfinite(q.d_b)))
        return fail(SP_ERR_INVALID_ARG, "uniform diameter range must satisfy 0 < d_a <= d_b");
    if (q.d_dist == SP_DIST_NORMAL_CLIPPED &&
        !(q.d_b >= 0.0f && q.d_lo > 0.0f && q.d_lo <= q.d_hi && std::isfinite(q.d_hi) && std::isfinite(q.d_a)))
        return fail(SP_ERR_INVALID_ARG, "normal diameter needs std >= 0 and 0 < d_lo <= d_hi");
    if (!(q.I0_lo >= 0.0f && q.I0_lo <= q.I0_hi && std::isfinite(q.I0_hi)))
        return fail(SP_ERR_INVALID_ARG, "intensity range must satisfy 0 <= lo <= hi");
    if (!(q.z_lo <= q.z_hi && std::isfinite(q.z_lo) && std::isfinite(q.z_hi)))
        return fail(SP_ERR_INVALID_ARG, "z range must satisfy lo <= hi, finite");
    if (!dev_ptr_ok(x) || !dev_ptr_ok(y) || !dev_ptr_ok(z) || !dev_ptr_ok(d) || !dev_ptr_ok(I0))
        return fail(SP_ERR_INVALID_ARG, "x, y, z, d, I0 must be non-NULL, 4-byte aligned device pointers");
    for (int32_t p = 0; p < n_pairs; ++p) {
        const double hw = (double)pairs_host[p].H * (double)pairs_host[p].W;
        if ((double)pairs_host[p].n_max != std::floor(hw * q.ppp_hi + 0.5))
            return fail(SP_ERR_INVALID_ARG, "pair %d: n_max %d is not floor(H W ppp_hi + 1/2)", p,
                        pairs_host[p].n_max);
    }
    const hipError_t e = sp::launch_seed(pairs_dev, n_pairs, span, q, seed, x, y, z, d, I0, n_active_dev, ppp_dev,
                                         as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "seed launch");
    return SP_OK;
}

synthpix_status synthpix_advect(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev, int32_t n_pairs,
                                const float* flow, const synthpix_advect_params* ap, const float* x1,
                                const float* y1, float* x2, float* y2, void* stream)
{
    int64_t span;
    synthpix_status st = check_pairs(pairs_host, pairs_dev, n_pairs, &span);
    if (st) return st;
    if (!ap) return fail(SP_ERR_INVALID_ARG, "advect params must be non-NULL");
    if (!std::isfinite(ap->dt)) return fail(SP_ERR_INVALID_ARG, "dt must be finite");
    if (ap->substeps < 1 || ap->substeps > 1024) return fail(SP_ERR_INVALID_ARG, "substeps must be in [1, 1024]");
    if (ap->integrator != SP_EULER && ap->integrator != SP_RK4)
        return fail(SP_ERR_INVALID_ARG, "unknown integrator %d", ap->integrator);
    if (!flow || !aligned(flow, 8)) return fail(SP_ERR_INVALID_ARG, "flow must be a non-NULL 8-byte aligned pointer");
    if (!dev_ptr_ok(x1) || !dev_ptr_ok(y1) || !dev_ptr_ok(x2) || !dev_ptr_ok(y2))
        return fail(SP_ERR_INVALID_ARG, "x1, y1, x2, y2 must be non-NULL, 4-byte aligned device pointers");
    if (x1 == x2 || y1 == y2) return fail(SP_ERR_INVALID_ARG, "x2/y2 must not alias x1/y1");
    const hipError_t e = sp::launch_advect(pairs_dev, n_pairs, span, flow, *ap, x1, y1, x2, y2, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "advect launch");
    return SP_OK;
}

synthpix_status synthpix_render_pair(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev,
                                     int32_t n_pairs, const synthpix_tiling* tiling, const float* x1,
                                     const float* y1, const float* x2, const float* y2, const float* z,
                                     const float* d, const float* I0, const synthpix_render_params* rp,
                                     void* images, void* workspace, size_t ws_bytes, void* stream)
{
    int64_t span;
    synthpix_status st = check_pairs(pairs_host, pairs_dev, n_pairs, &span);
    if (st) return st;
    if ((st = check_render_params(rp))) return st;
    const synthpix_tiling t = tiling ? *tiling : default_tiling();
    if ((st = check_tiling(t))) return st;
    if (!dev_ptr_ok(x1) || !dev_ptr_ok(y1) || !dev_ptr_ok(x2) || !dev_ptr_ok(y2) || !dev_ptr_ok(z) ||
        !dev_ptr_ok(d) || !dev_ptr_ok(I0))
        return fail(SP_ERR_INVALID_ARG, "particle arrays must be non-NULL, 4-byte aligned device pointers");
    if (!images || !aligned(images, rp->bits ? 2 : 4))
        return fail(SP_ERR_INVALID_ARG, "images must be a non-NULL, aligned device pointer");
    const sp::RenderConfig cfg = make_config(*rp, t);
    sp::BatchTotals T;
    if ((st = batch_totals(pairs_host, n_pairs, cfg, &T))) return st;
    const sp::WorkspaceLayout wl = workspace_layout(n_pairs, T, 0, pairs_host);
    if (!workspace || !aligned(workspace, 256)) return fail(SP_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < wl.total)
        return fail(SP_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, wl.total);
    if (sp::render_lds_bytes(cfg) > 160 * 1024)
        return fail(SP_ERR_UNSUPPORTED, "tiling needs %zu bytes of LDS per workgroup (max 163840)",
                    sp::render_lds_bytes(cfg));
    sp::RenderArgs a{};
    a.pairs = pairs_dev;
    a.n_pairs = n_pairs;
    a.x[0] = x1; a.y[0] = y1; a.x[1] = x2; a.y[1] = y2;
    a.z = z; a.d = d; a.I0 = I0;
    a.images = images;
    a.sheet_sigma = rp->sheet_sigma;
    a.noise_sigma = rp->noise_sigma;
    a.bits = rp->bits;
    a.seed = rp->seed;
    blur_taps(rp->blur_radius, rp->blur_sigma, a.blur_w);
    const hipError_t e = sp::launch_render(a, cfg, T, static_cast<char*>(workspace), wl, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "render launch");
    return SP_OK;
}

synthpix_status synthpix_render_pair_backward(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev,
                                              int32_t n_pairs, const synthpix_tiling* tiling, const float* flow,
                                              const float* x1, const float* y1, const float* z, const float* d,
                                              const float* I0, const synthpix_render_params* rp,
                                              const float* grad_images, float* g_x1, float* g_y1, float* g_z,
                                              float* g_d, float* g_I0, float* g_sheet, float* g_flow,
                                              void* workspace, size_t ws_bytes, void* stream)
{
    (void)pairs_host; (void)pairs_dev; (void)n_pairs; (void)tiling; (void)flow; (void)x1; (void)y1; (void)z;
    (void)d; (void)I0; (void)rp; (void)grad_images; (void)g_x1; (void)g_y1; (void)g_z; (void)g_d; (void)g_I0;
    (void)g_sheet; (void)g_flow; (void)workspace; (void)ws_bytes; (void)stream;
    return fail(SP_ERR_UNSUPPORTED, "backward not built yet");
}

}  // extern "C"
