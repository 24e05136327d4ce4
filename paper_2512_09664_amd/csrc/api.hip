// C ABI of the generator: host-side validation, workspace sizing and kernel
// enqueueing.  See include/synthpix.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

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
    if (!(rp->hide_p >= 0.0f && rp->hide_p <= 1.0f)) return fail(SP_ERR_INVALID_ARG, "hide_p must be in [0, 1]");
    if (!(rp->jitter_d >= 0.0f) || !std::isfinite(rp->jitter_d) || !(rp->jitter_rho >= 0.0f) ||
        !std::isfinite(rp->jitter_rho) || !(rp->jitter_I0 >= 0.0f) || !std::isfinite(rp->jitter_I0))
        return fail(SP_ERR_INVALID_ARG, "frame-2 variation standard deviations must be >= 0 and finite");
    if (rp->sheet_law != SP_SHEET_GAUSS && rp->sheet_law != SP_SHEET_REMARK1)
        return fail(SP_ERR_INVALID_ARG, "unknown sheet law %d", rp->sheet_law);
    if (rp->sheet_law == SP_SHEET_REMARK1 &&
        !(rp->sheet_dz0 > 0.0f && std::isfinite(rp->sheet_dz0) && rp->sheet_shape > 0.0f &&
          std::isfinite(rp->sheet_shape)))
        return fail(SP_ERR_INVALID_ARG, "the Remark 1 sheet law needs sheet_dz0 > 0 and sheet_shape > 0");
    return SP_OK;
}

// The full particle model is in use (the model's prep kernel runs) ...
bool model_in_use(const synthpix_render_params& rp, const synthpix_particle_extras* ex)
{
    return rp.hide_p > 0.0f || rp.jitter_d > 0.0f || rp.jitter_rho > 0.0f || rp.jitter_I0 > 0.0f ||
           rp.sheet_law != SP_SHEET_GAUSS || (ex && (ex->dy || ex->rho || ex->z2));
}

// ... and its particles may be anisotropic (shape records, anisotropic kernels).
bool aniso_in_use(const synthpix_render_params& rp, const synthpix_particle_extras* ex)
{
    return rp.jitter_d > 0.0f || rp.jitter_rho > 0.0f || (ex && (ex->dy || ex->rho));
}

synthpix_status check_extras(const synthpix_particle_extras* ex)
{
    if (!ex) return SP_OK;
    if ((ex->dy && !dev_ptr_ok(ex->dy)) || (ex->rho && !dev_ptr_ok(ex->rho)) || (ex->z2 && !dev_ptr_ok(ex->z2)))
        return fail(SP_ERR_INVALID_ARG, "extras dy, rho, z2 must be NULL or 4-byte aligned device pointers");
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
    if (t.persistent != 0 && t.persistent != 1) return fail(SP_ERR_INVALID_ARG, "persistent must be 0 or 1");
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
    c.persistent = t.persistent;
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
    w.status = o; o = align256(o + 64);     // status words 0..3, render work queues 8..15
    w.layout = o; o = align256(o + sizeof(sp::PairLayout) * (size_t)n_pairs);
    w.tile_count = o; o = align256(o + sizeof(uint32_t) * 2 * (size_t)T.tiles);
    w.tile_offset = o; o = align256(o + sizeof(int64_t) * 2 * (size_t)T.tiles);
    w.hist = o; o = align256(o + sizeof(uint32_t) * (size_t)T.hist);
    w.entries = o; o = align256(o + sizeof(int32_t) * (size_t)T.entries);
    w.records = o; o = align256(o + 2 * 16 * (size_t)T.n_span);
    w.boxes = o; o = align256(o + 2 * 8 * (size_t)T.n_span);
    w.shapes = o; o = align256(o + 2 * 8 * (size_t)T.n_span);
    (void)backward;
    (void)ph;
    w.total = o;
    return w;
}

// End of the furthest pair grid in the flow array (floats).
int64_t flow_span(const synthpix_pair* ph, int32_t n_pairs)
{
    int64_t e = 0;
    for (int32_t p = 0; p < n_pairs; ++p)
        e = std::max<int64_t>(e, ph[p].flow_offset + 2 * (int64_t)ph[p].Gh * ph[p].Gw);
    return e;
}

// Backward workspace: particle-major, no bins.
struct BwdLayout {
    size_t status, scale, x2, y2, gx2, gy2, sheet, sheet_part, bound_part, wg_base, head, part, ovf, eblur, parts,
        loss_part, total;
};

// Workgroups of the flow adjoint: 256 particles of one pair each.
int64_t grid_workgroups(const synthpix_pair* ph, int32_t n_pairs)
{
    int64_t n = 0;
    for (int32_t p = 0; p < n_pairs; ++p) n += ((int64_t)ph[p].n_max + 255) / 256;
    return n;
}

BwdLayout bwd_layout(int64_t n_span, int64_t n_wg, int32_t n_pairs, int64_t n_eblur, bool tile, int64_t n_loss)
{
    BwdLayout w{};
    size_t o = 0;
    const size_t nf = sizeof(float) * (size_t)n_span;
    w.status = o; o = align256(o + 16);
    w.scale = o; o = align256(o + 16);
    w.x2 = o; o = align256(o + nf);
    w.y2 = o; o = align256(o + nf);
    w.gx2 = o; o = align256(o + nf);
    w.gy2 = o; o = align256(o + nf);
    w.sheet = o; o = align256(o + nf);
    w.sheet_part = o; o = align256(o + sizeof(double) * sp::BWD_SLICES * (size_t)n_pairs);
    w.bound_part = o; o = align256(o + sizeof(float) * 2 * sp::BWD_SLICES * (size_t)n_pairs);
    w.wg_base = o; o = align256(o + sizeof(int64_t) * ((size_t)n_pairs + 1));
    w.head = o; o = align256(o + sizeof(sp::GridHeader) * (size_t)n_wg);
    w.part = o; o = align256(o + sizeof(uint64_t) * 2 * sp::WIN_NODES * (size_t)n_wg);
    w.ovf = o; o = align256(o + sizeof(sp::GridRecord) * sp::GRID_OVF_CAP * (size_t)n_wg);
    w.eblur = o; o = align256(o + sizeof(float) * (size_t)n_eblur);
    w.parts = o; o = align256(o + (tile ? 2 * 16 * (size_t)n_span : 0));
    w.loss_part = o; o = align256(o + sizeof(double) * (size_t)n_loss);
    w.total = o;
    return w;
}

// Elements of the blurred-gradient images the backward keeps (B^T dL/dJ, the
// images' layout): for any blur under the tile-major gather, else when the blur
// is wide enough (radius >= 2) for the particle-major gather to pay for a
// per-pixel pass, and always for the loss-fused form (mse); otherwise none.
int64_t eblur_span(const synthpix_pair* ph, int32_t n_pairs, int blur_radius, bool tile, bool mse)
{
    if (!mse && blur_radius < (tile ? 1 : 2)) return 0;
    int64_t span = 0;
    for (int32_t p = 0; p < n_pairs; ++p)
        span = std::max<int64_t>(span, ph[p].image_offset + 2 * (int64_t)ph[p].H * ph[p].W);
    return span;
}

// ceil(log2(samples)) for the fixed-point scale of the flow gradient.
int sample_exponent(int64_t n_span, const synthpix_advect_params& ap)
{
    const double n = (double)std::max<int64_t>(n_span, 1) * ap.substeps * (ap.integrator == SP_RK4 ? 4 : 1);
    int e = 0;
    while (std::ldexp(1.0, e) < n) ++e;
    return e;
}

// Seeding parameters and the particle-count rule n_max = floor(H W ppp_hi + 1/2).
synthpix_status check_seed_params(const synthpix_seed_params* sp_, const synthpix_pair* ph, int32_t n_pairs)
{
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
    for (int32_t p = 0; p < n_pairs; ++p) {
        const double hw = (double)ph[p].H * (double)ph[p].W;
        if ((double)ph[p].n_max != std::floor(hw * q.ppp_hi + 0.5))
            return fail(SP_ERR_INVALID_ARG, "pair %d: n_max %d is not floor(H W ppp_hi + 1/2)", p, ph[p].n_max);
    }
    return SP_OK;
}

synthpix_status check_advect_params(const synthpix_advect_params* ap)
{
    if (!ap) return fail(SP_ERR_INVALID_ARG, "advect params must be non-NULL");
    if (!std::isfinite(ap->dt)) return fail(SP_ERR_INVALID_ARG, "dt must be finite");
    if (ap->substeps < 1 || ap->substeps > 1024) return fail(SP_ERR_INVALID_ARG, "substeps must be in [1, 1024]");
    if (ap->integrator != SP_EULER && ap->integrator != SP_RK4)
        return fail(SP_ERR_INVALID_ARG, "unknown integrator %d", ap->integrator);
    return SP_OK;
}

hipError_t enqueue_render(const synthpix_pair* pairs_dev, int32_t n_pairs, const sp::RenderConfig& cfg,
                          const sp::BatchTotals& T, const sp::WorkspaceLayout& wl, const float* x1, const float* y1,
                          const float* x2, const float* y2, const float* z, const float* d, const float* I0,
                          const synthpix_render_params& rp, void* images, void* workspace, hipStream_t stream,
                          const synthpix_batch_io* iod = nullptr, const synthpix_particle_extras* ex = nullptr,
                          const int32_t* live = nullptr)
{
    sp::RenderArgs a{};
    if (ex) {
        a.dy = ex->dy;
        a.rho = ex->rho;
        a.z2 = ex->z2;
    }
    a.hide_p = rp.hide_p;
    a.jit_d = rp.jitter_d;
    a.jit_rho = rp.jitter_rho;
    a.jit_I0 = rp.jitter_I0;
    a.sheet_law = rp.sheet_law;
    a.sheet_dz0 = rp.sheet_dz0;
    a.sheet_shape = rp.sheet_shape;
    a.model = model_in_use(rp, ex);
    a.aniso = aniso_in_use(rp, ex);
    a.iod = iod;
    a.live = live;
    a.pairs = pairs_dev;
    a.n_pairs = n_pairs;
    a.x[0] = x1; a.y[0] = y1; a.x[1] = x2; a.y[1] = y2;
    a.z = z; a.d = d; a.I0 = I0;
    a.images = images;
    a.sheet_sigma = rp.sheet_sigma;
    a.noise_sigma = rp.noise_sigma;
    a.bits = rp.bits;
    a.seed = rp.seed;
    blur_taps(rp.blur_radius, rp.blur_sigma, a.blur_w);
    return sp::launch_render(a, cfg, T, static_cast<char*>(workspace), wl, stream);
}

synthpix_tiling default_tiling()
{
    synthpix_tiling t;
    t.tile_w = 64;
    t.tile_h = 32;
    t.chunk = 2048;    // smaller binning blocks keep more of each tile list's writes in L2
    t.cap = 64;
    t.persistent = 0;
    return t;
}

}  // namespace

// Home blocks of the advection order: 32 x 32 pixels, or larger where a pair
// would have more than 16384 blocks (the count pass holds one pair's block
// histogram in LDS).
sp::RenderConfig order_config(const synthpix_pair* ph, int32_t n_pairs)
{
    int lb = 5;
    for (int32_t p = 0; p < n_pairs; ++p)
        while ((int64_t)((ph[p].W + (1 << lb) - 1) >> lb) * ((ph[p].H + (1 << lb) - 1) >> lb) > 16384) ++lb;
    // 2048-particle chunks, larger for pairs with many particles (the per-chunk
    // block histograms would outgrow the particles)
    int chunk = 2048;
    for (int32_t p = 0; p < n_pairs; ++p)
        while (chunk < 16384 && ph[p].n_max / chunk > 512) chunk *= 2;
    sp::RenderConfig c{};
    c.tile_w = c.tile_h = 1 << lb;
    c.log_tw = c.log_th = lb;
    c.chunk = chunk;
    c.cap = 32;
    c.apron = 0;
    c.kx = c.ky = 1;     // one entry per particle
    c.d_max = 1.0f;
    return c;
}

sp::OrderLayout order_layout(int32_t n_pairs, const sp::BatchTotals& T, size_t base)
{
    sp::OrderLayout w{};
    size_t o = base;
    w.status = o; o = align256(o + 16);
    w.layout = o; o = align256(o + sizeof(sp::PairLayout) * (size_t)n_pairs);
    w.tile_count = o; o = align256(o + sizeof(uint32_t) * 2 * (size_t)T.tiles);
    w.tile_offset = o; o = align256(o + sizeof(int64_t) * 2 * (size_t)T.tiles);
    w.hist = o; o = align256(o + sizeof(uint32_t) * (size_t)T.hist);
    w.entries = o; o = align256(o + sizeof(int32_t) * (size_t)T.entries);
    w.total = o;
    return w;
}

// Order workspace bytes for a batch (0 when the batch is invalid).
size_t order_bytes(const synthpix_pair* ph, int32_t n_pairs)
{
    sp::BatchTotals T;
    if (batch_totals(ph, n_pairs, order_config(ph, n_pairs), &T) != SP_OK) return 0;
    return order_layout(n_pairs, T, 0).total;
}

// Backward workspace: the gradient layout, then the frame-1 home-block order
// and, for the tile-major gather, the frame-2 one.
struct BwdPlan {
    BwdLayout wl;
    size_t ob;
    bool tile;
    size_t total;
};

BwdPlan bwd_plan(const synthpix_pair* ph, int32_t n_pairs, int64_t span, const synthpix_render_params& rp, bool mse)
{
    BwdPlan b{};
    b.ob = order_bytes(ph, n_pairs);
    b.tile = sp::tile_gather_fits(rp.d_max, order_config(ph, n_pairs).log_tw, rp.blur_radius);
    int max_h = 0, max_w = 0;
    for (int32_t p = 0; p < n_pairs; ++p) {
        max_h = std::max(max_h, (int)ph[p].H);
        max_w = std::max(max_w, (int)ph[p].W);
    }
    const int64_t n_loss = mse ? sp::blur_grad_blocks(n_pairs, max_w, max_h, true) : 0;
    b.wl = bwd_layout(span, grid_workgroups(ph, n_pairs), n_pairs,
                      eblur_span(ph, n_pairs, rp.blur_radius, b.tile, mse), b.tile, n_loss);
    b.total = b.wl.total + b.ob * (b.tile ? 2 : 1);
    return b;
}

// Builds the home-block order of (x, y) in `ws` at byte offset `base` and
// returns it for the advection launch.
hipError_t enqueue_order(const synthpix_pair* ph, const synthpix_pair* pd, int32_t n_pairs, const float* x,
                         const float* y, char* ws, size_t base, hipStream_t s, sp::AdvectOrder* out,
                         const synthpix_batch_io* iod = nullptr, const int32_t* live = nullptr)
{
    const sp::RenderConfig cfg = order_config(ph, n_pairs);
    sp::BatchTotals T;
    if (batch_totals(ph, n_pairs, cfg, &T) != SP_OK) return hipErrorInvalidValue;
    const sp::OrderLayout ol = order_layout(n_pairs, T, base);
    out->L = reinterpret_cast<const sp::PairLayout*>(ws + ol.layout);
    out->entries = reinterpret_cast<const int32_t*>(ws + ol.entries);
    out->log_block = cfg.log_tw;
    out->blocks = T.tiles;
    out->count = reinterpret_cast<const uint32_t*>(ws + ol.tile_count);
    out->offset = reinterpret_cast<const int64_t*>(ws + ol.tile_offset);
    out->live = live;
    return sp::launch_order(pd, n_pairs, x, y, cfg, T, ws, ol, s, iod, live);
}

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
    const size_t ob = order_bytes(pairs_host, n_pairs);
    if (!ob) return fail(SP_ERR_UNSUPPORTED, "batch too large for the advection order");
    if (backward < 0 || backward > 2) return fail(SP_ERR_INVALID_ARG, "backward must be 0, 1 or 2");
    if (backward) {
        *bytes_out = bwd_plan(pairs_host, n_pairs, span, *rp, backward == 2).total;
        return SP_OK;
    }
    const sp::RenderConfig cfg = make_config(*rp, t);
    sp::BatchTotals T;
    if ((st = batch_totals(pairs_host, n_pairs, cfg, &T))) return st;
    *bytes_out = std::max(workspace_layout(n_pairs, T, 0, pairs_host).total, ob);
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

synthpix_status synthpix_probe(int32_t kind, void* buf, size_t bytes, int32_t iters, void* stream,
                               double* work_out)
{
    if (!work_out || !buf) return fail(SP_ERR_INVALID_ARG, "buf and work_out must be non-NULL");
    if (kind < SP_PROBE_STORE || kind > SP_PROBE_INT) return fail(SP_ERR_INVALID_ARG, "unknown probe kind %d", kind);
    const bool mem = kind <= SP_PROBE_COPY || kind == SP_PROBE_STORE_NT;
    if (mem && (!aligned(buf, 16) || bytes < 32))
        return fail(SP_ERR_INVALID_ARG, "store/copy probes need a 16-byte aligned buffer of >= 32 bytes");
    if (!mem && (bytes < 1024 || iters <= 0 || (iters & 3)))
        return fail(SP_ERR_INVALID_ARG, "ALU probes need >= 1 KiB of buffer and iters a positive multiple of 4");
    const hipError_t e = sp::launch_probe(kind, buf, bytes, iters, as_stream(stream), work_out);
    if (e != hipSuccess) return hip_fail(e, "probe launch");
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
    if ((st = check_seed_params(sp_, pairs_host, n_pairs))) return st;
    const synthpix_seed_params& q = *sp_;
    if (!dev_ptr_ok(x) || !dev_ptr_ok(y) || !dev_ptr_ok(z) || !dev_ptr_ok(d) || !dev_ptr_ok(I0))
        return fail(SP_ERR_INVALID_ARG, "x, y, z, d, I0 must be non-NULL, 4-byte aligned device pointers");
    const hipError_t e = sp::launch_seed(pairs_dev, n_pairs, span, q, seed, x, y, z, d, I0, n_active_dev, ppp_dev,
                                         as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "seed launch");
    return SP_OK;
}

synthpix_status synthpix_seed_shape(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev, int32_t n_pairs,
                                    const synthpix_seed_params* sp_, float rho_lo, float rho_hi, uint64_t seed,
                                    float* dy, float* rho, void* stream)
{
    int64_t span;
    synthpix_status st = check_pairs(pairs_host, pairs_dev, n_pairs, &span);
    if (st) return st;
    if ((st = check_seed_params(sp_, pairs_host, n_pairs))) return st;
    if (!(rho_lo >= -0.99f && rho_lo <= rho_hi && rho_hi <= 0.99f))
        return fail(SP_ERR_INVALID_ARG, "rho range must satisfy -0.99 <= rho_lo <= rho_hi <= 0.99");
    if (!dev_ptr_ok(dy) || !dev_ptr_ok(rho))
        return fail(SP_ERR_INVALID_ARG, "dy, rho must be non-NULL, 4-byte aligned device pointers");
    const hipError_t e = sp::launch_seed_shape(pairs_dev, n_pairs, span, *sp_, rho_lo, rho_hi, seed, dy, rho,
                                               as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "seed_shape launch");
    return SP_OK;
}

synthpix_status synthpix_flow_field(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev, int32_t n_pairs,
                                    const float* flow, float* out, void* stream)
{
    int64_t span;
    synthpix_status st = check_pairs(pairs_host, pairs_dev, n_pairs, &span);
    if (st) return st;
    if (n_pairs > 65535) return fail(SP_ERR_UNSUPPORTED, "at most 65535 pairs per call");
    if (!flow || !aligned(flow, 8)) return fail(SP_ERR_INVALID_ARG, "flow must be a non-NULL 8-byte aligned pointer");
    if (!out || !aligned(out, 8)) return fail(SP_ERR_INVALID_ARG, "out must be a non-NULL 8-byte aligned pointer");
    int64_t max_px = 0;
    for (int32_t p = 0; p < n_pairs; ++p) {
        if (pairs_host[p].image_offset & 1) return fail(SP_ERR_INVALID_ARG, "pair %d: image_offset must be even", p);
        max_px = std::max<int64_t>(max_px, (int64_t)pairs_host[p].H * pairs_host[p].W);
    }
    const hipError_t e = sp::launch_flow_field(pairs_dev, n_pairs, max_px, flow, out, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "flow field launch");
    return SP_OK;
}

synthpix_status synthpix_histogram_workspace_size(int32_t n_pairs, int32_t bits, size_t* bytes_out)
{
    if (!bytes_out) return fail(SP_ERR_INVALID_ARG, "bytes_out must be non-NULL");
    if (n_pairs <= 0 || n_pairs > 32767) return fail(SP_ERR_INVALID_ARG, "n_pairs must be in [1, 32767]");
    if (bits < 1 || bits > 14) return fail(SP_ERR_UNSUPPORTED, "histogram adjustment needs bits in [1, 14]");
    *bytes_out = sp::hist_workspace_bytes(n_pairs, bits);
    return SP_OK;
}

synthpix_status synthpix_histogram_match(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev,
                                         int32_t n_pairs, int32_t bits, const uint32_t* target, void* images,
                                         void* workspace, size_t ws_bytes, void* stream)
{
    int64_t span;
    synthpix_status st = check_pairs(pairs_host, pairs_dev, n_pairs, &span);
    if (st) return st;
    size_t need = 0;
    if ((st = synthpix_histogram_workspace_size(n_pairs, bits, &need))) return st;
    if (!target || !aligned(target, 4)) return fail(SP_ERR_INVALID_ARG, "target must be a 4-byte aligned device pointer");
    if (!images || !aligned(images, 2)) return fail(SP_ERR_INVALID_ARG, "images must be a 2-byte aligned device pointer");
    if (!workspace || !aligned(workspace, 256)) return fail(SP_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return fail(SP_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    int64_t max_px = 0;
    for (int32_t p = 0; p < n_pairs; ++p) max_px = std::max<int64_t>(max_px, (int64_t)pairs_host[p].H * pairs_host[p].W);
    const hipError_t e = sp::launch_histogram_match(pairs_dev, n_pairs, max_px, bits, target,
                                                    static_cast<uint16_t*>(images), static_cast<char*>(workspace),
                                                    as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "histogram launch");
    return SP_OK;
}

synthpix_status synthpix_advect_workspace_size(const synthpix_pair* pairs_host, int32_t n_pairs, size_t* bytes_out)
{
    if (!bytes_out) return fail(SP_ERR_INVALID_ARG, "bytes_out must be non-NULL");
    int64_t span;
    synthpix_status st = check_pairs(pairs_host, pairs_host, n_pairs, &span);
    if (st) return st;
    const size_t b = order_bytes(pairs_host, n_pairs);
    if (!b) return fail(SP_ERR_UNSUPPORTED, "batch too large for the advection order");
    *bytes_out = b;
    return SP_OK;
}

synthpix_status synthpix_advect(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev, int32_t n_pairs,
                                const float* flow, const synthpix_advect_params* ap, const float* x1,
                                const float* y1, float* x2, float* y2, const float* wflow, const float* z1,
                                float* z2, void* workspace, size_t ws_bytes, void* stream)
{
    int64_t span;
    synthpix_status st = check_pairs(pairs_host, pairs_dev, n_pairs, &span);
    if (st) return st;
    if ((st = check_advect_params(ap))) return st;
    if (!flow || !aligned(flow, 8)) return fail(SP_ERR_INVALID_ARG, "flow must be a non-NULL 8-byte aligned pointer");
    if (!dev_ptr_ok(x1) || !dev_ptr_ok(y1) || !dev_ptr_ok(x2) || !dev_ptr_ok(y2))
        return fail(SP_ERR_INVALID_ARG, "x1, y1, x2, y2 must be non-NULL, 4-byte aligned device pointers");
    if (x1 == x2 || y1 == y2) return fail(SP_ERR_INVALID_ARG, "x2/y2 must not alias x1/y1");
    if ((wflow == nullptr) != (z1 == nullptr) || (wflow == nullptr) != (z2 == nullptr))
        return fail(SP_ERR_INVALID_ARG, "wflow, z1 and z2 must be all NULL or all set");
    if (wflow) {
        if (!dev_ptr_ok(wflow) || !dev_ptr_ok(z1) || !dev_ptr_ok(z2))
            return fail(SP_ERR_INVALID_ARG, "wflow, z1, z2 must be 4-byte aligned device pointers");
        if (z1 == z2) return fail(SP_ERR_INVALID_ARG, "z2 must not alias z1");
        const hipError_t e = sp::launch_advect3(pairs_dev, n_pairs, span, flow, wflow, *ap, x1, y1, z1, x2, y2, z2,
                                                as_stream(stream));
        if (e != hipSuccess) return hip_fail(e, "advect launch");
        return SP_OK;
    }
    sp::AdvectOrder order{nullptr, nullptr};
    if (workspace) {
        if (!aligned(workspace, 256)) return fail(SP_ERR_WORKSPACE, "workspace must be 256-byte aligned");
        const size_t need = order_bytes(pairs_host, n_pairs);
        if (!need) return fail(SP_ERR_UNSUPPORTED, "batch too large for the advection order");
        if (ws_bytes < need) return fail(SP_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
        const hipError_t e = enqueue_order(pairs_host, pairs_dev, n_pairs, x1, y1, static_cast<char*>(workspace), 0,
                                           as_stream(stream), &order);
        if (e != hipSuccess) return hip_fail(e, "advect order launch");
    }
    const hipError_t e = sp::launch_advect(pairs_dev, n_pairs, span, flow, *ap, x1, y1, x2, y2, as_stream(stream),
                                           order);
    if (e != hipSuccess) return hip_fail(e, "advect launch");
    return SP_OK;
}

synthpix_status synthpix_render_pair(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev,
                                     int32_t n_pairs, const synthpix_tiling* tiling, const float* x1,
                                     const float* y1, const float* x2, const float* y2, const float* z,
                                     const float* d, const float* I0, const synthpix_particle_extras* extras,
                                     const synthpix_render_params* rp, void* images, void* workspace,
                                     size_t ws_bytes, void* stream)
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
    if ((st = check_extras(extras))) return st;
    const bool aniso = aniso_in_use(*rp, extras);
    if (sp::render_lds_bytes(cfg, aniso) > 160 * 1024)
        return fail(SP_ERR_UNSUPPORTED, "tiling needs %zu bytes of LDS per workgroup (max 163840)",
                    sp::render_lds_bytes(cfg, aniso));
    const hipError_t e = enqueue_render(pairs_dev, n_pairs, cfg, T, wl, x1, y1, x2, y2, z, d, I0, *rp, images,
                                        workspace, as_stream(stream), nullptr, extras);
    if (e != hipSuccess) return hip_fail(e, "render launch");
    return SP_OK;
}

size_t synthpix_mse_workspace_size(int64_t n)
{
    (void)n;
    return align256(sizeof(double) * sp::MSE_BLOCKS);
}

synthpix_status synthpix_mse_grad(const float* J, const float* T, int64_t n, float scale, float* grad,
                                  double* loss, void* workspace, size_t ws_bytes, void* stream)
{
    if (n < 0) return fail(SP_ERR_INVALID_ARG, "n must be >= 0");
    if ((n > 0 && (!J || !T || !grad)) || !aligned(J, 16) || !aligned(T, 16) || !aligned(grad, 16))
        return fail(SP_ERR_INVALID_ARG, "J, T and grad must be 16-byte aligned device pointers (non-NULL for n > 0)");
    if (!std::isfinite(scale)) return fail(SP_ERR_INVALID_ARG, "scale must be finite");
    if (loss) {
        if (!aligned(loss, 8)) return fail(SP_ERR_INVALID_ARG, "loss must be an 8-byte aligned device pointer");
        if (!workspace || !aligned(workspace, 256)) return fail(SP_ERR_WORKSPACE, "workspace must be 256-byte aligned");
        if (ws_bytes < synthpix_mse_workspace_size(n))
            return fail(SP_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes,
                        synthpix_mse_workspace_size(n));
    }
    if (n == 0 && !loss) return SP_OK;
    const hipError_t e = sp::launch_mse_grad(J, T, n, scale, grad, loss, static_cast<double*>(workspace),
                                             as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "loss gradient launch");
    return SP_OK;
}

}  // extern "C"

namespace {

// The body of both backward entry points: dL/dJ handed in (grad_images), or,
// with mse, formed from the images J and the target T as scale (J - T) inside
// the backward's per-pixel pass (loss: optional device double, the mean of
// (J - T)^2 over the pairs' pixels).
synthpix_status backward_common(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev, int32_t n_pairs,
                                const synthpix_tiling* tiling, const float* flow, const float* x1, const float* y1,
                                const float* x2, const float* y2, const float* z, const float* d, const float* I0,
                                const synthpix_render_params* rp, bool mse, const float* grad_images,
                                const float* J, const float* T, float scale, double* loss, float* g_x1,
                                float* g_y1, float* g_z, float* g_d, float* g_I0, float* g_sheet,
                                float* g_sheet_total, float* g_flow, void* workspace, size_t ws_bytes, void* stream)
{
    int64_t span;
    synthpix_status st = check_pairs(pairs_host, pairs_dev, n_pairs, &span);
    if (st) return st;
    if ((st = check_render_params(rp))) return st;
    if (tiling && (st = check_tiling(*tiling))) return st;
    if (rp->bits != 0) return fail(SP_ERR_UNSUPPORTED, "the backward differentiates float images (bits must be 0)");
    if (model_in_use(*rp, nullptr))
        return fail(SP_ERR_UNSUPPORTED, "the backward differentiates the isotropic model (no frame-2 variation, no "
                    "hiding, the Gaussian sheet)");
    if ((st = check_advect_params(&rp->advect))) return st;
    if (!flow || !aligned(flow, 8)) return fail(SP_ERR_INVALID_ARG, "flow must be a non-NULL 8-byte aligned pointer");
    if (!dev_ptr_ok(x1) || !dev_ptr_ok(y1) || !dev_ptr_ok(z) || !dev_ptr_ok(d) || !dev_ptr_ok(I0) ||
        (mse ? (!dev_ptr_ok(J) || !dev_ptr_ok(T)) : !dev_ptr_ok(grad_images)))
        return fail(SP_ERR_INVALID_ARG, "inputs must be non-NULL, 4-byte aligned device pointers");
    if (mse && !std::isfinite(scale)) return fail(SP_ERR_INVALID_ARG, "scale must be finite");
    if (loss && !aligned(loss, 8)) return fail(SP_ERR_INVALID_ARG, "loss must be NULL or an 8-byte aligned pointer");
    if ((x2 == nullptr) != (y2 == nullptr) || (x2 && (!dev_ptr_ok(x2) || !dev_ptr_ok(y2))))
        return fail(SP_ERR_INVALID_ARG, "x2 and y2 must both be NULL or both aligned device pointers");
    if (!dev_ptr_ok(g_x1) || !dev_ptr_ok(g_y1) || !dev_ptr_ok(g_z) || !dev_ptr_ok(g_d) || !dev_ptr_ok(g_I0) ||
        !dev_ptr_ok(g_sheet) || !dev_ptr_ok(g_flow))
        return fail(SP_ERR_INVALID_ARG, "gradient outputs must be non-NULL, 4-byte aligned device pointers");
    if (g_sheet_total && !dev_ptr_ok(g_sheet_total))
        return fail(SP_ERR_INVALID_ARG, "g_sheet_total must be NULL or a 4-byte aligned device pointer");
    const int64_t n_flow = flow_span(pairs_host, n_pairs);
    const BwdPlan bp = bwd_plan(pairs_host, n_pairs, span, *rp, mse);
    const BwdLayout& wl = bp.wl;
    if (!bp.ob) return fail(SP_ERR_UNSUPPORTED, "batch too large for the advection order");
    if (!workspace || !aligned(workspace, 256)) return fail(SP_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < bp.total)
        return fail(SP_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, bp.total);
    char* ws = static_cast<char*>(workspace);
    hipStream_t hs = as_stream(stream);
    sp::BwdArgs a{};
    {
        const hipError_t e = enqueue_order(pairs_host, pairs_dev, n_pairs, x1, y1, ws, wl.total, hs, &a.order);
        if (e != hipSuccess) return hip_fail(e, "backward order launch");
    }
    a.pairs = pairs_dev;
    a.n_pairs = n_pairs;
    a.flow = flow;
    a.x1 = x1;
    a.y1 = y1;
    a.x2w = reinterpret_cast<float*>(ws + wl.x2);
    a.y2w = reinterpret_cast<float*>(ws + wl.y2);
    a.x2 = x2 ? x2 : a.x2w;
    a.y2 = y2 ? y2 : a.y2w;
    a.recompute_x2 = x2 == nullptr;
    if (bp.tile) {
        // the tile gather groups frame 2 by its own positions: recompute them
        // first when the caller did not pass them, then order them
        if (a.recompute_x2) {
            const hipError_t e = sp::launch_advect(pairs_dev, n_pairs, span, flow, rp->advect, x1, y1, a.x2w, a.y2w,
                                                   hs, a.order);
            if (e != hipSuccess) return hip_fail(e, "backward advect launch");
            a.recompute_x2 = false;
        }
        const hipError_t e = enqueue_order(pairs_host, pairs_dev, n_pairs, a.x2, a.y2, ws, wl.total + bp.ob, hs,
                                           &a.order2);
        if (e != hipSuccess) return hip_fail(e, "backward order launch");
        a.parts = reinterpret_cast<float4*>(ws + wl.parts);
    }
    a.z = z;
    a.d = d;
    a.I0 = I0;
    a.grad = mse ? nullptr : grad_images;
    a.mse = mse;
    a.J = J;
    a.T = T;
    a.mse_scale = scale;
    a.loss = mse ? loss : nullptr;
    a.loss_part = a.loss ? reinterpret_cast<double*>(ws + wl.loss_part) : nullptr;
    for (int32_t p = 0; p < n_pairs; ++p) a.loss_n += 2 * (int64_t)pairs_host[p].H * pairs_host[p].W;
    a.eblur = wl.parts > wl.eblur ? reinterpret_cast<float*>(ws + wl.eblur) : nullptr;
    a.g_x1 = g_x1;
    a.g_y1 = g_y1;
    a.g_z = g_z;
    a.g_d = g_d;
    a.g_I0 = g_I0;
    a.g_sheet = g_sheet;
    a.g_sheet_total = g_sheet_total;
    a.g_flow = g_flow;
    a.gx2 = reinterpret_cast<float*>(ws + wl.gx2);
    a.gy2 = reinterpret_cast<float*>(ws + wl.gy2);
    a.sheet = reinterpret_cast<float*>(ws + wl.sheet);
    a.sheet_part = reinterpret_cast<double*>(ws + wl.sheet_part);
    a.bound_part = reinterpret_cast<float*>(ws + wl.bound_part);
    a.grid.wg_base = reinterpret_cast<int64_t*>(ws + wl.wg_base);
    a.grid.head = reinterpret_cast<sp::GridHeader*>(ws + wl.head);
    a.grid.part = reinterpret_cast<unsigned long long*>(ws + wl.part);
    a.grid.ovf = reinterpret_cast<sp::GridRecord*>(ws + wl.ovf);
    a.grid.n_wg = grid_workgroups(pairs_host, n_pairs);
    for (int32_t p = 0; p < n_pairs; ++p) {
        a.grid.max_gh = std::max(a.grid.max_gh, (int)pairs_host[p].Gh);
        a.grid.max_gw = std::max(a.grid.max_gw, (int)pairs_host[p].Gw);
    }
    a.scale = reinterpret_cast<uint32_t*>(ws + wl.scale);
    a.status = reinterpret_cast<uint32_t*>(ws + wl.status);
    a.sheet_sigma = rp->sheet_sigma;
    a.d_max = rp->d_max;
    blur_taps(rp->blur_radius, rp->blur_sigma, a.blur_w);
    for (int32_t p = 0; p < n_pairs; ++p) {
        a.max_h = std::max(a.max_h, (int)pairs_host[p].H);
        a.max_w = std::max(a.max_w, (int)pairs_host[p].W);
    }
    const hipError_t e = sp::launch_backward(a, span, n_flow, rp->advect, rp->blur_radius,
                                             sample_exponent(span, rp->advect), hs);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return SP_OK;
}


}  // namespace

extern "C" {

synthpix_status synthpix_render_pair_backward(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev,
                                              int32_t n_pairs, const synthpix_tiling* tiling, const float* flow,
                                              const float* x1, const float* y1, const float* x2,
                                              const float* y2, const float* z, const float* d,
                                              const float* I0, const synthpix_render_params* rp,
                                              const float* grad_images, float* g_x1, float* g_y1, float* g_z,
                                              float* g_d, float* g_I0, float* g_sheet, float* g_sheet_total,
                                              float* g_flow, void* workspace, size_t ws_bytes, void* stream)
{
    return backward_common(pairs_host, pairs_dev, n_pairs, tiling, flow, x1, y1, x2, y2, z, d, I0, rp, false,
                           grad_images, nullptr, nullptr, 0.0f, nullptr, g_x1, g_y1, g_z, g_d, g_I0, g_sheet,
                           g_sheet_total, g_flow, workspace, ws_bytes, stream);
}

synthpix_status synthpix_render_pair_backward_mse(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev,
                                                  int32_t n_pairs, const synthpix_tiling* tiling, const float* flow,
                                                  const float* x1, const float* y1, const float* x2,
                                                  const float* y2, const float* z, const float* d,
                                                  const float* I0, const synthpix_render_params* rp,
                                                  const float* images, const float* target, float scale,
                                                  double* loss, float* g_x1, float* g_y1, float* g_z, float* g_d,
                                                  float* g_I0, float* g_sheet, float* g_sheet_total, float* g_flow,
                                                  void* workspace, size_t ws_bytes, void* stream)
{
    return backward_common(pairs_host, pairs_dev, n_pairs, tiling, flow, x1, y1, x2, y2, z, d, I0, rp, true,
                           nullptr, images, target, scale, loss, g_x1, g_y1, g_z, g_d, g_I0, g_sheet, g_sheet_total,
                           g_flow, workspace, ws_bytes, stream);
}

}  // extern "C"

// ------------------------------------------------------------------ static scratch

// Library-held workspace of synthpix_render_pair_noalloc: one copy per device,
// held until the process ends.  Host code never uses the array's name as an
// address (on the host it is a stand-in, not device memory): each device's
// address comes from hipGetSymbolAddress, taken once per device with that
// device current.
static __device__ __align__(256) unsigned char scratch[SYNTHPIX_STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// The current device's scratch address (resolved on the first call per device).
synthpix_status scratch_of_current_device(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return fail(SP_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SP_OK;
}

}  // namespace

extern "C" synthpix_status synthpix_render_pair_noalloc(const synthpix_pair* pairs_host,
                                                        const synthpix_pair* pairs_dev, int32_t n_pairs,
                                                        const synthpix_tiling* tiling, const float* x1,
                                                        const float* y1, const float* x2, const float* y2,
                                                        const float* z, const float* d, const float* I0,
                                                        const synthpix_particle_extras* extras,
                                                        const synthpix_render_params* rp, void* images,
                                                        uint32_t* status_out, void* stream)
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
    if (status_out && !aligned(status_out, 4))
        return fail(SP_ERR_INVALID_ARG, "status_out must be NULL or a 4-byte aligned device pointer");
    const sp::RenderConfig cfg = make_config(*rp, t);
    sp::BatchTotals T;
    if ((st = batch_totals(pairs_host, n_pairs, cfg, &T))) return st;
    const sp::WorkspaceLayout wl = workspace_layout(n_pairs, T, 0, pairs_host);
    if (wl.total > (size_t)SYNTHPIX_STATIC_SCRATCH_BYTES)
        return fail(SP_ERR_WORKSPACE,
                    "batch needs %zu bytes of workspace; the static scratch holds %zu (split the batch or use "
                    "synthpix_render_pair with a caller workspace)",
                    wl.total, (size_t)SYNTHPIX_STATIC_SCRATCH_BYTES);
    if ((st = check_extras(extras))) return st;
    const bool aniso = aniso_in_use(*rp, extras);
    if (sp::render_lds_bytes(cfg, aniso) > 160 * 1024)
        return fail(SP_ERR_UNSUPPORTED, "tiling needs %zu bytes of LDS per workgroup (max 163840)",
                    sp::render_lds_bytes(cfg, aniso));
    void* ws = nullptr;
    if ((st = scratch_of_current_device(&ws))) return st;
    // every part of the workspace the kernels read is written earlier in the same
    // call (the status words are cleared by the layout kernel), so the previous
    // call's contents need no clearing
    hipError_t e = enqueue_render(pairs_dev, n_pairs, cfg, T, wl, x1, y1, x2, y2, z, d, I0, *rp, images, ws,
                                  as_stream(stream), nullptr, extras);
    if (e == hipSuccess && status_out)
        e = hipMemcpyAsync(status_out, static_cast<char*>(ws) + wl.status, sizeof(uint32_t),
                           hipMemcpyDeviceToDevice, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "render launch");
    return SP_OK;
}

// ------------------------------------------------------------------ plans

struct synthpix_plan {
    int device = 0;
    int32_t n_pairs = 0;
    std::vector<synthpix_pair> pairs_host;
    synthpix_pair* pairs_dev = nullptr;
    synthpix_batch_io* io_dev = nullptr;   // the descriptor the captured kernels read
    synthpix_seed_params sp{};
    synthpix_advect_params ap{};
    synthpix_render_params rp{};
    synthpix_batch_io io{};                // the creation io (autotuning runs on it)
    synthpix_tiling tiling{};
    int advance = 0;
    int64_t span = 0;
    void* workspace = nullptr;
    size_t ws_bytes = 0;
    int32_t* live = nullptr;               // each pair's active count (end of the workspace)
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// Pointer checks of one launch's io (flow: 8-byte nodes; images per the output type).
synthpix_status check_io(const synthpix_batch_io* io, int bits)
{
    if (!io) return fail(SP_ERR_INVALID_ARG, "io must be non-NULL");
    if (!io->flow || !aligned(io->flow, 8)) return fail(SP_ERR_INVALID_ARG, "io flow must be 8-byte aligned");
    if (!dev_ptr_ok(io->x1) || !dev_ptr_ok(io->y1) || !dev_ptr_ok(io->x2) || !dev_ptr_ok(io->y2) ||
        !dev_ptr_ok(io->z) || !dev_ptr_ok(io->d) || !dev_ptr_ok(io->I0))
        return fail(SP_ERR_INVALID_ARG, "io particle buffers must be non-NULL, 4-byte aligned device pointers");
    if (io->x1 == io->x2 || io->y1 == io->y2) return fail(SP_ERR_INVALID_ARG, "io x2/y2 must not alias x1/y1");
    if (!io->images || !aligned(io->images, bits ? 2 : 4))
        return fail(SP_ERR_INVALID_ARG, "io images must be a non-NULL, aligned device pointer");
    if ((io->n_active && !aligned(io->n_active, 4)) || (io->ppp && !aligned(io->ppp, 8)))
        return fail(SP_ERR_INVALID_ARG, "io n_active / ppp must be NULL or aligned");
    return SP_OK;
}

// The whole path for one batch on `s`, every buffer, the key and the pair-id
// offset taken from the plan's device-side descriptor.
hipError_t enqueue_batch(synthpix_plan* P, const synthpix_tiling& t, hipStream_t s, bool with_advance)
{
    const synthpix_batch_io& io = P->io;
    const synthpix_batch_io* iod = P->io_dev;
    // masked candidates (slots past each pair's active count) are seeded but not
    // ordered, advected, prepared or binned: the seed sets their frame-2
    // position to frame 1's
    hipError_t e = sp::launch_seed(P->pairs_dev, P->n_pairs, P->span, P->sp, io.seed, io.x1, io.y1, io.z, io.d,
                                   io.I0, io.n_active, io.ppp, s, iod, P->live);
    if (e != hipSuccess) return e;
    sp::AdvectOrder order{nullptr, nullptr};
    e = enqueue_order(P->pairs_host.data(), P->pairs_dev, P->n_pairs, io.x1, io.y1, static_cast<char*>(P->workspace),
                      0, s, &order, iod, P->live);
    if (e != hipSuccess) return e;
    e = sp::launch_advect(P->pairs_dev, P->n_pairs, P->span, io.flow, P->ap, io.x1, io.y1, io.x2, io.y2, s, order,
                          iod);
    if (e != hipSuccess) return e;
    const sp::RenderConfig cfg = make_config(P->rp, t);
    sp::BatchTotals T;
    if (batch_totals(P->pairs_host.data(), P->n_pairs, cfg, &T) != SP_OK) return hipErrorInvalidValue;
    const sp::WorkspaceLayout wl = workspace_layout(P->n_pairs, T, 0, P->pairs_host.data());
    e = enqueue_render(P->pairs_dev, P->n_pairs, cfg, T, wl, io.x1, io.y1, io.x2, io.y2, io.z, io.d, io.I0, P->rp,
                       io.images, P->workspace, s, iod, nullptr, P->live);
    if (e != hipSuccess) return e;
    if (with_advance && P->advance) e = sp::launch_advance(P->io_dev, (uint64_t)P->n_pairs, s);
    return e;
}

const int CHUNK_CANDIDATES[] = {1024, 4096, 8192};

// Tile shape x LDS capacity candidates (2048-particle binning blocks), default first.
std::vector<synthpix_tiling> shape_candidates(const synthpix_render_params& rp)
{
    std::vector<synthpix_tiling> out;
    out.push_back(default_tiling());
    const int shapes[][2] = {{32, 32}, {64, 32}, {64, 64}, {128, 32}, {32, 16}, {64, 16}};
    const int caps[] = {32, 64, 128};
    for (const auto& sh : shapes)
        for (int cap : caps) {
            synthpix_tiling t{sh[0], sh[1], 2048, cap, 0};
            if (t.tile_w == out[0].tile_w && t.tile_h == out[0].tile_h && t.cap == out[0].cap) continue;
            if (sp::render_lds_bytes(make_config(rp, t)) > 160 * 1024) continue;
            out.push_back(t);
        }
    return out;
}

void plan_free(synthpix_plan* P)
{
    if (!P) return;
    if (P->exec) hipGraphExecDestroy(P->exec);
    if (P->graph) hipGraphDestroy(P->graph);
    if (P->capture) hipStreamDestroy(P->capture);
    if (P->workspace) hipFree(P->workspace);
    if (P->io_dev) hipFree(P->io_dev);
    if (P->pairs_dev) hipFree(P->pairs_dev);
    delete P;
}

}  // namespace

extern "C" {

synthpix_status synthpix_tiling_candidates(const synthpix_render_params* rp, synthpix_tiling* out, int32_t max_out,
                                           int32_t* n_out)
{
    if (!n_out || (max_out > 0 && !out)) return fail(SP_ERR_INVALID_ARG, "out and n_out must be non-NULL");
    synthpix_status st = check_render_params(rp);
    if (st) return st;
    std::vector<synthpix_tiling> c = shape_candidates(*rp);
    for (int ch : CHUNK_CANDIDATES) c.push_back(synthpix_tiling{c[0].tile_w, c[0].tile_h, ch, c[0].cap, 0});
    c.push_back(synthpix_tiling{c[0].tile_w, c[0].tile_h, c[0].chunk, c[0].cap, 1});
    for (int32_t i = 0; i < max_out && i < (int32_t)c.size(); ++i) out[i] = c[i];
    *n_out = (int32_t)c.size();
    return SP_OK;
}

synthpix_status synthpix_plan_create(const synthpix_pair* pairs_host, int32_t n_pairs,
                                     const synthpix_seed_params* sp_, const synthpix_advect_params* ap,
                                     const synthpix_render_params* rp, const synthpix_batch_io* io,
                                     int32_t autotune, int32_t advance_pair_ids, void* stream, synthpix_plan** out)
{
    if (!out) return fail(SP_ERR_INVALID_ARG, "out must be non-NULL");
    *out = nullptr;
    int64_t span;
    synthpix_status st = check_pairs(pairs_host, pairs_host, n_pairs, &span);
    if (st) return st;
    if ((st = check_seed_params(sp_, pairs_host, n_pairs))) return st;
    if ((st = check_advect_params(ap))) return st;
    if ((st = check_render_params(rp))) return st;
    if ((st = check_io(io, rp->bits))) return st;
    if (model_in_use(*rp, nullptr))
        return fail(SP_ERR_UNSUPPORTED, "plans run the isotropic model (no frame-2 variation, no hiding, the Gaussian "
                    "sheet); use the eager calls for the full model");
    if (order_bytes(pairs_host, n_pairs) == 0) return fail(SP_ERR_UNSUPPORTED, "batch too large for the advection order");
    const synthpix_tiling t0 = default_tiling();
    {
        sp::BatchTotals T;
        if ((st = batch_totals(pairs_host, n_pairs, make_config(*rp, t0), &T))) return st;
    }
    synthpix_plan* P = new synthpix_plan();
    P->n_pairs = n_pairs;
    P->pairs_host.assign(pairs_host, pairs_host + n_pairs);
    P->sp = *sp_;
    P->ap = *ap;
    P->rp = *rp;
    P->io = *io;
    P->advance = advance_pair_ids ? 1 : 0;
    P->span = span;
    hipStream_t s = as_stream(stream);
    hipError_t e = hipGetDevice(&P->device);
    if (e == hipSuccess) e = hipMalloc(&P->pairs_dev, sizeof(synthpix_pair) * (size_t)n_pairs);
    if (e == hipSuccess) e = hipMalloc(&P->io_dev, sizeof(synthpix_batch_io));
    if (e == hipSuccess)
        e = hipMemcpy(P->pairs_dev, pairs_host, sizeof(synthpix_pair) * (size_t)n_pairs, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = sp::launch_store_io(P->io_dev, *io, s);
    if (e != hipSuccess) {
        plan_free(P);
        return hip_fail(e, "plan set-up");
    }
    // workspace for the largest candidate (every shape with every binning block size)
    std::vector<synthpix_tiling> shapes = autotune ? shape_candidates(*rp) : std::vector<synthpix_tiling>{t0};
    size_t ws = order_bytes(pairs_host, n_pairs);   // the advection order shares the render workspace
    std::vector<synthpix_tiling> ok;
    for (const auto& t : shapes) {
        sp::BatchTotals T;
        if (batch_totals(pairs_host, n_pairs, make_config(*rp, t), &T) != SP_OK) continue;
        ws = std::max(ws, workspace_layout(n_pairs, T, 0, pairs_host).total);
        if (autotune)
            for (int ch : CHUNK_CANDIDATES) {
                synthpix_tiling tc = t;
                tc.chunk = ch;
                if (batch_totals(pairs_host, n_pairs, make_config(*rp, tc), &T) == SP_OK)
                    ws = std::max(ws, workspace_layout(n_pairs, T, 0, pairs_host).total);
            }
        ok.push_back(t);
    }
    g_err.clear();
    if (ok.empty()) {
        plan_free(P);
        return fail(SP_ERR_UNSUPPORTED, "no tiling fits this batch");
    }
    const size_t live_off = align256(ws);
    ws = live_off + align256(sizeof(int32_t) * (size_t)n_pairs);
    e = hipMalloc(&P->workspace, ws);
    P->ws_bytes = ws;
    if (e != hipSuccess) {
        plan_free(P);
        return hip_fail(e, "plan workspace");
    }
    P->live = reinterpret_cast<int32_t*>(static_cast<char*>(P->workspace) + live_off);
    P->tiling = ok[0];
    if (autotune) {
        // time each candidate's render of this batch (seed/advect once, render warm-up + 3 runs):
        // first every shape x capacity, then the binning block sizes for the fastest
        e = enqueue_batch(P, ok[0], s, false);
        hipEvent_t a = nullptr, b = nullptr;
        if (e == hipSuccess) e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        float best = 1e30f;
        auto time_one = [&](const synthpix_tiling& t) {
            const sp::RenderConfig cfg = make_config(*rp, t);
            sp::BatchTotals T;
            if (batch_totals(pairs_host, n_pairs, cfg, &T) != SP_OK) return;
            const sp::WorkspaceLayout wl = workspace_layout(n_pairs, T, 0, pairs_host);
            auto run = [&]() {
                return enqueue_render(P->pairs_dev, n_pairs, cfg, T, wl, io->x1, io->y1, io->x2, io->y2, io->z,
                                      io->d, io->I0, *rp, io->images, P->workspace, s, P->io_dev);
            };
            e = run();
            if (e == hipSuccess) e = hipEventRecord(a, s);
            for (int r = 0; r < 3 && e == hipSuccess; ++r) e = run();
            if (e == hipSuccess) e = hipEventRecord(b, s);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            if (e == hipSuccess && ms < best) {
                best = ms;
                P->tiling = t;
            }
        };
        for (size_t i = 0; i < ok.size() && e == hipSuccess; ++i) time_one(ok[i]);
        const synthpix_tiling shape_best = P->tiling;
        for (int ch : CHUNK_CANDIDATES) {
            if (e != hipSuccess) break;
            synthpix_tiling tc = shape_best;
            tc.chunk = ch;
            time_one(tc);
        }
        // then the persistent form of the fastest
        if (e == hipSuccess) {
            synthpix_tiling tp = P->tiling;
            tp.persistent = 1;
            time_one(tp);
        }
        if (a) hipEventDestroy(a);
        if (b) hipEventDestroy(b);
        if (e != hipSuccess) {
            plan_free(P);
            return hip_fail(e, "autotuning");
        }
    }
    // capture the whole path once
    e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->capture, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(P->capture, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t ee = enqueue_batch(P, P->tiling, P->capture, true);
        e = hipStreamEndCapture(P->capture, &P->graph);
        if (ee != hipSuccess) e = ee;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        plan_free(P);
        return hip_fail(e, "graph capture");
    }
    *out = P;
    return SP_OK;
}

synthpix_status synthpix_plan_launch(synthpix_plan* plan, const synthpix_batch_io* io, void* stream)
{
    if (!plan || !plan->exec) return fail(SP_ERR_INVALID_ARG, "plan must be a created plan");
    if (io) {
        const synthpix_status st = check_io(io, plan->rp.bits);
        if (st) return st;
        const hipError_t e = sp::launch_store_io(plan->io_dev, *io, as_stream(stream));
        if (e != hipSuccess) return hip_fail(e, "io descriptor store");
    }
    const hipError_t e = hipGraphLaunch(plan->exec, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return SP_OK;
}

synthpix_status synthpix_plan_read_status(const synthpix_plan* plan, void* stream, uint32_t* flags)
{
    if (!plan || !plan->workspace) return fail(SP_ERR_INVALID_ARG, "plan must be a created plan");
    return synthpix_read_status(plan->workspace, stream, flags);
}

synthpix_status synthpix_plan_tiling(const synthpix_plan* plan, synthpix_tiling* out)
{
    if (!plan || !out) return fail(SP_ERR_INVALID_ARG, "plan and out must be non-NULL");
    *out = plan->tiling;
    return SP_OK;
}

synthpix_status synthpix_plan_destroy(synthpix_plan* plan)
{
    plan_free(plan);
    return SP_OK;
}

}  // extern "C"
