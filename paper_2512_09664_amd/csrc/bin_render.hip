// Screen-tile binning and the fused tile renderer (gfx950).
//
// Rendering follows Eq. 1 (rho = 0, sigma = d/4) with a Gaussian laser-sheet
// peak (Remark 1), point-sampled at pixel centres (Remark 2), summed over all
// particles (Section 2, "Considerations on the aggregation") on per-particle
// square patches |dx|, |dy| <= 1.5 d (Section 2, "Efficient rasterization").
//
// Pipeline of one call (all pairs of a batch at once):
//   bin_layout  : per-pair prefix tables (one block)
//   prep        : per particle and frame, a 16-byte record (x, y, d, fixed-point
//                 peak); d < 0 marks a particle that adds nothing
//   bin_count   : per (pair, frame, particle chunk) LDS histogram of tile hits
//   bin_scan    : per tile, chunk bases inside its list and its total; per
//                 (pair, frame), the exclusive scan of the totals -> list offsets
//   bin_scatter : per chunk, LDS cursors -> particle indices into tile lists
//   render_tile : per (pair, frame, tile) stage the list in LDS, splat footprints
//                 into an LDS fixed-point accumulator (tile + blur apron), then
//                 blur, noise, quantise and store.
// No global atomics: counts, cursors and pixel sums all live in LDS.  Pixel sums
// are exact 32-bit fixed point, so the LDS atomics' order does not matter.
#include <map>
#include <mutex>
#include <utility>

#include "device_math.hpp"
#include "launch.hpp"

namespace sp {

__device__ __forceinline__ int find_pair_by_chunk(const PairLayout* L, int n_pairs, int64_t c)
{
    int lo = 0, hi = n_pairs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L[mid].chunk_base <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------------ layout

__global__ void __launch_bounds__(256)
bin_layout(const synthpix_pair* __restrict__ pairs, int n_pairs, RenderConfig cfg,
           PairLayout* __restrict__ L, uint32_t* __restrict__ status)
{
    __shared__ int64_t s_part[4][256];
    __shared__ int64_t s_carry[4];
    const int t = threadIdx.x;
    if (t < 4) s_carry[t] = 0;
    // status words, and the renderer's per-XCD work queues (words 8 .. 15)
    if (t < 16) status[t] = 0u;
    __syncthreads();
    for (int base = 0; base < n_pairs; base += 256) {
        const int p = base + t;
        int64_t v[4] = {0, 0, 0, 0};
        int n_chunks = 0, ntx = 0, nty = 0;
        int64_t cap = 0;
        if (p < n_pairs) {
            const synthpix_pair P = pairs[p];
            n_chunks = (P.n_max + cfg.chunk - 1) / cfg.chunk;
            ntx = (P.W + cfg.tile_w - 1) / cfg.tile_w;
            nty = (P.H + cfg.tile_h - 1) / cfg.tile_h;
            cap = (int64_t)P.n_max * cfg.kx * cfg.ky;
            v[0] = n_chunks;
            v[1] = (int64_t)ntx * nty;
            v[2] = 2 * (int64_t)n_chunks * ntx * nty;
            v[3] = 2 * cap;
        }
        for (int k = 0; k < 4; ++k) s_part[k][t] = v[k];
        __syncthreads();
        // Hillis-Steele inclusive scan of the four columns
        for (int off = 1; off < 256; off <<= 1) {
            int64_t add[4];
            for (int k = 0; k < 4; ++k) add[k] = t >= off ? s_part[k][t - off] : 0;
            __syncthreads();
            for (int k = 0; k < 4; ++k) s_part[k][t] += add[k];
            __syncthreads();
        }
        if (p < n_pairs) {
            PairLayout o;
            o.chunk_base = (int32_t)(s_carry[0] + s_part[0][t] - v[0]);
            o.n_chunks = n_chunks;
            o.tile_base = (int32_t)(s_carry[1] + s_part[1][t] - v[1]);
            o.ntx = ntx;
            o.nty = nty;
            o.pad_ = 0;
            o.hist_base = s_carry[2] + s_part[2][t] - v[2];
            o.entry_base = s_carry[3] + s_part[3][t] - v[3];
            o.entry_cap = cap;
            L[p] = o;
        }
        __syncthreads();
        if (t < 4) s_carry[t] += s_part[t][255];
        __syncthreads();
    }
}

// ------------------------------------------------------------------ particle records

// Per particle and frame: the record (x, y, kappa, Af) with kappa = 8 / (d d)
// and Af = min(2^24 I0 exp(-z^2 / (2 s^2)), 2^32 - 256), and the patch box
// |dx|, |dy| <= 1.5 d clipped to the image (computed once here for every tile
// list and tile that uses the particle).  Particles that add nothing (I0 <= 0,
// d <= 0 or not a number, non-finite position) or whose d exceeds d_max
// (flagged) get an empty box.  With live counts (captured plans), the masked
// slots past a pair's count are skipped: the binning passes skip them too.
__global__ void __launch_bounds__(256)
prep_records(const synthpix_pair* __restrict__ pairs, int n_pairs, int64_t n_span, RenderArgs a,
             float d_max, float4* __restrict__ rec0, float4* __restrict__ rec1, uint2* __restrict__ box0,
             uint2* __restrict__ box1, uint32_t* __restrict__ status)
{
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t g = g0 + threadIdx.x;
    if (g >= n_span) return;
    const int p = find_pair_from(pairs, n_pairs, g0, g);
    const int64_t i = g - pairs[p].particle_offset;
    if (i < 0 || i >= (a.live ? (int64_t)min(a.live[p], pairs[p].n_max) : (int64_t)pairs[p].n_max)) return;
    if (a.iod) {
        a.x[0] = a.iod->x1;
        a.y[0] = a.iod->y1;
        a.x[1] = a.iod->x2;
        a.y[1] = a.iod->y2;
        a.z = a.iod->z;
        a.d = a.iod->d;
        a.I0 = a.iod->I0;
    }
    const int W = pairs[p].W, H = pairs[p].H;
    const float cs = 0.5f / (a.sheet_sigma * a.sheet_sigma);
    const float z = a.z[g], d = a.d[g], I0 = a.I0[g];
    const float x1 = a.x[0][g], y1 = a.y[0][g], x2 = a.x[1][g], y2 = a.y[1][g];
    const float Af = fixed_peak(I0 * expneg((z * z) * cs));
    bool live = (I0 > 0.0f) && (d > 0.0f);
    if (live && !(d <= d_max)) {
        atomicOr(status, SP_STATUS_D_ABOVE_MAX);
        live = false;
    }
    const float R = 1.5f * d;
    const uint2 empty = make_uint2(EMPTY_BOX, EMPTY_BOX);
    const float kap = live ? 8.0f / (d * d) : 0.0f;
    rec0[g] = make_float4(x1, y1, kap, Af);
    rec1[g] = make_float4(x2, y2, kap, Af);
    box0[g] = live ? patch_box(x1, y1, R, R, W, H) : empty;
    box1[g] = live ? patch_box(x2, y2, R, R, W, H) : empty;
}

// The full particle model's records (Eq. 1 with sigma_y and rho; frame-2
// parameter variation, the sentence after Eq. 1; per-frame hiding, Section 2
// "Considerations on the aggregation"; the Remark 1 sheet law; frame-2 z from
// the out-of-plane motion).  Per particle and frame: the record (x, y, d or -1,
// 2^24 A) and, in the anisotropic layout, (d_y, rho).  Frame-2 parameters are
// frame 1's plus zero-mean Gaussians (Philox stream 2: Box-Muller of words 0, 1
// and 2, 3, cosine then sine, for d, d_y, rho, I0), clipped to [0, d_max],
// [-0.99, 0.99] and [0, inf) (masked particles stay dark); a particle is hidden
// in frame f when word f of stream 7 is below hide_p.
__device__ __forceinline__ float model_peak(float I0, float z, const RenderArgs& a)
{
    if (a.sheet_law == 0) return I0 * expneg((z * z) * (0.5f / (a.sheet_sigma * a.sheet_sigma)));
    // Remark 1: exp(-(1/sqrt(2 pi)) v^s), v = z^2 (2 / DZ0^2); v^s = exp(s ln v)
    const float v = (z * z) * (2.0f / (a.sheet_dz0 * a.sheet_dz0));
    float pw = 0.0f;
    if (v >= 0x1p-126f) {
        const float e = a.sheet_shape * log_ra(v);
        if (!(e < 80.0f)) return 0.0f;
        pw = expneg(-e);
    }
    return I0 * expneg((float)0.39894228040143267794 * pw);
}

__global__ void __launch_bounds__(256)
prep_records_model(const synthpix_pair* __restrict__ pairs, int n_pairs, int64_t n_span, RenderArgs a, float d_max,
                   float4* __restrict__ rec0, float4* __restrict__ rec1, uint2* __restrict__ box0,
                   uint2* __restrict__ box1, float2* __restrict__ shp0, float2* __restrict__ shp1,
                   uint32_t* __restrict__ status)
{
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t g = g0 + threadIdx.x;
    if (g >= n_span) return;
    const int p = find_pair_from(pairs, n_pairs, g0, g);
    const int64_t i = g - pairs[p].particle_offset;
    if (i < 0 || i >= pairs[p].n_max) return;
    const uint64_t pid = pairs[p].pair_id;
    const float x1 = a.x[0][g], y1 = a.y[0][g], x2 = a.x[1][g], y2 = a.y[1][g];
    const float z1 = a.z[g];
    const float z2 = a.z2 ? a.z2[g] : z1;
    const float d = a.d[g];
    const float dy = a.dy ? a.dy[g] : d;
    const float r = a.rho ? a.rho[g] : 0.0f;
    const float I = a.I0[g];
    float d2 = d, dy2 = dy, r2 = r, I2 = I;
    if (a.jit_d > 0.0f || a.jit_rho > 0.0f || a.jit_I0 > 0.0f) {
        const u32x4 w = draw((uint32_t)i, STREAM_JITTER, pid, a.seed);
        const float R0 = __builtin_sqrtf(-2.0f * log_ra(u24_open0(w.a)));
        const float R1 = __builtin_sqrtf(-2.0f * log_ra(u24_open0(w.c)));
        const float2 t0 = cossin2pi_ra(u24(w.b));
        const float2 t1 = cossin2pi_ra(u24(w.d));
        if (a.jit_d > 0.0f) {
            d2 = __builtin_fminf(__builtin_fmaxf(__builtin_fmaf(a.jit_d, R0 * t0.x, d), 0.0f), d_max);
            dy2 = __builtin_fminf(__builtin_fmaxf(__builtin_fmaf(a.jit_d, R0 * t0.y, dy), 0.0f), d_max);
        }
        if (a.jit_rho > 0.0f) r2 = __builtin_fminf(__builtin_fmaxf(__builtin_fmaf(a.jit_rho, R1 * t1.x, r), -0.99f), 0.99f);
        if (a.jit_I0 > 0.0f) I2 = I > 0.0f ? __builtin_fmaxf(__builtin_fmaf(a.jit_I0, R1 * t1.y, I), 0.0f) : 0.0f;
    }
    float I1 = I;
    if (a.hide_p > 0.0f) {
        const u32x4 w = draw((uint32_t)i, STREAM_HIDE, pid, a.seed);
        if (u24(w.a) < a.hide_p) I1 = 0.0f;
        if (u24(w.b) < a.hide_p) I2 = 0.0f;
    }
    const float dd[2] = {d, d2}, ddy[2] = {dy, dy2}, rr[2] = {r, r2}, II[2] = {I1, I2};
    const float xx[2] = {x1, x2}, yy[2] = {y1, y2}, zz[2] = {z1, z2};
    const int W = pairs[p].W, H = pairs[p].H;
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        bool live = (II[f] > 0.0f) && (dd[f] > 0.0f) && (ddy[f] > 0.0f);
        if (live && !(dd[f] <= d_max && ddy[f] <= d_max)) {
            atomicOr(status, SP_STATUS_D_ABOVE_MAX);
            live = false;
        }
        if (live && !(__builtin_fabsf(rr[f]) <= 0.99f)) {
            atomicOr(status, SP_STATUS_BAD_SHAPE);
            live = false;
        }
        // om = 1 - rho^2; kappa_x = 8 / (om d^2), kappa_y = 8 / (om d_y^2),
        // kappa_xy = -16 rho / (om d d_y) (0 for rho = 0: the separable form)
        const float om = __builtin_fmaf(-rr[f], rr[f], 1.0f);
        const float kx = live ? 8.0f / (om * (dd[f] * dd[f])) : 0.0f;
        const float ky = live ? 8.0f / (om * (ddy[f] * ddy[f])) : 0.0f;
        const float kxy = (live && rr[f] != 0.0f) ? (-16.0f * rr[f]) / (om * (dd[f] * ddy[f])) : 0.0f;
        (f ? rec1 : rec0)[g] = make_float4(xx[f], yy[f], kx, fixed_peak(model_peak(II[f], zz[f], a)));
        (f ? box1 : box0)[g] = live ? patch_box(xx[f], yy[f], 1.5f * dd[f], 1.5f * ddy[f], W, H)
                                    : make_uint2(EMPTY_BOX, EMPTY_BOX);
        if (a.aniso) (f ? shp1 : shp0)[g] = make_float2(ky, kxy);
    }
}

// ------------------------------------------------------------------ membership

// ------------------------------------------------------------------ count / scatter

template <bool SCATTER>
__global__ void __launch_bounds__(256)
bin_pass(const synthpix_pair* __restrict__ pairs, const PairLayout* __restrict__ L, int n_pairs,
         const uint2* __restrict__ box0, const uint2* __restrict__ box1, RenderConfig cfg, uint32_t* __restrict__ hist,
         const int64_t* __restrict__ tile_offset, int64_t tiles_total, int32_t* __restrict__ entries,
         unsigned n_chunks_total, const int32_t* __restrict__ live)
{
    extern __shared__ uint32_t lh[];
    const int f = blockIdx.y;
    const unsigned cb = xcd_contiguous(blockIdx.x, n_chunks_total);
    const int p = find_pair_by_chunk(L, n_pairs, cb);
    const synthpix_pair P = pairs[p];
    const PairLayout PL = L[p];
    const int chunk = (int)cb - PL.chunk_base;
    const int nt = PL.ntx * PL.nty;
    uint32_t* gh = hist + PL.hist_base + ((int64_t)f * PL.n_chunks + chunk) * nt;
    int32_t* seg = entries + PL.entry_base + (int64_t)f * PL.entry_cap;
    // scatter cursors start at the chunk's first slot in each tile list
    const int64_t* toff = tile_offset + f * tiles_total + PL.tile_base;
    const int64_t seg0 = PL.entry_base + (int64_t)f * PL.entry_cap;
    const int i_end = min(live ? min(live[p], P.n_max) : P.n_max, (chunk + 1) * cfg.chunk);
    // a chunk past the live slots holds nothing (and is not scanned): the whole
    // workgroup returns before its barrier
    if (live && chunk * cfg.chunk >= i_end) return;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) lh[t] = SCATTER ? gh[t] + (uint32_t)(toff[t] - seg0) : 0u;
    __syncthreads();
    const uint2* __restrict__ bxs = f ? box1 : box0;
    // BIN_ILP particles per thread and step: their box loads and LDS atomic
    // round trips overlap
    constexpr int BIN_ILP = 4;
    for (int i0 = chunk * cfg.chunk + threadIdx.x; i0 < i_end; i0 += BIN_ILP * blockDim.x) {
        uint2 r[BIN_ILP];
#pragma unroll
        for (int q = 0; q < BIN_ILP; ++q) {
            const int i = i0 + q * blockDim.x;
            r[q] = i < i_end ? bxs[P.particle_offset + i] : make_uint2(EMPTY_BOX, EMPTY_BOX);
        }
#pragma unroll
        for (int q = 0; q < BIN_ILP; ++q) {
            const int i = i0 + q * blockDim.x;
            int tx0, tx1, ty0, ty1;
            if (!tile_rect(r[q], cfg, PL.ntx, PL.nty, tx0, tx1, ty0, ty1)) continue;
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) {
                    const uint32_t slot = atomicAdd(&lh[ty * PL.ntx + tx], 1u);
                    if (SCATTER) seg[slot] = i;
                }
        }
    }
    if (!SCATTER) {
        __syncthreads();
        for (int t = threadIdx.x; t < nt; t += blockDim.x) gh[t] = lh[t];
    }
}

// ------------------------------------------------------------------ home order

// A spatial processing order for per-particle work that samples the flow grid:
// particle i of a pair goes to the block (a "tile" of the order's config) that
// holds its clamped position.  Blocks are numbered in strips of four block
// rows, column by column inside a strip, odd strips from right to left (so the
// last block of a strip and the first of the next are neighbours): a run of
// consecutive entries (one workgroup's particles) covers a compact patch of
// the image.  Count and
// scatter passes as for the tile lists, one entry per particle, in the frame-1
// half of the lists.
__device__ __forceinline__ int home_block(float x, float y, int W, int H, const PairLayout& PL,
                                          const RenderConfig& cfg)
{
    const int cx = !(x >= 0.0f) ? 0 : (x >= (float)W ? W - 1 : (int)x);
    const int cy = !(y >= 0.0f) ? 0 : (y >= (float)H ? H - 1 : (int)y);
    const int bx = cx >> cfg.log_tw, by = cy >> cfg.log_th;
    const int s0 = by & ~3;                                   // first block row of the strip
    const int rows = PL.nty - s0 < 4 ? PL.nty - s0 : 4;       // rows in this strip
    const int col = (by & 4) ? PL.ntx - 1 - bx : bx;          // odd strips run right to left
    return s0 * PL.ntx + col * rows + (by - s0);
}

template <bool SCATTER>
__global__ void __launch_bounds__(256)
order_pass(const synthpix_pair* __restrict__ pairs, const PairLayout* __restrict__ L, int n_pairs,
           const float* __restrict__ x, const float* __restrict__ y, RenderConfig cfg, uint32_t* __restrict__ hist,
           const int64_t* __restrict__ tile_offset, int32_t* __restrict__ entries, unsigned n_chunks_total,
           const synthpix_batch_io* __restrict__ iod, const int32_t* __restrict__ live)
{
    extern __shared__ uint32_t lh[];
    if (iod) {
        x = iod->x1;
        y = iod->y1;
    }
    const unsigned cb = xcd_contiguous(blockIdx.x, n_chunks_total);
    const int p = find_pair_by_chunk(L, n_pairs, cb);
    const synthpix_pair P = pairs[p];
    const PairLayout PL = L[p];
    const int chunk = (int)cb - PL.chunk_base;
    const int nt = PL.ntx * PL.nty;
    uint32_t* gh = hist + PL.hist_base + (int64_t)chunk * nt;
    int32_t* seg = entries + PL.entry_base;
    const int64_t* toff = tile_offset + PL.tile_base;
    const int i_end = min(live ? min(live[p], P.n_max) : P.n_max, (chunk + 1) * cfg.chunk);
    // a chunk past the live slots holds nothing (and is not scanned): the whole
    // workgroup returns before its barrier
    if (live && chunk * cfg.chunk >= i_end) return;
    for (int t = threadIdx.x; t < nt; t += blockDim.x)
        lh[t] = SCATTER ? gh[t] + (uint32_t)(toff[t] - PL.entry_base) : 0u;
    __syncthreads();
    for (int i = chunk * cfg.chunk + threadIdx.x; i < i_end; i += blockDim.x) {
        const int64_t g = P.particle_offset + i;
        const uint32_t slot = atomicAdd(&lh[home_block(x[g], y[g], P.W, P.H, PL, cfg)], 1u);
        if (SCATTER) seg[slot] = i;
    }
    if (!SCATTER) {
        __syncthreads();
        for (int t = threadIdx.x; t < nt; t += blockDim.x) gh[t] = lh[t];
    }
}

// Per (pair, frame, tile), one thread each: exclusive prefix of the chunk
// histograms over the chunks, in place (each chunk's first slot inside the
// tile's list), and the tile's total.  Consecutive threads take consecutive
// tiles, so every chunk row is read and written with coalesced accesses.  With
// live counts only the chunks that hold a live slot are scanned (the count and
// scatter passes of the others return at once).
__global__ void __launch_bounds__(256)
scan_chunks(const PairLayout* __restrict__ L, int n_pairs, uint32_t* __restrict__ hist,
            uint32_t* __restrict__ tile_count, int64_t tiles_total, const int32_t* __restrict__ live, int chunk)
{
    const int f = blockIdx.y;
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gt >= tiles_total) return;
    const int p = find_pair_by_tile(L, n_pairs, gt);
    const PairLayout PL = L[p];
    const int nt = PL.ntx * PL.nty;
    const int t = (int)(gt - PL.tile_base);
    const int nc = live ? min(PL.n_chunks, (max(live[p], 0) + chunk - 1) / chunk) : PL.n_chunks;
    uint32_t* h = hist + PL.hist_base + (int64_t)f * PL.n_chunks * nt + t;
    constexpr int U = 8;                 // chunk rows loaded together
    uint32_t run = 0;
    for (int c0 = 0; c0 < nc; c0 += U) {
        uint32_t v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = c0 + k < nc ? h[(int64_t)(c0 + k) * nt] : 0u;
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (c0 + k < nc) h[(int64_t)(c0 + k) * nt] = run;
            run += v[k];
        }
    }
    tile_count[f * tiles_total + gt] = run;
}

// Per (pair, frame): exclusive scan of the tile totals -> absolute offsets of
// the tile lists (the pair-frame segment's base plus the prefix).
__global__ void __launch_bounds__(256)
scan_tiles(const PairLayout* __restrict__ L, const uint32_t* __restrict__ tile_count,
           int64_t* __restrict__ tile_offset, int64_t tiles_total)
{
    __shared__ uint32_t s_wave[4];
    const int p = blockIdx.x;
    const int f = blockIdx.y;
    const PairLayout PL = L[p];
    const int nt = PL.ntx * PL.nty;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t* cnt = tile_count + f * tiles_total + PL.tile_base;
    int64_t* out = tile_offset + f * tiles_total + PL.tile_base;
    int64_t carry = PL.entry_base + (int64_t)f * PL.entry_cap;
    for (int b = 0; b < nt; b += 256) {
        const int t = b + threadIdx.x;
        const uint32_t v = t < nt ? cnt[t] : 0u;
        uint32_t inc = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t x = __shfl_up(inc, off, 64);
            if (lane >= off) inc += x;
        }
        if (lane == 63) s_wave[wid] = inc;
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint32_t sw = s_wave[w];
            if (w < wid) before += sw;
            total += sw;
        }
        if (t < nt) out[t] = carry + (int64_t)(before + inc - v);
        carry += total;
        __syncthreads();
    }
}

// ------------------------------------------------------------------ render

// LDS carve-up of one render workgroup (all offsets 16-byte aligned).
struct RenderLds {
    int acc_words;           // RH * RW + 8 of slack, rounded up to a multiple of 4
    int tables;              // CAP * WM4 floats per table
    size_t bytes;
};

__host__ __device__ inline RenderLds render_lds_shape(int tw, int th, int apron, int cap, int wm4, bool aniso)
{
    RenderLds L;
    const int RW = tw + 2 * apron, RH = th + 2 * apron;
    L.acc_words = (RH * RW + 8 + 3) & ~3;
    L.tables = cap * wm4;
    size_t work = (size_t)cap * 16                                  // staged (x, y, kappa_x, Af)
                + (size_t)cap * 4                                   // staged patch box
                + (aniso ? (size_t)cap * 8 : 0)                     // staged (kappa_y, kappa_xy)
                + (size_t)L.tables * sizeof(float)                  // column factors gx
                + (size_t)L.tables * sizeof(uint16_t)               // work items
                + 64;                                                // scan scratch
    size_t blur = (size_t)RH * tw * sizeof(float);
    L.bytes = (size_t)L.acc_words * 4 + (work > blur ? work : blur);
    return L;
}

__host__ __device__ inline RenderLds render_lds(const RenderConfig& c, bool aniso)
{
    return render_lds_shape(c.tile_w, c.tile_h, c.apron, c.cap, c.wm4, aniso);
}

// Exclusive scan of one counter over a workgroup of 256 threads (4 waves of
// 64) in which only the first n threads can hold a nonzero value: waves past
// them skip their in-wave scan.  In-wave inclusive scan with DPP: row shifts
// by 1, 2, 4, 8 within each row of 16 lanes, then the row broadcasts of lanes
// 15 and 31 into the rows above.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_add(int v)
{
    return v + __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, false);
}

__device__ __forceinline__ int stage_scan(int v, int n, int* s_wave, int& total)
{
    const int wid = threadIdx.x >> 6;
    int inc = v;
    if (wid * 64 < n) {
        inc = dpp_add<0x111, 0xF>(inc);
        inc = dpp_add<0x112, 0xF>(inc);
        inc = dpp_add<0x114, 0xF>(inc);
        inc = dpp_add<0x118, 0xF>(inc);
        inc = dpp_add<0x142, 0xA>(inc);
        inc = dpp_add<0x143, 0xC>(inc);
    }
    if ((threadIdx.x & 63) == 63) s_wave[wid] = inc;
    __syncthreads();
    int before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const int sw = s_wave[w];
        if (w < wid) before += sw;
        total += sw;
    }
    return before + inc - v;
}

__device__ __forceinline__ uint32_t pack_box(int c0, int w, int r0, int h)
{
    return (uint32_t)c0 | ((uint32_t)w << 8) | ((uint32_t)r0 << 16) | ((uint32_t)h << 24);
}

// Tile renderer, templated on the tile shape and the blur radius (tile-local
// index arithmetic becomes shifts, blur loops unroll).  ANISO: the full model's
// particle images (Eq. 1 with sigma_y = d_y / 4 and rho, from the shape
// records): kappa_x = 8 / (om d^2), kappa_y = 8 / (om d_y^2), om = 1 - rho^2;
// rho = 0 keeps the separable factors (with kappa_y for the rows), rho != 0
// evaluates exp(-q) per pixel, q = dx (kappa_x dx + kappa_xy dy) + kappa_y dy^2,
// kappa_xy = -16 rho / (om d d_y); the patch is |dx| <= 1.5 d, |dy| <= 1.5 d_y.
template <int TW, int TH, int B, bool ANISO, bool PERSIST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PERSIST ? 6 : 8)))
render_tile(const synthpix_pair* __restrict__ pairs, const PairLayout* __restrict__ L, int n_pairs,
            const float4* __restrict__ rec0, const float4* __restrict__ rec1, const uint2* __restrict__ box0,
            const uint2* __restrict__ box1, const float2* __restrict__ shp0,
            const float2* __restrict__ shp1, EpilogueArgs a, int cap, int wm4,
            const uint32_t* __restrict__ tile_count, const int64_t* __restrict__ tile_offset,
            const int32_t* __restrict__ entries, int64_t tiles_total, uint32_t* __restrict__ status,
            uint32_t* __restrict__ queue)
{
    static_assert(TW % 4 == 0 && (TW & (TW - 1)) == 0 && (TH & (TH - 1)) == 0, "power-of-two tiles");
    static_assert(TW + 6 < 256 && TH + 6 < 256, "patch boxes are packed in bytes");
    static_assert(B >= 0 && B <= 3, "blur radius 0..3");
    constexpr int Q4 = TW / 4;
    float wb[2 * B + 1];
#pragma unroll
    for (int q = 0; q <= 2 * B; ++q) wb[q] = a.blur_w[q];
    extern __shared__ __align__(16) unsigned char smem[];
    const RenderLds lay = render_lds_shape(TW, TH, B, cap, wm4, ANISO);
    constexpr int b = B;
    constexpr int RW = TW + 2 * B;
    constexpr int RH = TH + 2 * B;
    const int WM = wm4;
    uint32_t* acc = reinterpret_cast<uint32_t*>(smem);
    float4* stg = reinterpret_cast<float4*>(acc + lay.acc_words);       // (x, y, kappa, Af)
    uint32_t* box = reinterpret_cast<uint32_t*>(stg + cap);              // c0 | w | r0 | h bytes
    float2* stg2 = reinterpret_cast<float2*>(box + cap);                // (kappa_y, kappa_xy), ANISO only
    float* gx = reinterpret_cast<float*>(ANISO ? reinterpret_cast<uint32_t*>(stg2 + cap) : box + cap);
    uint16_t* items = reinterpret_cast<uint16_t*>(gx + lay.tables);     // tables entries
    int* s_wave = reinterpret_cast<int*>(items + lay.tables);
    float* tmp = reinterpret_cast<float*>(stg);   // blur scratch, reuses the particle tables
    // fixed-point range bound: a difference array over the region's rows of the
    // staged particles' integer peaks (each particle's peak added over the rows
    // its patch covers).  Every term a particle adds to a pixel is at most its
    // peak, so a row's prefix sum bounds every pixel sum of that row.
    __shared__ unsigned long long s_rows[RH + 1];

    // PERSIST: a persistent work list.  Each workgroup pops (frame, tile) items
    // from the queue of its XCD until the queue is empty; the items of one XCD
    // form a contiguous range (workgroups are dispatched to the 8 XCDs
    // round-robin), so the neighbouring tiles in flight on an XCD share particle
    // records in its L2, and the grid is at most what the chip holds at once.
    // Otherwise one item per workgroup, numbered XCD-contiguously.
    __shared__ unsigned s_pop;
    uint64_t pid_base = 0;
    if (a.iod) {
        a.images = a.iod->images;
        a.seed = a.iod->seed;
        pid_base = a.iod->pair_id_base;
    }
    const unsigned n_items = (unsigned)(2 * tiles_total);
    const bool split = gridDim.x >= 8;
    const unsigned xq = split ? (blockIdx.x & 7u) : 0u;
    const unsigned q8 = n_items >> 3, r8 = n_items & 7u;
    const unsigned lo = split ? (xq < r8 ? xq * (q8 + 1) : r8 * (q8 + 1) + (xq - r8) * q8) : 0u;
    const unsigned len = split ? (xq < r8 ? q8 + 1 : q8) : n_items;
    for (;;) {
    int64_t item;
    if (PERSIST) {
        if (threadIdx.x == 0) s_pop = atomicAdd(&queue[xq], 1u);
        __syncthreads();
        const unsigned kq = (unsigned)__builtin_amdgcn_readfirstlane((int)s_pop);   // uniform: one scalar value
        if (kq >= len) break;             // the same value in every thread of the workgroup
        item = (int64_t)lo + kq;
    } else {
        item = xcd_contiguous(blockIdx.x, gridDim.x);
    }
    const int f = item >= tiles_total ? 1 : 0;
    const int64_t tile = item - (int64_t)f * tiles_total;
    const int p = find_pair_by_tile(L, n_pairs, tile);
    const int pW = pairs[p].W, pH = pairs[p].H;
    const int64_t p_off = pairs[p].particle_offset, p_img = pairs[p].image_offset;
    const uint64_t pid = pairs[p].pair_id + pid_base;
    const int64_t tile_base = L[p].tile_base;
    const int ntx = L[p].ntx;
    const int tl = (int)(tile - tile_base);
    const int ty = tl / ntx;
    const int tx = tl - ty * ntx;
    const int rx0 = tx * TW - b;          // region origin in image pixels
    const int ry0 = ty * TH - b;
    const int cnt = (int)tile_count[item];
    const int64_t off = tile_offset[item];
    const float4* __restrict__ rec = f ? rec1 : rec0;
    const uint2* __restrict__ bxs = f ? box1 : box0;
    const float2* __restrict__ shp = f ? shp1 : shp0;

    for (int k = threadIdx.x; k < (lay.acc_words >> 2); k += 256)
        reinterpret_cast<uint4*>(acc)[k] = make_uint4(0u, 0u, 0u, 0u);
    for (int k = threadIdx.x; k <= RH; k += 256) s_rows[k] = 0ull;

    // the record of a thread's particle in the next pass is loaded one pass ahead,
    // so its two dependent loads overlap the current pass's factor and splat work
    float4 next = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    uint2 next_bx = make_uint2(EMPTY_BOX, EMPTY_BOX);
    float2 next_sh = make_float2(0.0f, 0.0f);
    if ((int)threadIdx.x < min(cap, cnt)) {
        const int e = entries[off + threadIdx.x];
        next = rec[p_off + e];
        next_bx = bxs[p_off + e];
        if (ANISO) next_sh = shp[p_off + e];
    }
    for (int base = 0; base < cnt; base += cap) {
        const int n = min(cap, cnt - base);
        const float4 r = next;
        const uint2 pb = next_bx;
        const float2 rs = next_sh;
        if ((int)threadIdx.x < cap && base + cap + (int)threadIdx.x < cnt) {
            const int e = entries[off + base + cap + threadIdx.x];
            next = rec[p_off + e];
            next_bx = bxs[p_off + e];
            if (ANISO) next_sh = shp[p_off + e];
        }
        __syncthreads();
        // stage: one particle per thread; its patch box (image pixels) clipped to the region
        int w = 0, h = 0, c0 = 0, r0 = 0;
        if ((int)threadIdx.x < n) {
            if (!box_empty(pb)) {
                int a0 = (int)(pb.x & 0xffffu), a1 = (int)(pb.x >> 16);
                int b0 = (int)(pb.y & 0xffffu), b1 = (int)(pb.y >> 16);
                a0 = max(a0, rx0);
                a1 = min(a1, rx0 + RW - 1);
                b0 = max(b0, ry0);
                b1 = min(b1, ry0 + RH - 1);
                if (a0 <= a1 && b0 <= b1) {
                    w = a1 - a0 + 1;
                    h = b1 - b0 + 1;
                    if (w > WM || h > WM) {            // cannot happen for d <= d_max
                        atomicOr(status, SP_STATUS_D_ABOVE_MAX);
                        w = 0;
                        h = 0;
                    }
                    c0 = a0 - rx0;
                    r0 = b0 - ry0;
                }
            }
            stg[threadIdx.x] = r;                                   // (x, y, kappa_x, Af)
            if (ANISO) stg2[threadIdx.x] = rs;                      // (kappa_y, kappa_xy)
            box[threadIdx.x] = pack_box(c0, w, r0, h);
            if (w > 0) {
                const unsigned long long pk = (unsigned long long)r.w;
                atomicAdd(&s_rows[r0], pk);
                atomicAdd(&s_rows[r0 + h], 0ull - pk);
            }
            // zero column factors up to the next multiple of four: the splat adds
            // whole quads, the columns past the patch adding zero (the factor pass
            // then overwrites the quad's columns inside the patch)
            if (w & 3)
                *reinterpret_cast<float4*>(gx + threadIdx.x * WM + (w & ~3)) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        // work items: one per patch line j < max(w, h); item j carries the j-th
        // column factor (if j < w) and the j-th row factor (if j < h)
        const int m = w > h ? w : h;
        int tm_;
        const int em = stage_scan(m, n, s_wave, tm_);
        const uint16_t tag = (uint16_t)(threadIdx.x << 8);
        for (int j = 0; j < m; ++j) items[em + j] = tag | (uint16_t)j;
        __syncthreads();
        // separable factors: gx per patch column here; the row factor Af * gy of
        // a patch row is formed by the splat item that adds that row (every
        // argument lies in [0, 18.1]: no range check needed)
        for (int i = threadIdx.x; i < tm_; i += 256) {
            const int it = items[i];
            const int k = it >> 8, j = it & 255;
            const uint32_t bx = box[k];
            if (j < (int)((bx >> 8) & 255u) && (!ANISO || stg2[k].y == 0.0f)) {
                const float4 sf = stg[k];
                const float dx = ((float)(rx0 + (int)(bx & 255u) + j) + 0.5f) - sf.x;
                gx[k * WM + j] = expneg_lt80(sf.z * (dx * dx));
            }
        }
        __syncthreads();
        // splat: one patch row per work item, eight columns per step; columns past
        // the patch edge carry zero factors (the accumulator has slack for the overrun)
        for (int i = threadIdx.x; i < tm_; i += 256) {
            const int it = items[i];
            const int k = it >> 8, j = it & 255;
            const uint32_t bx = box[k];
            if (j >= (int)(bx >> 24)) continue;
            const int pc0 = (int)(bx & 255u), pw = (int)((bx >> 8) & 255u), pr0 = (int)((bx >> 16) & 255u);
            const float4 sf = stg[k];
            const float dy = ((float)(ry0 + pr0 + j) + 0.5f) - sf.y;
            uint32_t* dst = acc + (pr0 + j) * RW + pc0;
            if (ANISO) {
                const float2 s2 = stg2[k];
                if (s2.y != 0.0f) {
                    // rho != 0: one exponential per pixel of the row
                    const float ra = s2.y * dy, rb = s2.x * (dy * dy);
                    for (int c = 0; c < pw; ++c) {
                        const float dx = ((float)(rx0 + pc0 + c) + 0.5f) - sf.x;
                        const float q = __builtin_fmaxf(__builtin_fmaf(dx, __builtin_fmaf(sf.z, dx, ra), rb), 0.0f);
                        atomicAdd(dst + c, (uint32_t)(sf.w * expneg(q)));
                    }
                    continue;
                }
            }
            const float rv = sf.w * expneg_lt80((ANISO ? stg2[k].x : sf.z) * (dy * dy));
            const float* gk = gx + k * WM;
            for (int cs0 = 0; cs0 < pw; cs0 += 8) {
                const float4 g0 = *reinterpret_cast<const float4*>(gk + cs0);
                atomicAdd(dst + cs0 + 0, (uint32_t)(rv * g0.x));
                atomicAdd(dst + cs0 + 1, (uint32_t)(rv * g0.y));
                atomicAdd(dst + cs0 + 2, (uint32_t)(rv * g0.z));
                atomicAdd(dst + cs0 + 3, (uint32_t)(rv * g0.w));
                if (pw - cs0 > 4) {
                    const float4 g1 = *reinterpret_cast<const float4*>(gk + cs0 + 4);
                    atomicAdd(dst + cs0 + 4, (uint32_t)(rv * g1.x));
                    atomicAdd(dst + cs0 + 5, (uint32_t)(rv * g1.y));
                    atomicAdd(dst + cs0 + 6, (uint32_t)(rv * g1.z));
                    atomicAdd(dst + cs0 + 7, (uint32_t)(rv * g1.w));
                }
            }
        }
    }
    // prefix sums of the row bounds (wave 0): flag a row whose bound reaches 2^32
    __syncthreads();
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        unsigned long long carry = 0ull, top = 0ull;
        for (int c = 0; c <= RH; c += 64) {
            unsigned long long v = c + lane <= RH ? s_rows[c + lane] : 0ull;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const unsigned long long u = __shfl_up(v, o, 64);
                if (lane >= o) v += u;
            }
            v += carry;
            top = v > top ? v : top;
            carry = __shfl(v, 63, 64);
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const unsigned long long u = __shfl_xor(top, o, 64);
            top = u > top ? u : top;
        }
        if (lane == 0 && top >= (1ull << 32)) atomicOr(status, SP_STATUS_FIXED_RANGE);
    }

    // fixed point -> float happens as the blur / store passes read the accumulator
    constexpr float FIX = 0x1p-24f;
    if constexpr (B > 0) {
        // horizontal pass over all region rows: four tile columns per work item
        for (int k = threadIdx.x; k < RH * Q4; k += 256) {
            const int r = k / Q4;
            const int c = (k % Q4) * 4;
            // the fixed-point scale rides on the weights: w (v 2^-24) and (w 2^-24) v
            // are the same binary32 products (exact power-of-two scaling, no underflow)
            const uint32_t* src = acc + r * RW + c;
            float vv[4 + 2 * B];
#pragma unroll
            for (int q = 0; q < 4 + 2 * B; ++q) vv[q] = (float)src[q];
            float o0 = 0.0f, o1 = 0.0f, o2 = 0.0f, o3 = 0.0f;
#pragma unroll
            for (int q = 0; q <= 2 * B; ++q) {
                const float wq = wb[q] * FIX;
                o0 = __builtin_fmaf(wq, vv[q], o0);
                o1 = __builtin_fmaf(wq, vv[q + 1], o1);
                o2 = __builtin_fmaf(wq, vv[q + 2], o2);
                o3 = __builtin_fmaf(wq, vv[q + 3], o3);
            }
            *reinterpret_cast<float4*>(tmp + r * TW + c) = make_float4(o0, o1, o2, o3);
        }
        __syncthreads();
    }

    // vertical pass, noise, codes, store: four consecutive pixels per work item
    const int64_t plane = (int64_t)pH * pW;
    const int Wq = (pW + 3) >> 2;
    const float Lq = a.bits > 0 ? (float)((1u << a.bits) - 1u) : 0.0f;
    // the noise words of a thread's next work item are drawn while it finishes
    // the current one (the Philox rounds are one long dependent chain)
    const bool noisy = a.noise_sigma > 0.0f;
    u32x4 w_next = {0u, 0u, 0u, 0u};
    if (noisy && (int)threadIdx.x < TH * Q4)
        w_next = draw((uint32_t)((ty * TH + (int)threadIdx.x / Q4) * Wq + ((tx * TW) >> 2) + (int)threadIdx.x % Q4),
                      STREAM_NOISE0 + f, pid, a.seed);
#pragma unroll 1
    for (int gi = threadIdx.x; gi < TH * Q4; gi += 256) {
        const int r = gi / Q4;
        const int c4 = (gi % Q4) * 4;
        const int R = ty * TH + r;
        const int C = tx * TW + c4;
        const u32x4 w = w_next;
        const int gn = gi + 256;
        if (noisy && gn < TH * Q4)
            w_next = draw((uint32_t)((ty * TH + gn / Q4) * Wq + ((tx * TW) >> 2) + gn % Q4), STREAM_NOISE0 + f, pid,
                          a.seed);
        if (R >= pH || C >= pW) continue;
        float o[4];
        if constexpr (B > 0) {
            float4 s4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
            for (int q = 0; q <= 2 * B; ++q) {
                const float wq = wb[q];
                const float4 t4 = *reinterpret_cast<const float4*>(tmp + (r + q) * TW + c4);
                s4.x = __builtin_fmaf(wq, t4.x, s4.x);
                s4.y = __builtin_fmaf(wq, t4.y, s4.y);
                s4.z = __builtin_fmaf(wq, t4.z, s4.z);
                s4.w = __builtin_fmaf(wq, t4.w, s4.w);
            }
            o[0] = s4.x; o[1] = s4.y; o[2] = s4.z; o[3] = s4.w;
        } else {
            const uint32_t* src = acc + r * RW + c4;
            o[0] = (float)src[0] * FIX; o[1] = (float)src[1] * FIX;
            o[2] = (float)src[2] * FIX; o[3] = (float)src[3] * FIX;
        }
        if (noisy) {
            const uint32_t wa[2] = {w.a, w.c};
            const uint32_t wb[2] = {w.b, w.d};
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
                const float u1 = u24_open0(wa[h2]);
                const float u2 = u24(wb[h2]);
                // v_log_f32 is log2 (so -2 ln u = -2 ln2 log2 u); v_sin/v_cos take revolutions
                const float rad = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u1));
                o[2 * h2] = __builtin_fmaf(a.noise_sigma, rad * __builtin_amdgcn_cosf(u2), o[2 * h2]);
                o[2 * h2 + 1] = __builtin_fmaf(a.noise_sigma, rad * __builtin_amdgcn_sinf(u2), o[2 * h2 + 1]);
            }
        }
        const int64_t pix = p_img + (int64_t)f * plane + (int64_t)R * pW + C;
        const int ne = min(4, pW - C);
        if (a.bits > 0) {
            uint32_t qv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                // clamp to [0, L] with one median (the value is finite)
                const float t = __builtin_amdgcn_fmed3f(__builtin_rintf(o[e] * Lq), 0.0f, Lq);
                qv[e] = (uint32_t)t;
            }
            uint16_t* dst = reinterpret_cast<uint16_t*>(a.images) + pix;
            if (ne == 4 && ((uintptr_t)dst & 7) == 0) {
                *reinterpret_cast<uint2*>(dst) = make_uint2(qv[0] | (qv[1] << 16), qv[2] | (qv[3] << 16));
            } else {
                for (int e = 0; e < ne; ++e) dst[e] = (uint16_t)qv[e];
            }
        } else {
            float* dst = reinterpret_cast<float*>(a.images) + pix;
            if (ne == 4 && ((uintptr_t)dst & 15) == 0) {
                *reinterpret_cast<float4*>(dst) = make_float4(o[0], o[1], o[2], o[3]);
            } else {
                for (int e = 0; e < ne; ++e) dst[e] = o[e];
            }
        }
    }
    if (!PERSIST) break;
    // the next item's accumulator reset and queue pop wait for this epilogue
    __syncthreads();
    }
}

size_t render_lds_bytes(const RenderConfig& cfg, bool aniso) { return render_lds(cfg, aniso).bytes; }

// Tile shapes with a compiled renderer (width x height).
bool render_shape_supported(int tw, int th)
{
    switch (tw * 1000 + th) {
    case 8008: case 16016: case 32016: case 32032: case 64016: case 64032: case 64064: case 128032:
        return true;
    default:
        return false;
    }
}

// ------------------------------------------------------------------ launcher

static void launch_scans(const PairLayout* L, int n_pairs, uint32_t* hist, uint32_t* tile_count,
                         int64_t* tile_offset, int64_t tiles, int frames, hipStream_t s, const int32_t* live,
                         int chunk)
{
    hipLaunchKernelGGL(scan_chunks, dim3((unsigned)((tiles + 255) / 256), frames), dim3(256), 0, s, L, n_pairs, hist,
                       tile_count, tiles, live, chunk);
    hipLaunchKernelGGL(scan_tiles, dim3((unsigned)n_pairs, frames), dim3(256), 0, s, L, tile_count, tile_offset,
                       tiles);
}

// Launches one renderer instantiation: one workgroup per item, or (persistent
// kernels) as many workgroups as the device holds at once, from the kernel's
// occupancy at this LDS size (cached per kernel and size).  The persistent
// form is compiled for the isotropic renderer; anisotropic batches run one
// workgroup per item.
template <typename K, typename... Args>
static void launch_tile_kernel(K kernel, dim3 grid, size_t lds, hipStream_t s, bool persistent, Args... args)
{
    if (persistent) {
        static std::mutex mu;
        static std::map<std::pair<const void*, size_t>, int> cache;
        int per_cu = 0;
        {
            std::lock_guard<std::mutex> lk(mu);
            const auto key = std::make_pair(reinterpret_cast<const void*>(kernel), lds);
            auto it = cache.find(key);
            if (it == cache.end()) {
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, lds) != hipSuccess)
                    per_cu = 0;
                cache[key] = per_cu;
            } else {
                per_cu = it->second;
            }
        }
        if (per_cu > 0) {
            const unsigned cap = (unsigned)per_cu * (unsigned)device_cu_count();
            if (grid.x > cap) grid.x = cap;
        }
    }
    hipLaunchKernelGGL(kernel, grid, dim3(256), lds, s, args...);
}

template <int TW, int TH>
static void launch_render_shape(dim3 grid, size_t lds, hipStream_t s, const RenderArgs& a, const RenderConfig& cfg,
                                const PairLayout* L, const float4* r0, const float4* r1, const uint2* b0,
                                const uint2* b1, const float2* h0, const float2* h1, const uint32_t* tile_count,
                                const int64_t* tile_offset, const int32_t* entries, int64_t tiles, uint32_t* status)
{
    EpilogueArgs ea;
    ea.images = a.images;
    ea.noise_sigma = a.noise_sigma;
    ea.bits = a.bits;
    ea.seed = a.seed;
    ea.iod = a.iod;
    for (int q = 0; q < 7; ++q) ea.blur_w[q] = a.blur_w[q];
#define SP_B(B_)                                                                                                 \
    case B_:                                                                                                     \
        if (a.aniso)                                                                                             \
            launch_tile_kernel(render_tile<TW, TH, B_, true, false>, grid, lds, s, false, a.pairs, L, a.n_pairs, \
                               r0, r1, b0, b1, h0, h1, ea, cfg.cap, cfg.wm4, tile_count, tile_offset, entries,   \
                               tiles,                                                                            \
                               status, status + 8);                                                              \
        else if (cfg.persistent)                                                                                 \
            launch_tile_kernel(render_tile<TW, TH, B_, false, true>, grid, lds, s, true, a.pairs, L, a.n_pairs,  \
                               r0, r1, b0, b1, h0, h1, ea, cfg.cap, cfg.wm4, tile_count, tile_offset, entries,   \
                               tiles,                                                                            \
                               status, status + 8);                                                              \
        else                                                                                                     \
            launch_tile_kernel(render_tile<TW, TH, B_, false, false>, grid, lds, s, false, a.pairs, L,           \
                               a.n_pairs, r0, r1, b0, b1, h0, h1, ea, cfg.cap, cfg.wm4, tile_count,              \
                               tile_offset, entries, tiles, status, status + 8);                                 \
        break;
    switch (cfg.apron) { SP_B(0) SP_B(1) SP_B(2) SP_B(3) default: break; }
#undef SP_B
}

hipError_t launch_bins(const RenderArgs& a, const RenderConfig& cfg, const BatchTotals& tot, char* ws,
                       const WorkspaceLayout& wl, hipStream_t s)
{
    uint32_t* status = reinterpret_cast<uint32_t*>(ws + wl.status);
    PairLayout* L = reinterpret_cast<PairLayout*>(ws + wl.layout);
    uint32_t* tile_count = reinterpret_cast<uint32_t*>(ws + wl.tile_count);
    int64_t* tile_offset = reinterpret_cast<int64_t*>(ws + wl.tile_offset);
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws + wl.hist);
    int32_t* entries = reinterpret_cast<int32_t*>(ws + wl.entries);
    float4* rec0 = reinterpret_cast<float4*>(ws + wl.records);
    float4* rec1 = rec0 + tot.n_span;
    uint2* box0 = reinterpret_cast<uint2*>(ws + wl.boxes);
    uint2* box1 = box0 + tot.n_span;
    float2* shp0 = reinterpret_cast<float2*>(ws + wl.shapes);
    float2* shp1 = shp0 + tot.n_span;

    {
        TimedScope ts("bin_layout", s);
        hipLaunchKernelGGL(bin_layout, dim3(1), dim3(256), 0, s, a.pairs, a.n_pairs, cfg, L, status);
    }
    if (tot.n_span > 0) {
        TimedScope ts("prep", s);
        if (a.model)
            hipLaunchKernelGGL(prep_records_model, dim3((unsigned)((tot.n_span + 255) / 256)), dim3(256), 0, s,
                               a.pairs, a.n_pairs, tot.n_span, a, cfg.d_max, rec0, rec1, box0, box1, shp0, shp1,
                               status);
        else
            hipLaunchKernelGGL(prep_records, dim3((unsigned)((tot.n_span + 255) / 256)), dim3(256), 0, s, a.pairs,
                               a.n_pairs, tot.n_span, a, cfg.d_max, rec0, rec1, box0, box1, status);
    }
    const size_t hist_lds = (size_t)tot.max_tiles * sizeof(uint32_t);
    const dim3 bgrid((unsigned)tot.chunks, 2);
    // the full model's prep writes every slot; live counts only with the isotropic prep
    const int32_t* live = a.model ? nullptr : a.live;
    if (tot.chunks > 0) {
        TimedScope ts("bin_count", s);
        hipLaunchKernelGGL(bin_pass<false>, bgrid, dim3(256), hist_lds, s, a.pairs, L, a.n_pairs, box0, box1, cfg,
                           hist, tile_offset, tot.tiles, entries, (unsigned)tot.chunks, live);
    }
    if (tot.tiles > 0) {
        TimedScope ts("bin_scan", s);
        launch_scans(L, a.n_pairs, hist, tile_count, tile_offset, tot.tiles, 2, s, live, cfg.chunk);
    }
    if (tot.chunks > 0) {
        TimedScope ts("bin_scatter", s);
        hipLaunchKernelGGL(bin_pass<true>, bgrid, dim3(256), hist_lds, s, a.pairs, L, a.n_pairs, box0, box1, cfg,
                           hist, tile_offset, tot.tiles, entries, (unsigned)tot.chunks, live);
    }
    return hipGetLastError();
}

hipError_t launch_render(const RenderArgs& a, const RenderConfig& cfg, const BatchTotals& tot, char* ws,
                         const WorkspaceLayout& wl, hipStream_t s)
{
    uint32_t* status = reinterpret_cast<uint32_t*>(ws + wl.status);
    PairLayout* L = reinterpret_cast<PairLayout*>(ws + wl.layout);
    uint32_t* tile_count = reinterpret_cast<uint32_t*>(ws + wl.tile_count);
    int64_t* tile_offset = reinterpret_cast<int64_t*>(ws + wl.tile_offset);
    int32_t* entries = reinterpret_cast<int32_t*>(ws + wl.entries);
    float4* rec0 = reinterpret_cast<float4*>(ws + wl.records);
    float4* rec1 = rec0 + tot.n_span;
    uint2* box0 = reinterpret_cast<uint2*>(ws + wl.boxes);
    uint2* box1 = box0 + tot.n_span;
    float2* shp0 = reinterpret_cast<float2*>(ws + wl.shapes);
    float2* shp1 = shp0 + tot.n_span;
    const hipError_t e = launch_bins(a, cfg, tot, ws, wl, s);
    if (e != hipSuccess) return e;
    if (tot.tiles > 0) {
        TimedScope ts("render_tile", s);
        const size_t lds = render_lds_bytes(cfg, a.aniso);
        const dim3 grid((unsigned)(2 * tot.tiles));
#define SP_SHAPE(W_, H_)                                                                                        \
    if (cfg.tile_w == W_ && cfg.tile_h == H_)                                                                   \
        launch_render_shape<W_, H_>(grid, lds, s, a, cfg, L, rec0, rec1, box0, box1, shp0, shp1, tile_count,   \
                                    tile_offset, entries, tot.tiles, status);                                   \
    else
        SP_SHAPE(8, 8) SP_SHAPE(16, 16) SP_SHAPE(32, 16) SP_SHAPE(32, 32) SP_SHAPE(64, 16) SP_SHAPE(64, 32)
        SP_SHAPE(64, 64) SP_SHAPE(128, 32)
        return hipErrorInvalidValue;
#undef SP_SHAPE
    }
    return hipGetLastError();
}

hipError_t launch_order(const synthpix_pair* pairs_dev, int n_pairs, const float* x, const float* y,
                        const RenderConfig& cfg, const BatchTotals& tot, char* ws, const OrderLayout& ol,
                        hipStream_t s, const synthpix_batch_io* iod, const int32_t* live)
{
    uint32_t* status = reinterpret_cast<uint32_t*>(ws + ol.status);
    PairLayout* L = reinterpret_cast<PairLayout*>(ws + ol.layout);
    uint32_t* tile_count = reinterpret_cast<uint32_t*>(ws + ol.tile_count);
    int64_t* tile_offset = reinterpret_cast<int64_t*>(ws + ol.tile_offset);
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws + ol.hist);
    int32_t* entries = reinterpret_cast<int32_t*>(ws + ol.entries);
    TimedScope ts("order", s);
    hipLaunchKernelGGL(bin_layout, dim3(1), dim3(256), 0, s, pairs_dev, n_pairs, cfg, L, status);
    if (tot.chunks == 0) return hipGetLastError();
    const size_t hist_lds = (size_t)tot.max_tiles * sizeof(uint32_t);
    hipLaunchKernelGGL(order_pass<false>, dim3((unsigned)tot.chunks), dim3(256), hist_lds, s, pairs_dev, L, n_pairs, x,
                       y, cfg, hist, tile_offset, entries, (unsigned)tot.chunks, iod, live);
    launch_scans(L, n_pairs, hist, tile_count, tile_offset, tot.tiles, 1, s, live, cfg.chunk);
    hipLaunchKernelGGL(order_pass<true>, dim3((unsigned)tot.chunks), dim3(256), hist_lds, s, pairs_dev, L, n_pairs, x,
                       y, cfg, hist, tile_offset, entries, (unsigned)tot.chunks, iod, live);
    return hipGetLastError();
}

}  // namespace sp
