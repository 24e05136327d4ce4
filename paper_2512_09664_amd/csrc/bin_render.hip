// Screen-tile binning and the fused tile renderer (gfx950).
//
// Rendering follows Eq. 1 (rho = 0, sigma = d/4) with a Gaussian laser-sheet
// peak (Remark 1), point-sampled at pixel centres (Remark 2), summed over all
// particles (Section 2, "Considerations on the aggregation") on per-particle
// square patches |dx|, |dy| <= 1.5 d (Section 2, "Efficient rasterization").
//
// Pipeline of one call (all pairs of a batch at once):
//   bin_layout  : per-pair prefix tables (one block)
//   bin_count   : per (pair, frame, particle chunk) LDS histogram of tile hits
//   bin_scan    : per (pair, frame) exclusive scan -> tile offsets and per-chunk bases
//   bin_scatter : per chunk, LDS cursors -> particle indices into tile lists
//   render_tile : per (pair, frame, tile) stage the list in LDS, splat footprints
//                 into an LDS fixed-point accumulator (tile + blur apron), then
//                 blur, noise, quantise and store.
// No global atomics: counts, cursors and pixel sums all live in LDS.  Pixel sums
// are exact 32-bit fixed point, so the LDS atomics' order does not matter.
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

__device__ __forceinline__ int find_pair_by_tile(const PairLayout* L, int n_pairs, int64_t t)
{
    int lo = 0, hi = n_pairs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L[mid].tile_base <= t) lo = mid; else hi = mid - 1;
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
    if (t == 0) { status[0] = 0u; status[1] = 0u; status[2] = 0u; status[3] = 0u; }
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

// ------------------------------------------------------------------ membership

// Tile rectangle touched by one particle in one frame: its support, clipped to
// the image, grown by the blur apron.  False when the particle adds nothing.
__device__ __forceinline__ bool tile_rect(float x, float y, float d, float I0, int H, int W,
                                          const RenderConfig& cfg, int ntx, int nty,
                                          int& tx0, int& tx1, int& ty0, int& ty1,
                                          uint32_t* status)
{
    if (!particle_valid(x, y, d, I0)) return false;
    if (!(d <= cfg.d_max)) {
        atomicOr(status, SP_STATUS_D_ABOVE_MAX);
        return false;
    }
    const float R = 1.5f * d;
    int c0, c1, r0, r1;
    if (!support_range(x, R, W, c0, c1)) return false;
    if (!support_range(y, R, H, r0, r1)) return false;
    const int b = cfg.apron;
    tx0 = c0 - b < 0 ? 0 : (c0 - b) / cfg.tile_w;
    ty0 = r0 - b < 0 ? 0 : (r0 - b) / cfg.tile_h;
    tx1 = (c1 + b) / cfg.tile_w;
    ty1 = (r1 + b) / cfg.tile_h;
    tx1 = tx1 > ntx - 1 ? ntx - 1 : tx1;
    ty1 = ty1 > nty - 1 ? nty - 1 : ty1;
    return true;
}

// ------------------------------------------------------------------ count / scatter

template <bool SCATTER>
__global__ void __launch_bounds__(256)
bin_pass(const synthpix_pair* __restrict__ pairs, const PairLayout* __restrict__ L, int n_pairs,
         RenderArgs a, RenderConfig cfg, uint32_t* __restrict__ hist, int32_t* __restrict__ entries,
         uint32_t* __restrict__ status)
{
    extern __shared__ uint32_t lh[];
    const int f = blockIdx.y;
    const int p = find_pair_by_chunk(L, n_pairs, blockIdx.x);
    const synthpix_pair P = pairs[p];
    const PairLayout PL = L[p];
    const int chunk = blockIdx.x - PL.chunk_base;
    const int nt = PL.ntx * PL.nty;
    uint32_t* gh = hist + PL.hist_base + ((int64_t)f * PL.n_chunks + chunk) * nt;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) lh[t] = SCATTER ? gh[t] : 0u;
    __syncthreads();
    const int i_end = min(P.n_max, (chunk + 1) * cfg.chunk);
    const float* __restrict__ xf = a.x[f];
    const float* __restrict__ yf = a.y[f];
    int32_t* seg = entries + PL.entry_base + (int64_t)f * PL.entry_cap;
    for (int i = chunk * cfg.chunk + threadIdx.x; i < i_end; i += blockDim.x) {
        const int64_t g = P.particle_offset + i;
        int tx0, tx1, ty0, ty1;
        if (!tile_rect(xf[g], yf[g], a.d[g], a.I0[g], P.H, P.W, cfg, PL.ntx, PL.nty, tx0, tx1, ty0, ty1,
                       status))
            continue;
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx) {
                const uint32_t slot = atomicAdd(&lh[ty * PL.ntx + tx], 1u);
                if (SCATTER) seg[slot] = i;
            }
    }
    if (!SCATTER) {
        __syncthreads();
        for (int t = threadIdx.x; t < nt; t += blockDim.x) gh[t] = lh[t];
    }
}

// Per (pair, frame): tile totals, exclusive tile offsets (within the pair-frame
// segment) and, in place, each chunk's starting slot inside every tile list.
__global__ void __launch_bounds__(256)
bin_scan(const PairLayout* __restrict__ L, uint32_t* __restrict__ hist, uint32_t* __restrict__ tile_count,
         int64_t* __restrict__ tile_offset, int64_t tiles_total)
{
    __shared__ uint32_t s_sum[256];
    const int p = blockIdx.x;
    const int f = blockIdx.y;
    const PairLayout PL = L[p];
    const int nt = PL.ntx * PL.nty;
    uint32_t* h = hist + PL.hist_base + (int64_t)f * PL.n_chunks * nt;
    const int per = (nt + 255) / 256;
    const int t0 = threadIdx.x * per;
    const int t1 = min(nt, t0 + per);
    // pass 1: within-tile exclusive prefix over chunks; tile totals; thread sum
    uint32_t mine = 0;
    for (int t = t0; t < t1; ++t) {
        uint32_t run = 0;
        for (int c = 0; c < PL.n_chunks; ++c) {
            const uint32_t v = h[(int64_t)c * nt + t];
            h[(int64_t)c * nt + t] = run;
            run += v;
        }
        tile_count[f * tiles_total + PL.tile_base + t] = run;
        mine += run;
    }
    s_sum[threadIdx.x] = mine;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t add = threadIdx.x >= off ? s_sum[threadIdx.x - off] : 0u;
        __syncthreads();
        s_sum[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t base = s_sum[threadIdx.x] - mine;
    // pass 2: tile offsets; shift chunk bases by the tile offset
    for (int t = t0; t < t1; ++t) {
        const uint32_t cnt = tile_count[f * tiles_total + PL.tile_base + t];
        tile_offset[f * tiles_total + PL.tile_base + t] = PL.entry_base + (int64_t)f * PL.entry_cap + base;
        for (int c = 0; c < PL.n_chunks; ++c) h[(int64_t)c * nt + t] += base;
        base += cnt;
    }
}

// ------------------------------------------------------------------ render

struct StagedParticle {
    int c0, w, r0, h;        // patch rectangle in region-local pixels
    float Af, kap, x, y;     // 2^24 * peak, 8/d^2, position
};

__global__ void __launch_bounds__(256)
render_tile(const synthpix_pair* __restrict__ pairs, const PairLayout* __restrict__ L, int n_pairs,
            RenderArgs a, RenderConfig cfg, const uint32_t* __restrict__ tile_count,
            const int64_t* __restrict__ tile_offset, const int32_t* __restrict__ entries,
            int64_t tiles_total, uint32_t* __restrict__ status)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int b = cfg.apron;
    const int RW = cfg.tile_w + 2 * b;
    const int RH = cfg.tile_h + 2 * b;
    const int CAP = cfg.cap;
    const int WM = cfg.wmax;
    uint32_t* acc = reinterpret_cast<uint32_t*>(smem);                       // RH * RW
    StagedParticle* sp_ = reinterpret_cast<StagedParticle*>(acc + RH * RW);  // CAP
    float* gx = reinterpret_cast<float*>(sp_ + CAP);                         // CAP * WM
    float* rs = gx + CAP * WM;                                               // CAP * WM
    float* tmp = reinterpret_cast<float*>(sp_);   // blur scratch RH * tile_w, reuses the tables
    __shared__ unsigned long long s_asum;

    const int64_t item = blockIdx.x;
    const int f = (int)(item / tiles_total);
    const int64_t tile = item - (int64_t)f * tiles_total;
    const int p = find_pair_by_tile(L, n_pairs, tile);
    const synthpix_pair P = pairs[p];
    const PairLayout PL = L[p];
    const int tl = (int)(tile - PL.tile_base);
    const int tx = tl % PL.ntx;
    const int ty = tl / PL.ntx;
    const int rx0 = tx * cfg.tile_w - b;   // region origin in image pixels
    const int ry0 = ty * cfg.tile_h - b;
    const int cnt = (int)tile_count[item];
    const int64_t off = tile_offset[item];
    const float cs = 0.5f / (a.sheet_sigma * a.sheet_sigma);
    const float* __restrict__ xf = a.x[f];
    const float* __restrict__ yf = a.y[f];

    for (int k = threadIdx.x; k < RH * RW; k += blockDim.x) acc[k] = 0u;
    if (threadIdx.x == 0) s_asum = 0ull;

    for (int base = 0; base < cnt; base += CAP) {
        const int n = min(CAP, cnt - base);
        __syncthreads();
        if ((int)threadIdx.x < n) {
            const int idx = entries[off + base + threadIdx.x];
            const int64_t g = P.particle_offset + idx;
            const float x = xf[g], y = yf[g], z = a.z[g], d = a.d[g], I0 = a.I0[g];
            const float R = 1.5f * d;
            int c0 = 0, c1 = -1, r0 = 0, r1 = -1;
            StagedParticle s;
            s.w = 0;
            s.h = 0;
            if (support_range(x, R, P.W, c0, c1) && support_range(y, R, P.H, r0, r1)) {
                c0 = max(c0, rx0);
                c1 = min(c1, rx0 + RW - 1);
                r0 = max(r0, ry0);
                r1 = min(r1, ry0 + RH - 1);
                if (c0 <= c1 && r0 <= r1) {
                    s.c0 = c0 - rx0;
                    s.r0 = r0 - ry0;
                    s.w = c1 - c0 + 1;
                    s.h = r1 - r0 + 1;
                    if (s.w > WM || s.h > WM) {          // cannot happen for d <= d_max
                        atomicOr(status, SP_STATUS_D_ABOVE_MAX);
                        s.w = 0;
                        s.h = 0;
                    }
                }
            }
            const float A = I0 * expneg((z * z) * cs);
            s.Af = A * 16777216.0f;
            s.kap = 8.0f / (d * d);
            s.x = x;
            s.y = y;
            sp_[threadIdx.x] = s;
            atomicAdd(&s_asum, (unsigned long long)quant24(s.Af));
        }
        __syncthreads();
        // separable factors: column factors gx and row factors rs = Af * gy
        for (int it = threadIdx.x; it < n * WM; it += blockDim.x) {
            const int k = it / WM;
            const int j = it - k * WM;
            const StagedParticle s = sp_[k];
            if (j < s.w) {
                const float dx = ((float)(rx0 + s.c0 + j) + 0.5f) - s.x;
                gx[it] = expneg(s.kap * (dx * dx));
            }
            if (j < s.h) {
                const float dy = ((float)(ry0 + s.r0 + j) + 0.5f) - s.y;
                rs[it] = s.Af * expneg(s.kap * (dy * dy));
            }
        }
        __syncthreads();
        // splat one patch row per work item
        for (int it = threadIdx.x; it < n * WM; it += blockDim.x) {
            const int k = it / WM;
            const int j = it - k * WM;
            const StagedParticle s = sp_[k];
            if (j >= s.h) continue;
            const float rv = rs[it];
            const float* gxk = gx + k * WM;
            uint32_t* dst = acc + (s.r0 + j) * RW + s.c0;
            for (int c = 0; c < s.w; ++c) atomicAdd(dst + c, quant24(rv * gxk[c]));
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_asum >= 4294967296ull) atomicOr(status, SP_STATUS_FIXED_RANGE);

    // fixed point -> float, in place
    float* v = reinterpret_cast<float*>(acc);
    for (int k = threadIdx.x; k < RH * RW; k += blockDim.x) v[k] = (float)acc[k] * 0x1p-24f;
    __syncthreads();

    const int TW = cfg.tile_w;
    if (b > 0) {
        // horizontal pass over all region rows, tile columns
        for (int k = threadIdx.x; k < RH * TW; k += blockDim.x) {
            const int r = k / TW;
            const int c = k - r * TW;
            const float* src = v + r * RW + c;
            float s = 0.0f;
            for (int q = 0; q <= 2 * b; ++q) s = __builtin_fmaf(a.blur_w[q], src[q], s);
            tmp[k] = s;
        }
        __syncthreads();
    }

    // vertical pass, noise, quantise, store; 4 consecutive pixels per work item
    const int groups = cfg.tile_h * (TW >> 2);
    const int64_t plane = (int64_t)P.H * P.W;
    const int Wq = (P.W + 3) >> 2;
    for (int gi = threadIdx.x; gi < groups; gi += blockDim.x) {
        const int r = gi / (TW >> 2);
        const int c4 = (gi - r * (TW >> 2)) << 2;
        const int R = ty * cfg.tile_h + r;
        const int C = tx * TW + c4;
        if (R >= P.H || C >= P.W) continue;
        float o[4];
        for (int e = 0; e < 4; ++e) {
            const int c = c4 + e;
            if (b > 0) {
                const float* src = tmp + r * TW + c;
                float s = 0.0f;
                for (int q = 0; q <= 2 * b; ++q) s = __builtin_fmaf(a.blur_w[q], src[q * TW], s);
                o[e] = s;
            } else {
                o[e] = v[r * RW + c];
            }
        }
        if (a.noise_sigma > 0.0f) {
            const u32x4 w = draw((uint32_t)(R * Wq + (C >> 2)), STREAM_NOISE0 + f, P.pair_id, a.seed);
            const uint32_t wa[2] = {w.a, w.c};
            const uint32_t wb[2] = {w.b, w.d};
            for (int h2 = 0; h2 < 2; ++h2) {
                const float u1 = u24_open0(wa[h2]);
                const float u2 = u24(wb[h2]);
                // v_log_f32 is log2; v_sin/v_cos take revolutions
                const float rad = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u1));
                o[2 * h2] = __builtin_fmaf(a.noise_sigma, rad * __builtin_amdgcn_cosf(u2), o[2 * h2]);
                o[2 * h2 + 1] = __builtin_fmaf(a.noise_sigma, rad * __builtin_amdgcn_sinf(u2), o[2 * h2 + 1]);
            }
        }
        const int64_t pix = P.image_offset + (int64_t)f * plane + (int64_t)R * P.W + C;
        const int ne = min(4, P.W - C);
        if (a.bits > 0) {
            const float Lq = (float)((1u << a.bits) - 1u);
            uint16_t* dst = reinterpret_cast<uint16_t*>(a.images) + pix;
            for (int e = 0; e < ne; ++e) {
                float t = __builtin_rintf(o[e] * Lq);
                t = __builtin_fmaxf(t, 0.0f);
                t = __builtin_fminf(t, Lq);
                dst[e] = (uint16_t)t;
            }
        } else {
            float* dst = reinterpret_cast<float*>(a.images) + pix;
            for (int e = 0; e < ne; ++e) dst[e] = o[e];
        }
    }
}

// ------------------------------------------------------------------ launcher

size_t render_lds_bytes(const RenderConfig& cfg)
{
    const int RW = cfg.tile_w + 2 * cfg.apron;
    const int RH = cfg.tile_h + 2 * cfg.apron;
    size_t tables = (size_t)cfg.cap * sizeof(StagedParticle) + 2 * (size_t)cfg.cap * cfg.wmax * sizeof(float);
    size_t blur = (size_t)RH * cfg.tile_w * sizeof(float);
    return (size_t)RH * RW * sizeof(uint32_t) + (tables > blur ? tables : blur);
}

hipError_t launch_render(const RenderArgs& a, const RenderConfig& cfg, const BatchTotals& tot, char* ws,
                         const WorkspaceLayout& wl, hipStream_t s)
{
    uint32_t* status = reinterpret_cast<uint32_t*>(ws + wl.status);
    PairLayout* L = reinterpret_cast<PairLayout*>(ws + wl.layout);
    uint32_t* tile_count = reinterpret_cast<uint32_t*>(ws + wl.tile_count);
    int64_t* tile_offset = reinterpret_cast<int64_t*>(ws + wl.tile_offset);
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws + wl.hist);
    int32_t* entries = reinterpret_cast<int32_t*>(ws + wl.entries);

    {
        TimedScope ts("bin_layout", s);
        hipLaunchKernelGGL(bin_layout, dim3(1), dim3(256), 0, s, a.pairs, a.n_pairs, cfg, L, status);
    }
    const size_t hist_lds = (size_t)tot.max_tiles * sizeof(uint32_t);
    if (tot.chunks > 0) {
        TimedScope ts("bin_count", s);
        hipLaunchKernelGGL(bin_pass<false>, dim3((unsigned)tot.chunks, 2), dim3(256), hist_lds, s,
                           a.pairs, L, a.n_pairs, a, cfg, hist, entries, status);
    }
    {
        TimedScope ts("bin_scan", s);
        hipLaunchKernelGGL(bin_scan, dim3((unsigned)a.n_pairs, 2), dim3(256), 0, s, L, hist, tile_count,
                           tile_offset, tot.tiles);
    }
    if (tot.chunks > 0) {
        TimedScope ts("bin_scatter", s);
        hipLaunchKernelGGL(bin_pass<true>, dim3((unsigned)tot.chunks, 2), dim3(256), hist_lds, s,
                           a.pairs, L, a.n_pairs, a, cfg, hist, entries, status);
    }
    if (tot.tiles > 0) {
        TimedScope ts("render_tile", s);
        hipLaunchKernelGGL(render_tile, dim3((unsigned)(2 * tot.tiles)), dim3(256), render_lds_bytes(cfg), s,
                           a.pairs, L, a.n_pairs, a, cfg, tile_count, tile_offset, entries, tot.tiles, status);
    }
    return hipGetLastError();
}

}  // namespace sp
