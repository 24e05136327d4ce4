// Adjoint of advect -> render -> blur (gfx950): given dL/dJ of the float images,
// the gradients with respect to frame-1 positions, z, d, I0, each pair's sheet
// width and each pair's flow grid.
//
// Render adjoint (Eq. 1 with sigma = d/4 and peak A = I0 exp(-z^2 / (2 s^2))):
// every particle's footprint is separable, t = A gx(c) gy(r), so with the
// zero-padded blur B (also separable) the four per-particle sums the chain rule
// needs,
//     S0 = sum_q e_q G_q,  Sx = sum e G dx,  Sy = sum e G dy,  Sr = sum e G (dx^2 + dy^2),
// e = B^T dL/dJ, equal sum_q (dL/dJ)_q Ty_j(r) Tx_k(c) with 1-D tables
// Tx_k = w * (gx dx^k) (the blur folded into the particle's factor tables).
// The gather is particle-major (a group of 8 or 16 lanes per particle reads
// its patch rows of dL/dJ with coalesced loads) or, for wide blurs, tile-major
// (a home block of the image and its halo staged in LDS, the block's particles
// gathered from it); nothing is scattered, no partial sums cross tiles.
//
// Flow adjoint: a reverse sweep through the recomputed Euler / RK4 substeps
// (checkpointed).  Each bilinear sample passes its upstream gradient to its
// four grid nodes; consecutive samples in one cell are merged per particle,
// and node sums are accumulated in 64-bit fixed point, so the result does not
// depend on the order of the additions.  The fixed-point scale is a power of
// two from an a-priori bound on every upstream value (largest dL/dx2 and the
// flow's Lipschitz constant through the stage recurrences) and the sample
// count, so no sum can leave the int64 range.
#include "device_math.hpp"
#include "flow.hpp"
#include "launch.hpp"

namespace sp {

// Patch rows loaded per batch of the column walk (independent loads in
// flight): 8 from global memory, 4 from a region staged in LDS (16 measured
// slower for both, 4 slower from global memory and 2 the same from LDS).  The
// rows' terms are added in row order whatever the batch.
constexpr int GROWS_GLOBAL = 8;
constexpr int GROWS_LDS = 4;

// A particle's lane group: G = 16 lanes (a DPP row) or 8 (half of one); a
// workgroup of 256 threads holds 256 / G particles.  BT table slots cover the
// pixel range (<= 3 d_max + 3 pixels) plus 4 b of zero padding.  The raw
// factors are stored as the Gaussian values e alone (their dx and dx^2
// multiples are formed where they are read); the raw row factors are kept
// only where a blur is folded in (RY).
template <int G, int BT, bool RY = true>
struct GatherLds {
    float rx[256 / G][BT];                      // raw column factors e(c) (slot = c - c0 + 2b)
    float ry[RY ? 256 / G : 1][RY ? BT : 1];    // raw row factors e(r)
    float4 ty[256 / G][BT];                     // blurred row tables (Ty0, Ty1, Ty2, 0)
};

// Sum over a particle's G lanes, result in every lane: quad butterflies
// (quad_perm [1,0,3,2] and [2,3,0,1]), then, for 16 lanes, rotations of the
// row by 4 and 8 lanes, for 8 lanes the mirror of each half row (the other
// quad of the eight).
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// A particle's lane group lies inside one wavefront and its LDS tables are
// private to it, so the group synchronises with a wave-level fence instead of
// a workgroup barrier (LDS operations of one wave complete in issue order).
__device__ __forceinline__ void group_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int G>
__device__ __forceinline__ float group_sum(float v)
{
    static_assert(G == 8 || G == 16, "a lane group is a DPP row or half of one");
    v += dpp<0xB1>(v);
    v += dpp<0x4E>(v);
    if constexpr (G == 16) {
        v += dpp<0x124>(v);
        v += dpp<0x128>(v);
    } else {
        v += dpp<0x141>(v);
    }
    return v;
}

// exp(-q) for the gradient's factor tables: the hardware base-2 exponential
// (relative error about 1e-6 over the support's q <= 18, well inside the
// gradient's tolerance; the images themselves use the exact polynomial).
// Zero for q >= 80 or not a number.
__device__ __forceinline__ float expneg_hw(float q)
{
    return q < 80.0f ? __builtin_amdgcn_exp2f(q * -LOG2E_F) : 0.0f;
}

// Pixel indices that may hold the support |(k + 1/2) - p| <= R, clipped to
// [0, n): a superset by at most one index per side (the exact binary32 test
// is applied per pixel where the factor tables are filled).
__device__ __forceinline__ bool cover_range(float p, float R, int n, int& lo, int& hi)
{
    if (!__builtin_isfinite(p)) return false;
    const float a = p - R - 0.5f, b = p + R - 0.5f;
    if (b < -1.0f || a > (float)n) return false;
    const int l = (int)__builtin_floorf(a), h = (int)__builtin_ceilf(b);
    lo = l < 0 ? 0 : l;
    hi = h > n - 1 ? n - 1 : h;
    return lo <= hi;
}

// One lane group's sums for one frame of its particle: the raw factor tables,
// the blurred row tables (B > 0) and the gather
//     S0 = sum e G,  Sx = sum e G dx,  Sy = sum e G dy,  Sr = sum e G (dx^2 + dy^2)
// over the blurred support inside the image, reading pixel (r, c) of the
// frame's dL/dJ (B > 0) or B^T dL/dJ (B = 0) at src[(r - sr) * stride + (c - sc)]
// (global memory, or a region staged in LDS).  Every lane returns the group's
// sums.  on: the particle is valid and its support [c0, c1] x [r0, r1] is not
// empty.
// CS: the source's row stride in elements when known at compile time (rows
// then load at immediate offsets), 0 for the runtime stride.  GROWS: rows per
// batch of the column walk.
template <int B, int BT, bool RY, int G, int CS = 0, int GROWS = GROWS_GLOBAL>
__device__ __forceinline__ float4 frame_sums(GatherLds<G, BT, RY>& S, int grp, int lane, bool on, float x, float y,
                                             float kap, float R, int c0, int c1, int r0, int r1, int W, int H,
                                             const float* __restrict__ src, int64_t stride, int sr, int sc,
                                             const float* blur_w)
{
    // raw factor tables over the slots the gather reads, 0 .. max(c1 - c0, r1 - r0)
    // + 4b (zeros outside the support); a group stops after its last one
    const int n_raw = on ? max(c1 - c0, r1 - r0) + 4 * B + 1 : 0;
#pragma unroll
    for (int m = 0; m < BT / G; ++m) {
        if (G * m >= n_raw) break;
        const int slot = lane + G * m;
        const int c = c0 - 2 * B + slot;
        float v0 = 0.0f;
        const float dx = ((float)c + 0.5f) - x;
        if (on && c >= c0 && c <= c1 && __builtin_fabsf(dx) <= R) v0 = expneg_hw(kap * (dx * dx));
        S.rx[grp][slot] = v0;
        const int r = r0 - 2 * B + slot;
        float u0 = 0.0f;
        const float dy = ((float)r + 0.5f) - y;
        if (on && r >= r0 && r <= r1 && __builtin_fabsf(dy) <= R) u0 = expneg_hw(kap * (dy * dy));
        if constexpr (B == 0) {
            const float u1 = u0 * dy;
            S.ty[grp][slot] = make_float4(u0, u1, u1 * dy, 0.0f);
        } else {
            static_assert(RY, "a folded blur needs the raw row factors");
            S.ry[grp][slot] = u0;
        }
    }
    group_sync();
    if constexpr (B > 0) {
        // blurred row tables (the column ones are formed per column in the gather);
        // table slot t is pixel r0 - b + t; raw slot t + 2b - k holds pixel
        // r0 + t - k, whose offset dy gives the e dy and e dy^2 terms
        const int n_ty = on ? (r1 - r0 + 1) + 2 * B : 0;
#pragma unroll
        for (int m = 0; m < BT / G; ++m) {
            if (G * m >= n_ty) break;
            const int t = lane + G * m;
            if (t < BT - 2 * B) {
                float Y0 = 0.0f, Y1 = 0.0f, Y2 = 0.0f;
#pragma unroll
                for (int k = 0; k <= 2 * B; ++k) {
                    const float w = blur_w[k];
                    const float u0 = S.ry[grp][t + 2 * B - k];
                    const float dy = ((float)(r0 + t - k) + 0.5f) - y;
                    const float u1 = u0 * dy;
                    Y0 = __builtin_fmaf(w, u0, Y0);
                    Y1 = __builtin_fmaf(w, u1, Y1);
                    Y2 = __builtin_fmaf(w, u1 * dy, Y2);
                }
                S.ty[grp][t] = make_float4(Y0, Y1, Y2, 0.0f);
            }
        }
        group_sync();
    }

    // gather: sum_q (dL/dJ)_q Ty(r) Tx(c) over the blurred support, inside the
    // image.  The column factors are constant along a column, so each lane
    // first forms P_j = sum_r (dL/dJ) Ty_j(r) down a column, or a slice of one
    // (three FMAs per pixel), and applies Tx afterwards.  Columns go to lanes
    // in blocks of G; a block of m < G columns splits its rows into
    // G / m' slices (m' = m rounded up to a power of two), so the lanes a
    // narrow block would leave idle shorten its walk instead.
    float s0 = 0.0f, s_x = 0.0f, s_y = 0.0f, s_r = 0.0f;
    if (on) {
        const int nt = (c1 - c0 + 1) + 2 * B, nu = (r1 - r0 + 1) + 2 * B;
        const int tlo = B - c0 > 0 ? B - c0 : 0;
        const int thi = nt < W - c0 + B ? nt : W - c0 + B;
        const int ulo = B - r0 > 0 ? B - r0 : 0;
        const int uhi = nu < H - r0 + B ? nu : H - r0 + B;
        constexpr int LG = G == 16 ? 4 : 3;
        const float* T = S.rx[grp];
        const int ncol = thi - tlo, nrow = uhi - ulo;
        for (int cb = 0; cb < ncol; cb += G) {
            const int m = ncol - cb < G ? ncol - cb : G;
            const int lm = m > 8 ? 4 : m > 4 ? 3 : m > 2 ? 2 : m > 1 ? 1 : 0;   // log2 m'
            const int cl = lane & ((1 << lm) - 1);
            const int per = (nrow + (G >> lm) - 1) >> (LG - lm);                // rows per slice
            const int ua = ulo + (lane >> lm) * per;
            const int ub = ua + per < uhi ? ua + per : uhi;
            if (cl >= m || ua >= ub) continue;
            const int t = tlo + cb + cl;
            // walk down the column slice with a row pointer: whole batches of GROWS
            // rows (their loads issued together), then batches of 4, 2 and 1
            const int64_t str = CS > 0 ? (int64_t)CS : stride;
            const float* __restrict__ q = src + (int64_t)(r0 - B + ua - sr) * str + (c0 - B + t - sc);
            float P0 = 0.0f, P1 = 0.0f, P2 = 0.0f;
            int u = ua;
#pragma unroll 1
            for (; u + GROWS <= ub; u += GROWS) {
                float e[GROWS];
                if constexpr (CS > 0) {
#pragma unroll
                    for (int k = 0; k < GROWS; ++k) e[k] = q[k * CS];
                    q += GROWS * CS;
                } else {
#pragma unroll
                    for (int k = 0; k < GROWS; ++k) {
                        e[k] = *q;
                        q += str;
                    }
                }
#pragma unroll
                for (int k = 0; k < GROWS; ++k) {
                    const float4 ty = S.ty[grp][u + k];
                    P0 = __builtin_fmaf(ty.x, e[k], P0);
                    P1 = __builtin_fmaf(ty.y, e[k], P1);
                    P2 = __builtin_fmaf(ty.z, e[k], P2);
                }
            }
#pragma unroll
            for (int nb = GROWS / 2; nb >= 1; nb >>= 1) {
                if (ub - u >= nb) {
                    float e[GROWS / 2];
                    if constexpr (CS > 0) {
#pragma unroll
                        for (int k = 0; k < nb; ++k) e[k] = q[k * CS];
                        q += nb * CS;
                    } else {
#pragma unroll
                        for (int k = 0; k < nb; ++k) {
                            e[k] = *q;
                            q += str;
                        }
                    }
#pragma unroll
                    for (int k = 0; k < nb; ++k) {
                        const float4 ty = S.ty[grp][u + k];
                        P0 = __builtin_fmaf(ty.x, e[k], P0);
                        P1 = __builtin_fmaf(ty.y, e[k], P1);
                        P2 = __builtin_fmaf(ty.z, e[k], P2);
                    }
                    u += nb;
                }
            }
            // blurred column factors of this column, from the raw ones (raw slot
            // t + 2b - k holds column c0 + t - k)
            float X0 = 0.0f, X1 = 0.0f, X2 = 0.0f;
#pragma unroll
            for (int k = 0; k <= 2 * B; ++k) {
                const float w = B > 0 ? blur_w[k] : 1.0f;
                const float v0 = T[t + 2 * B - k];
                const float dx = ((float)(c0 + t - k) + 0.5f) - x;
                const float v1 = v0 * dx;
                X0 = __builtin_fmaf(w, v0, X0);
                X1 = __builtin_fmaf(w, v1, X1);
                X2 = __builtin_fmaf(w, v1 * dx, X2);
            }
            s0 = __builtin_fmaf(P0, X0, s0);
            s_x = __builtin_fmaf(P0, X1, s_x);
            s_y = __builtin_fmaf(P1, X0, s_y);
            s_r = __builtin_fmaf(P0, X2, __builtin_fmaf(P2, X0, s_r));
        }
    }
    const float4 out = make_float4(group_sum<G>(s0), group_sum<G>(s_x), group_sum<G>(s_y), group_sum<G>(s_r));
    group_sync();
    return out;
}

// Gradients of one particle from its two frames' sums.
struct ParticleGrads {
    float gx1, gy1, gx2, gy2, gd, gz, gI0, sheet;
};

__device__ __forceinline__ ParticleGrads particle_grads(float z, float d, float I0, float sheet_sigma, float4 f0,
                                                        float4 f1)
{
    const float kap = 8.0f / (d * d);
    const float sum0 = f0.x + f1.x, sumr = f0.w + f1.w;
    const float s = sheet_sigma;
    const float Sz = expneg((z * z) * (0.5f / (s * s)));
    const float A = I0 * Sz;
    const float k2 = 2.0f * kap;                // d/dx of -kap dx^2 is 2 kap dx
    ParticleGrads o;
    o.gx1 = A * k2 * f0.y;
    o.gy1 = A * k2 * f0.z;
    o.gx2 = A * k2 * f1.y;
    o.gy2 = A * k2 * f1.z;
    o.gd = A * (k2 / d) * sumr;                 // d kap / d d = -2 kap / d
    o.gI0 = sum0 * Sz;
    o.gz = sum0 * A * (-z / (s * s));
    o.sheet = sum0 * A * ((z * z) / (s * s * s));
    return o;
}

// Particle-major gather: G lanes per particle read their patch rows of the
// frame's gradient image from global memory (any diameter bound and blur).
template <int B, int BT, int G>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(G == 8 ? 6 : BT == 32 ? 7 : 4)))
bwd_gather(BwdArgs a, int64_t n_span)
{
    __shared__ GatherLds<G, BT> S;
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int64_t g0 = (int64_t)xcd_contiguous(blockIdx.x, gridDim.x) * (256 / G);
    int64_t g = g0 + grp;

    bool in_pair = false, valid = false;
    int H = 1, W = 1;
    int64_t img = 0;
    float z = 0.0f, d = 1.0f, I0 = 0.0f;
    if (g < n_span) {
        const int p = find_pair_from(a.pairs, a.n_pairs, g0, g);
        const synthpix_pair P = a.pairs[p];
        int64_t i = g - P.particle_offset;
        if (i >= 0 && i < P.n_max) {
            // slots follow the home-block order: neighbouring groups read
            // overlapping rows of dL/dJ
            if (a.order.entries) i = a.order.entries[a.order.L[p].entry_base + i];
            g = P.particle_offset + i;
            in_pair = true;
            H = P.H;
            W = P.W;
            img = P.image_offset;
            z = a.z[g];
            d = a.d[g];
            I0 = a.I0[g];
            valid = (I0 > 0.0f) && (d > 0.0f);
            if (valid && !(d <= a.d_max)) {
                if (lane == 0) atomicOr(a.status, SP_STATUS_D_ABOVE_MAX);
                valid = false;
            }
        }
    }
    const float kap = 8.0f / (d * d);
    const float R = 1.5f * d;
    float4 fs[2];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        float x = 0.0f, y = 0.0f;
        if (in_pair) {
            x = f ? a.x2[g] : a.x1[g];
            y = f ? a.y2[g] : a.y1[g];
        }
        int c0 = 0, c1 = -1, r0 = 0, r1 = -1;
        bool on = valid && cover_range(x, R, W, c0, c1);
        on = on && cover_range(y, R, H, r0, r1);
        fs[f] = frame_sums<B, BT, true, G>(S, grp, lane, on, x, y, kap, R, c0, c1, r0, r1, W, H,
                                  a.grad + img + (int64_t)f * H * W, W, 0, 0, a.blur_w);
    }

    if (lane != 0) return;
    if (!in_pair) {
        // a slot in no pair's particle range (a gap of the packed arrays): zero gradients
        if (g < n_span) {
            a.g_x1[g] = 0.0f;
            a.g_y1[g] = 0.0f;
            a.g_z[g] = 0.0f;
            a.g_d[g] = 0.0f;
            a.g_I0[g] = 0.0f;
        }
        return;
    }
    ParticleGrads o{};
    if (valid) o = particle_grads(z, d, I0, a.sheet_sigma, fs[0], fs[1]);
    a.g_x1[g] = o.gx1;
    a.g_y1[g] = o.gy1;
    a.g_z[g] = o.gz;
    a.g_d[g] = o.gd;
    a.g_I0[g] = o.gI0;
    a.gx2[g] = o.gx2;
    a.gy2[g] = o.gy2;
    a.sheet[g] = o.sheet;
}

// Tile-major gather.  Frame f's particles are grouped by the home block
// (2^lb x 2^lb pixels) of their frame-f position; a workgroup takes one
// (frame, block), stages the frame's B^T dL/dJ over the block grown by a halo
// of hb pixels into LDS (zeros outside the image), then runs the lane-group
// sums of the block's particles, 16 per pass, from LDS.  With hb >=
// ceil(1.5 d_max) + 2 every in-image pixel of the support of a particle whose
// position lies in the block (or beyond the image edge next to it, where the
// home block is clamped) is inside the staged region.  The sums go to
// parts[f * n_span + slot]; bwd_particles turns them into gradients.
// RS: the staged region's row stride (a multiple of 8 at least its width, so
// the gather's row loads take immediate offsets), 0 for a stride equal to the
// width.
template <int RS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
bwd_tile_gather(BwdArgs a, int64_t n_span, int lb, int hb)
{
    extern __shared__ __align__(16) float region[];
    // sixteen lanes per particle here: eight (more particles per wave, deeper
    // walks for the wide supports this gather serves) measured slower
    constexpr int G = 16, NP = 256 / G;
    __shared__ GatherLds<G, 32, false> S;
    const int64_t blocks = a.order.blocks;
    const int64_t item = xcd_contiguous(blockIdx.x, gridDim.x);
    const int f = item >= blocks ? 1 : 0;
    const int64_t b = item - (int64_t)f * blocks;
    const AdvectOrder& O = f ? a.order2 : a.order;
    const int cnt = (int)O.count[b];
    if (cnt == 0) return;                      // the whole workgroup, before its barrier
    const int p = find_pair_by_tile(O.L, a.n_pairs, b);
    const synthpix_pair P = a.pairs[p];
    const PairLayout PL = O.L[p];
    // home blocks are numbered in strips of four block rows, column by column
    // inside a strip, odd strips right to left (the order's numbering)
    const int tl = (int)(b - PL.tile_base);
    const int s0 = (tl / (4 * PL.ntx)) * 4;
    const int rows = PL.nty - s0 < 4 ? PL.nty - s0 : 4;
    const int wi = tl - s0 * PL.ntx;
    const int col = wi / rows, by = s0 + (wi - col * rows);
    const int bx = (s0 & 4) ? PL.ntx - 1 - col : col;
    const int side = 1 << lb, rw = side + 2 * hb;
    const int rs = RS > 0 ? RS : rw;
    const int ox = (bx << lb) - hb, oy = (by << lb) - hb;
    const int H = P.H, W = P.W;
    const float* __restrict__ src = a.grad + P.image_offset + (int64_t)f * H * W;
    // one region row per wave and step, lanes along the row
    {
        const int wave = threadIdx.x >> 6, ln = threadIdx.x & 63;
        for (int r = wave; r < rw; r += 4) {
            const int R = oy + r;
            const bool rin = R >= 0 && R < H;
            const float* __restrict__ row = src + (int64_t)(rin ? R : 0) * W;
            for (int c = ln; c < rw; c += 64) {
                const int C = ox + c;
                region[r * rs + c] = (rin && C >= 0 && C < W) ? row[C] : 0.0f;
            }
        }
    }
    __syncthreads();

    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int64_t off = O.offset[b];
    const float* __restrict__ fx = f ? a.x2 : a.x1;
    const float* __restrict__ fy = f ? a.y2 : a.y1;
    for (int base = 0; base < cnt; base += NP) {
        const int k = base + grp;
        bool act = k < cnt, on = false;
        int64_t g = 0;
        float x = 0.0f, y = 0.0f, d = 1.0f;
        if (act) {
            g = P.particle_offset + O.entries[off + k];
            d = a.d[g];
            x = fx[g];
            y = fy[g];
            on = (a.I0[g] > 0.0f) && (d > 0.0f) && (d <= a.d_max);
        }
        const float kap = 8.0f / (d * d);
        const float R = 1.5f * d;
        int c0 = 0, c1 = -1, r0 = 0, r1 = -1;
        on = on && cover_range(x, R, W, c0, c1);
        on = on && cover_range(y, R, H, r0, r1);
        // in-image support inside the staged region (always, for d <= d_max)
        on = on && c0 >= ox && c1 < ox + rw && r0 >= oy && r1 < oy + rw;
        const float4 sums = frame_sums<0, 32, false, G, RS, GROWS_LDS>(S, grp, lane, on, x, y, kap, R, c0, c1, r0,
                                                                     r1, W, H, region, rs, oy, ox, a.blur_w);
        if (act && lane == 0) a.parts[(int64_t)f * n_span + g] = sums;
    }
}

// Per-slot gradients from the tile gather's frame sums (zeros for slots in no
// pair's particle range and for invalid particles).
__global__ void __launch_bounds__(256) bwd_particles(BwdArgs a, int64_t n_span)
{
    const int64_t g0 = (int64_t)xcd_contiguous(blockIdx.x, gridDim.x) * 256;
    const int64_t g = g0 + threadIdx.x;
    if (g >= n_span) return;
    const int p = find_pair_from(a.pairs, a.n_pairs, g0, g);
    const synthpix_pair P = a.pairs[p];
    const int64_t i = g - P.particle_offset;
    ParticleGrads o{};
    const bool in_pair = i >= 0 && i < P.n_max;
    if (in_pair) {
        const float z = a.z[g], d = a.d[g], I0 = a.I0[g];
        bool valid = (I0 > 0.0f) && (d > 0.0f);
        if (valid && !(d <= a.d_max)) {
            atomicOr(a.status, SP_STATUS_D_ABOVE_MAX);
            valid = false;
        }
        if (valid) o = particle_grads(z, d, I0, a.sheet_sigma, a.parts[g], a.parts[n_span + g]);
    }
    a.g_x1[g] = o.gx1;
    a.g_y1[g] = o.gy1;
    a.g_z[g] = o.gz;
    a.g_d[g] = o.gd;
    a.g_I0[g] = o.gI0;
    if (in_pair) {
        a.gx2[g] = o.gx2;
        a.gy2[g] = o.gy2;
        a.sheet[g] = o.sheet;
    }
}

// One input column x of a strip of the per-pixel pass: its SH + 2b rows from
// Y0 - b (zeros outside the image) blurred vertically into vb[.][k].  MSE: the
// values are scale (J - T); returns the float64 sum of (J - T)^2 over the
// strip's own rows (Y0 .. Y0 + SH - 1, inside the image), 0 otherwise.
template <int B, bool MSE, int SH, int VW>
__device__ __forceinline__ double blur_column(const BwdArgs& a, int64_t base, int W, int H, int x, int Y0, int k,
                                              float (*vb)[VW])
{
    const bool xin = x >= 0 && x < W;
    float g[SH + 2 * B];
    double sq = 0.0;
#pragma unroll
    for (int r = 0; r < SH + 2 * B; ++r) {
        const int y = Y0 - B + r;
        const bool in = xin && y >= 0 && y < H;
        if constexpr (MSE) {
            const int64_t i = base + (int64_t)(in ? y : 0) * W + (in ? x : 0);
            const float j = in ? a.J[i] : 0.0f, tv = in ? a.T[i] : 0.0f;
            g[r] = a.mse_scale * (j - tv);
            if (in && r >= B && r < SH + B) {
                const double e = (double)j - (double)tv;
                sq = __builtin_fma(e, e, sq);
            }
        } else {
            g[r] = in ? a.grad[base + (int64_t)y * W + x] : 0.0f;
        }
    }
#pragma unroll
    for (int r = 0; r < SH; ++r) {
        float v = 0.0f;
#pragma unroll
        for (int q = 0; q <= 2 * B; ++q) v = __builtin_fmaf(a.blur_w[q], g[r + q], v);
        vb[r][k] = v;
    }
    return sq;
}

// e = B^T dL/dJ, once per pixel: the zero-padded blur's adjoint sums
// w_k dL/dJ(q + k) over the taps that land inside the image (the same blur,
// its weights being symmetric).  A workgroup owns a strip of SH output rows
// by 256 output columns of one frame: each thread takes one column (the first
// 2b threads also one of the b apron columns on either side), issues its
// SH + 2b loads together and blurs them vertically in registers; the rows then
// pass through LDS for the horizontal taps.  Rows of 256 floats keep the reads
// and writes in whole 1 KB segments, and images 256 k pixels wide split into
// whole strips.  Workgroups are numbered (pair, frame, strip row, strip
// column) over the batch's largest pair, XCD-contiguously.
// MSE: dL/dJ is the mean-squared-difference loss's gradient scale (J - T),
// formed from the images and the target as they are read (the same binary32
// products synthpix_mse_grad stores), and with loss_part each workgroup also
// writes the float64 sum of (J - T)^2 over the pixels of its strip (every
// pixel lies in exactly one strip); b = 0 is then a plain pass.
template <int B, bool MSE>
__global__ void __launch_bounds__(256)
bwd_blur_grad(BwdArgs a, int nsx, int nsy)
{
    constexpr int SH = blur_strip_rows(MSE), VW = 256 + 2 * B;
    __shared__ float vb[SH][VW];
    __shared__ double red[MSE ? 256 : 1];
    const int64_t bid = xcd_contiguous(blockIdx.x, gridDim.x);
    const int64_t per_pair = (int64_t)2 * nsx * nsy;
    const int p = (int)(bid / per_pair);
    int rem = (int)(bid - (int64_t)p * per_pair);
    const int f = rem / (nsx * nsy);
    rem -= f * nsx * nsy;
    const int sy = rem / nsx, sx = rem - sy * nsx;
    const int H = a.pairs[p].H, W = a.pairs[p].W;
    const int X0 = sx * 256, Y0 = sy * SH;
    if (X0 >= W || Y0 >= H) {                    // the whole workgroup, before its barrier
        if (MSE && a.loss_part && threadIdx.x == 0) a.loss_part[bid] = 0.0;
        return;
    }
    const int64_t base = a.pairs[p].image_offset + (int64_t)f * H * W;
    const int t = (int)threadIdx.x;
    // vb column k holds input column X0 - b + k
    double sq = 0.0;
    const int nc = t < 2 * B ? 2 : 1;
#pragma unroll 1
    for (int c = 0; c < nc; ++c) {             // own column, then an apron column
        const int xc = c == 0 ? X0 + t : t < B ? X0 - B + t : X0 + 256 + (t - B);
        const int k = c == 0 ? B + t : t < B ? t : 256 + t;
        const double s2 = blur_column<B, MSE, SH, VW>(a, base, W, H, xc, Y0, k, vb);
        if (c == 0) sq = s2;
    }
    if (MSE && a.loss_part) {
        red[t] = sq;
        __syncthreads();
        for (int w = 128; w >= 1; w >>= 1) {
            if (t < w) red[t] += red[t + w];
            __syncthreads();
        }
        if (t == 0) a.loss_part[bid] = red[0];
    }
    __syncthreads();
    const int x = X0 + t;
    if (x >= W) return;
    const int nr = H - Y0 < SH ? H - Y0 : SH;
#pragma unroll 4
    for (int r = 0; r < nr; ++r) {
        float e = 0.0f;
#pragma unroll
        for (int q = 0; q <= 2 * B; ++q) e = __builtin_fmaf(a.blur_w[q], vb[r][t + q], e);
        a.eblur[base + (int64_t)(Y0 + r) * W + x] = e;
    }
}

// ------------------------------------------------------------------ flow adjoint

struct Sample {
    float2 val;
    float2 jx, jy;        // dU/dpx, dU/dpy (zero along clamped axes)
    int i0, j0;
    float fx, fy;
};

// Value bit-identical to sample_flow, plus Jacobian and node weights.
__device__ __forceinline__ Sample sample_jac(const FlowView& fv, float px, float py)
{
    Sample o;
    const float gxr = px * fv.sx - 0.5f;
    const float gyr = py * fv.sy - 0.5f;
    const float gx = __builtin_fminf(__builtin_fmaxf(gxr, 0.0f), (float)(fv.Gw - 1));
    const float gy = __builtin_fminf(__builtin_fmaxf(gyr, 0.0f), (float)(fv.Gh - 1));
    int j0 = (int)__builtin_floorf(gx);
    int i0 = (int)__builtin_floorf(gy);
    j0 = j0 > fv.Gw - 2 ? fv.Gw - 2 : j0;
    i0 = i0 > fv.Gh - 2 ? fv.Gh - 2 : i0;
    const float fx = gx - (float)j0;
    const float fy = gy - (float)i0;
    const float2* row0 = fv.F + (size_t)i0 * fv.Gw + j0;
    const float4 r0 = load_pair(row0);
    const float4 r1 = load_pair(row0 + fv.Gw);
    const float2 A = make_float2(r0.x, r0.y), Bn = make_float2(r0.z, r0.w);
    const float2 C = make_float2(r1.x, r1.y), E = make_float2(r1.z, r1.w);
    {
        const float top = __builtin_fmaf(fx, Bn.x - A.x, A.x);
        const float bot = __builtin_fmaf(fx, E.x - C.x, C.x);
        o.val.x = __builtin_fmaf(fy, bot - top, top);
    }
    {
        const float top = __builtin_fmaf(fx, Bn.y - A.y, A.y);
        const float bot = __builtin_fmaf(fx, E.y - C.y, C.y);
        o.val.y = __builtin_fmaf(fy, bot - top, top);
    }
    const float inx = (gxr > 0.0f && gxr < (float)(fv.Gw - 1)) ? fv.sx : 0.0f;
    const float iny = (gyr > 0.0f && gyr < (float)(fv.Gh - 1)) ? fv.sy : 0.0f;
    o.jx.x = ((1.0f - fy) * (Bn.x - A.x) + fy * (E.x - C.x)) * inx;
    o.jx.y = ((1.0f - fy) * (Bn.y - A.y) + fy * (E.y - C.y)) * inx;
    o.jy.x = ((1.0f - fx) * (C.x - A.x) + fx * (E.x - Bn.x)) * iny;
    o.jy.y = ((1.0f - fx) * (C.y - A.y) + fx * (E.y - Bn.y)) * iny;
    o.i0 = i0;
    o.j0 = j0;
    o.fx = fx;
    o.fy = fy;
    return o;
}

// Per-particle accumulation of node contributions, merged while consecutive
// samples stay in one grid cell, flushed as 64-bit fixed-point atomic adds
// (integer sums: the result does not depend on their order).  A run is flushed
// as soon as the sample leaves its cell (holding the two runs before it back,
// so that lanes flush together, took 40 more registers and a wave per SIMD).
struct CellRun {
    int i0 = -1, j0 = 0;
    float acc[8];
};

struct NodeRun {
    CellRun cur;
    int Gw;
    double scale;         // 2^e; 0 when the flow gradient is not accumulated
    // the workgroup's LDS window of node sums (rows wi0 .., cols wj0 .., wh x ww
    // nodes, (u, v) interleaved); nodes outside it become overflow records
    unsigned long long* win;
    int wi0, wj0, wh, ww;
    GridRecord* ovf;      // the workgroup's overflow records (global memory)
    unsigned* n_ovf;      // their count (LDS)

    __device__ void add_node(int ni, int nj, int c, unsigned long long q)
    {
        const int li = ni - wi0, lj = nj - wj0;
        if ((unsigned)li < (unsigned)wh && (unsigned)lj < (unsigned)ww) {
            atomicAdd(win + 2 * (li * ww + lj) + c, q);
        } else {
            const unsigned k = atomicAdd(n_ovf, 1u);
            if (k < GRID_OVF_CAP) ovf[k] = GridRecord{2 * (ni * Gw + nj) + c, 0u, q};
        }
    }

    __device__ void flush(const CellRun& r)
    {
        if (r.i0 < 0) return;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const float v = r.acc[2 * n + c];
                if (v != 0.0f)
                    add_node(r.i0 + (n >> 1), r.j0 + (n & 1), c,
                             (unsigned long long)(long long)__builtin_rint((double)v * scale));
            }
        }
    }

    __device__ void finish() { flush(cur); }

    __device__ void add(const Sample& s, float ku, float kv)
    {
        if (scale == 0.0) return;
        if (s.i0 != cur.i0 || s.j0 != cur.j0) {
            flush(cur);
            cur.i0 = s.i0;
            cur.j0 = s.j0;
#pragma unroll
            for (int k = 0; k < 8; ++k) cur.acc[k] = 0.0f;
        }
        const float w[4] = {(1.0f - s.fx) * (1.0f - s.fy), s.fx * (1.0f - s.fy), (1.0f - s.fx) * s.fy, s.fx * s.fy};
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            cur.acc[2 * n] = __builtin_fmaf(w[n], ku, cur.acc[2 * n]);
            cur.acc[2 * n + 1] = __builtin_fmaf(w[n], kv, cur.acc[2 * n + 1]);
        }
    }
};

// Back-propagate one sample with upstream (ku, kv); returns J^T k in (bx, by).
__device__ __forceinline__ void stage_back(const FlowView& fv, NodeRun& run, float px, float py, float ku, float kv,
                                           float& bx, float& by)
{
    const Sample s = sample_jac(fv, px, py);
    run.add(s, ku, kv);
    bx = s.jx.x * ku + s.jx.y * kv;
    by = s.jy.x * ku + s.jy.y * kv;
}

__device__ __forceinline__ void substep_adjoint(const FlowView& fv, NodeRun& run, float px, float py, float h,
                                                float hh, int integrator, float& gpx, float& gpy)
{
    float bx, by;
    if (integrator == SP_EULER) {
        stage_back(fv, run, px, py, h * gpx, h * gpy, bx, by);
        gpx += bx;
        gpy += by;
        return;
    }
    const float2 k1 = sample_flow(fv, px, py);
    const float p2x = __builtin_fmaf(hh, k1.x, px), p2y = __builtin_fmaf(hh, k1.y, py);
    const float2 k2 = sample_flow(fv, p2x, p2y);
    const float p3x = __builtin_fmaf(hh, k2.x, px), p3y = __builtin_fmaf(hh, k2.y, py);
    const float2 k3 = sample_flow(fv, p3x, p3y);
    const float p4x = __builtin_fmaf(h, k3.x, px), p4y = __builtin_fmaf(h, k3.y, py);
    const float c = h / 6.0f;
    float b4x, b4y, b3x, b3y, b2x, b2y, b1x, b1y;
    stage_back(fv, run, p4x, p4y, c * gpx, c * gpy, b4x, b4y);
    stage_back(fv, run, p3x, p3y, 2.0f * c * gpx + h * b4x, 2.0f * c * gpy + h * b4y, b3x, b3y);
    stage_back(fv, run, p2x, p2y, 2.0f * c * gpx + hh * b3x, 2.0f * c * gpy + hh * b3y, b2x, b2y);
    stage_back(fv, run, px, py, c * gpx + hh * b2x, c * gpy + hh * b2y, b1x, b1y);
    gpx += ((b1x + b2x) + b3x) + b4x;
    gpy += ((b1y + b2y) + b3y) + b4y;
}

// Words of the fixed-point scale block in the workspace.
enum { SC_G2MAX = 0, SC_LIP = 1, SC_EXP = 2, SC_STATE = 3 };
enum { SC_NONE = 0, SC_VALID = 1, SC_NONFINITE = 2 };

// Reverse sweep of every particle: final position gradient (added to g_x1,
// g_y1) and node sums into the fixed-point grid.  CK checkpoints of the
// trajectory are kept, one every L = ceil(substeps / CK) substeps; each segment
// is recomputed into SK >= L slots during the sweep.

template <int CK, int SK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CK <= 8 ? 4 : 3)))
bwd_advect(BwdArgs a, synthpix_advect_params ap)
{
    __shared__ unsigned long long win[2 * WIN_NODES];
    __shared__ int s_box[4][4];
    __shared__ unsigned s_novf;
    // workgroup -> (pair, 256-particle chunk of the pair's ordered particles)
    const int64_t wg = xcd_contiguous(blockIdx.x, gridDim.x);
    int p = 0;
    {
        int lo = 0, hi = a.n_pairs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.grid.wg_base[mid] <= wg) lo = mid;
            else hi = mid - 1;
        }
        p = lo;
    }
    const synthpix_pair P = a.pairs[p];
    const int64_t chunk = wg - a.grid.wg_base[p];
    int64_t i = chunk * 256 + threadIdx.x;
    int64_t g = 0;
    bool live = false;
    float gpx = 0.0f, gpy = 0.0f, px = 0.0f, py = 0.0f;
    if (i < P.n_max) {
        // slots follow the home-block order: neighbouring lanes sample, and add
        // into, neighbouring grid cells
        if (a.order.entries) i = a.order.entries[a.order.L[p].entry_base + i];
        g = P.particle_offset + i;
        gpx = a.gx2[g];
        gpy = a.gy2[g];
        px = a.x1[g];
        py = a.y1[g];
        live = (gpx != 0.0f || gpy != 0.0f) && __builtin_isfinite(px) && __builtin_isfinite(py);
    }
    NodeRun run;
    run.Gw = P.Gw;
    run.scale = a.scale[SC_STATE] == SC_VALID ? __builtin_ldexp(1.0, (int)a.scale[SC_EXP]) : 0.0;
    const FlowView fv = flow_view(P, a.flow);

    // window: the box of the live particles' starting cells, grown on every side
    // by as many cells as the LDS window holds (at least one)
    int bi0 = 1 << 30, bj0 = 1 << 30, bi1 = -1, bj1 = -1;
    if (live) {
        const float gx = __builtin_fminf(__builtin_fmaxf(px * fv.sx - 0.5f, 0.0f), (float)(fv.Gw - 1));
        const float gy = __builtin_fminf(__builtin_fmaxf(py * fv.sy - 0.5f, 0.0f), (float)(fv.Gh - 1));
        bj0 = bj1 = (int)gx;
        bi0 = bi1 = (int)gy;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        bi0 = min(bi0, __shfl_xor(bi0, o, 64));
        bj0 = min(bj0, __shfl_xor(bj0, o, 64));
        bi1 = max(bi1, __shfl_xor(bi1, o, 64));
        bj1 = max(bj1, __shfl_xor(bj1, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        s_box[threadIdx.x >> 6][0] = bi0;
        s_box[threadIdx.x >> 6][1] = bj0;
        s_box[threadIdx.x >> 6][2] = bi1;
        s_box[threadIdx.x >> 6][3] = bj1;
    }
    if (threadIdx.x == 0) s_novf = 0u;
    __syncthreads();
    bi0 = min(min(s_box[0][0], s_box[1][0]), min(s_box[2][0], s_box[3][0]));
    bj0 = min(min(s_box[0][1], s_box[1][1]), min(s_box[2][1], s_box[3][1]));
    bi1 = max(max(s_box[0][2], s_box[1][2]), max(s_box[2][2], s_box[3][2])) + 1;
    bj1 = max(max(s_box[0][3], s_box[1][3]), max(s_box[2][3], s_box[3][3])) + 1;
    const bool any = bi1 >= bi0 && run.scale != 0.0;
    int m = 0;                                   // margin in cells
    if (any) {
        const int h0 = bi1 - bi0 + 1, w0 = bj1 - bj0 + 1;
        m = 1;
        while ((h0 + 2 * (m + 1)) * (w0 + 2 * (m + 1)) <= WIN_NODES) ++m;
        if (h0 + 2 * m > WIN_NODES || (h0 + 2 * m) * (w0 + 2 * m) > WIN_NODES) m = 0;
    }
    const int wh = any ? bi1 - bi0 + 1 + 2 * m : 0, ww = any ? bj1 - bj0 + 1 + 2 * m : 0;
    const bool use_win = any && wh * ww <= WIN_NODES;
    run.win = win;
    run.wi0 = bi0 - m;
    run.wj0 = bj0 - m;
    run.wh = use_win ? wh : 0;                   // no window: every node becomes a record
    run.ww = ww;
    run.ovf = a.grid.ovf + wg * GRID_OVF_CAP;
    run.n_ovf = &s_novf;
    if (use_win) {
        for (int k = threadIdx.x; k < 2 * wh * ww; k += 256) win[k] = 0ull;
    }
    __syncthreads();

    if (live) {
        const int S = ap.substeps;
        const float h = ap.dt / (float)S;
        const float hh = h * 0.5f;
        const int L = (S + CK - 1) / CK;
        const int nseg = (S + L - 1) / L;
        float cpx[CK], cpy[CK];
        float qx = px, qy = py;
        for (int s = 0; s < S; ++s) {
            if (s % L == 0) {
                cpx[s / L] = qx;
                cpy[s / L] = qy;
            }
            if (s + 1 < S) substep(fv, qx, qy, h, hh, ap.integrator);
        }
        if constexpr (SK == 1) {
            // S <= CK: every substep's start is a checkpoint, the sweep walks them
            // (no segment slots, whose runtime indexing would live in scratch)
            for (int seg = nseg - 1; seg >= 0; --seg)
                substep_adjoint(fv, run, cpx[seg], cpy[seg], h, hh, ap.integrator, gpx, gpy);
        } else {
            float spx[SK], spy[SK];
            for (int seg = nseg - 1; seg >= 0; --seg) {
                const int s0 = seg * L;
                const int len = (S - s0) < L ? (S - s0) : L;
                spx[0] = cpx[seg];
                spy[0] = cpy[seg];
                for (int k = 1; k < len; ++k) {
                    float tx = spx[k - 1], ty = spy[k - 1];
                    substep(fv, tx, ty, h, hh, ap.integrator);
                    spx[k] = tx;
                    spy[k] = ty;
                }
                for (int k = len - 1; k >= 0; --k)
                    substep_adjoint(fv, run, spx[k], spy[k], h, hh, ap.integrator, gpx, gpy);
            }
        }
        run.finish();
        a.g_x1[g] += gpx;
        a.g_y1[g] += gpy;
    }
    __syncthreads();

    // the window's nonzero box, then its sums into this workgroup's partial
    // (rows of the box, (u, v) interleaved) and the header
    int ti0 = 1 << 30, tj0 = 1 << 30, ti1 = -1, tj1 = -1;
    if (use_win) {
        for (int k = threadIdx.x; k < wh * ww; k += 256) {
            if (win[2 * k] != 0ull || win[2 * k + 1] != 0ull) {
                const int li = k / ww, lj = k - li * ww;
                ti0 = min(ti0, li);
                ti1 = max(ti1, li);
                tj0 = min(tj0, lj);
                tj1 = max(tj1, lj);
            }
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        ti0 = min(ti0, __shfl_xor(ti0, o, 64));
        tj0 = min(tj0, __shfl_xor(tj0, o, 64));
        ti1 = max(ti1, __shfl_xor(ti1, o, 64));
        tj1 = max(tj1, __shfl_xor(tj1, o, 64));
    }
    __syncthreads();                             // s_box is reused
    if ((threadIdx.x & 63) == 0) {
        s_box[threadIdx.x >> 6][0] = ti0;
        s_box[threadIdx.x >> 6][1] = tj0;
        s_box[threadIdx.x >> 6][2] = ti1;
        s_box[threadIdx.x >> 6][3] = tj1;
    }
    __syncthreads();
    ti0 = min(min(s_box[0][0], s_box[1][0]), min(s_box[2][0], s_box[3][0]));
    tj0 = min(min(s_box[0][1], s_box[1][1]), min(s_box[2][1], s_box[3][1]));
    ti1 = max(max(s_box[0][2], s_box[1][2]), max(s_box[2][2], s_box[3][2]));
    tj1 = max(max(s_box[0][3], s_box[1][3]), max(s_box[2][3], s_box[3][3]));
    const int th = ti1 >= ti0 ? ti1 - ti0 + 1 : 0, tw = ti1 >= ti0 ? tj1 - tj0 + 1 : 0;
    unsigned long long* part = a.grid.part + wg * (2 * WIN_NODES);
    for (int k = threadIdx.x; k < th * tw; k += 256) {
        const int r = k / tw, c = k - r * tw;
        const int src = (ti0 + r) * ww + (tj0 + c);
        part[2 * k] = win[2 * src];
        part[2 * k + 1] = win[2 * src + 1];
    }
    if (threadIdx.x == 0) {
        const unsigned n = s_novf;
        if (n > GRID_OVF_CAP) atomicOr(a.status, SP_STATUS_GRID_OVERFLOW);
        GridHeader hd;
        hd.i0 = run.wi0 + ti0;
        hd.j0 = run.wj0 + tj0;
        hd.h = th;
        hd.w = tw;
        hd.n_ovf = n < GRID_OVF_CAP ? n : GRID_OVF_CAP;
        a.grid.head[wg] = hd;
    }
}

// Flow-grid gradient of one 32 x 32-node tile of one pair: each thread holds
// four nodes' two fixed-point sums and adds, in workgroup order, the partial
// of every workgroup of the pair whose box covers them, then the overflow
// records that fall in the tile; the sums leave as floats (scaled by 2^-e).
// Workgroups are (pair, tile row, tile column) over the batch's largest grid.
constexpr int GRID_TILE = 32;

__global__ void __launch_bounds__(256)
bwd_grid_reduce(BwdArgs a, int ntx, int nty)
{
    const int64_t bid = blockIdx.x;
    const int p = (int)(bid / ((int64_t)ntx * nty));
    const int rem = (int)(bid - (int64_t)p * ntx * nty);
    const int ty = rem / ntx, tx = rem - ty * ntx;
    const synthpix_pair P = a.pairs[p];
    const int i0 = ty * GRID_TILE, j0 = tx * GRID_TILE;
    if (i0 >= P.Gh || j0 >= P.Gw) return;
    const uint32_t state = a.scale[SC_STATE];
    float* out = a.g_flow + P.flow_offset;
    // thread -> nodes (i0 + r + 8 q, j0 + c), r = threadIdx / 32, c = threadIdx % 32, q = 0..3
    const int r = threadIdx.x >> 5, c = threadIdx.x & 31;
    unsigned long long su[4] = {0ull, 0ull, 0ull, 0ull}, sv[4] = {0ull, 0ull, 0ull, 0ull};
    __shared__ int s_list[256];
    if (state == SC_VALID) {
        const int64_t w0 = a.grid.wg_base[p], w1 = a.grid.wg_base[p + 1];
        for (int64_t wb = w0; wb < w1; wb += 256) {
            // the covering workgroups of this stretch, in order
            const int64_t w = wb + threadIdx.x;
            bool hit = false;
            if (w < w1) {
                const GridHeader hd = a.grid.head[w];
                hit = (hd.h > 0 && hd.i0 < i0 + GRID_TILE && hd.i0 + hd.h > i0 && hd.j0 < j0 + GRID_TILE &&
                       hd.j0 + hd.w > j0) || hd.n_ovf > 0;
            }
            // ordered compaction: a workgroup-wide prefix count of the hits
            const unsigned long long bal = __ballot(hit);
            __shared__ int s_cnt[4];
            if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = __popcll(bal);
            __syncthreads();
            int before = 0;
            for (int k = 0; k < (int)(threadIdx.x >> 6); ++k) before += s_cnt[k];
            const int lane = threadIdx.x & 63;
            const unsigned long long lower = lane ? (bal & ((~0ull) >> (64 - lane))) : 0ull;
            if (hit) s_list[before + __popcll(lower)] = (int)(w - wb);
            const int nl = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
            __syncthreads();
            for (int k = 0; k < nl; ++k) {
                const int64_t wi = wb + s_list[k];
                const GridHeader hd = a.grid.head[wi];
                const unsigned long long* part = a.grid.part + wi * (2 * WIN_NODES);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int ni = i0 + r + 8 * q, nj = j0 + c;
                    const int li = ni - hd.i0, lj = nj - hd.j0;
                    if ((unsigned)li < (unsigned)hd.h && (unsigned)lj < (unsigned)hd.w) {
                        su[q] += part[2 * (li * hd.w + lj)];
                        sv[q] += part[2 * (li * hd.w + lj) + 1];
                    }
                }
                for (unsigned e = 0; e < hd.n_ovf; ++e) {
                    const GridRecord rec = a.grid.ovf[wi * GRID_OVF_CAP + e];
                    const int node = rec.elem >> 1;
                    const int ni = node / P.Gw, nj = node - ni * P.Gw;
                    const int q = (ni - i0 - r) >> 3;
                    if (nj == j0 + c && ni >= i0 + r && ((ni - i0 - r) & 7) == 0 && q < 4) {
                        if (rec.elem & 1) sv[q] += rec.value;
                        else su[q] += rec.value;
                    }
                }
            }
            __syncthreads();
        }
    }
    const double inv = state == SC_VALID ? __builtin_ldexp(1.0, -(int)a.scale[SC_EXP]) : 0.0;
    const float fill = state == SC_NONFINITE ? __builtin_nanf("") : 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int ni = i0 + r + 8 * q, nj = j0 + c;
        if (ni < P.Gh && nj < P.Gw) {
            const int64_t k = 2 * ((int64_t)ni * P.Gw + nj);
            out[k] = state == SC_VALID ? (float)((double)(long long)su[q] * inv) : fill;
            out[k + 1] = state == SC_VALID ? (float)((double)(long long)sv[q] * inv) : fill;
        }
    }
}

// Inputs of the fixed-point scale: the largest |dL/dx2|, |dL/dy2| and a bound L
// on the transposed velocity Jacobian's max-row-sum over every cell (the
// bilinear x-derivative is a blend of the cell's two edge differences, so its
// magnitude is at most the larger one).  Also each slice's float64 sum of the
// sheet-width terms, in a fixed order.  Blocks (pair, slice), ns <= BWD_SLICES
// slices per pair (more for pairs with many particles); float bits of
// non-negative values order like unsigned integers.
__global__ void __launch_bounds__(256)
bwd_bounds(BwdArgs a, int ns)
{
    const synthpix_pair P = a.pairs[blockIdx.x];
    const int sl = blockIdx.y;
    float gm = 0.0f;
    double sh = 0.0;
#pragma unroll 4
    for (int64_t i = (int64_t)sl * 256 + threadIdx.x; i < P.n_max; i += (int64_t)ns * 256) {
        const int64_t g = P.particle_offset + i;
        const float u = a.gx2[g], v = a.gy2[g];
        gm = __builtin_fmaxf(gm, __builtin_fmaxf(__builtin_fabsf(u), __builtin_fabsf(v)));
        if (!__builtin_isfinite(u) || !__builtin_isfinite(v)) gm = __builtin_inff();
        sh += (double)a.sheet[g];
    }
    const float2* F = reinterpret_cast<const float2*>(a.flow + P.flow_offset);
    const float sx = (float)P.Gw / (float)P.W, sy = (float)P.Gh / (float)P.H;
    float lm = 0.0f;
    for (int i = sl; i < P.Gh - 1; i += ns)
        for (int j = threadIdx.x; j < P.Gw - 1; j += 256) {
            const float2 A = F[(int64_t)i * P.Gw + j], B = F[(int64_t)i * P.Gw + j + 1];
            const float2 C = F[(int64_t)(i + 1) * P.Gw + j], E = F[(int64_t)(i + 1) * P.Gw + j + 1];
            const float lx = sx * (__builtin_fmaxf(__builtin_fabsf(B.x - A.x), __builtin_fabsf(E.x - C.x)) +
                                   __builtin_fmaxf(__builtin_fabsf(B.y - A.y), __builtin_fabsf(E.y - C.y)));
            const float ly = sy * (__builtin_fmaxf(__builtin_fabsf(C.x - A.x), __builtin_fabsf(E.x - B.x)) +
                                   __builtin_fmaxf(__builtin_fabsf(C.y - A.y), __builtin_fabsf(E.y - B.y)));
            lm = __builtin_fmaxf(lm, __builtin_fmaxf(lx, ly));
            if (!__builtin_isfinite(lx) || !__builtin_isfinite(ly)) lm = __builtin_inff();
        }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        gm = __builtin_fmaxf(gm, __shfl_xor(gm, o, 64));
        lm = __builtin_fmaxf(lm, __shfl_xor(lm, o, 64));
    }
    __shared__ float red[2][4];
    __shared__ double sred[256];
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = gm;
        red[1][threadIdx.x >> 6] = lm;
    }
    sred[threadIdx.x] = sh;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) sred[threadIdx.x] += sred[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // per-block results (no same-address atomics); bwd_scale reduces them
        const int64_t k = (int64_t)blockIdx.x * ns + sl;
        a.bound_part[2 * k] = __builtin_fmaxf(__builtin_fmaxf(red[0][0], red[0][1]),
                                              __builtin_fmaxf(red[0][2], red[0][3]));
        a.bound_part[2 * k + 1] = __builtin_fmaxf(__builtin_fmaxf(red[1][0], red[1][1]),
                                                  __builtin_fmaxf(red[1][2], red[1][3]));
        a.sheet_part[k] = sred[0];
    }
}

// The fixed-point exponent e.  Every upstream value k of the reverse sweep obeys
// |k| <= K = G0 kfac growth^(S-1), from the stage recurrences with |J^T k| <= L |k|
// (Euler: kfac = |h|, growth = 1 + |h| L; RK4: k4 = c, k3 = 2c + |h| L k4,
// k2 = 2c + |h|/2 L k3, k1 = c + |h|/2 L k2 with c = |h|/6, growth = 1 + L sum k).
// A node sum has at most 2^en such terms of weight <= 1, so with
// e = 61 - ceil(log2 K) - en no partial sum leaves the int64 range.
__global__ void __launch_bounds__(256)
bwd_scale(uint32_t* __restrict__ sc, synthpix_advect_params ap, int en, const double* __restrict__ sheet_part,
          const float* __restrict__ bound_part, int n_pairs, int ns, float* __restrict__ g_sheet,
          float* __restrict__ g_sheet_total)
{
    // per-pair sheet-width gradient: the slices' float64 sums in slice order; each
    // thread takes a contiguous run of pairs, and the shared-sheet total adds
    // the runs' float64 sums in a fixed tree, so it too is reproducible
    __shared__ double s_tot[256];
    const int per = (n_pairs + 255) / 256;
    const int pa = (int)threadIdx.x * per, pb = min(n_pairs, pa + per);
    double run = 0.0;
    for (int p = pa; p < pb; ++p) {
        double t = 0.0;
        // unrolled so that the loads are issued together; the additions stay in slice order
#pragma unroll 16
        for (int k = 0; k < ns; ++k) t += sheet_part[(int64_t)p * ns + k];
        g_sheet[p] = (float)t;
        run += t;
    }
    s_tot[threadIdx.x] = run;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) s_tot[threadIdx.x] += s_tot[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && g_sheet_total) *g_sheet_total = (float)s_tot[0];
    // maxima over all (pair, slice) blocks
    float gm = 0.0f, lm = 0.0f;
    for (int64_t k = threadIdx.x; k < (int64_t)n_pairs * ns; k += blockDim.x) {
        gm = __builtin_fmaxf(gm, bound_part[2 * k]);
        lm = __builtin_fmaxf(lm, bound_part[2 * k + 1]);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        gm = __builtin_fmaxf(gm, __shfl_xor(gm, o, 64));
        lm = __builtin_fmaxf(lm, __shfl_xor(lm, o, 64));
    }
    __shared__ float red[2][4];
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = gm;
        red[1][threadIdx.x >> 6] = lm;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double G0 = (double)__builtin_fmaxf(__builtin_fmaxf(red[0][0], red[0][1]),
                                              __builtin_fmaxf(red[0][2], red[0][3]));
    const double L = (double)__builtin_fmaxf(__builtin_fmaxf(red[1][0], red[1][1]),
                                             __builtin_fmaxf(red[1][2], red[1][3]));
    sc[SC_G2MAX] = __float_as_uint((float)G0);
    sc[SC_LIP] = __float_as_uint((float)L);
    const int S = ap.substeps;
    const double h = __builtin_fabs((double)ap.dt / (double)S);
    double kfac, growth;
    if (ap.integrator == SP_EULER) {
        kfac = h;
        growth = 1.0 + h * L;
    } else {
        const double c = h / 6.0;
        const double k4 = c, k3 = 2.0 * c + h * L * k4, k2 = 2.0 * c + 0.5 * h * L * k3, k1 = c + 0.5 * h * L * k2;
        kfac = __builtin_fmax(__builtin_fmax(k1, k2), __builtin_fmax(k3, k4));
        growth = 1.0 + L * (k1 + k2 + k3 + k4);
    }
    const double K = G0 * kfac * pow(growth, (double)(S - 1)) * 1.0009765625;
    uint32_t state = SC_VALID;
    int e = 0;
    if (!(G0 > 0.0) || !(h > 0.0)) {
        state = SC_NONE;
    } else if (!__builtin_isfinite(K) || !(K > 0.0)) {
        state = SC_NONFINITE;
    } else {
        int k;
        (void)__builtin_frexp(K, &k);   // K < 2^k
        e = 61 - k - en;
    }
    sc[SC_EXP] = (uint32_t)e;
    sc[SC_STATE] = state;
}

// Status, scale block and sheet outputs cleared; the flow gradient zeroed (its
// pairs' grids are overwritten by the reduction, gaps between them stay 0).
__global__ void bwd_init(float* __restrict__ g_flow, int64_t n, uint32_t* __restrict__ status,
                         uint32_t* __restrict__ sc, float* __restrict__ g_sheet, int n_pairs,
                         float* __restrict__ g_sheet_total, const synthpix_pair* __restrict__ pairs,
                         int64_t* __restrict__ wg_base)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 4) {
        status[t] = 0u;
        sc[t] = 0u;
    }
    if (blockIdx.x == 0) {
        // workgroups of the flow adjoint, each pair's particles in chunks of 256:
        // an exclusive prefix over the pairs, 256 at a time (wave scans, then
        // the four wave totals)
        __shared__ int64_t s_tot[4];
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        int64_t carry = 0;
        for (int b = 0; b < n_pairs; b += 256) {
            const int p = b + (int)threadIdx.x;
            const int64_t v = p < n_pairs ? (pairs[p].n_max + 255) / 256 : 0;
            int64_t inc = v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int64_t u = __shfl_up(inc, o, 64);
                if (lane >= o) inc += u;
            }
            if (lane == 63) s_tot[wid] = inc;
            __syncthreads();
            int64_t before = 0, total = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                if (w < wid) before += s_tot[w];
                total += s_tot[w];
            }
            if (p < n_pairs) wg_base[p] = carry + before + inc - v;
            carry += total;
            __syncthreads();
        }
        if (threadIdx.x == 0) wg_base[n_pairs] = carry;
    }
    // sheet gradients of a batch without particles (otherwise overwritten later)
    if (t < n_pairs) g_sheet[t] = 0.0f;
    if (t == 0 && g_sheet_total) *g_sheet_total = 0.0f;
    for (int64_t k = t; k < n; k += (int64_t)gridDim.x * blockDim.x) g_flow[k] = 0.0f;
}


// ------------------------------------------------------------------ image loss

// grad = scale (J - T) over float4 groups, grid-stride in a fixed grid of
// MSE_BLOCKS workgroups; with loss partials, each workgroup's float64 sum of
// (J - T)^2 (each thread's terms in index order, then a fixed tree) goes to
// part[block].  The last n % 4 elements are workgroup 0's.
__global__ void __launch_bounds__(256)
mse_grad_kernel(const float* __restrict__ J, const float* __restrict__ T, int64_t n, float scale,
                float* __restrict__ grad, double* __restrict__ part)
{
    const int64_t n4 = n >> 2;
    const float4* J4 = reinterpret_cast<const float4*>(J);
    const float4* T4 = reinterpret_cast<const float4*>(T);
    float4* G4 = reinterpret_cast<float4*>(grad);
    double acc = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n4; k += (int64_t)gridDim.x * 256) {
        const float4 j = J4[k], t = T4[k];
        const float4 d = make_float4(j.x - t.x, j.y - t.y, j.z - t.z, j.w - t.w);
        G4[k] = make_float4(scale * d.x, scale * d.y, scale * d.z, scale * d.w);
        if (part) {     // the differences exactly, in float64
            const double ex = (double)j.x - (double)t.x, ey = (double)j.y - (double)t.y;
            const double ez = (double)j.z - (double)t.z, ew = (double)j.w - (double)t.w;
            acc = __builtin_fma(ex, ex, acc);
            acc = __builtin_fma(ey, ey, acc);
            acc = __builtin_fma(ez, ez, acc);
            acc = __builtin_fma(ew, ew, acc);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < (n & 3)) {
        const int64_t i = 4 * n4 + threadIdx.x;
        const float j = J[i], t = T[i];          // read before the write: grad may be J or T
        grad[i] = scale * (j - t);
        if (part) {
            const double e = (double)j - (double)t;
            acc = __builtin_fma(e, e, acc);
        }
    }
    if (!part) return;
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// loss = (sum of the MSE_BLOCKS partials, as a fixed tree) / n
__global__ void __launch_bounds__(256)
mse_finish(const double* __restrict__ part, int64_t n_part, int64_t n, double* __restrict__ loss)
{
    __shared__ double red[256];
    double v = 0.0;
    for (int64_t k = threadIdx.x; k < n_part; k += 256) v += part[k];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = n > 0 ? red[0] / (double)n : 0.0;
}

hipError_t launch_mse_grad(const float* J, const float* T, int64_t n, float scale, float* grad, double* loss,
                           double* part, hipStream_t s)
{
    TimedScope ts("mse_grad", s);
    const int64_t want = (n / 4 + 255) / 256;
    const unsigned grid = loss ? (unsigned)MSE_BLOCKS : (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, MSE_BLOCKS));
    hipLaunchKernelGGL(mse_grad_kernel, dim3(grid), dim3(256), 0, s, J, T, n, scale, grad, loss ? part : nullptr);
    if (loss) hipLaunchKernelGGL(mse_finish, dim3(1), dim3(256), 0, s, part, (int64_t)MSE_BLOCKS, n, loss);
    return hipGetLastError();
}

// Workgroups of the per-pixel blur adjoint: (pair, frame, strip row, strip
// column) over the batch's largest pair.
int64_t blur_grad_blocks(int n_pairs, int max_w, int max_h, bool mse)
{
    const int sh = blur_strip_rows(mse);
    return (int64_t)n_pairs * 2 * ((max_w + 255) / 256) * ((max_h + sh - 1) / sh);
}

// Workgroups of the particle-major gather: 256 / G particles each.
static unsigned gather_blocks(int64_t n_span, int G)
{
    return (unsigned)((n_span + 256 / G - 1) / (256 / G));
}

void launch_advect_adjoint(const BwdArgs& a, const synthpix_advect_params& ap, unsigned blocks, hipStream_t s)
{
    const int S = ap.substeps;
#define SP_ADJ(CK, SK) hipLaunchKernelGGL((bwd_advect<CK, SK>), dim3(blocks), dim3(256), 0, s, a, ap)
    if (S <= 1) SP_ADJ(1, 1);
    else if (S <= 2) SP_ADJ(2, 1);
    else if (S <= 4) SP_ADJ(4, 1);
    else if (S <= 8) SP_ADJ(8, 1);
    else if (S <= 16) SP_ADJ(16, 1);
    else if (S <= 32) SP_ADJ(32, 1);
    else SP_ADJ(32, 32);       // substeps <= 1024 = 32 * 32
#undef SP_ADJ
}

hipError_t launch_backward(const BwdArgs& a, int64_t n_span, int64_t n_flow, const synthpix_advect_params& ap,
                           int blur, int en, hipStream_t s)
{
    {
        TimedScope ts("bwd_init", s);
        const int64_t blocks = std::min<int64_t>(std::max<int64_t>((n_flow + 255) / 256 + 1, (a.n_pairs + 255) / 256),
                                                 65536);
        hipLaunchKernelGGL(bwd_init, dim3((unsigned)blocks), dim3(256), 0, s, a.g_flow, n_flow, a.status, a.scale,
                           a.g_sheet, a.n_pairs, a.g_sheet_total, a.pairs, a.grid.wg_base);
    }
    if (a.mse && !a.eblur) return hipErrorInvalidValue;
    const bool tile = a.order2.entries && a.parts;
    // the blur's adjoint once per pixel (the gather then runs on the unblurred
    // footprints of B^T dL/dJ): for wide blurs and the tile gather, and always
    // for the loss-fused form, whose pass also forms dL/dJ (and the loss, which
    // the images define even when no pair holds a particle)
    const bool per_pixel = a.eblur && (a.mse || (blur >= 1 && (tile || blur >= 2)));
    if (per_pixel && (n_span > 0 || (a.mse && a.loss))) {
        TimedScope ts("bwd_blur", s);
        const int64_t nb = blur_grad_blocks(a.n_pairs, a.max_w, a.max_h, a.mse);
        if (nb < 1 || nb > 0xFFFFFFFFll) return hipErrorInvalidValue;
        const int sh = blur_strip_rows(a.mse);
        const int nsx = (a.max_w + 255) / 256, nsy = (a.max_h + sh - 1) / sh;
#define SP_BLUR(BB)                                                                                             \
    case BB:                                                                                                    \
        if (a.mse) hipLaunchKernelGGL((bwd_blur_grad<BB, true>), dim3((unsigned)nb), dim3(256), 0, s, a, nsx, nsy); \
        else hipLaunchKernelGGL((bwd_blur_grad<BB, false>), dim3((unsigned)nb), dim3(256), 0, s, a, nsx, nsy);     \
        break;
        switch (blur) {
        SP_BLUR(0) SP_BLUR(1) SP_BLUR(2) SP_BLUR(3)
        default: return hipErrorInvalidValue;
        }
#undef SP_BLUR
        if (a.mse && a.loss)
            hipLaunchKernelGGL(mse_finish, dim3(1), dim3(256), 0, s, a.loss_part, nb, a.loss_n, a.loss);
    }
    if (n_span > 0) {
        if (a.recompute_x2) {
            const hipError_t e = launch_advect(a.pairs, a.n_pairs, n_span, a.flow, ap, a.x1, a.y1, a.x2w, a.y2w, s,
                                               a.order);
            if (e != hipSuccess) return e;
        }
        BwdArgs b = a;
        if (per_pixel) b.grad = a.eblur;
        if (tile) {
            TimedScope ts("bwd_gather", s);
            const int hb = tile_halo(a.d_max);
            const int rw = (1 << a.order.log_block) + 2 * hb;
            const int64_t items = 2 * a.order.blocks;
            if (items > 0xFFFFFFFFll) return hipErrorInvalidValue;
            // the region's row stride rounded up to one of the compiled ones
            const int rs = rw <= 40 ? 40 : rw <= 48 ? 48 : rw <= 56 ? 56 : rw <= 64 ? 64 : rw;
            const size_t lds = sizeof(float) * (size_t)rs * rw;
#define SP_TILE(RS_) hipLaunchKernelGGL(bwd_tile_gather<RS_>, dim3((unsigned)items), dim3(256), lds, s, b, n_span, \
                                        a.order.log_block, hb)
            switch (rs) {
            case 40: SP_TILE(40); break;
            case 48: SP_TILE(48); break;
            case 56: SP_TILE(56); break;
            case 64: SP_TILE(64); break;
            default: SP_TILE(0); break;
            }
#undef SP_TILE
            hipLaunchKernelGGL(bwd_particles, dim3((unsigned)((n_span + 255) / 256)), dim3(256), 0, s, b, n_span);
        } else if (per_pixel) {
            TimedScope ts("bwd_gather", s);
            if ((int)(3.0f * a.d_max) + 4 <= 32) hipLaunchKernelGGL((bwd_gather<0, 32, 8>), dim3(gather_blocks(n_span, 8)), dim3(256), 0, s, b, n_span);
            else hipLaunchKernelGGL((bwd_gather<0, 64, 16>), dim3(gather_blocks(n_span, 16)), dim3(256), 0, s, b, n_span);
        } else {
            TimedScope ts("bwd_gather", s);
            // slots needed: floor(3 d_max) + 4 covered pixels + 4 b padding
            const bool small = (int)(3.0f * a.d_max) + 4 + 4 * blur <= 32;
#define SP_GATHER(BB)                                                                  \
    do {                                                                               \
        if (small) hipLaunchKernelGGL((bwd_gather<BB, 32, 8>), dim3(gather_blocks(n_span, 8)), dim3(256), 0, s, a, n_span); \
        else hipLaunchKernelGGL((bwd_gather<BB, 64, 16>), dim3(gather_blocks(n_span, 16)), dim3(256), 0, s, a, n_span);       \
    } while (0)
            switch (blur) {
            case 0: SP_GATHER(0); break;
            case 1: SP_GATHER(1); break;
            default: return hipErrorInvalidValue;
            }
#undef SP_GATHER
        }
        {
            TimedScope ts("bwd_bounds", s);
            // about 768 particles per slice (3 per thread), at least 32 slices per
            // pair: enough workgroups to keep the loads of every CU in flight
            const int64_t per = (n_span + (int64_t)a.n_pairs * 768 - 1) / ((int64_t)a.n_pairs * 768);
            const int ns = (int)std::min<int64_t>(std::max<int64_t>(per, 32), BWD_SLICES);
            hipLaunchKernelGGL(bwd_bounds, dim3((unsigned)a.n_pairs, ns), dim3(256), 0, s, a, ns);
            hipLaunchKernelGGL(bwd_scale, dim3(1), dim3(256), 0, s, a.scale, ap, en, a.sheet_part, a.bound_part,
                               a.n_pairs, ns, a.g_sheet, a.g_sheet_total);
        }
        if (a.grid.n_wg > 0) {
            TimedScope ts("bwd_advect", s);
            if (a.grid.n_wg > 0xFFFFFFFFll) return hipErrorInvalidValue;
            launch_advect_adjoint(a, ap, (unsigned)a.grid.n_wg, s);
        }
        {
            TimedScope ts("bwd_flow", s);
            const int ntx = (a.grid.max_gw + GRID_TILE - 1) / GRID_TILE, nty = (a.grid.max_gh + GRID_TILE - 1) / GRID_TILE;
            const int64_t nb = (int64_t)a.n_pairs * ntx * nty;
            if (nb > 0xFFFFFFFFll) return hipErrorInvalidValue;
            if (nb > 0) hipLaunchKernelGGL(bwd_grid_reduce, dim3((unsigned)nb), dim3(256), 0, s, a, ntx, nty);
        }
    }
    return hipGetLastError();
}

}  // namespace sp
