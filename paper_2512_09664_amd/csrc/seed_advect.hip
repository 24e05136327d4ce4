// Particle seeding and inter-frame advection kernels (gfx950).
//
// Seeding follows Section 2, "Sampling the particles": n_max candidates per
// pair drawn over the image, the pair's ppp drawn uniformly, particles past
// n_active masked with zero intensity; per-particle parameters uniform in
// their ranges (the paragraph after Eq. 1), the diameter optionally a clipped
// normal.  Advection implements the same passage's x -> x + u(x), generalised to
// dt with Euler or RK4 substeps on a bilinear, cell-centred flow grid.
//
// One thread per particle; SoA float stores are fully coalesced.  Both kernels
// are bound by Philox / interpolation arithmetic, not by memory.
#include "device_math.hpp"
#include "flow.hpp"
#include "launch.hpp"

namespace sp {

// The pair's drawn ppp and active-particle count (Philox stream 5, index 0).
__device__ __forceinline__ int pair_active(const synthpix_pair& P, uint64_t pid, const synthpix_seed_params& prm,
                                           uint64_t seed, double* ppp_out)
{
    const u32x4 w = draw(0u, STREAM_PAIR, pid, seed);
    const double ppp = prm.ppp_lo + (prm.ppp_hi - prm.ppp_lo) * (double)u24(w.a);
    const double na = floor((double)P.H * (double)P.W * ppp + 0.5);
    *ppp_out = ppp;
    return na < (double)P.n_max ? (int)na : P.n_max;
}

__global__ void __launch_bounds__(256)
pair_scalars_kernel(const synthpix_pair* __restrict__ pairs, int n_pairs, synthpix_seed_params prm,
                    uint64_t seed, int32_t* __restrict__ n_active_out, double* __restrict__ ppp_out,
                    const synthpix_batch_io* __restrict__ iod, int32_t* __restrict__ live_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_pairs) return;
    uint64_t base = 0;
    if (iod) {
        seed = iod->seed;
        base = iod->pair_id_base;
        n_active_out = iod->n_active;
        ppp_out = iod->ppp;
    }
    double ppp;
    const int na = pair_active(pairs[p], pairs[p].pair_id + base, prm, seed, &ppp);
    if (n_active_out) n_active_out[p] = na;
    if (ppp_out) ppp_out[p] = ppp;
    if (live_out) live_out[p] = na;
}

__global__ void __launch_bounds__(256)
seed_kernel(const synthpix_pair* __restrict__ pairs, int n_pairs, int64_t n_span,
            synthpix_seed_params prm, uint64_t seed,
            float* __restrict__ x, float* __restrict__ y, float* __restrict__ z,
            float* __restrict__ d, float* __restrict__ I0, const synthpix_batch_io* __restrict__ iod,
            bool masked_still)
{
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t g = g0 + threadIdx.x;
    if (g >= n_span) return;
    const int p = find_pair_from(pairs, n_pairs, g0, g);
    const synthpix_pair P = pairs[p];
    const int64_t i64 = g - P.particle_offset;
    if (i64 < 0 || i64 >= P.n_max) return;
    const uint32_t i = (uint32_t)i64;
    uint64_t pid = P.pair_id;
    if (iod) {
        x = iod->x1;
        y = iod->y1;
        z = iod->z;
        d = iod->d;
        I0 = iod->I0;
        seed = iod->seed;
        pid += iod->pair_id_base;
    }

    double ppp;
    const int n_active = pair_active(P, pid, prm, seed, &ppp);

    const u32x4 gw = draw(i, STREAM_GEOM, pid, seed);
    const u32x4 hw = draw(i, STREAM_PHOTO, pid, seed);
    const float px = u24(gw.a) * (float)P.W, py = u24(gw.b) * (float)P.H;
    x[g] = px;
    y[g] = py;
    if (masked_still && (int)i >= n_active) {
        // a masked candidate is not advected: its frame-2 position is its frame-1 one
        iod->x2[g] = px;
        iod->y2[g] = py;
    }
    z[g] = __builtin_fmaf(prm.z_hi - prm.z_lo, u24(gw.c), prm.z_lo);
    float dv;
    if (prm.d_dist == SP_DIST_UNIFORM) {
        dv = __builtin_fmaf(prm.d_b - prm.d_a, u24(gw.d), prm.d_a);
    } else {
        const float l = log_ra(u24_open0(hw.b));
        const float R = __builtin_sqrtf(-2.0f * l);
        const float n = R * cos2pi_ra(u24(hw.c));
        float v = __builtin_fmaf(prm.d_b, n, prm.d_a);
        v = __builtin_fmaxf(v, prm.d_lo);
        dv = __builtin_fminf(v, prm.d_hi);
    }
    d[g] = dv;
    I0[g] = ((int)i < n_active) ? __builtin_fmaf(prm.I0_hi - prm.I0_lo, u24(hw.a), prm.I0_lo) : 0.0f;
}

// Bilinear sample of the pair's (u, v) grid at image position (px, py).
// One frozen-field substep sequence; the update order is fixed (see the
// reference arithmetic): Euler p = fma(h, u, p); RK4 stages at fma(h/2, k, p)
// and fma(h, k3, p), update p = fma(h, (((k1 + 2 k2) + 2 k3) + k4) / 6, p).
__device__ __forceinline__ float2 integrate(const FlowView& fv, float px, float py, float dt,
                                            int substeps, int integrator)
{
    const float h = dt / (float)substeps;
    const float hh = h * 0.5f;
    for (int s = 0; s < substeps; ++s) {
        if (integrator == SP_EULER) {
            const float2 u = sample_flow(fv, px, py);
            px = __builtin_fmaf(h, u.x, px);
            py = __builtin_fmaf(h, u.y, py);
        } else {
            const float2 k1 = sample_flow(fv, px, py);
            const float2 k2 = sample_flow(fv, __builtin_fmaf(hh, k1.x, px), __builtin_fmaf(hh, k1.y, py));
            const float2 k3 = sample_flow(fv, __builtin_fmaf(hh, k2.x, px), __builtin_fmaf(hh, k2.y, py));
            const float2 k4 = sample_flow(fv, __builtin_fmaf(h, k3.x, px), __builtin_fmaf(h, k3.y, py));
            const float su = ((k1.x + 2.0f * k2.x) + 2.0f * k3.x) + k4.x;
            const float sv = ((k1.y + 2.0f * k2.y) + 2.0f * k3.y) + k4.y;
            px = __builtin_fmaf(h, su / 6.0f, px);
            py = __builtin_fmaf(h, sv / 6.0f, py);
        }
    }
    return make_float2(px, py);
}

// N particles per thread, integrated in lockstep: each substep's bilinear
// samples are chains of dependent L2 reads, so independent particles in one
// thread overlap those latencies.
template <int N>
__device__ __forceinline__ void integrate_n(const FlowView* fv, float* px, float* py, float dt, int substeps,
                                            int integrator, const FlowWin* win, lds_float* lds)
{
    const float h = dt / (float)substeps;
    const float hh = h * 0.5f;
    for (int s = 0; s < substeps; ++s) {
        if (integrator == SP_EULER) {
            float2 u[N];
#pragma unroll
            for (int q = 0; q < N; ++q) u[q] = sample_flow(fv[q], px[q], py[q], win[q], lds);
#pragma unroll
            for (int q = 0; q < N; ++q) {
                px[q] = __builtin_fmaf(h, u[q].x, px[q]);
                py[q] = __builtin_fmaf(h, u[q].y, py[q]);
            }
        } else {
            float2 k1[N], k2[N], k3[N], k4[N];
#pragma unroll
            for (int q = 0; q < N; ++q) k1[q] = sample_flow(fv[q], px[q], py[q], win[q], lds);
#pragma unroll
            for (int q = 0; q < N; ++q)
                k2[q] = sample_flow(fv[q], __builtin_fmaf(hh, k1[q].x, px[q]), __builtin_fmaf(hh, k1[q].y, py[q]),
                                    win[q], lds);
#pragma unroll
            for (int q = 0; q < N; ++q)
                k3[q] = sample_flow(fv[q], __builtin_fmaf(hh, k2[q].x, px[q]), __builtin_fmaf(hh, k2[q].y, py[q]),
                                    win[q], lds);
#pragma unroll
            for (int q = 0; q < N; ++q)
                k4[q] = sample_flow(fv[q], __builtin_fmaf(h, k3[q].x, px[q]), __builtin_fmaf(h, k3[q].y, py[q]),
                                    win[q], lds);
#pragma unroll
            for (int q = 0; q < N; ++q) {
                const float su = ((k1[q].x + 2.0f * k2[q].x) + 2.0f * k3[q].x) + k4[q].x;
                const float sv = ((k1[q].y + 2.0f * k2[q].y) + 2.0f * k3[q].y) + k4[q].y;
                px[q] = __builtin_fmaf(h, su / 6.0f, px[q]);
                py[q] = __builtin_fmaf(h, sv / 6.0f, py[q]);
            }
        }
    }
}

constexpr int ADVECT_ILP = 1;
constexpr int ADVECT_WIN_NODES = 2048;   // LDS window of grid nodes (16 KB)
constexpr int ADVECT_WIN_MARGIN = 4;     // cells added around the starting cells

// SORTED: thread slots follow the home-block order (neighbouring lanes sample
// neighbouring grid cells, so the bilinear gathers share cache lines); each
// slot reads its particle index from the order's entry list.
template <bool SORTED>
__global__ void __launch_bounds__(256)
advect_kernel(const synthpix_pair* __restrict__ pairs, int n_pairs, int64_t n_span,
              const float* __restrict__ flow, synthpix_advect_params ap,
              const float* __restrict__ x1, const float* __restrict__ y1,
              float* __restrict__ x2, float* __restrict__ y2, AdvectOrder order,
              const synthpix_batch_io* __restrict__ iod)
{
    if (iod) {
        flow = iod->flow;
        x1 = iod->x1;
        y1 = iod->y1;
        x2 = iod->x2;
        y2 = iod->y2;
    }
    // consecutive particle blocks (same pair, same flow grid) stay on one XCD
    const int64_t g0 = (int64_t)xcd_contiguous(blockIdx.x, gridDim.x) * (256 * ADVECT_ILP);
    const int64_t base = g0 + threadIdx.x;
    FlowView fv[ADVECT_ILP];
    float px[ADVECT_ILP], py[ADVECT_ILP];
    int64_t gi[ADVECT_ILP];
#pragma unroll
    for (int q = 0; q < ADVECT_ILP; ++q) {
        const int64_t g = base + 256 * q;
        gi[q] = -1;
        px[q] = py[q] = 0.0f;
        fv[q] = FlowView{reinterpret_cast<const float2*>(flow), 2, 2, 1.0f, 1.0f};
        if (g < n_span) {
            const int p = find_pair_from(pairs, n_pairs, g0, g);
            const synthpix_pair P = pairs[p];
            const int64_t i = g - P.particle_offset;
            if (i >= 0 && i < (order.live ? (int64_t)order.live[p] : (int64_t)P.n_max)) {
                gi[q] = SORTED ? P.particle_offset + order.entries[order.L[p].entry_base + i] : g;
                fv[q] = flow_view(P, flow);
                px[q] = x1[gi[q]];
                py[q] = y1[gi[q]];
            }
        }
    }
    // SORTED: the workgroup's particles start in a compact patch of the image;
    // the grid nodes around their starting cells (those of the first slot's
    // pair, grown by a margin) are copied to LDS when they fit
    __shared__ float2 s_win[ADVECT_WIN_NODES];
    __shared__ int s_box[4][4];
    __shared__ int s_pair;
    FlowWin win[ADVECT_ILP];
#pragma unroll
    for (int q = 0; q < ADVECT_ILP; ++q) win[q] = NO_WIN;
    if (SORTED) {
        if (threadIdx.x == 0) s_pair = gi[0] >= 0 ? find_pair_from(pairs, n_pairs, g0, g0) : -1;
        __syncthreads();
        const int sp_ = s_pair;
        int bi0 = 1 << 30, bj0 = 1 << 30, bi1 = -1, bj1 = -1;
        bool mine[ADVECT_ILP];
#pragma unroll
        for (int q = 0; q < ADVECT_ILP; ++q) {
            mine[q] = gi[q] >= 0 && sp_ >= 0 && fv[q].F == flow_view(pairs[sp_], flow).F;
            if (mine[q]) {
                const float gx = __builtin_fminf(__builtin_fmaxf(px[q] * fv[q].sx - 0.5f, 0.0f), (float)(fv[q].Gw - 1));
                const float gy = __builtin_fminf(__builtin_fmaxf(py[q] * fv[q].sy - 0.5f, 0.0f), (float)(fv[q].Gh - 1));
                bj0 = min(bj0, (int)gx);
                bj1 = max(bj1, (int)gx);
                bi0 = min(bi0, (int)gy);
                bi1 = max(bi1, (int)gy);
            }
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
        __syncthreads();
        if (sp_ >= 0) {
            const synthpix_pair Q = pairs[sp_];
            bi0 = max(min(min(s_box[0][0], s_box[1][0]), min(s_box[2][0], s_box[3][0])) - ADVECT_WIN_MARGIN, 0);
            bj0 = max(min(min(s_box[0][1], s_box[1][1]), min(s_box[2][1], s_box[3][1])) - ADVECT_WIN_MARGIN, 0);
            bi1 = min(max(max(s_box[0][2], s_box[1][2]), max(s_box[2][2], s_box[3][2])) + ADVECT_WIN_MARGIN + 1,
                      Q.Gh - 1);
            bj1 = min(max(max(s_box[0][3], s_box[1][3]), max(s_box[2][3], s_box[3][3])) + ADVECT_WIN_MARGIN + 1,
                      Q.Gw - 1);
            const int wh = bi1 - bi0 + 1, ww = bj1 - bj0 + 1;
            if (bi1 >= bi0 && bj1 >= bj0 && wh * ww <= ADVECT_WIN_NODES) {
                const float2* F = reinterpret_cast<const float2*>(flow + Q.flow_offset);
                // window row of node k without an integer division: (k + 1/2) / ww lies at
                // least 1/(2 ww) from an integer and, for k < 2048, the float product errs
                // by under 2048 * 2^-21 / ww, so truncation gives floor(k / ww)
                const float inv_ww = 1.0f / (float)ww;
                for (int k = threadIdx.x; k < wh * ww; k += 256) {
                    const int r = (int)(((float)k + 0.5f) * inv_ww);
                    s_win[k] = F[(int64_t)(bi0 + r) * Q.Gw + bj0 + (k - r * ww)];
                }
#pragma unroll
                for (int q = 0; q < ADVECT_ILP; ++q)
                    if (mine[q]) win[q] = FlowWin{bi0, bj0, wh, ww};
            }
        }
        __syncthreads();
    }
    // a wave none of whose slots holds a particle to move (slots past every
    // pair's range or, with live counts, masked candidates) skips the steps
    bool any = false;
#pragma unroll
    for (int q = 0; q < ADVECT_ILP; ++q) any = any || gi[q] >= 0;
    if (__builtin_amdgcn_ballot_w64(any) != 0)
        integrate_n<ADVECT_ILP>(fv, px, py, ap.dt, ap.substeps, ap.integrator, win, (lds_float*)s_win);
#pragma unroll
    for (int q = 0; q < ADVECT_ILP; ++q) {
        if (gi[q] >= 0) {
            x2[gi[q]] = px[q];
            y2[gi[q]] = py[q];
        }
    }
}

// Second diameter d_y and correlation rho of Eq. 1 per candidate particle
// (anisotropic particle images; the sentence after Eq. 1 draws every shape
// parameter per particle): d_y from the seed's diameter distribution, rho
// uniform in [rho_lo, rho_hi]; Philox stream 6 (word 0: uniform d_y; words 1, 2:
// Box-Muller of a normal d_y; word 3: rho).
__global__ void __launch_bounds__(256)
seed_shape_kernel(const synthpix_pair* __restrict__ pairs, int n_pairs, int64_t n_span, synthpix_seed_params prm,
                  float rho_lo, float rho_hi, uint64_t seed, float* __restrict__ dy, float* __restrict__ rho)
{
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t g = g0 + threadIdx.x;
    if (g >= n_span) return;
    const int p = find_pair_from(pairs, n_pairs, g0, g);
    const synthpix_pair P = pairs[p];
    const int64_t i64 = g - P.particle_offset;
    if (i64 < 0 || i64 >= P.n_max) return;
    const u32x4 w = draw((uint32_t)i64, STREAM_SHAPE, P.pair_id, seed);
    float v;
    if (prm.d_dist == SP_DIST_UNIFORM) {
        v = __builtin_fmaf(prm.d_b - prm.d_a, u24(w.a), prm.d_a);
    } else {
        const float R = __builtin_sqrtf(-2.0f * log_ra(u24_open0(w.b)));
        v = __builtin_fmaf(prm.d_b, R * cos2pi_ra(u24(w.c)), prm.d_a);
        v = __builtin_fminf(__builtin_fmaxf(v, prm.d_lo), prm.d_hi);
    }
    dy[g] = v;
    rho[g] = __builtin_fmaf(rho_hi - rho_lo, u24(w.d), rho_lo);
}

// Bilinear, clamped sample of a pair's scalar grid (the out-of-plane velocity w,
// one float per node, registered like the (u, v) grid).
__device__ __forceinline__ float sample_scalar(const float* __restrict__ G, const FlowView& fv, float px, float py)
{
    float gx = px * fv.sx - 0.5f;
    float gy = py * fv.sy - 0.5f;
    gx = __builtin_fminf(__builtin_fmaxf(gx, 0.0f), (float)(fv.Gw - 1));
    gy = __builtin_fminf(__builtin_fmaxf(gy, 0.0f), (float)(fv.Gh - 1));
    int j0 = (int)__builtin_floorf(gx);
    int i0 = (int)__builtin_floorf(gy);
    j0 = j0 > fv.Gw - 2 ? fv.Gw - 2 : j0;
    i0 = i0 > fv.Gh - 2 ? fv.Gh - 2 : i0;
    const float fx = gx - (float)j0;
    const float fy = gy - (float)i0;
    const float* a = G + (size_t)i0 * fv.Gw + j0;
    const float* c = a + fv.Gw;
    const float top = __builtin_fmaf(fx, a[1] - a[0], a[0]);
    const float bot = __builtin_fmaf(fx, c[1] - c[0], c[0]);
    return __builtin_fmaf(fy, bot - top, top);
}

// Three-dimensional motion (Remark 1's particles in 3-D space under a 3-D
// flow): the in-plane trajectory of advect_kernel, and z integrating the
// out-of-plane velocity w(x, y) with the same stages (Euler z = fma(h, w, z);
// RK4 z = fma(h, (((w1 + 2 w2) + 2 w3) + w4) / 6, z), w_k at the k-th stage
// position).  One particle per thread in index order.
__global__ void __launch_bounds__(256)
advect3_kernel(const synthpix_pair* __restrict__ pairs, int n_pairs, int64_t n_span, const float* __restrict__ flow,
               const float* __restrict__ wflow, synthpix_advect_params ap, const float* __restrict__ x1,
               const float* __restrict__ y1, const float* __restrict__ z1, float* __restrict__ x2,
               float* __restrict__ y2, float* __restrict__ z2)
{
    const int64_t g0 = (int64_t)xcd_contiguous(blockIdx.x, gridDim.x) * 256;
    const int64_t g = g0 + threadIdx.x;
    if (g >= n_span) return;
    const int p = find_pair_from(pairs, n_pairs, g0, g);
    const synthpix_pair P = pairs[p];
    const int64_t i = g - P.particle_offset;
    if (i < 0 || i >= P.n_max) return;
    const FlowView fv = flow_view(P, flow);
    const float* W = wflow + P.flow_offset / 2;
    float px = x1[g], py = y1[g], pz = z1[g];
    const float h = ap.dt / (float)ap.substeps;
    const float hh = h * 0.5f;
    for (int s = 0; s < ap.substeps; ++s) {
        if (ap.integrator == SP_EULER) {
            const float2 u = sample_flow(fv, px, py);
            const float w = sample_scalar(W, fv, px, py);
            px = __builtin_fmaf(h, u.x, px);
            py = __builtin_fmaf(h, u.y, py);
            pz = __builtin_fmaf(h, w, pz);
        } else {
            const float2 k1 = sample_flow(fv, px, py);
            const float w1 = sample_scalar(W, fv, px, py);
            const float ax = __builtin_fmaf(hh, k1.x, px), ay = __builtin_fmaf(hh, k1.y, py);
            const float2 k2 = sample_flow(fv, ax, ay);
            const float w2 = sample_scalar(W, fv, ax, ay);
            const float bx = __builtin_fmaf(hh, k2.x, px), by = __builtin_fmaf(hh, k2.y, py);
            const float2 k3 = sample_flow(fv, bx, by);
            const float w3 = sample_scalar(W, fv, bx, by);
            const float cx = __builtin_fmaf(h, k3.x, px), cy = __builtin_fmaf(h, k3.y, py);
            const float2 k4 = sample_flow(fv, cx, cy);
            const float w4 = sample_scalar(W, fv, cx, cy);
            const float su = ((k1.x + 2.0f * k2.x) + 2.0f * k3.x) + k4.x;
            const float sv = ((k1.y + 2.0f * k2.y) + 2.0f * k3.y) + k4.y;
            const float sw = ((w1 + 2.0f * w2) + 2.0f * w3) + w4;
            px = __builtin_fmaf(h, su / 6.0f, px);
            py = __builtin_fmaf(h, sv / 6.0f, py);
            pz = __builtin_fmaf(h, sw / 6.0f, pz);
        }
    }
    x2[g] = px;
    y2[g] = py;
    z2[g] = pz;
}

// Ground-truth flow of each pair (the sampler's flow_fields): the pair's (u, v)
// grid sampled bilinearly at every pixel centre, (c + 1/2, r + 1/2), exactly
// as the advection samples it; written as [H][W][2] floats at the pair's image
// offset (2 H W floats, the extent of its two float frames).  One thread per
// pixel; grid y = pair.
__global__ void __launch_bounds__(256)
flow_field_kernel(const synthpix_pair* __restrict__ pairs, const float* __restrict__ flow, float* __restrict__ out)
{
    const synthpix_pair P = pairs[blockIdx.y];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)P.H * P.W) return;
    const int r = (int)(k / P.W), c = (int)(k - (int64_t)r * P.W);
    const float2 u = sample_flow(flow_view(P, flow), (float)c + 0.5f, (float)r + 0.5f);
    *reinterpret_cast<float2*>(out + P.image_offset + 2 * k) = u;
}

hipError_t launch_flow_field(const synthpix_pair* pairs_dev, int n_pairs, int64_t max_px, const float* flow, float* out,
                             hipStream_t s)
{
    if (max_px <= 0) return hipSuccess;
    TimedScope ts("flow_field", s);
    hipLaunchKernelGGL(flow_field_kernel, dim3((unsigned)((max_px + 255) / 256), (unsigned)n_pairs), dim3(256), 0, s,
                       pairs_dev, flow, out);
    return hipGetLastError();
}

hipError_t launch_seed_shape(const synthpix_pair* pairs_dev, int n_pairs, int64_t n_span,
                             const synthpix_seed_params& prm, float rho_lo, float rho_hi, uint64_t seed, float* dy,
                             float* rho, hipStream_t s)
{
    if (n_span <= 0) return hipSuccess;
    TimedScope ts("seed_shape", s);
    hipLaunchKernelGGL(seed_shape_kernel, dim3((unsigned)((n_span + 255) / 256)), dim3(256), 0, s, pairs_dev, n_pairs,
                       n_span, prm, rho_lo, rho_hi, seed, dy, rho);
    return hipGetLastError();
}

hipError_t launch_advect3(const synthpix_pair* pairs_dev, int n_pairs, int64_t n_span, const float* flow,
                          const float* wflow, const synthpix_advect_params& ap, const float* x1, const float* y1,
                          const float* z1, float* x2, float* y2, float* z2, hipStream_t s)
{
    if (n_span <= 0) return hipSuccess;
    TimedScope ts("advect", s);
    hipLaunchKernelGGL(advect3_kernel, dim3((unsigned)((n_span + 255) / 256)), dim3(256), 0, s, pairs_dev, n_pairs,
                       n_span, flow, wflow, ap, x1, y1, z1, x2, y2, z2);
    return hipGetLastError();
}

// Moves a captured plan's descriptor on to the next batch of the same shape:
// the pair-id offset grows by `step` (the batch size), so replays draw fresh
// particles.
__global__ void advance_pair_ids(synthpix_batch_io* __restrict__ iod, uint64_t step)
{
    if (threadIdx.x == 0) iod->pair_id_base += step;
}

__global__ void store_io(synthpix_batch_io* __restrict__ iod, synthpix_batch_io io)
{
    if (threadIdx.x == 0) *iod = io;
}

hipError_t launch_advance(synthpix_batch_io* iod, uint64_t step, hipStream_t s)
{
    hipLaunchKernelGGL(advance_pair_ids, dim3(1), dim3(64), 0, s, iod, step);
    return hipGetLastError();
}

hipError_t launch_store_io(synthpix_batch_io* iod, const synthpix_batch_io& io, hipStream_t s)
{
    hipLaunchKernelGGL(store_io, dim3(1), dim3(64), 0, s, iod, io);
    return hipGetLastError();
}

hipError_t launch_seed(const synthpix_pair* pairs_dev, int n_pairs, int64_t n_span,
                       const synthpix_seed_params& prm, uint64_t seed, float* x, float* y, float* z,
                       float* d, float* I0, int32_t* n_active, double* ppp, hipStream_t s,
                       const synthpix_batch_io* iod, int32_t* live)
{
    TimedScope ts("seed", s);
    if (n_active || ppp || iod || live)
        hipLaunchKernelGGL(pair_scalars_kernel, dim3((unsigned)((n_pairs + 255) / 256)), dim3(256), 0, s, pairs_dev,
                           n_pairs, prm, seed, n_active, ppp, iod, live);
    if (n_span > 0) {
        const int64_t blocks = (n_span + 255) / 256;
        hipLaunchKernelGGL(seed_kernel, dim3((unsigned)blocks), dim3(256), 0, s, pairs_dev, n_pairs, n_span,
                           prm, seed, x, y, z, d, I0, iod, iod != nullptr && live != nullptr);
    }
    return hipGetLastError();
}

hipError_t launch_advect(const synthpix_pair* pairs_dev, int n_pairs, int64_t n_span, const float* flow,
                         const synthpix_advect_params& ap, const float* x1, const float* y1, float* x2,
                         float* y2, hipStream_t s, AdvectOrder order, const synthpix_batch_io* iod)
{
    if (n_span <= 0) return hipSuccess;
    const int64_t blocks = (n_span + 256 * ADVECT_ILP - 1) / (256 * ADVECT_ILP);
    TimedScope ts("advect", s);
    if (order.entries)
        hipLaunchKernelGGL(advect_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, pairs_dev, n_pairs, n_span,
                           flow, ap, x1, y1, x2, y2, order, iod);
    else
        hipLaunchKernelGGL(advect_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, pairs_dev, n_pairs, n_span,
                           flow, ap, x1, y1, x2, y2, order, iod);
    return hipGetLastError();
}

}  // namespace sp
