// Bilinear sampling of a pair's cell-centred flow grid (shared by the
// advection kernel and its adjoint).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "synthpix.h"

namespace sp {

// Two consecutive (u, v) nodes as one 16-byte load (8-byte aligned address; the
// hardware handles the unaligned vector access).
__device__ __forceinline__ float4 load_pair(const float2* p)
{
    float4 v;
    __builtin_memcpy(&v, p, sizeof(v));
    return v;
}

struct FlowView {
    const float2* __restrict__ F;
    int Gh, Gw;
    float sx, sy;      // Gw / W, Gh / H (correctly rounded)
};

// A rectangle of a pair's grid nodes copied to LDS (rows wi0 .., columns wj0 ..,
// wh x ww nodes, row-major, wh and ww >= 1); NO_WIN (a single node, which holds
// no whole cell) means none.  The nodes themselves are passed separately, as
// the workgroup's LDS array of (u, v) floats.
struct FlowWin {
    int wi0, wj0, wh, ww;
};

constexpr FlowWin NO_WIN = {0, 0, 1, 1};

typedef __attribute__((address_space(3))) const float lds_float;   // LDS (group segment) word

__device__ __forceinline__ float2 sample_flow(const FlowView& fv, float px, float py,
                                              const FlowWin& win = NO_WIN,
                                              lds_float* lds = nullptr)
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
    // the cell's two nodes of one grid row are adjacent: one 16-byte load per row,
    // from the LDS window when the cell lies inside it
    float4 r0, r1;
    const int li = i0 - win.wi0, lj = j0 - win.wj0;
    // 0 <= li < wh - 1 and 0 <= lj < ww - 1, each as one unsigned comparison
    if ((unsigned)li < (unsigned)(win.wh - 1) && (unsigned)lj < (unsigned)(win.ww - 1)) {
        // (u, v) nodes as float pairs: row li from node lj on, then row li + 1
        lds_float* w0 = lds + 2 * (li * win.ww + lj);
        lds_float* w1 = w0 + 2 * win.ww;
        r0 = make_float4(w0[0], w0[1], w0[2], w0[3]);
        r1 = make_float4(w1[0], w1[1], w1[2], w1[3]);
    } else {
        const float2* row0 = fv.F + (size_t)i0 * fv.Gw + j0;
        r0 = load_pair(row0);
        r1 = load_pair(row0 + fv.Gw);
    }
    const float2 a = make_float2(r0.x, r0.y), b = make_float2(r0.z, r0.w);
    const float2 c = make_float2(r1.x, r1.y), e = make_float2(r1.z, r1.w);
    float2 out;
    {
        const float top = __builtin_fmaf(fx, b.x - a.x, a.x);
        const float bot = __builtin_fmaf(fx, e.x - c.x, c.x);
        out.x = __builtin_fmaf(fy, bot - top, top);
    }
    {
        const float top = __builtin_fmaf(fx, b.y - a.y, a.y);
        const float bot = __builtin_fmaf(fx, e.y - c.y, c.y);
        out.y = __builtin_fmaf(fy, bot - top, top);
    }
    return out;
}

__device__ __forceinline__ FlowView flow_view(const synthpix_pair& P, const float* flow)
{
    FlowView fv;
    fv.F = reinterpret_cast<const float2*>(flow + P.flow_offset);
    fv.Gh = P.Gh;
    fv.Gw = P.Gw;
    fv.sx = (float)P.Gw / (float)P.W;
    fv.sy = (float)P.Gh / (float)P.H;
    return fv;
}

// One substep of the frozen-field integrator, the same operations in the same
// order as the advection kernel: Euler p = fma(h, u, p); RK4 stages at
// fma(h/2, k, p) and fma(h, k3, p), update fma(h, (((k1 + 2 k2) + 2 k3) + k4) / 6, p).
__device__ __forceinline__ void substep(const FlowView& fv, float& px, float& py, float h, float hh, int integrator)
{
    if (integrator == SP_EULER) {
        const float2 u = sample_flow(fv, px, py);
        px = __builtin_fmaf(h, u.x, px);
        py = __builtin_fmaf(h, u.y, py);
        return;
    }
    const float2 k1 = sample_flow(fv, px, py);
    const float2 k2 = sample_flow(fv, __builtin_fmaf(hh, k1.x, px), __builtin_fmaf(hh, k1.y, py));
    const float2 k3 = sample_flow(fv, __builtin_fmaf(hh, k2.x, px), __builtin_fmaf(hh, k2.y, py));
    const float2 k4 = sample_flow(fv, __builtin_fmaf(h, k3.x, px), __builtin_fmaf(h, k3.y, py));
    const float su = ((k1.x + 2.0f * k2.x) + 2.0f * k3.x) + k4.x;
    const float sv = ((k1.y + 2.0f * k2.y) + 2.0f * k3.y) + k4.y;
    px = __builtin_fmaf(h, su / 6.0f, px);
    py = __builtin_fmaf(h, sv / 6.0f, py);
}

}  // namespace sp
