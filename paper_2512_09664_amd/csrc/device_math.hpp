// Device-side arithmetic shared by the generator's kernels (gfx950).
//
// Everything that decides an integer (tile membership, stored codes) or that
// must reproduce bit for bit is written here with explicit roundings:
// the translation unit is compiled with -ffp-contract=off, so a fused
// multiply-add happens only where __builtin_fmaf is written.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "synthpix.h"

namespace sp {

// ---------------------------------------------------------------- Philox4x32-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11).  Counter (index, stream, pair_id lo, pair_id hi), key (seed lo, hi).

struct u32x4 { uint32_t a, b, c, d; };

__device__ __forceinline__ u32x4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return {c0, c1, c2, c3};
}

__device__ __forceinline__ u32x4 draw(uint32_t index, uint32_t stream, uint64_t pair_id, uint64_t seed)
{
    return philox(index, stream, (uint32_t)pair_id, (uint32_t)(pair_id >> 32),
                  (uint32_t)seed, (uint32_t)(seed >> 32));
}

enum : uint32_t { STREAM_GEOM = 0, STREAM_PHOTO = 1, STREAM_NOISE0 = 3, STREAM_PAIR = 5 };

__device__ __forceinline__ float u24(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }
__device__ __forceinline__ float u24_open0(uint32_t w) { return (float)((w >> 8) + 1u) * 0x1p-24f; }

// ---------------------------------------------------------------- elementary functions
// exp(-q): Cody-Waite reduction by ln 2 (16-bit head + tail), degree-7 Taylor
// polynomial of exp(-r) in Horner form, exact scaling by 2^-k.  Zero for q >= 80.

constexpr float LN2_HI = (float)(45426.0 / 65536.0);
constexpr float LN2_LO = (float)(0.69314718055994530942 - 45426.0 / 65536.0);
constexpr float LOG2E_F = (float)1.44269504088896340736;

__device__ __forceinline__ float expneg(float q)
{
    if (!(q < 80.0f)) return 0.0f;
    const float kf = __builtin_rintf(q * LOG2E_F);
    float r = __builtin_fmaf(kf, -LN2_HI, q);
    r = __builtin_fmaf(kf, -LN2_LO, r);
    float p = (float)(-1.0 / 5040.0);
    p = __builtin_fmaf(p, r, (float)(1.0 / 720.0));
    p = __builtin_fmaf(p, r, (float)(-1.0 / 120.0));
    p = __builtin_fmaf(p, r, (float)(1.0 / 24.0));
    p = __builtin_fmaf(p, r, (float)(-1.0 / 6.0));
    p = __builtin_fmaf(p, r, 0.5f);
    p = __builtin_fmaf(p, r, -1.0f);
    p = __builtin_fmaf(p, r, 1.0f);
    const int k = (int)kf;
    return p * __uint_as_float((uint32_t)(127 - k) << 23);
}

// ln(u), u a positive normal float: exponent split, mantissa in [sqrt(1/2), sqrt(2)),
// atanh series 2 f (1 + f^2/3 + f^4/5 + f^6/7 + f^8/9), f = (m - 1) / (m + 1).
__device__ __forceinline__ float log_ra(float u)
{
    const uint32_t b = __float_as_uint(u);
    int e = (int)(b >> 23) - 127;
    float m = __uint_as_float((b & 0x7fffffu) | 0x3f800000u);
    if (m > (float)1.41421356237309504880) { m = m * 0.5f; e += 1; }
    const float f = (m - 1.0f) / (m + 1.0f);
    const float s = f * f;
    float p = __builtin_fmaf(s, (float)(1.0 / 9.0), (float)(1.0 / 7.0));
    p = __builtin_fmaf(s, p, (float)(1.0 / 5.0));
    p = __builtin_fmaf(s, p, (float)(1.0 / 3.0));
    p = __builtin_fmaf(s, p, 1.0f);
    const float lnm = (f + f) * p;
    const float ef = (float)e;
    return __builtin_fmaf(ef, LN2_HI, __builtin_fmaf(ef, LN2_LO, lnm));
}

// cos(2 pi u), u in [0, 1): quadrant reduction t = 4u = k + f, x = f pi/2,
// Taylor cos/sin of x through degree 8/9.
__device__ __forceinline__ float cos2pi_ra(float u)
{
    const float t = u * 4.0f;
    const float kf = __builtin_rintf(t);
    const float f = t - kf;
    const float x = f * (float)1.57079632679489661923;
    const float x2 = x * x;
    float c = __builtin_fmaf(x2, (float)(1.0 / 40320.0), (float)(-1.0 / 720.0));
    c = __builtin_fmaf(x2, c, (float)(1.0 / 24.0));
    c = __builtin_fmaf(x2, c, -0.5f);
    c = __builtin_fmaf(x2, c, 1.0f);
    float s = __builtin_fmaf(x2, (float)(1.0 / 362880.0), (float)(-1.0 / 5040.0));
    s = __builtin_fmaf(x2, s, (float)(1.0 / 120.0));
    s = __builtin_fmaf(x2, s, (float)(-1.0 / 6.0));
    s = __builtin_fmaf(x2, s, 1.0f);
    s = x * s;
    switch (((int)kf) & 3) {
    case 0: return c;
    case 1: return -s;
    case 2: return -c;
    default: return s;
    }
}

// ---------------------------------------------------------------- support ranges
// Pixel indices k in [0, n) with |(k + 1/2) - p| <= R, the difference and the
// comparison in binary32.  The float offset is monotone in k, so the set is an
// interval; it is found from a float estimate and corrected by re-testing.

__device__ __forceinline__ bool in_support(int k, float p, float R)
{
    const float dx = ((float)k + 0.5f) - p;
    return __builtin_fabsf(dx) <= R;
}

__device__ __forceinline__ bool support_range(float p, float R, int n, int& lo, int& hi)
{
    if (!(R > 0.0f) || !__builtin_isfinite(p)) return false;
    const float a = __builtin_floorf(p - R) - 2.0f;
    const float b = __builtin_ceilf(p + R) + 2.0f;
    if (b < 0.0f || a > (float)(n - 1)) return false;
    int k0 = a < 0.0f ? 0 : (int)a;
    int k1 = b > (float)(n - 1) ? n - 1 : (int)b;
    // The float estimate is within a couple of pixels: at most a few iterations.
    while (k0 <= k1 && !in_support(k0, p, R)) ++k0;
    while (k1 >= k0 && !in_support(k1, p, R)) --k1;
    if (k0 > k1) return false;
    lo = k0;
    hi = k1;
    return true;
}

__device__ __forceinline__ uint32_t quant24(float t)
{
    // t already carries the 2^24 scale; truncate, saturate, NaN -> 0.
    if (!(t > 0.0f)) return 0u;
    if (t >= 4294967296.0f) return 0xffffffffu;
    return (uint32_t)t;
}

__device__ __forceinline__ bool particle_valid(float x, float y, float d, float I0)
{
    return (I0 > 0.0f) && (d > 0.0f) && __builtin_isfinite(x) && __builtin_isfinite(y);
}

// Pair lookup: the pair whose particle range [offset, offset + n_max) holds g.
// Pairs are sorted by particle_offset (validated on the host).
__device__ __forceinline__ int find_pair_by_particle(const synthpix_pair* pairs, int n_pairs, int64_t g)
{
    int lo = 0, hi = n_pairs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pairs[mid].particle_offset <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace sp
