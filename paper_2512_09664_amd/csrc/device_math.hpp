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

// a ^ b ^ k in one VALU instruction (gfx950's v_bitop3_b32, truth table 0x96:
// set for an odd number of set inputs), k a wave-uniform key word in an SGPR.
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

// The key must be wave-uniform (it is the generator seed everywhere).  The
// empty asm keeps the ten round keys from being hoisted out of callers' loops
// as twenty live scalar registers: each round's key is one scalar add.
__device__ __forceinline__ u32x4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
{
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3_key((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3_key((uint32_t)(p0 >> 32), c3, k1);
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

enum : uint32_t {
    STREAM_GEOM = 0, STREAM_PHOTO = 1, STREAM_JITTER = 2, STREAM_NOISE0 = 3, STREAM_PAIR = 5, STREAM_SHAPE = 6,
    STREAM_HIDE = 7
};

__device__ __forceinline__ float u24(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }
__device__ __forceinline__ float u24_open0(uint32_t w) { return (float)((w >> 8) + 1u) * 0x1p-24f; }

// ---------------------------------------------------------------- elementary functions
// exp(-q): Cody-Waite reduction by ln 2 (16-bit head + tail), degree-7 Taylor
// polynomial of exp(-r) in Horner form, exact scaling by 2^-k.  Zero for q >= 80.

constexpr float LN2_HI = (float)(45426.0 / 65536.0);
constexpr float LN2_LO = (float)(0.69314718055994530942 - 45426.0 / 65536.0);
constexpr float LOG2E_F = (float)1.44269504088896340736;

// exp(-q) for 0 <= q < 80 (no range check): the polynomial times the exact power 2^-k.
__device__ __forceinline__ float expneg_lt80(float q)
{
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
    return __builtin_amdgcn_ldexpf(p, -(int)kf);
}

__device__ __forceinline__ float expneg(float q)
{
    if (!(q < 80.0f)) return 0.0f;
    return expneg_lt80(q);
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

// cos(2 pi u) and sin(2 pi u) of one reduction (the same polynomials as cos2pi_ra;
// sin(k pi/2 + x) picks sin x, cos x, -sin x, -cos x by quadrant).
__device__ __forceinline__ float2 cossin2pi_ra(float u)
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
    case 0: return make_float2(c, s);
    case 1: return make_float2(-s, c);
    case 2: return make_float2(-c, -s);
    default: return make_float2(s, -c);
    }
}

// ---------------------------------------------------------------- support ranges
// Pixel indices k in [0, n) with |(k + 1/2) - p| <= R, the difference and the
// comparison in binary32.  The float offset is monotone in k, so the set is an
// interval [K0, K1].  Its ends are estimated as ceil(p - R - 1/2) and
// floor(p + R - 1/2); for |p| < 2^15 the estimates' rounding errors are far
// below one pixel, so each is within one of the exact end and a single
// re-test on either side fixes it.

__device__ __forceinline__ bool in_support(int k, float p, float R)
{
    const float dx = ((float)k + 0.5f) - p;
    return __builtin_fabsf(dx) <= R;
}

__device__ __forceinline__ bool support_range(float p, float R, int n, int& lo, int& hi)
{
    if (!(R > 0.0f) || !__builtin_isfinite(p)) return false;
    const float a = p - R, b = p + R;
    if (b < -1.0f || a > (float)n + 1.0f) {
        // far outside the image: nothing in [0, n); still exact since |dx| > R for every k
        return false;
    }
    int k0 = (int)__builtin_ceilf(a - 0.5f);
    int k1 = (int)__builtin_floorf(b - 0.5f);
    k0 = in_support(k0 - 1, p, R) ? k0 - 1 : (in_support(k0, p, R) ? k0 : k0 + 1);
    k1 = in_support(k1 + 1, p, R) ? k1 + 1 : (in_support(k1, p, R) ? k1 : k1 - 1);
    k0 = k0 < 0 ? 0 : k0;
    k1 = k1 > n - 1 ? n - 1 : k1;
    if (k0 > k1) return false;
    lo = k0;
    hi = k1;
    return true;
}

// Fixed-point scale of a particle's peak: 2^24 A, capped at 2^32 - 256 so that
// every product (Af gy) gx with gx, gy in [0, 1] truncates into a uint32.
__device__ __forceinline__ float fixed_peak(float A) { return __builtin_fminf(A * 16777216.0f, 4294967040.0f); }

__device__ __forceinline__ bool particle_valid(float x, float y, float d, float I0)
{
    return (I0 > 0.0f) && (d > 0.0f) && __builtin_isfinite(x) && __builtin_isfinite(y);
}

// Blocks are dispatched round-robin over the 8 XCDs; renumber them so that each
// XCD works on one contiguous range of the logical index space (neighbouring
// work shares data, and each XCD has its own L2).
__device__ __forceinline__ unsigned xcd_contiguous(unsigned b, unsigned n)
{
    const unsigned xcd = b & 7u, slot = b >> 3;
    const unsigned q = n >> 3, rem = n & 7u;
    return xcd < rem ? xcd * (q + 1) + slot : rem * (q + 1) + (xcd - rem) * q + slot;
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

// Pair of particle g when g0 <= g is a particle index common to the whole
// workgroup: the search for g0 is uniform (scalar loads), then each lane steps
// forward over the few pair starts between g0 and g.
__device__ __forceinline__ int find_pair_from(const synthpix_pair* __restrict__ pairs, int n_pairs, int64_t g0,
                                              int64_t g)
{
    int p = find_pair_by_particle(pairs, n_pairs, g0);
    while (p + 1 < n_pairs && pairs[p + 1].particle_offset <= g) ++p;
    return p;
}

}  // namespace sp
