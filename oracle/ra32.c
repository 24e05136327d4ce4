/*
 * Binary32 mirror of the generator -- TEST INFRASTRUCTURE ONLY (oracle).
 *
 * Plain host C.  Every step of the float64 oracle is repeated here with each
 * rounding written out, so that where a float decides an integer (the tile
 * membership, the stored integer codes) the decision is taken in the same
 * precision as the GPU kernels.  Build with -ffp-contract=off: every fused
 * multiply-add below is an explicit fmaf(); no other operation is fused.
 *
 * Paper passages followed (SynthPix, Terpin et al.):
 *   Eq. 1 (single-particle Gaussian, here rho = 0, sigma = d/4);
 *   Section 2 "Sampling the particles" (ppp_max allocation, ppp draw, masking,
 *   flow mapping x -> x + u);
 *   Section 2 "Considerations on the aggregation" (plain superposition);
 *   Section 2 "Efficient rasterization" (patch side 3 d + 1 -> support 1.5 d);
 *   Remark 1 / Remark 2 (sheet profile deferred, point sampling).
 *
 * Reference arithmetic (all binary32, round-to-nearest-even):
 *   - exp(-q) is E(q): Cody-Waite reduction by ln 2 and a degree-7 Taylor
 *     polynomial in fmaf Horner form, scaled by an exact power of two; E = 0
 *     for q >= 80 (or NaN).
 *   - ln and cos(2 pi u) for the Box-Muller normal of the diameter use the same
 *     style of reduction (atanh series, quadrant reduction).
 *   - a particle's contribution to a pixel is quantised to 2^-24 full-scale
 *     units, t = (min(A * 2^24, 2^32 - 256) * gy) * gx truncated to an unsigned
 *     32-bit integer, and summed in 32-bit integers: the sum is exact and
 *     order-free.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* ------------------------------------------------------------------ Philox */

#define PX_M0 0xD2511F53u
#define PX_M1 0xCD9E8D57u
#define PX_W0 0x9E3779B9u
#define PX_W1 0xBB67AE85u

void ra_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += PX_W0; k1 += PX_W1; }
        uint64_t p0 = (uint64_t)PX_M0 * c0;
        uint64_t p1 = (uint64_t)PX_M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint32_t index, uint32_t stream, uint64_t pid, uint64_t seed, uint32_t w[4])
{
    uint32_t c[4] = {index, stream, (uint32_t)pid, (uint32_t)(pid >> 32)};
    uint32_t k[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    ra_philox(c, k, w);
}

static float u24(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }
static float u24o(uint32_t w) { return (float)((w >> 8) + 1u) * 0x1p-24f; }

/* ------------------------------------------------------- elementary functions */

static const float LN2_HI = (float)(45426.0 / 65536.0);                 /* ln2 to 16 bits */
static const float LN2_LO = (float)(0.69314718055994530942 - 45426.0 / 65536.0);
static const float LOG2E_F = (float)1.44269504088896340736;

float ra_E(float q)
{
    if (!(q < 80.0f)) return 0.0f;
    float kf = rintf(q * LOG2E_F);
    float r = fmaf(kf, -LN2_HI, q);
    r = fmaf(kf, -LN2_LO, r);
    float p = (float)(-1.0 / 5040.0);
    p = fmaf(p, r, (float)(1.0 / 720.0));
    p = fmaf(p, r, (float)(-1.0 / 120.0));
    p = fmaf(p, r, (float)(1.0 / 24.0));
    p = fmaf(p, r, (float)(-1.0 / 6.0));
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, -1.0f);
    p = fmaf(p, r, 1.0f);
    int k = (int)kf;
    uint32_t bits = (uint32_t)(127 - k) << 23;
    float sc;
    memcpy(&sc, &bits, 4);
    return p * sc;
}

float ra_ln(float u)
{
    uint32_t b;
    memcpy(&b, &u, 4);
    int e = (int)(b >> 23) - 127;
    uint32_t mb = (b & 0x7fffffu) | 0x3f800000u;
    float m;
    memcpy(&m, &mb, 4);
    if (m > (float)1.41421356237309504880) { m = m * 0.5f; e += 1; }
    float f = (m - 1.0f) / (m + 1.0f);
    float s = f * f;
    float p = fmaf(s, (float)(1.0 / 9.0), (float)(1.0 / 7.0));
    p = fmaf(s, p, (float)(1.0 / 5.0));
    p = fmaf(s, p, (float)(1.0 / 3.0));
    p = fmaf(s, p, 1.0f);
    float lnm = (f + f) * p;
    float ef = (float)e;
    return fmaf(ef, LN2_HI, fmaf(ef, LN2_LO, lnm));
}

float ra_cos2pi(float u)
{
    float t = u * 4.0f;
    float kf = rintf(t);
    float f = t - kf;
    float x = f * (float)1.57079632679489661923;
    float x2 = x * x;
    float c = fmaf(x2, (float)(1.0 / 40320.0), (float)(-1.0 / 720.0));
    c = fmaf(x2, c, (float)(1.0 / 24.0));
    c = fmaf(x2, c, -0.5f);
    c = fmaf(x2, c, 1.0f);
    float s = fmaf(x2, (float)(1.0 / 362880.0), (float)(-1.0 / 5040.0));
    s = fmaf(x2, s, (float)(1.0 / 120.0));
    s = fmaf(x2, s, (float)(-1.0 / 6.0));
    s = fmaf(x2, s, 1.0f);
    s = x * s;
    switch (((int)kf) & 3) {
    case 0: return c;
    case 1: return -s;
    case 2: return -c;
    default: return s;
    }
}

/* ----------------------------------------------------------------- seeding */

int ra_seed_pair(int H, int W, int n_max, double ppp_lo, double ppp_hi, uint64_t pid, uint64_t seed,
                 int d_normal, const float dp[4], const float I0r[2], const float zr[2],
                 float* x, float* y, float* z, float* d, float* I0, double* ppp_out)
{
    uint32_t w[4], g[4], h[4];
    draw(0u, 5u, pid, seed, w);
    double ppp = ppp_lo + (ppp_hi - ppp_lo) * (double)u24(w[0]);
    double na = floor((double)H * (double)W * ppp + 0.5);
    int n_active = na < (double)n_max ? (int)na : n_max;
    if (ppp_out) *ppp_out = ppp;
    const float Wf = (float)W, Hf = (float)H;
    for (int i = 0; i < n_max; ++i) {
        draw((uint32_t)i, 0u, pid, seed, g);
        draw((uint32_t)i, 1u, pid, seed, h);
        x[i] = u24(g[0]) * Wf;
        y[i] = u24(g[1]) * Hf;
        z[i] = fmaf(zr[1] - zr[0], u24(g[2]), zr[0]);
        if (!d_normal) {
            d[i] = fmaf(dp[1] - dp[0], u24(g[3]), dp[0]);
        } else {
            float l = ra_ln(u24o(h[1]));
            float R = sqrtf(-2.0f * l);
            float n = R * ra_cos2pi(u24(h[2]));
            float v = fmaf(dp[1], n, dp[0]);
            v = fmaxf(v, dp[2]);
            d[i] = fminf(v, dp[3]);
        }
        I0[i] = (i < n_active) ? fmaf(I0r[1] - I0r[0], u24(h[0]), I0r[0]) : 0.0f;
    }
    return n_active;
}

/* ---------------------------------------------------------------- advection */

static void sample(const float* F, int Gh, int Gw, float sx, float sy, float px, float py,
                   float* u, float* v)
{
    float gx = px * sx - 0.5f;
    float gy = py * sy - 0.5f;
    gx = fminf(fmaxf(gx, 0.0f), (float)(Gw - 1));
    gy = fminf(fmaxf(gy, 0.0f), (float)(Gh - 1));
    int j0 = (int)floorf(gx);
    int i0 = (int)floorf(gy);
    if (j0 > Gw - 2) j0 = Gw - 2;
    if (i0 > Gh - 2) i0 = Gh - 2;
    float fx = gx - (float)j0;
    float fy = gy - (float)i0;
    const float* a = F + 2 * ((size_t)i0 * Gw + j0);
    const float* b = a + 2;
    const float* c = a + 2 * (size_t)Gw;
    const float* e = c + 2;
    for (int k = 0; k < 2; ++k) {
        float top = fmaf(fx, b[k] - a[k], a[k]);
        float bot = fmaf(fx, e[k] - c[k], c[k]);
        float val = fmaf(fy, bot - top, top);
        if (k == 0) *u = val; else *v = val;
    }
}

void ra_advect(const float* F, int Gh, int Gw, int H, int W, int n, const float* x1, const float* y1,
               float dt, int substeps, int rk4, float* x2, float* y2)
{
    const float sx = (float)Gw / (float)W;
    const float sy = (float)Gh / (float)H;
    const float h = dt / (float)substeps;
    const float hh = h * 0.5f;
    for (int i = 0; i < n; ++i) {
        float px = x1[i], py = y1[i];
        for (int s = 0; s < substeps; ++s) {
            if (!rk4) {
                float u, v;
                sample(F, Gh, Gw, sx, sy, px, py, &u, &v);
                px = fmaf(h, u, px);
                py = fmaf(h, v, py);
            } else {
                float k1u, k1v, k2u, k2v, k3u, k3v, k4u, k4v;
                sample(F, Gh, Gw, sx, sy, px, py, &k1u, &k1v);
                sample(F, Gh, Gw, sx, sy, fmaf(hh, k1u, px), fmaf(hh, k1v, py), &k2u, &k2v);
                sample(F, Gh, Gw, sx, sy, fmaf(hh, k2u, px), fmaf(hh, k2v, py), &k3u, &k3v);
                sample(F, Gh, Gw, sx, sy, fmaf(h, k3u, px), fmaf(h, k3v, py), &k4u, &k4v);
                float su = ((k1u + 2.0f * k2u) + 2.0f * k3u) + k4u;
                float sv = ((k1v + 2.0f * k2v) + 2.0f * k3v) + k4v;
                px = fmaf(h, su / 6.0f, px);
                py = fmaf(h, sv / 6.0f, py);
            }
        }
        x2[i] = px;
        y2[i] = py;
    }
}

/* ------------------------------------------------------------------ support */

static int in_support(int k, float p, float R)
{
    float dx = ((float)k + 0.5f) - p;
    return fabsf(dx) <= R;
}

/* Pixel index range [lo, hi] in [0, n) whose centre offset (k + 1/2) - p lies
 * in [-R, R] (binary32).  Returns 0 if empty. */
int ra_support_range(float p, float R, int n, int* lo, int* hi)
{
    if (!(R > 0.0f) || !isfinite(p)) return 0;
    double a = floor((double)p - (double)R) - 2.0;
    double b = ceil((double)p + (double)R) + 2.0;
    if (b < 0.0 || a > (double)(n - 1)) return 0;
    int k0 = a < 0.0 ? 0 : (int)a;
    int k1 = b > (double)(n - 1) ? n - 1 : (int)b;
    while (k0 <= k1 && !in_support(k0, p, R)) ++k0;
    while (k1 >= k0 && !in_support(k1, p, R)) --k1;
    if (k0 > k1) return 0;
    *lo = k0;
    *hi = k1;
    return 1;
}

/* --------------------------------------------------------------- rendering */

/* t = (Af gy) gx with 0 <= gx, gy <= 1 and 0 <= Af <= 2^32 - 256, so t fits an
 * unsigned 32-bit integer: plain truncation. */
static uint32_t quant(float t) { return (uint32_t)t; }

/* Fixed-point exposure: acc[r*W + c] = sum over particles of the 2^-24-quantised
 * contribution.  sheet_sigma is the Gaussian laser-sheet width s. */
void ra_render_fixed(int H, int W, int n, const float* x, const float* y, const float* z,
                     const float* d, const float* I0, float sheet_sigma, uint32_t* acc)
{
    const float cs = 0.5f / (sheet_sigma * sheet_sigma);
    memset(acc, 0, sizeof(uint32_t) * (size_t)H * (size_t)W);
    float gxt[1024];
    for (int i = 0; i < n; ++i) {
        if (!(I0[i] > 0.0f) || !(d[i] > 0.0f) || !isfinite(x[i]) || !isfinite(y[i])) continue;
        const float R = 1.5f * d[i];
        int c0, c1, r0, r1;
        if (!ra_support_range(x[i], R, W, &c0, &c1)) continue;
        if (!ra_support_range(y[i], R, H, &r0, &r1)) continue;
        if (c1 - c0 >= 1024) continue;             /* diameters beyond ~340 px are not modelled */
        const float A = I0[i] * ra_E((z[i] * z[i]) * cs);
        const float Af = fminf(A * 16777216.0f, 4294967040.0f);   /* 2^24 A, at most 2^32 - 256 */
        const float kap = 8.0f / (d[i] * d[i]);
        for (int c = c0; c <= c1; ++c) {
            float dx = ((float)c + 0.5f) - x[i];
            gxt[c - c0] = ra_E(kap * (dx * dx));
        }
        for (int r = r0; r <= r1; ++r) {
            float dy = ((float)r + 0.5f) - y[i];
            float rs = Af * ra_E(kap * (dy * dy));
            uint32_t* row = acc + (size_t)r * W;
            for (int c = c0; c <= c1; ++c) row[c] += quant(rs * gxt[c - c0]);
        }
    }
}

void ra_fixed_to_float(const uint32_t* acc, size_t n, float* out)
{
    for (size_t i = 0; i < n; ++i) out[i] = (float)acc[i] * 0x1p-24f;
}

/* ------------------------------------------------------------------ epilogue */

/* Separable zero-padded blur: horizontal then vertical, taps summed in
 * ascending offset with fmaf from +0. */
void ra_blur(const float* in, int H, int W, const float* w, int b, float* tmp, float* out)
{
    for (int r = 0; r < H; ++r)
        for (int c = 0; c < W; ++c) {
            float acc = 0.0f;
            for (int k = -b; k <= b; ++k) {
                int cc = c + k;
                if (cc < 0 || cc >= W) continue;
                acc = fmaf(w[k + b], in[(size_t)r * W + cc], acc);
            }
            tmp[(size_t)r * W + c] = acc;
        }
    for (int r = 0; r < H; ++r)
        for (int c = 0; c < W; ++c) {
            float acc = 0.0f;
            for (int k = -b; k <= b; ++k) {
                int rr = r + k;
                if (rr < 0 || rr >= H) continue;
                acc = fmaf(w[k + b], tmp[(size_t)rr * W + c], acc);
            }
            out[(size_t)r * W + c] = acc;
        }
}

void ra_quantise(const float* v, size_t n, int bits, uint16_t* q)
{
    const float L = (float)((1u << bits) - 1u);
    for (size_t i = 0; i < n; ++i) {
        float t = rintf(v[i] * L);
        t = fmaxf(t, 0.0f);
        t = fminf(t, L);
        q[i] = (uint16_t)t;
    }
}

/* ============================================================ full model */
/*
 * Binary32 mirror of the full per-particle model (Eq. 1 with sigma_x = d / 4,
 * sigma_y = d_y / 4 and rho; frame-2 parameter variation; per-frame hiding;
 * the out-of-focus sheet law of Remark 1; out-of-plane motion).
 */

#define RHO_MAX 0.99f

float ra_sin2pi(float u)
{
    float t = u * 4.0f;
    float kf = rintf(t);
    float f = t - kf;
    float x = f * (float)1.57079632679489661923;
    float x2 = x * x;
    float c = fmaf(x2, (float)(1.0 / 40320.0), (float)(-1.0 / 720.0));
    c = fmaf(x2, c, (float)(1.0 / 24.0));
    c = fmaf(x2, c, -0.5f);
    c = fmaf(x2, c, 1.0f);
    float s = fmaf(x2, (float)(1.0 / 362880.0), (float)(-1.0 / 5040.0));
    s = fmaf(x2, s, (float)(1.0 / 120.0));
    s = fmaf(x2, s, (float)(-1.0 / 6.0));
    s = fmaf(x2, s, 1.0f);
    s = x * s;
    switch (((int)kf) & 3) {
    case 0: return s;
    case 1: return c;
    case 2: return -s;
    default: return -c;
    }
}

/* Second diameter and correlation (stream 6): d_y from the diameter
 * distribution (uniform: word 0; clipped normal: Box-Muller of words 1, 2),
 * rho = rho_lo + (rho_hi - rho_lo) u(word 3). */
void ra_seed_shape(int n_max, uint64_t pid, uint64_t seed, int d_normal, const float dp[4], float rho_lo,
                   float rho_hi, float* dy, float* rho)
{
    uint32_t w[4];
    for (int i = 0; i < n_max; ++i) {
        draw((uint32_t)i, 6u, pid, seed, w);
        if (!d_normal) {
            dy[i] = fmaf(dp[1] - dp[0], u24(w[0]), dp[0]);
        } else {
            float R = sqrtf(-2.0f * ra_ln(u24o(w[1])));
            float v = fmaf(dp[1], R * ra_cos2pi(u24(w[2])), dp[0]);
            v = fmaxf(v, dp[2]);
            dy[i] = fminf(v, dp[3]);
        }
        rho[i] = fmaf(rho_hi - rho_lo, u24(w[3]), rho_lo);
    }
}

/* Per-frame parameters.  In: frame-1 d, dy, rho, I0.  Out: I0_1 (frame 1 after
 * hiding) and d2, dy2, rho2, I0_2 (frame 2).  jit = (diameters, rho,
 * intensity) standard deviations; a zero one leaves the parameter as is. */
void ra_frame_params(int n, uint64_t pid, uint64_t seed, const float jit[3], float hide_p, float d_max,
                     const float* d, const float* dy, const float* rho, const float* I0,
                     float* I0_1, float* d2, float* dy2, float* rho2, float* I0_2)
{
    uint32_t w[4];
    for (int i = 0; i < n; ++i) {
        float a = d[i], b = dy[i], r = rho[i], I = I0[i];
        if (jit[0] > 0.0f || jit[1] > 0.0f || jit[2] > 0.0f) {
            draw((uint32_t)i, 2u, pid, seed, w);
            float R0 = sqrtf(-2.0f * ra_ln(u24o(w[0])));
            float R1 = sqrtf(-2.0f * ra_ln(u24o(w[2])));
            float n0 = R0 * ra_cos2pi(u24(w[1]));
            float n1 = R0 * ra_sin2pi(u24(w[1]));
            float n2 = R1 * ra_cos2pi(u24(w[3]));
            float n3 = R1 * ra_sin2pi(u24(w[3]));
            if (jit[0] > 0.0f) {
                a = fminf(fmaxf(fmaf(jit[0], n0, a), 0.0f), d_max);
                b = fminf(fmaxf(fmaf(jit[0], n1, b), 0.0f), d_max);
            }
            if (jit[1] > 0.0f) r = fminf(fmaxf(fmaf(jit[1], n2, r), -RHO_MAX), RHO_MAX);
            if (jit[2] > 0.0f) I = I > 0.0f ? fmaxf(fmaf(jit[2], n3, I), 0.0f) : 0.0f;
        }
        float I1 = I0[i];
        if (hide_p > 0.0f) {
            draw((uint32_t)i, 7u, pid, seed, w);
            if (u24(w[0]) < hide_p) I1 = 0.0f;
            if (u24(w[1]) < hide_p) I = 0.0f;
        }
        I0_1[i] = I1;
        d2[i] = a;
        dy2[i] = b;
        rho2[i] = r;
        I0_2[i] = I;
    }
}

/* Peak of a particle: I0 S(z).  law 0: Gaussian sheet S = E(z^2 / (2 s^2))
 * (c = 0.5 / (s s)); law 1: Remark 1, S = exp(-k v^shape) with
 * v = z^2 (2 / (DZ0 DZ0)), k = 1 / sqrt(2 pi): v^shape = E(-(shape ln v))
 * (v below the smallest normal float counts as 0; shape ln v >= 80 gives S = 0). */
float ra_peak(float I0, float z, int law, float sheet_sigma, float dz0, float shape)
{
    if (law == 0) return I0 * ra_E((z * z) * (0.5f / (sheet_sigma * sheet_sigma)));
    const float c2 = 2.0f / (dz0 * dz0);
    const float v = (z * z) * c2;
    float p = 0.0f;
    if (v >= 0x1p-126f) {
        const float a = shape * ra_ln(v);
        if (!(a < 80.0f)) return 0.0f;
        p = ra_E(-a);
    }
    return I0 * ra_E((float)0.39894228040143267794 * p);
}

void ra_peaks(int n, const float* I0, const float* z, int law, float sheet_sigma, float dz0, float shape,
              float* A)
{
    for (int i = 0; i < n; ++i) A[i] = ra_peak(I0[i], z[i], law, sheet_sigma, dz0, shape);
}

/* Fixed-point exposure of the full model from per-particle peaks A.
 * om = 1 - rho^2 (one fmaf), kx = 8 / (om (d d)), ky = 8 / (om (dy dy)).
 * rho == 0: separable, t = (Af E(ky dy^2)) E(kx dx^2), as the isotropic path.
 * rho != 0: kxy = (-16 rho) / (om (d dy)); per row a = kxy dy, b = ky (dy dy);
 * per pixel q = max(fmaf(dx, fmaf(kx, dx, a), b), 0), t = Af E(q).
 * Patch: |dx| <= 1.5 d, |dy| <= 1.5 d_y. */
void ra_render_model_fixed(int H, int W, int n, const float* x, const float* y, const float* A,
                           const float* d, const float* dy, const float* rho, uint32_t* acc)
{
    memset(acc, 0, sizeof(uint32_t) * (size_t)H * (size_t)W);
    float gxt[1024];
    for (int i = 0; i < n; ++i) {
        if (!(A[i] > 0.0f) || !(d[i] > 0.0f) || !(dy[i] > 0.0f) || !isfinite(x[i]) || !isfinite(y[i])) continue;
        int c0, c1, r0, r1;
        if (!ra_support_range(x[i], 1.5f * d[i], W, &c0, &c1)) continue;
        if (!ra_support_range(y[i], 1.5f * dy[i], H, &r0, &r1)) continue;
        if (c1 - c0 >= 1024) continue;
        const float Af = fminf(A[i] * 16777216.0f, 4294967040.0f);
        const float r = rho[i];
        const float om = fmaf(-r, r, 1.0f);
        const float kx = 8.0f / (om * (d[i] * d[i]));
        const float ky = 8.0f / (om * (dy[i] * dy[i]));
        if (r == 0.0f) {
            for (int c = c0; c <= c1; ++c) {
                float dx = ((float)c + 0.5f) - x[i];
                gxt[c - c0] = ra_E(kx * (dx * dx));
            }
            for (int rr = r0; rr <= r1; ++rr) {
                float ddy = ((float)rr + 0.5f) - y[i];
                float rs = Af * ra_E(ky * (ddy * ddy));
                uint32_t* row = acc + (size_t)rr * W;
                for (int c = c0; c <= c1; ++c) row[c] += quant(rs * gxt[c - c0]);
            }
        } else {
            const float kxy = (-16.0f * r) / (om * (d[i] * dy[i]));
            for (int rr = r0; rr <= r1; ++rr) {
                float ddy = ((float)rr + 0.5f) - y[i];
                float a = kxy * ddy;
                float b = ky * (ddy * ddy);
                uint32_t* row = acc + (size_t)rr * W;
                for (int c = c0; c <= c1; ++c) {
                    float dx = ((float)c + 0.5f) - x[i];
                    float q = fmaxf(fmaf(dx, fmaf(kx, dx, a), b), 0.0f);
                    row[c] += quant(Af * ra_E(q));
                }
            }
        }
    }
}

/* Scalar bilinear sample of a cell-centred [Gh][Gw] grid (same registration
 * and clamping as the (u, v) grid). */
static float sample_scalar(const float* G, int Gh, int Gw, float sx, float sy, float px, float py)
{
    float gx = px * sx - 0.5f;
    float gy = py * sy - 0.5f;
    gx = fminf(fmaxf(gx, 0.0f), (float)(Gw - 1));
    gy = fminf(fmaxf(gy, 0.0f), (float)(Gh - 1));
    int j0 = (int)floorf(gx);
    int i0 = (int)floorf(gy);
    if (j0 > Gw - 2) j0 = Gw - 2;
    if (i0 > Gh - 2) i0 = Gh - 2;
    float fx = gx - (float)j0;
    float fy = gy - (float)i0;
    const float* a = G + (size_t)i0 * Gw + j0;
    const float* c = a + Gw;
    float top = fmaf(fx, a[1] - a[0], a[0]);
    float bot = fmaf(fx, c[1] - c[0], c[0]);
    return fmaf(fy, bot - top, top);
}

/* Out-of-plane motion: z2 = z1 + integral of w along the in-plane trajectory,
 * with the stages of ra_advect (Euler: z = fmaf(h, w, z); RK4: z = fmaf(h,
 * (((w1 + 2 w2) + 2 w3) + w4) / 6, z), w_k sampled at the k-th stage position). */
void ra_advect_z(const float* F, const float* Gw_, int Gh, int Gw, int H, int W, int n, const float* x1,
                 const float* y1, const float* z1, float dt, int substeps, int rk4, float* z2)
{
    const float sx = (float)Gw / (float)W;
    const float sy = (float)Gh / (float)H;
    const float h = dt / (float)substeps;
    const float hh = h * 0.5f;
    for (int i = 0; i < n; ++i) {
        float px = x1[i], py = y1[i], pz = z1[i];
        for (int s = 0; s < substeps; ++s) {
            if (!rk4) {
                float u, v;
                sample(F, Gh, Gw, sx, sy, px, py, &u, &v);
                float w = sample_scalar(Gw_, Gh, Gw, sx, sy, px, py);
                px = fmaf(h, u, px);
                py = fmaf(h, v, py);
                pz = fmaf(h, w, pz);
            } else {
                float k1u, k1v, k2u, k2v, k3u, k3v, k4u, k4v;
                sample(F, Gh, Gw, sx, sy, px, py, &k1u, &k1v);
                float w1 = sample_scalar(Gw_, Gh, Gw, sx, sy, px, py);
                float ax = fmaf(hh, k1u, px), ay = fmaf(hh, k1v, py);
                sample(F, Gh, Gw, sx, sy, ax, ay, &k2u, &k2v);
                float w2 = sample_scalar(Gw_, Gh, Gw, sx, sy, ax, ay);
                float bx = fmaf(hh, k2u, px), by = fmaf(hh, k2v, py);
                sample(F, Gh, Gw, sx, sy, bx, by, &k3u, &k3v);
                float w3 = sample_scalar(Gw_, Gh, Gw, sx, sy, bx, by);
                float cx = fmaf(h, k3u, px), cy = fmaf(h, k3v, py);
                sample(F, Gh, Gw, sx, sy, cx, cy, &k4u, &k4v);
                float w4 = sample_scalar(Gw_, Gh, Gw, sx, sy, cx, cy);
                float su = ((k1u + 2.0f * k2u) + 2.0f * k3u) + k4u;
                float sv = ((k1v + 2.0f * k2v) + 2.0f * k3v) + k4v;
                float sw = ((w1 + 2.0f * w2) + 2.0f * w3) + w4;
                px = fmaf(h, su / 6.0f, px);
                py = fmaf(h, sv / 6.0f, py);
                pz = fmaf(h, sw / 6.0f, pz);
            }
        }
        z2[i] = pz;
    }
}

/* Ground-truth flow field: the (u, v) grid sampled at every pixel centre
 * (c + 1/2, r + 1/2), as the advection samples it; out [H][W][2]. */
void ra_flow_field(const float* F, int Gh, int Gw, int H, int W, float* out)
{
    const float sx = (float)Gw / (float)W;
    const float sy = (float)Gh / (float)H;
    for (int r = 0; r < H; ++r)
        for (int c = 0; c < W; ++c) {
            float u, v;
            sample(F, Gh, Gw, sx, sy, (float)c + 0.5f, (float)r + 0.5f, &u, &v);
            out[2 * ((size_t)r * W + c)] = u;
            out[2 * ((size_t)r * W + c) + 1] = v;
        }
}
