// Histogram adjustment of the stored images (Section 2, after Remark 2: the
// output may be remapped so that its intensities follow a histogram the user
// chooses), gfx950.
//
// Histogram specification of every stored image (each frame of each pair, its
// integer codes) to one target histogram t[0 .. B - 1], B = 2^bits: with the
// image's cumulative counts S(k) (N pixels) and the target's T(m) (total
// T_tot), code k becomes the smallest m with T(m) N >= S(k) T_tot.  Everything
// is integer arithmetic (T_tot < 2^32 and N < 2^31, so both products fit in 64
// bits), so the result is exact and independent of the launch shape.  bits is
// at most 14: a workgroup holds one image's histogram (64 KB) and both
// cumulative tables (128 KB) in LDS.
//
//   hist_clear : zero the per-image histograms
//   hist_count : per (image, pixel chunk) LDS histogram, flushed with one
//                global atomic per non-empty bin
//   hist_lut   : per image, the prefix sums of its histogram and of the target
//                in LDS and a binary search per code -> look-up table
//   hist_apply : every pixel through its image's table
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace sp {
namespace {

constexpr int HIST_CHUNK = 256 * 64;    // pixels per counting / applying workgroup

__device__ __forceinline__ void image_of(const synthpix_pair* __restrict__ pairs, int img, int64_t& off, int64_t& n)
{
    const synthpix_pair P = pairs[img >> 1];
    n = (int64_t)P.H * P.W;
    off = P.image_offset + (img & 1) * n;
}

__global__ void __launch_bounds__(256) hist_clear(uint32_t* __restrict__ h, int64_t n, uint32_t* __restrict__ status)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) status[0] = 0u;
    if (i < n) h[i] = 0u;
}

__global__ void __launch_bounds__(256)
hist_count(const synthpix_pair* __restrict__ pairs, const uint16_t* __restrict__ images, int B,
           uint32_t* __restrict__ hist, uint32_t* __restrict__ status)
{
    extern __shared__ uint32_t lh[];
    const int img = blockIdx.y;
    int64_t off, n;
    image_of(pairs, img, off, n);
    const int64_t c0 = (int64_t)blockIdx.x * HIST_CHUNK;
    if (c0 >= n) return;
    for (int b = threadIdx.x; b < B; b += 256) lh[b] = 0u;
    __syncthreads();
    const int64_t c1 = c0 + HIST_CHUNK < n ? c0 + HIST_CHUNK : n;
    bool wide = false;
    for (int64_t i = c0 + threadIdx.x; i < c1; i += 256) {
        int v = images[off + i];
        if (v >= B) {
            wide = true;
            v = B - 1;
        }
        atomicAdd(&lh[v], 1u);
    }
    if (wide) atomicOr(status, SP_STATUS_HIST_CODE);
    __syncthreads();
    uint32_t* g = hist + (int64_t)img * B;
    for (int b = threadIdx.x; b < B; b += 256)
        if (lh[b]) atomicAdd(&g[b], lh[b]);
}

// In-place inclusive scan of s[0 .. Bp) (Bp a multiple of 256) over 256
// threads: each thread sums its run of Bp / 256 entries, a workgroup scan of
// the run totals, then each run adds its offset.
__device__ void block_scan(uint32_t* s, int Bp, uint32_t* part)
{
    const int t = threadIdx.x, per = Bp / 256;
    uint32_t run = 0;
    for (int k = 0; k < per; ++k) run += s[t * per + k];
    part[t] = run;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t v = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t acc = part[t] - run;
    for (int k = 0; k < per; ++k) {
        acc += s[t * per + k];
        s[t * per + k] = acc;
    }
    __syncthreads();
}

// One workgroup per image.  The target's total is summed in 64 bits first; with
// it below 2^32 every cumulative count fits 32 bits (the image's: N < 2^31).
__global__ void __launch_bounds__(256)
hist_lut(const synthpix_pair* __restrict__ pairs, const uint32_t* __restrict__ target, int B,
         const uint32_t* __restrict__ hist, uint16_t* __restrict__ lut, uint32_t* __restrict__ status)
{
    extern __shared__ uint32_t ls[];
    const int Bp = B < 256 ? 256 : B;
    uint32_t* S = ls;           // [Bp] image cumulative counts
    uint32_t* T = ls + Bp;      // [Bp] target cumulative counts
    __shared__ uint32_t part[256];
    __shared__ unsigned long long s_tot;
    const int img = blockIdx.x;
    int64_t off, n;
    image_of(pairs, img, off, n);
    unsigned long long tsum = 0;
    for (int b = threadIdx.x; b < B; b += 256) tsum += target[b];
    if (threadIdx.x == 0) s_tot = 0ull;
    __syncthreads();
    atomicAdd(&s_tot, tsum);
    __syncthreads();
    const unsigned long long Tt = s_tot;
    uint16_t* out = lut + (int64_t)img * B;
    if (Tt == 0ull || Tt >= (1ull << 32)) {
        // no usable target: the images stay as they are
        if (threadIdx.x == 0) atomicOr(status, SP_STATUS_HIST_TARGET);
        for (int b = threadIdx.x; b < B; b += 256) out[b] = (uint16_t)b;
        return;
    }
    const uint32_t* h = hist + (int64_t)img * B;
    for (int b = threadIdx.x; b < Bp; b += 256) {
        S[b] = b < B ? h[b] : 0u;
        T[b] = b < B ? target[b] : 0u;
    }
    __syncthreads();
    block_scan(S, Bp, part);
    block_scan(T, Bp, part);
    const unsigned long long N = (unsigned long long)n;
    for (int k = threadIdx.x; k < B; k += 256) {
        const unsigned long long need = (unsigned long long)S[k] * Tt;     // < 2^31 * 2^32
        int lo = 0, hi = B - 1;                                             // T[B - 1] N >= S[k] Tt holds
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((unsigned long long)T[mid] * N >= need) hi = mid; else lo = mid + 1;
        }
        out[k] = (uint16_t)lo;
    }
}

__global__ void __launch_bounds__(256)
hist_apply(const synthpix_pair* __restrict__ pairs, uint16_t* __restrict__ images, int B,
           const uint16_t* __restrict__ lut)
{
    const int img = blockIdx.y;
    int64_t off, n;
    image_of(pairs, img, off, n);
    const int64_t c0 = (int64_t)blockIdx.x * HIST_CHUNK;
    if (c0 >= n) return;
    const int64_t c1 = c0 + HIST_CHUNK < n ? c0 + HIST_CHUNK : n;
    const uint16_t* L = lut + (int64_t)img * B;
    for (int64_t i = c0 + threadIdx.x; i < c1; i += 256) {
        const int v = images[off + i];
        images[off + i] = L[v < B ? v : B - 1];
    }
}

}  // namespace

size_t hist_workspace_bytes(int n_pairs, int bits)
{
    const size_t B = (size_t)1 << bits, nimg = 2 * (size_t)n_pairs;
    return 256 + ((nimg * B * 4 + 255) & ~(size_t)255) + ((nimg * B * 2 + 255) & ~(size_t)255);
}

hipError_t launch_histogram_match(const synthpix_pair* pairs_dev, int n_pairs, int64_t max_pixels, int bits,
                                  const uint32_t* target, uint16_t* images, char* ws, hipStream_t s)
{
    const int B = 1 << bits;
    const int nimg = 2 * n_pairs;
    uint32_t* status = reinterpret_cast<uint32_t*>(ws);
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws + 256);
    uint16_t* lut = reinterpret_cast<uint16_t*>(ws + 256 + (((size_t)nimg * B * 4 + 255) & ~(size_t)255));
    const int64_t nh = (int64_t)nimg * B;
    const dim3 grid((unsigned)((max_pixels + HIST_CHUNK - 1) / HIST_CHUNK), (unsigned)nimg);
    TimedScope ts("histogram_match", s);
    hipLaunchKernelGGL(hist_clear, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0, s, hist, nh, status);
    hipLaunchKernelGGL(hist_count, grid, dim3(256), (size_t)B * 4, s, pairs_dev, images, B, hist, status);
    hipLaunchKernelGGL(hist_lut, dim3((unsigned)nimg), dim3(256), (size_t)(B < 256 ? 256 : B) * 8, s, pairs_dev,
                       target, B, hist, lut, status);
    hipLaunchKernelGGL(hist_apply, grid, dim3(256), 0, s, pairs_dev, images, B, lut);
    return hipGetLastError();
}

}  // namespace sp
