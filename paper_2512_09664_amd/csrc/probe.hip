// Peak-rate probes for the roofline figures: small kernels whose work per
// launch is known exactly, timed by the caller.  They measure what the chip
// sustains for the instruction classes the generator's kernels use (16-byte
// stores to HBM, float32 FMA, the transcendental unit, the 32x32 -> 64-bit
// integer multiply of the Philox rounds), so that a kernel's fraction of peak
// is taken against a measured ceiling as well as the datasheet one.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace sp {
namespace {

constexpr int PROBE_CHAINS = 8;     // independent dependency chains per thread

typedef unsigned int vec4u __attribute__((ext_vector_type(4)));

// Streaming store of zeros: each workgroup writes 16 KiB runs (four 16-byte
// vectors per thread, the workgroup's 4 KiB rows one after another), grid-stride
// over the runs; NT: non-temporal stores (no cache allocation).
template <bool NT>
__global__ void __launch_bounds__(256) probe_store(uint4* __restrict__ dst, size_t n16)
{
    const size_t run = 4 * 256;
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (size_t b = (size_t)blockIdx.x * run; b < n16; b += (size_t)gridDim.x * run) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const size_t i = b + (size_t)k * 256 + threadIdx.x;
            if (i < n16) {
                if (NT) __builtin_nontemporal_store(vec4u{0u, 0u, 0u, 0u}, reinterpret_cast<vec4u*>(dst + i));
                else dst[i] = z;
            }
        }
    }
}

// Streaming copy of the first half of the buffer into the second half.
__global__ void __launch_bounds__(256) probe_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n16)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

// PROBE_CHAINS chains of `iters` dependent float32 FMAs per thread.  The
// result is stored only if it equals a value it never takes, so nothing is
// optimised away and nothing is written.
__global__ void __launch_bounds__(256) probe_fma(float* __restrict__ sink, int iters, float a, float b)
{
    float v[PROBE_CHAINS];
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) v[k] = (float)(threadIdx.x + k) * 1e-3f;
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < PROBE_CHAINS; ++k) v[k] = __builtin_fmaf(v[k], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) s += v[k];
    if (s == -1.0f) sink[threadIdx.x] = s;
}

// Transcendental chains: per iteration and chain one v_sin_f32 (argument in
// revolutions; values stay in [-1, 1]).
__global__ void __launch_bounds__(256) probe_trans(float* __restrict__ sink, int iters)
{
    float v[PROBE_CHAINS];
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) v[k] = (float)(threadIdx.x + k) * 1e-3f;
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < PROBE_CHAINS; ++k) v[k] = __builtin_amdgcn_sinf(v[k]);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) s += v[k];
    if (s == -100.0f) sink[threadIdx.x] = s;
}

// Integer multiply chains: per iteration and chain one 32 x 32 -> 64-bit
// product (v_mad_u64_u32, the Philox round's multiply), its halves folded back
// by a xor: two VALU instructions per chain and iteration.
__global__ void __launch_bounds__(256) probe_mul64(uint32_t* __restrict__ sink, int iters, uint32_t m)
{
    uint32_t v[PROBE_CHAINS];
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) v[k] = threadIdx.x * 2654435761u + k;
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < PROBE_CHAINS; ++k) {
            const uint64_t p = (uint64_t)v[k] * m;
            v[k] = (uint32_t)p ^ (uint32_t)(p >> 32);
        }
    }
    uint32_t s = 0u;
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) s ^= v[k];
    if (s == 0x9e3779b9u) sink[threadIdx.x] = s;
}

// Mixed chains in the proportions of the renderer's inner loops: per
// iteration and chain nine VALU instructions as compiled for gfx950 (one
// float32 FMA, two multiplies, a float -> u32 and a u32 -> float conversion,
// an integer add, a shift, a xor and a three-input bit operation).
__global__ void __launch_bounds__(256) probe_mix(uint32_t* __restrict__ sink, int iters, float a)
{
    float v[PROBE_CHAINS];
    uint32_t u[PROBE_CHAINS];
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) {
        v[k] = (float)(threadIdx.x + k) * 1e-3f;
        u[k] = threadIdx.x * 2654435761u + k;
    }
#pragma unroll 2
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < PROBE_CHAINS; ++k) {
            const float w = __builtin_fmaf(v[k], a, 0.5f) * 0.75f;
            const uint32_t q = (uint32_t)w;
            u[k] = (u[k] + q) ^ (u[k] >> 3);
            v[k] = (float)(u[k] & 0xffffu) * 1e-5f;
        }
    }
    uint32_t s = 0u;
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) s ^= u[k];
    if (s == 0x9e3779b9u) sink[threadIdx.x] = s;
}

// 32-bit integer chains: per iteration and chain an add, a shift and a xor;
// gfx950 code for two iterations of the eight chains is 40 VALU instructions
// (v_add_u32, v_lshlrev_b32, v_xor_b32 and the fused v_xad_u32): 2.5 per
// iteration and chain.
__global__ void __launch_bounds__(256) probe_int(uint32_t* __restrict__ sink, int iters, uint32_t k)
{
    uint32_t u[PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) u[c] = threadIdx.x * 2654435761u + c;
#pragma unroll 2
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < PROBE_CHAINS; ++c) {
            const uint32_t t = u[c] + k;
            u[c] = t ^ (t << 5);
        }
    }
    uint32_t s = 0u;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) s ^= u[c];
    if (s == 0x9e3779b9u) sink[threadIdx.x] = s;
}

}  // namespace

// Enqueues one probe; *work gets the launch's unit count: bytes moved to or
// from HBM (store, store_nt: written bytes; copy: read + written), or the wave64 VALU
// instructions of the probe's loop (fma: FMAs; trans: v_sin; mul64: the
// multiply and xor pairs).  iters must be a multiple of 4 (the loops are
// unrolled by four).
hipError_t launch_probe(int kind, void* buf, size_t bytes, int iters, hipStream_t s, double* work)
{
    const int cus = device_cu_count();
    switch (kind) {
    case 0: case 5: {
        const size_t n16 = bytes / 16;
        const unsigned grid = (unsigned)std::min<size_t>((n16 + 1023) / 1024, (size_t)cus * 16);
        if (kind == 0) {
            TimedScope ts("probe_store", s);
            hipLaunchKernelGGL(probe_store<false>, dim3(grid), dim3(256), 0, s, static_cast<uint4*>(buf), n16);
        } else {
            TimedScope ts("probe_store_nt", s);
            hipLaunchKernelGGL(probe_store<true>, dim3(grid), dim3(256), 0, s, static_cast<uint4*>(buf), n16);
        }
        *work = (double)(n16 * 16);
        break;
    }
    case 1: {
        const size_t n16 = bytes / 32;
        const unsigned grid = (unsigned)std::min<size_t>((n16 + 255) / 256, (size_t)cus * 32);
        uint4* b = static_cast<uint4*>(buf);
        TimedScope ts("probe_copy", s);
        hipLaunchKernelGGL(probe_copy, dim3(grid), dim3(256), 0, s, b, b + n16, n16);
        *work = (double)(n16 * 32);
        break;
    }
    case 2: case 3: case 4: case 6: case 7: {
        // 8 waves per SIMD on every CU: 8 workgroups of 4 waves per CU
        const unsigned grid = (unsigned)cus * 8;
        const double waves = (double)grid * 4.0;
        *work = waves * (double)iters * PROBE_CHAINS * (kind == 4 ? 2.0 : kind == 6 ? 9.0 : kind == 7 ? 2.5 : 1.0);
        if (kind == 2) {
            TimedScope ts("probe_fma", s);
            hipLaunchKernelGGL(probe_fma, dim3(grid), dim3(256), 0, s, static_cast<float*>(buf), iters, 0.999f,
                               1e-3f);
        } else if (kind == 3) {
            TimedScope ts("probe_trans", s);
            hipLaunchKernelGGL(probe_trans, dim3(grid), dim3(256), 0, s, static_cast<float*>(buf), iters);
        } else if (kind == 7) {
            TimedScope ts("probe_int", s);
            hipLaunchKernelGGL(probe_int, dim3(grid), dim3(256), 0, s, static_cast<uint32_t*>(buf), iters, 0x9E3779B9u);
        } else if (kind == 6) {
            TimedScope ts("probe_mix", s);
            hipLaunchKernelGGL(probe_mix, dim3(grid), dim3(256), 0, s, static_cast<uint32_t*>(buf), iters, 0.999f);
        } else {
            TimedScope ts("probe_mul64", s);
            hipLaunchKernelGGL(probe_mul64, dim3(grid), dim3(256), 0, s, static_cast<uint32_t*>(buf), iters,
                               0xD2511F53u);
        }
        break;
    }
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sp
