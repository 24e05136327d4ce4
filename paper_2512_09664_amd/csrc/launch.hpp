// Kernel launchers shared between the kernel translation units and the C ABI.
#pragma once

#include <cmath>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "device_math.hpp"
#include "synthpix.h"

namespace sp {

// RAII bracket of one kernel launch with timing events (no-op unless enabled).
class TimedScope {
public:
    TimedScope(const char* name, hipStream_t s);
    ~TimedScope();
    TimedScope(const TimedScope&) = delete;
    TimedScope& operator=(const TimedScope&) = delete;
private:
    const char* name_;
    hipStream_t stream_;
    hipEvent_t start_;
};
void timing_enable(bool on);
int timing_read(const char* name, double* total_ms, int64_t* launches);

// Per-pair derived sizes of one render call (computed identically on host
// and device from the pair table and the tiling).
struct PairLayout {
    int32_t chunk_base;     // first binning block of the pair (prefix over pairs)
    int32_t n_chunks;       // ceil(n_max / chunk)
    int32_t tile_base;      // first tile of the pair (prefix over pairs)
    int32_t ntx, nty;       // tiles per row / column
    int32_t pad_;
    int64_t hist_base;      // first per-(frame, chunk, tile) count of the pair
    int64_t entry_base;     // first entry slot of the pair (frame 2 at + entry_cap)
    int64_t entry_cap;      // entry slots per frame
};

// Pair owning a (flattened) tile index.
__device__ __forceinline__ int find_pair_by_tile(const PairLayout* L, int n_pairs, int64_t t)
{
    int lo = 0, hi = n_pairs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L[mid].tile_base <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

struct RenderConfig {
    int tile_w, tile_h, chunk, cap;
    int log_tw, log_th;     // tile sizes are powers of two
    int apron;              // blur radius b
    int wmax;               // largest per-particle patch side the LDS tables hold
    int wm4;                // wmax rounded up to a multiple of 4 (row stride of the tables)
    int kx, ky;             // bound on tiles touched per particle per axis
    float d_max;
    int persistent;         // renderer grid capped at the device's resident workgroups
};

// Totals of a batch (host side).
// Tile rectangle touched by one particle record: its support, clipped to the
// image, grown by the blur apron.  False when the particle adds nothing.
// A particle's patch in image pixels, clipped to the image: columns c0 .. c1 in
// the low and high halves of .x, rows r0 .. r1 in those of .y.  A particle that
// adds nothing has c1 < c0 (EMPTY_BOX).
constexpr uint32_t EMPTY_BOX = 1u;

__device__ __forceinline__ uint2 patch_box(float x, float y, float Rx, float Ry, int W, int H)
{
    int c0, c1, r0, r1;
    if (!support_range(x, Rx, W, c0, c1) || !support_range(y, Ry, H, r0, r1)) return make_uint2(EMPTY_BOX, EMPTY_BOX);
    return make_uint2((uint32_t)c0 | ((uint32_t)c1 << 16), (uint32_t)r0 | ((uint32_t)r1 << 16));
}

__device__ __forceinline__ bool box_empty(uint2 b) { return (b.x >> 16) < (b.x & 0xffffu); }

// Tile rectangle touched by one particle's patch box, grown by the blur apron.
// False when the particle adds nothing.
__device__ __forceinline__ bool tile_rect(const uint2 bx, const RenderConfig& cfg, int ntx, int nty, int& tx0,
                                          int& tx1, int& ty0, int& ty1)
{
    if (box_empty(bx)) return false;
    const int c0 = (int)(bx.x & 0xffffu), c1 = (int)(bx.x >> 16);
    const int r0 = (int)(bx.y & 0xffffu), r1 = (int)(bx.y >> 16);
    const int b = cfg.apron;
    tx0 = c0 - b < 0 ? 0 : (c0 - b) >> cfg.log_tw;
    ty0 = r0 - b < 0 ? 0 : (r0 - b) >> cfg.log_th;
    tx1 = (c1 + b) >> cfg.log_tw;
    ty1 = (r1 + b) >> cfg.log_th;
    tx1 = tx1 > ntx - 1 ? ntx - 1 : tx1;
    ty1 = ty1 > nty - 1 ? nty - 1 : ty1;
    return true;
}

struct BatchTotals {
    int64_t n_span;         // max(particle_offset + n_max)
    int64_t chunks;         // sum n_chunks
    int64_t tiles;          // sum ntx * nty
    int64_t hist;           // 2 * sum n_chunks * tiles
    int64_t entries;        // 2 * sum entry_cap
    int64_t max_tiles;      // max ntx * nty over pairs (LDS histogram size)
};

// Workspace layout (byte offsets, 256-aligned).
struct WorkspaceLayout {
    size_t status;          // uint32 [4]
    size_t layout;          // PairLayout [n_pairs]
    size_t tile_count;      // uint32 [2 * tiles]
    size_t tile_offset;     // int64  [2 * tiles]
    size_t hist;            // uint32 [hist]
    size_t entries;         // int32  [entries]
    size_t records;         // float4 [2 * n_span] per-frame particle records (x, y, kappa_x, 2^24 A)
    size_t boxes;           // uint2 [2 * n_span] per-frame patch boxes in image pixels
    size_t shapes;          // float2 [2 * n_span] per-frame (kappa_y, kappa_xy) of the anisotropic model
    size_t total;
};

// Workspace of the spatial order used by the advection kernels: a pair layout,
// per-block counts and offsets, per-chunk histograms and one entry per particle.
struct OrderLayout {
    size_t status, layout, tile_count, tile_offset, hist, entries, total;
};

// A captured plan's kernels read their buffers, draw key and pair-id offset from
// a device-side descriptor (iod); eager calls pass the buffers directly and a
// null descriptor.
hipError_t launch_order(const synthpix_pair* pairs_dev, int n_pairs, const float* x, const float* y,
                        const RenderConfig& cfg, const BatchTotals& tot, char* ws, const OrderLayout& ol,
                        hipStream_t s, const synthpix_batch_io* iod = nullptr, const int32_t* live = nullptr);

// The order a launch of the advection kernel follows (null: particle index order).
struct AdvectOrder {
    const PairLayout* L;
    const int32_t* entries;
    int log_block;              // home blocks are 2^log_block pixels square
    int64_t blocks;             // home blocks over all pairs
    const uint32_t* count;      // particles per home block
    const int64_t* offset;      // first entry of each home block
    const int32_t* live;        // per pair: only slots below this are ordered and advected (null: all n_max)
};

hipError_t launch_seed(const synthpix_pair* pairs_dev, int n_pairs, int64_t n_span,
                       const synthpix_seed_params& prm, uint64_t seed, float* x, float* y, float* z,
                       float* d, float* I0, int32_t* n_active, double* ppp, hipStream_t s,
                       const synthpix_batch_io* iod = nullptr, int32_t* live = nullptr);

// Moves a descriptor's pair_id_base on by `step` (the next batch of pairs).
hipError_t launch_advance(synthpix_batch_io* iod, uint64_t step, hipStream_t s);

// Stores *io into the device-side descriptor (one thread; the value travels as
// a kernel argument, so the call is stream-ordered and io may be reused at once).
hipError_t launch_store_io(synthpix_batch_io* iod, const synthpix_batch_io& io, hipStream_t s);

hipError_t launch_advect(const synthpix_pair* pairs_dev, int n_pairs, int64_t n_span, const float* flow,
                         const synthpix_advect_params& ap, const float* x1, const float* y1, float* x2,
                         float* y2, hipStream_t s, AdvectOrder order = AdvectOrder{nullptr, nullptr},
                         const synthpix_batch_io* iod = nullptr);

// Second diameter and correlation per candidate particle (Philox stream 6).
hipError_t launch_seed_shape(const synthpix_pair* pairs_dev, int n_pairs, int64_t n_span,
                             const synthpix_seed_params& prm, float rho_lo, float rho_hi, uint64_t seed, float* dy,
                             float* rho, hipStream_t s);

// Three-dimensional motion: (x2, y2, z2) under the (u, v) grid and the w grid.
hipError_t launch_advect3(const synthpix_pair* pairs_dev, int n_pairs, int64_t n_span, const float* flow,
                          const float* wflow, const synthpix_advect_params& ap, const float* x1, const float* y1,
                          const float* z1, float* x2, float* y2, float* z2, hipStream_t s);

struct RenderArgs {
    const synthpix_pair* pairs;
    int n_pairs;
    const float* x[2];
    const float* y[2];
    const float* z;
    const float* d;
    const float* I0;
    void* images;
    float sheet_sigma;
    float noise_sigma;
    int bits;
    uint64_t seed;
    float blur_w[7];
    const synthpix_batch_io* iod;   // captured plans: buffers, key and pair-id offset (else null)
    const int32_t* live;            // captured plans: each pair's active count; the masked slots past
                                    // it are neither prepared nor binned (else null: every slot)
    // the full particle model (all zero / null: the isotropic Gaussian-sheet path)
    const float* dy;                // second diameter per particle (null: d)
    const float* rho;               // correlation per particle (null: 0)
    const float* z2;                // frame-2 out-of-plane position (null: z)
    float hide_p;                   // per-frame hiding probability
    float jit_d, jit_rho, jit_I0;   // std of the frame-2 parameter changes
    int sheet_law;                  // 0 Gaussian sheet, 1 Remark 1
    float sheet_dz0, sheet_shape;   // Remark 1: thickness and shape factor
    bool model;                     // any of the above in use (the model's prep kernel runs)
    bool aniso;                     // shape records in use (d_y != d or rho != 0 possible)
};

// What the tile renderer's epilogue needs (kept small: kernel arguments live in SGPRs).
struct EpilogueArgs {
    void* images;
    uint64_t seed;
    float noise_sigma;
    int bits;
    float blur_w[7];
    const synthpix_batch_io* iod;
};

// Particle records and tile lists of both frames (layout, prep, count, scan,
// scatter): what the tile renderer and the tile-major backward read.
hipError_t launch_bins(const RenderArgs& a, const RenderConfig& cfg, const BatchTotals& tot, char* ws,
                       const WorkspaceLayout& wl, hipStream_t s);

size_t render_lds_bytes(const RenderConfig& cfg, bool aniso = false);
bool render_shape_supported(int tile_w, int tile_h);

hipError_t launch_render(const RenderArgs& a, const RenderConfig& cfg, const BatchTotals& tot,
                         char* ws, const WorkspaceLayout& wl, hipStream_t s);

// Most particle slices per pair of the backward's bound and sheet-sum pass.
constexpr int BWD_SLICES = 128;

// Everything the backward kernels read and write.
// Flow-grid gradient without global atomics: the flow adjoint runs one
// workgroup per 256 particles of one pair; each accumulates its node sums (64-bit
// fixed point) in an LDS window and writes the window's nonzero box to its own
// partial (and any contribution outside the window as a record); a reduction
// then adds, per node, the partials and records of the pair's workgroups.
constexpr int WIN_NODES = 2048;      // LDS window capacity (nodes; 32 KB of (u, v) sums)
constexpr int GRID_OVF_CAP = 512;    // records per workgroup for nodes outside its window

struct GridHeader {
    int32_t i0, j0;                  // first node row / column of the partial's box
    int32_t h, w;                    // box rows / columns (0: no partial)
    uint32_t n_ovf;                  // records written (<= GRID_OVF_CAP)
    uint32_t pad_[3];
};

struct GridRecord {
    int32_t elem;                    // 2 (i Gw + j) + component in the pair's grid
    uint32_t pad_;
    unsigned long long value;        // fixed-point contribution
};

struct GridAccum {
    int64_t* wg_base;                // [n_pairs + 1] first workgroup of each pair
    GridHeader* head;                // [n_wg]
    unsigned long long* part;        // [n_wg][2 WIN_NODES]
    GridRecord* ovf;                 // [n_wg][GRID_OVF_CAP]
    int64_t n_wg;                    // sum over pairs of ceil(n_max / 256)
    int max_gh, max_gw;              // largest grid of the batch (nodes)
};

struct BwdArgs {
    AdvectOrder order;           // home-block order of the frame-1 positions
    AdvectOrder order2;          // the same for the frame-2 positions (tile gather only)
    float4* parts;               // per-frame particle sums (S0, Sx, Sy, Sr), 2 x n_span (tile gather only)
    const synthpix_pair* pairs;
    int n_pairs;
    const float* flow;
    const float* x1;
    const float* y1;
    const float* x2;             // frame-2 positions: the caller's, or the recomputed ones
    const float* y2;
    float* x2w;                  // recomputed frame-2 positions (workspace)
    float* y2w;
    bool recompute_x2;
    const float* z;
    const float* d;
    const float* I0;
    const float* grad;           // dL/dJ, the images' layout (unless mse)
    // mse: dL/dJ = mse_scale (J - T) is formed from the float images J and the
    // target T (the images' layout) by the per-pixel pass, which also writes
    // float64 partial sums of (J - T)^2 to loss_part when loss is non-null;
    // *loss = their sum / loss_n
    bool mse;
    const float* J;
    const float* T;
    float mse_scale;
    double* loss_part;
    double* loss;
    int64_t loss_n;
    float* eblur;                // B^T dL/dJ (workspace, the images' layout): blur radius >= 2, the
                                 // tile gather, or the mse form
    float* g_x1;
    float* g_y1;
    float* g_z;
    float* g_d;
    float* g_I0;
    float* g_sheet;
    float* g_sheet_total;        // optional (null): the sum over pairs
    float* g_flow;
    float* gx2;                  // dL/dx2, dL/dy2 (workspace)
    float* gy2;
    float* sheet;                // per-particle sheet-width terms (workspace)
    double* sheet_part;          // per (pair, slice) float64 sums of those terms (workspace)
    float* bound_part;           // per (pair, slice) max |dL/dx2| and Lipschitz bound (workspace)
    GridAccum grid;              // flow-gradient partials (workspace)
    uint32_t* scale;             // fixed-point scale block: max |dL/dx2|, Lipschitz bound, exponent, state
    uint32_t* status;
    float sheet_sigma;
    float d_max;
    float blur_w[7];
    int max_h, max_w;            // largest pair height and width of the batch
};

hipError_t launch_backward(const BwdArgs& a, int64_t n_span, int64_t n_flow, const synthpix_advect_params& ap,
                           int blur, int en, hipStream_t s);

// Rows per strip of the backward's per-pixel pass, and its workgroups over a
// batch whose largest pair is max_h x max_w (the loss partials of the
// loss-fused form, one each).
constexpr int blur_strip_rows(bool mse) { return mse ? 16 : 24; }
int64_t blur_grad_blocks(int n_pairs, int max_w, int max_h, bool mse);

// Image loss gradient grad = scale (J - T) and, with loss, the mean of (J - T)^2
// (float64 partials of MSE_BLOCKS workgroups in part, summed in a fixed order).
constexpr int MSE_BLOCKS = 1024;
hipError_t launch_mse_grad(const float* J, const float* T, int64_t n, float scale, float* grad, double* loss,
                           double* part, hipStream_t s);

// Halo (pixels) of the tile-major adjoint gather's staged region for a diameter
// bound: every in-image pixel of a footprint whose centre lies in a home block
// is within this distance of the block.
inline int tile_halo(float d_max) { return (int)std::ceil(1.5f * d_max) + 2; }

// Whether the tile-major gather serves a batch: a blur of radius >= 2 (whose
// adjoint then runs once per pixel; narrower blurs fold into the particle-major
// gather's tables, which costs less than staging and the second order), factor
// tables that hold the support (3 d_max + 4 slots <= 32) and a staged region of
// a home block of 2^log_block pixels within 64 KB of LDS.
inline bool tile_gather_fits(float d_max, int log_block, int blur_radius)
{
    if (blur_radius < 2 || !((int)(3.0f * d_max) + 4 <= 32)) return false;
    const int rw = (1 << log_block) + 2 * tile_halo(d_max);
    return (size_t)rw * rw * sizeof(float) <= 64 * 1024;
}

// Peak-rate probes (store, copy, fma, trans, mul64, store_nt = kinds 0..5); *work gets
// the launch's bytes or wave64 instructions.
hipError_t launch_probe(int kind, void* buf, size_t bytes, int iters, hipStream_t s, double* work);

// Ground-truth flow fields: each pair's grid sampled at its pixel centres.
hipError_t launch_flow_field(const synthpix_pair* pairs_dev, int n_pairs, int64_t max_px, const float* flow, float* out,
                             hipStream_t s);

// Histogram adjustment of uint16 images (bits 1..14): workspace bytes and launch.
size_t hist_workspace_bytes(int n_pairs, int bits);
hipError_t launch_histogram_match(const synthpix_pair* pairs_dev, int n_pairs, int64_t max_pixels, int bits,
                                  const uint32_t* target, uint16_t* images, char* ws, hipStream_t s);

// Compute units of the current device (cached per device).
int device_cu_count();

}  // namespace sp
