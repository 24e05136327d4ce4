/*
 * synthpix.h -- C ABI of the MI355X (gfx950) synthetic PIV image-pair generator.
 *
 * The generator follows SynthPix (Terpin, Bonomi, Banelli, D'Andrea):
 *   - particles are allocated for the largest seeding density, the pair's ppp is
 *     drawn uniformly and the excess particles are masked with zero intensity
 *     (Section 2, "Sampling the particles");
 *   - frame-2 particles are frame-1 particles moved by the flow (same passage);
 *   - each particle adds I0 * exp(-8 r^2 / d^2) (Eq. 1 with rho = 0 and
 *     sigma_x = sigma_y = d / 4), times a laser-sheet profile exp(-z^2 / (2 s^2))
 *     (Remark 1 defers the paper's own sheet law), on a square patch of side at
 *     most 3 d + 1 pixels (Section 2, "Efficient rasterization"), and the image
 *     is the plain sum (Section 2, "Considerations on the aggregation");
 *   - blur, noise and storage depth are acquisition parameters (Abstract, Section 1).
 *
 * Conventions.
 *   Images are row-major, H rows by W columns; pixel (r, c) is centred at
 *   (c + 0.5, r + 0.5); x points right, y down.  Positions and diameters are in
 *   pixels, z in laser-sheet units, intensities in full-scale units (1.0 = white),
 *   flows in pixels per frame on a cell-centred grid: node (i, j) sits at
 *   ((j + 0.5) W / Gw, (i + 0.5) H / Gh), stored as interleaved (u, v) floats
 *   [Gh][Gw][2].
 *   Particle data are structure-of-arrays float arrays indexed by
 *   pair.particle_offset + i, i < pair.n_max.
 *   Images are [pair][frame][H][W] at pair.image_offset (in elements of the
 *   output type): float when bits == 0, uint16 codes otherwise.
 *
 * Ownership and streams.
 *   The caller owns every buffer.  "dev" pointers are device pointers, "host"
 *   pointers are host pointers.  The library allocates nothing in these calls
 *   (scratch space comes from a caller-provided workspace sized by
 *   synthpix_workspace_size) except inside synthpix_plan_create.  Every call
 *   validates its arguments on the host before enqueuing anything, then
 *   enqueues its kernels asynchronously on `stream` (a hipStream_t; NULL is the
 *   null stream) and returns.  Host-side pair tables may be reused or freed as
 *   soon as the call returns; device-side ones must stay valid until the
 *   stream reaches the call.
 *
 * Errors.
 *   Every call returns a synthpix_status: SP_OK (0) or a negative code.  On an
 *   error nothing has been enqueued (argument errors) or the HIP error is
 *   reported (SP_ERR_HIP).  synthpix_last_error() returns a thread-local
 *   message describing the last failure.  No C++ exception crosses the ABI.
 *   Conditions only the device can see (a diameter above the declared d_max, a
 *   tile whose sum could leave the fixed-point range) are recorded as bits in a
 *   status word at the start of the workspace; synthpix_read_status returns it.
 *
 * Determinism.
 *   Outputs are a pure function of the inputs, the seed and each pair's pair_id.
 *   They do not depend on tiling, batching or the stream: particle contributions
 *   are summed in exact fixed point (2^-24 full-scale units, 32-bit), so any
 *   summation order gives the same bits.
 */
#ifndef SYNTHPIX_H
#define SYNTHPIX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SYNTHPIX_VERSION 4

typedef enum {
    SP_OK = 0,
    SP_ERR_INVALID_ARG = -1,   /* a pointer, size or parameter is out of its documented range */
    SP_ERR_WORKSPACE = -2,     /* workspace missing, misaligned or smaller than synthpix_workspace_size */
    SP_ERR_UNSUPPORTED = -3,   /* a configuration the kernels do not handle (e.g. too many tiles per image) */
    SP_ERR_HIP = -4,           /* a HIP runtime call failed (no device, launch failure, ...) */
    SP_ERR_DEVICE_STATUS = -5  /* synthpix_read_status found device-side flags */
} synthpix_status;

typedef enum { SP_EULER = 0, SP_RK4 = 1 } synthpix_integrator;
typedef enum { SP_DIST_UNIFORM = 0, SP_DIST_NORMAL_CLIPPED = 1 } synthpix_dist;

/* Device status bits (workspace word 0). */
#define SP_STATUS_D_ABOVE_MAX   0x1u   /* a particle had d (or d_y) > d_max; it was not rendered */
#define SP_STATUS_FIXED_RANGE   0x2u   /* the peaks of the particles covering one pixel row of a
                                          tile sum to >= 256 full scale: a pixel sum could have
                                          left the 32-bit fixed-point range */
#define SP_STATUS_BAD_SHAPE     0x4u   /* a particle had |rho| > 0.99; it was not rendered */
#define SP_STATUS_HIST_TARGET   0x8u   /* histogram adjustment: the target's total is 0 or >= 2^32;
                                          the images were left unchanged */
#define SP_STATUS_HIST_CODE     0x10u  /* histogram adjustment: a stored code >= 2^bits was taken
                                          as 2^bits - 1 */
#define SP_STATUS_GRID_OVERFLOW 0x20u  /* backward: a workgroup of 256 particles had more flow-grid
                                          contributions outside its node window than it keeps;
                                          g_flow is incomplete (the particles moved too far) */

/* Laser-sheet laws of the peak intensity. */
#define SP_SHEET_GAUSS   0   /* I0 exp(-z^2 / (2 s^2)), s = sheet_sigma                           */
#define SP_SHEET_REMARK1 1   /* I0 exp(-(1/sqrt(2 pi)) |2 z^2 / DZ0^2|^shape) (Remark 1, q = I0)   */

/* One image pair.  An array of these describes a batch, pairs of different size
 * included.  56 bytes, identical layout on host and device. */
typedef struct {
    int32_t  H, W;              /* image rows, columns (1 .. 16384)                         */
    int32_t  Gh, Gw;            /* flow grid rows, columns (2 .. 8192)                        */
    int32_t  n_max;             /* particles allocated for the pair (synthpix_particle_count) */
    int32_t  reserved;          /* must be 0                                                 */
    int64_t  particle_offset;   /* index of the pair's first particle in the SoA arrays      */
    int64_t  image_offset;      /* element offset of frame 1; frame 2 starts H*W later       */
    int64_t  flow_offset;       /* float offset of the pair's [Gh][Gw][2] flow grid          */
    uint64_t pair_id;           /* global pair index: Philox counter words 2 and 3           */
} synthpix_pair;

/* Seeding parameters (Section 2, "Sampling the particles"; the paragraph after Eq. 1). */
typedef struct {
    double  ppp_lo, ppp_hi;     /* seeding density range, particles per pixel, 0 < lo <= hi <= 1 */
    int32_t d_dist;             /* synthpix_dist                                                 */
    float   d_a, d_b;           /* uniform: d ~ U[d_a, d_b]; normal: mean d_a, std d_b           */
    float   d_lo, d_hi;         /* normal only: clip range                                      */
    float   I0_lo, I0_hi;       /* peak intensity range, full-scale units, 0 <= lo <= hi          */
    float   z_lo, z_hi;         /* out-of-plane position range, laser-sheet units               */
} synthpix_seed_params;

/* Inter-frame motion (Section 2, "Sampling the particles"; Euler, dt = 1, 1 substep
 * is the paper's x -> x + u(x)). */
typedef struct {
    float   dt;                 /* inter-frame time in frames, finite                 */
    int32_t substeps;           /* 1 .. 1024                                          */
    int32_t integrator;         /* synthpix_integrator                                */
} synthpix_advect_params;

/* Rendering and acquisition parameters. */
typedef struct {
    float    sheet_sigma;       /* Gaussian laser-sheet width s (> 0), sheet units             */
    float    d_max;             /* upper bound of every diameter passed in (0 < d_max <= 16)    */
    int32_t  blur_radius;       /* 0 (off) .. 3: taps -b..b                                      */
    float    blur_sigma;        /* > 0 when blur_radius > 0                                      */
    float    noise_sigma;       /* >= 0; additive N(0, sigma^2) full-scale units after the blur  */
    int32_t  bits;              /* 0: float images; 1..16: uint16 codes of that depth            */
    uint64_t seed;              /* key of the noise, frame-2 variation and hiding draws          */
    synthpix_advect_params advect;  /* used by the backward to recompute frame-2 positions  */
    /* The full particle model (all zero: the isotropic Gaussian-sheet path).  Frame 2
     * varies each particle parameter by a zero-mean Gaussian (the sentence after
     * Eq. 1): d and d_y by jitter_d (clipped to [0, d_max]), rho by jitter_rho
     * (clipped to [-0.99, 0.99]), I0 by jitter_I0 (clipped at 0; masked particles
     * stay dark).  Each particle is hidden (intensity 0) in each frame with
     * probability hide_p (Section 2, "Considerations on the aggregation"). */
    float    hide_p;            /* [0, 1]                                                         */
    float    jitter_d;          /* >= 0, pixels                                                   */
    float    jitter_rho;        /* >= 0                                                           */
    float    jitter_I0;         /* >= 0, full-scale units                                         */
    int32_t  sheet_law;         /* SP_SHEET_GAUSS or SP_SHEET_REMARK1                             */
    float    sheet_dz0;         /* SP_SHEET_REMARK1: laser-sheet thickness DZ0 (> 0)              */
    float    sheet_shape;       /* SP_SHEET_REMARK1: shape factor (> 0)                           */
} synthpix_render_params;

/* Optional per-particle inputs of the full model (any pointer may be NULL). */
typedef struct {
    const float* dy;            /* second diameter d_y: sigma_y = d_y / 4 (NULL: d_y = d)        */
    const float* rho;           /* correlation of Eq. 1, |rho| <= 0.99 (NULL: 0)                  */
    const float* z2;            /* frame-2 out-of-plane position (NULL: frame 1's z)              */
} synthpix_particle_extras;

/* Screen tiling used by the renderer.  Tiles are tile_w x tile_h pixels, one of
 * 8x8, 16x16, 32x16, 32x32, 64x16, 64x32, 64x64, 128x32.  NULL selects the
 * default. */
typedef struct {
    int32_t tile_w, tile_h;
    int32_t chunk;              /* particles per binning block (256 .. 16384, multiple of 256) */
    int32_t cap;                /* particles staged in LDS per render pass (32 .. 256)        */
    int32_t persistent;         /* 1: one persistent render launch whose workgroups (as many as
                                   the device holds) pop (frame, tile) items from per-XCD work
                                   queues; 0: one workgroup per item.  Same images either way. */
} synthpix_tiling;

/* ---------------------------------------------------------------- helpers */

int32_t synthpix_version(void);
const char* synthpix_last_error(void);

/* floor(H * W * ppp + 1/2) in float64 (Section 2, "Sampling the particles"). */
synthpix_status synthpix_particle_count(int32_t H, int32_t W, double ppp, int32_t* n_out);

/* The default tiling for a batch. */
synthpix_status synthpix_default_tiling(const synthpix_pair* pairs_host, int32_t n_pairs,
                                        const synthpix_render_params* rp, synthpix_tiling* out);

/* The tilings a plan's autotuner may choose for these parameters (the default
 * first): every compiled tile shape x LDS particle capacity whose LDS fits,
 * with 2048-particle binning blocks, then the binning block sizes it tries for
 * the fastest of those, then the persistent form of the fastest.  Writes at most max_out entries, the total count to
 * *n_out. */
synthpix_status synthpix_tiling_candidates(const synthpix_render_params* rp, synthpix_tiling* out,
                                           int32_t max_out, int32_t* n_out);

/* Bytes of workspace needed by synthpix_render_pair (backward = 0),
 * synthpix_render_pair_backward (backward = 1) or
 * synthpix_render_pair_backward_mse (backward = 2) for this batch and tiling;
 * other values of backward are refused.  The forward size also covers
 * synthpix_advect's optional workspace. */
synthpix_status synthpix_workspace_size(const synthpix_pair* pairs_host, int32_t n_pairs,
                                        const synthpix_render_params* rp,
                                        const synthpix_tiling* tiling, int32_t backward,
                                        size_t* bytes_out);

/* Where the binning results of the last synthpix_render_pair call live inside
 * its workspace (byte offsets from the workspace start), for inspection:
 *   tile_count  uint32 [2][tiles]  particles listed per tile (frame-major)
 *   tile_offset int64  [2][tiles]  index of each tile's first entry in `entries`
 *   entries     int32  [..]        pair-local particle indices; a tile's list is
 *                                  a set (its order is unspecified)
 * tiles = sum over pairs of ceil(W / tile_w) * ceil(H / tile_h), pairs in table
 * order, tiles row-major inside a pair. */
typedef struct {
    size_t tile_count, tile_offset, entries;
    int64_t tiles;
} synthpix_bin_views;

synthpix_status synthpix_bin_views_of(const synthpix_pair* pairs_host, int32_t n_pairs,
                                      const synthpix_render_params* rp, const synthpix_tiling* tiling,
                                      synthpix_bin_views* out);

/* Copies the device status word (workspace word 0) to *flags after the stream
 * has drained; returns SP_ERR_DEVICE_STATUS when any flag is set. */
synthpix_status synthpix_read_status(const void* workspace_dev, void* stream, uint32_t* flags);

/* Measurement helper: while enabled (on != 0), every kernel launch made by the
 * library is bracketed by two hipEvents recorded on its stream.
 * synthpix_timing_read waits for the recorded events of kernel `name` (NULL:
 * all kernels), returns their summed elapsed milliseconds and launch count,
 * and forgets them.  Kernel names: "seed", "advect", "bin_layout", "bin_count",
 * "bin_scan", "bin_scatter", "render_tile" (and the backward's kernels). */
synthpix_status synthpix_timing_enable(int32_t on);
synthpix_status synthpix_timing_read(const char* name, double* total_ms, int64_t* launches);

/* Measurement helper: one launch of a peak-rate probe, for roofline ceilings
 * measured on the device itself.  kind:
 *   SP_PROBE_STORE  16-byte stores of zeros over `bytes` of buf (HBM write rate)
 *   SP_PROBE_COPY   copy of the first half of buf into the second half
 *   SP_PROBE_FMA    8 chains of `iters` dependent float32 FMAs per thread, 8 waves
 *                   per SIMD on every compute unit (VALU issue rate)
 *   SP_PROBE_TRANS  the same with v_sin_f32 (transcendental rate)
 *   SP_PROBE_MUL64  the same with a 32 x 32 -> 64-bit multiply and a xor (the
 *                   Philox round's multiply)
 *   SP_PROBE_STORE_NT  as SP_PROBE_STORE with non-temporal stores
 *   SP_PROBE_MIX    the same with chains of nine mixed VALU instructions (FMA,
 *                   multiplies, float <-> u32 conversions, integer add, shift
 *                   and bit operations: the renderer's inner-loop mix)
 *   SP_PROBE_INT    the same with 32-bit integer add, shift and xor chains
 * buf: device memory of `bytes` bytes (store, copy; 16-byte aligned) or of at
 * least 1 KiB (the ALU probes never write it).  iters: a positive multiple of 4
 * (ALU probes).  *work_out: bytes moved (store: written; copy: read + written)
 * or wave64 VALU instructions of the probe loop.  The launch is timed like the
 * library's other kernels ("probe_store", "probe_copy", "probe_fma",
 * "probe_trans", "probe_mul64", "probe_store_nt", "probe_mix", "probe_int"). */
#define SP_PROBE_STORE 0
#define SP_PROBE_COPY  1
#define SP_PROBE_FMA   2
#define SP_PROBE_TRANS 3
#define SP_PROBE_MUL64 4
#define SP_PROBE_STORE_NT 5
#define SP_PROBE_MIX   6
#define SP_PROBE_INT   7
synthpix_status synthpix_probe(int32_t kind, void* buf, size_t bytes, int32_t iters, void* stream,
                               double* work_out);

/* -------------------------------------------------------------- hot path */

/* Seed every pair's n_max candidate particles (Section 2, "Sampling the
 * particles").  Per pair: ppp = ppp_lo + (ppp_hi - ppp_lo) u, n_active =
 * min(n_max, floor(H W ppp + 1/2)); per particle i: x = W u, y = H u,
 * z ~ U[z_lo, z_hi], d per d_dist, I0 ~ U[I0_lo, I0_hi] for i < n_active and
 * 0 otherwise.  Draws are Philox4x32-10 words of counter
 * (i, stream, pair_id lo, pair_id hi) under key (seed lo, seed hi).
 * pairs_host/pairs_dev: the same n_pairs table on host and device.
 * x, y, z, d, I0: device float arrays covering every pair's particle range.
 * n_active_dev, ppp_dev: optional per-pair outputs (int32, float64), may be NULL. */
synthpix_status synthpix_seed(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev,
                              int32_t n_pairs, const synthpix_seed_params* sp, uint64_t seed,
                              float* x, float* y, float* z, float* d, float* I0,
                              int32_t* n_active_dev, double* ppp_dev, void* stream);

/* Move frame-1 particles through the pair's frozen flow grid over dt
 * (Section 2, "Sampling the particles"): bilinear, clamped-to-edge sampling,
 * `substeps` steps of explicit Euler or classical RK4.
 * flow: device floats holding every pair's grid at pair.flow_offset.
 * x1, y1 -> x2, y2: device float arrays (x2/y2 may not alias x1/y1).
 * wflow, z1, z2: all NULL (planar motion) or all set: the three-dimensional
 * motion of Remark 1's particles, z2 = z1 + the integral of the out-of-plane
 * velocity w along the in-plane trajectory (same integrator stages); wflow
 * holds each pair's [Gh][Gw] w grid (sheet units per frame, registered like
 * the (u, v) grid) at float offset pair.flow_offset / 2.  The 3-D form runs in
 * particle index order (the workspace is not used).
 * workspace: optional device scratch, 256-byte aligned, of at least
 * synthpix_advect_workspace_size bytes (any workspace sized by
 * synthpix_workspace_size also fits).  With it, particles are first ordered by
 * home block so that neighbouring threads sample neighbouring grid cells; the
 * results are identical with or without it (NULL: particle index order). */
synthpix_status synthpix_advect(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev,
                                int32_t n_pairs, const float* flow, const synthpix_advect_params* ap,
                                const float* x1, const float* y1, float* x2, float* y2,
                                const float* wflow, const float* z1, float* z2,
                                void* workspace, size_t ws_bytes, void* stream);

/* Second diameter and correlation of every candidate particle for anisotropic
 * particle images (Eq. 1; the sentence after it draws every shape parameter
 * per particle): d_y from the seed's diameter distribution, rho ~ U[rho_lo,
 * rho_hi] with -0.99 <= rho_lo <= rho_hi <= 0.99.  Draws: Philox stream 6 at
 * the particle index (word 0 uniform d_y; words 1, 2 Box-Muller of a normal
 * d_y; word 3 rho).  dy, rho: device float arrays like synthpix_seed's. */
synthpix_status synthpix_seed_shape(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev,
                                    int32_t n_pairs, const synthpix_seed_params* sp, float rho_lo,
                                    float rho_hi, uint64_t seed, float* dy, float* rho, void* stream);

/* Bytes of the optional synthpix_advect workspace for this batch. */
synthpix_status synthpix_advect_workspace_size(const synthpix_pair* pairs_host, int32_t n_pairs,
                                               size_t* bytes_out);

/* Render both exposures of every pair and apply blur, noise and storage
 * (Eq. 1; Section 2, "Considerations on the aggregation", "Efficient
 * rasterization").  Frame 1 uses (x1, y1), frame 2 (x2, y2); z, d, I0 are
 * shared.  Particles with I0 <= 0, d <= 0 or non-finite position add nothing.
 * extras: NULL, or the full model's per-particle d_y, rho and frame-2 z (each
 * optional); with rp's frame-2 variation, hiding and sheet law they select the
 * full model (an anisotropic particle adds I0 S(z) times Eq. 1 with
 * sigma_x = d / 4, sigma_y = d_y / 4 on |dx| <= 1.5 d, |dy| <= 1.5 d_y).
 * tiling may be NULL (default); the output does not depend on it.
 * images: device buffer, float or uint16 per rp->bits; only the pairs' image
 * ranges are written.
 * workspace: device, 256-byte aligned, >= synthpix_workspace_size(..., 0). */
synthpix_status synthpix_render_pair(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev,
                                     int32_t n_pairs, const synthpix_tiling* tiling,
                                     const float* x1, const float* y1,
                                     const float* x2, const float* y2,
                                     const float* z, const float* d, const float* I0,
                                     const synthpix_particle_extras* extras,
                                     const synthpix_render_params* rp, void* images,
                                     void* workspace, size_t ws_bytes, void* stream);

/* Gradient of a loss L of the float images J (bits must be 0; the isotropic
 * model: no frame-2 variation, no hiding, the Gaussian sheet) with respect to
 * the frame-1 positions, z, d, I0, each pair's sheet width and each pair's flow
 * grid (differentiating Eq. 1 with the Gaussian sheet peak, the patch cutoff
 * held fixed, and the blur; noise is additive and has no gradient).
 * Frame-2 positions: x2, y2 as produced by synthpix_advect from (x1, y1) with
 * rp->advect, or both NULL to have them recomputed; footprints and the
 * trajectory are recomputed, nothing else from the forward is needed.
 * grad_images: device floats dL/dJ, same layout as the forward's images.
 * Outputs (device floats, overwritten): g_x1, g_y1, g_z, g_d, g_I0 per particle
 * (every index below the batch's particle span is written; indices in no
 * pair's range get 0), g_sheet [n_pairs] (each pair's sheet width),
 * g_sheet_total (optional, may be NULL: one float, the gradient with respect
 * to a sheet width shared by all pairs, the float64 sum of the per-pair terms
 * in pair order rounded once), g_flow with the flow's layout (zero outside the
 * pairs' grids).  Deterministic: flow-grid sums are 64-bit fixed point.
 * tiling is unused (may be NULL); workspace: >= synthpix_workspace_size(..., 1). */
synthpix_status synthpix_render_pair_backward(const synthpix_pair* pairs_host,
                                              const synthpix_pair* pairs_dev, int32_t n_pairs,
                                              const synthpix_tiling* tiling, const float* flow,
                                              const float* x1, const float* y1,
                                              const float* x2, const float* y2, const float* z,
                                              const float* d, const float* I0,
                                              const synthpix_render_params* rp,
                                              const float* grad_images,
                                              float* g_x1, float* g_y1, float* g_z, float* g_d,
                                              float* g_I0, float* g_sheet, float* g_sheet_total,
                                              float* g_flow, void* workspace, size_t ws_bytes,
                                              void* stream);

/* The backward of synthpix_render_pair_backward for the image loss of
 * synthpix_mse_grad, in one call: dL/dJ = scale (J - T) of the float images J
 * (`images`, the forward's output) and a target T of the same layout is formed
 * inside the backward's first per-pixel pass, where it is read (the same
 * binary32 values synthpix_mse_grad would store), instead of being written to
 * and read back from device memory; with a blur, that pass also applies the
 * blur's adjoint once per pixel (Section 2, "Considerations on the aggregation":
 * the blur is a fixed linear map of the images).  Arguments and outputs as in
 * synthpix_render_pair_backward; the pairs' image ranges of images and target
 * are read (16-byte alignment not needed).  scale: finite.  loss: optional
 * (NULL: skipped) device double, 8-byte aligned, receiving the mean of
 * (J - T)^2 over the pairs' pixels (2 H W per pair), summed in float64 in a
 * fixed order (bit-reproducible; equal to synthpix_mse_grad's value up to the
 * summation order).  workspace: >= synthpix_workspace_size(..., 2).  The
 * gradients equal those of synthpix_mse_grad followed by
 * synthpix_render_pair_backward up to float32 rounding (the same values with
 * no blur or a blur of radius >= 2; a radius-1 blur, which the two-step form
 * folds into its gather, is applied here once per pixel). */
synthpix_status synthpix_render_pair_backward_mse(const synthpix_pair* pairs_host,
                                                  const synthpix_pair* pairs_dev, int32_t n_pairs,
                                                  const synthpix_tiling* tiling, const float* flow,
                                                  const float* x1, const float* y1,
                                                  const float* x2, const float* y2, const float* z,
                                                  const float* d, const float* I0,
                                                  const synthpix_render_params* rp,
                                                  const float* images, const float* target, float scale,
                                                  double* loss,
                                                  float* g_x1, float* g_y1, float* g_z, float* g_d,
                                                  float* g_I0, float* g_sheet, float* g_sheet_total,
                                                  float* g_flow, void* workspace, size_t ws_bytes,
                                                  void* stream);

/* Image loss of a fitting loop through the generator (the acquisition and
 * parameter co-design the Abstract and Introduction name): the mean squared
 * difference L = sum_i (J_i - T_i)^2 / n of rendered float images J to a target
 * T of the same layout, and its gradient dL/dJ_i = scale (J_i - T_i), with
 * scale = 2 / n for L itself (the caller picks it, e.g. to weight several
 * terms), in one pass.  J, T, grad: n device floats, 16-byte aligned (NULL
 * allowed for n = 0); grad may be J or T itself.  loss: optional (NULL: skipped) device double receiving
 * sum_i (J_i - T_i)^2 / n, summed in a fixed order (bit-reproducible); it
 * needs the workspace: 256-byte aligned device memory of
 * synthpix_mse_workspace_size(n) bytes (NULL when loss is NULL). */
size_t synthpix_mse_workspace_size(int64_t n);
synthpix_status synthpix_mse_grad(const float* J, const float* T, int64_t n, float scale, float* grad,
                                  double* loss, void* workspace, size_t ws_bytes, void* stream);

/* Allocation-free form of synthpix_render_pair, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same inputs, outputs and results as
 * synthpix_render_pair (bit-identical images), but the workspace is a
 * library-held static device array of SYNTHPIX_STATIC_SCRATCH_BYTES, one per
 * device, resolved on the first call on each device and held until the
 * process ends.  Calls nothing that allocates.  A batch whose workspace
 * (synthpix_workspace_size) exceeds the array is refused with
 * SP_ERR_WORKSPACE before anything is enqueued.  Every call on a device shares
 * that device's array: calls that overlap on one device (different streams, or
 * host threads, without ordering between them) race and are not supported.
 * status_out: optional device uint32 that receives the call's device status
 * word (SP_STATUS_* bits), copied stream-ordered after the render; NULL drops
 * it. */
#define SYNTHPIX_STATIC_SCRATCH_BYTES (64u << 20)
synthpix_status synthpix_render_pair_noalloc(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev,
                                             int32_t n_pairs, const synthpix_tiling* tiling,
                                             const float* x1, const float* y1,
                                             const float* x2, const float* y2,
                                             const float* z, const float* d, const float* I0,
                                             const synthpix_particle_extras* extras,
                                             const synthpix_render_params* rp, void* images,
                                             uint32_t* status_out, void* stream);

/* Ground-truth flow of every pair (the flow_fields a sampler returns next to
 * the images, Section 2 "Usage"): the pair's (u, v) grid, pixels per frame,
 * sampled bilinearly at each pixel centre (c + 1/2, r + 1/2) exactly as the
 * advection samples it.  out: device floats, each pair's [H][W][2] field at
 * float offset pair.image_offset (8-byte aligned; the same extent as the
 * pair's two float frames).  n_pairs <= 65535. */
synthpix_status synthpix_flow_field(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev,
                                    int32_t n_pairs, const float* flow, float* out, void* stream);

/* Histogram adjustment of the stored images (Section 2, after Remark 2: the
 * output may be remapped so that its intensities follow a histogram the user
 * chooses).
 * Every image (each frame of each pair, uint16 codes of `bits` bits, 1..14) is
 * mapped in place onto the target histogram `target` (device uint32 counts
 * [2^bits], total in [1, 2^32)): code k becomes the smallest m with
 * T(m) / T_tot >= S(k) / N, where S and T are the cumulative counts of the
 * image (N pixels) and of the target (T_tot); the comparison is exact integer
 * arithmetic.  workspace: device, 256-byte aligned, at least
 * synthpix_histogram_workspace_size bytes; its first word is the call's
 * device status (SP_STATUS_HIST_*; synthpix_read_status reads it). */
synthpix_status synthpix_histogram_workspace_size(int32_t n_pairs, int32_t bits, size_t* bytes_out);
synthpix_status synthpix_histogram_match(const synthpix_pair* pairs_host, const synthpix_pair* pairs_dev,
                                         int32_t n_pairs, int32_t bits, const uint32_t* target, void* images,
                                         void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------- batched, captured form */

/* Device buffers and draw key of one launch of a plan.  synthpix_plan_create
 * takes the first launch's; synthpix_plan_launch may pass new ones for every
 * launch.  The plan copies them into a device-side descriptor that the captured
 * kernels read, so one captured graph serves any buffers of the plan's shapes. */
typedef struct {
    const float* flow;          /* every pair's flow grid at pair.flow_offset (8-byte aligned) */
    float *x1, *y1, *x2, *y2;   /* particle positions of frame 1 and frame 2                  */
    float *z, *d, *I0;          /* per-particle out-of-plane position, diameter, intensity    */
    void* images;               /* [pair][frame][H][W], float or uint16 per rp->bits          */
    int32_t* n_active;          /* optional per-pair outputs of the seed step (may be NULL)   */
    double* ppp;
    uint64_t seed;              /* key of every draw of the launch: particles and noise       */
    uint64_t pair_id_base;      /* added to every pair's pair_id (Philox counter words 2, 3)  */
} synthpix_batch_io;

typedef struct synthpix_plan synthpix_plan;

/* Build a plan for a fixed batch signature (pair table and parameters):
 * copies the pair table to plan-owned device memory, sizes and allocates the
 * render workspace and the device-side io descriptor, and, if `autotune` != 0,
 * times the compiled tiling candidates (synthpix_tiling_candidates: tile shape
 * x LDS particle capacity, then the binning block size of the fastest) on this
 * batch and keeps the fastest (all candidates give bit-identical images).  The
 * whole path -- seed, advect, bin, render, epilogue -- is then captured once
 * into a hipGraph whose kernels take their buffers, draw key and pair-id
 * offset from the descriptor.  io: the first launch's buffers (also used while
 * autotuning, so they must be valid device memory of the batch's sizes).  The
 * plan draws particles and noise with io->seed (rp->seed is not used).  This
 * call validates every parameter as the eager calls do, allocates device
 * memory and synchronises `stream`; it is the set-up call, not the hot path.
 * advance_pair_ids != 0: every launch moves the descriptor's pair_id_base on
 * by n_pairs after rendering, so consecutive launches without new io draw the
 * pairs with ids pair_id + pair_id_base + k * n_pairs.
 * Masked candidates (slots i >= the pair's drawn active count, whose I0 is 0)
 * are not advected by a plan: their x2, y2 are set to x1, y1.  Images and every
 * active particle's outputs equal the eager calls'. */
synthpix_status synthpix_plan_create(const synthpix_pair* pairs_host, int32_t n_pairs,
                                     const synthpix_seed_params* sp, const synthpix_advect_params* ap,
                                     const synthpix_render_params* rp, const synthpix_batch_io* io,
                                     int32_t autotune, int32_t advance_pair_ids, void* stream,
                                     synthpix_plan** out);

/* Replay the captured graph on `stream` (asynchronous, no allocation).  io:
 * NULL replays with the descriptor as it stands (the previous launch's
 * buffers, pair ids advanced if the plan advances them); otherwise its
 * pointers are validated on the host and a one-thread kernel stores *io into
 * the descriptor on `stream` before the graph runs (stream-ordered, so io may
 * be reused or freed on return).  Buffers must have the plan's sizes. */
synthpix_status synthpix_plan_launch(synthpix_plan* plan, const synthpix_batch_io* io, void* stream);

/* Device status word of the plan's last launch (see synthpix_read_status). */
synthpix_status synthpix_plan_read_status(const synthpix_plan* plan, void* stream, uint32_t* flags);

/* The tiling the plan runs with (after autotuning). */
synthpix_status synthpix_plan_tiling(const synthpix_plan* plan, synthpix_tiling* out);

/* Release the plan's graph, workspace and device pair table. */
synthpix_status synthpix_plan_destroy(synthpix_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* SYNTHPIX_H */
