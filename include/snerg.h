/*
 * snerg.h -- C ABI of the MI355X (gfx950) SNeRG renderer.
 *
 * Renders a Sparse Neural Radiance Grid as described in "Baking Neural
 * Radiance Fields for Real-Time View Synthesis" (Hedman et al., arXiv
 * 2103.14645): for every pixel a ray is marched through the block-sparse
 * grid (Section 5.1: a coarse indirection grid over an atlas of B^3
 * macroblocks holding density, diffuse colour and a 4-channel feature
 * vector), trilinearly sampled and alpha-composited front to back with
 * early termination (Section 5.2, Eq. 2, 5, 6); the deferred shading MLP
 * then runs once per pixel on the composited colour, features and view
 * direction and its residual is added (Eq. 7, Section 4.2).  A backward
 * entry point gives gradients with respect to the MLP and a float copy of
 * the grid values, for fine-tuning by a pixel loss (Eq. 3, Section 5.5),
 * with a squared-error loss and an Adam step beside it.  Two baking entry
 * points turn a densely evaluated field into the grid: the empty-space and
 * visibility culls of Section 5.3 and the 8-bit atlas of Section 5.4.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Device pointers ("device") are HIP device allocations owned by the
 *    caller; the library never allocates, frees or retains them.  Host
 *    pointers ("host") are read during the call only.
 *  - `stream` is a hipStream_t (NULL = the default stream).  All device
 *    work is enqueued asynchronously on it; results are valid once the
 *    stream has reached that point.
 *  - Validation is synchronous and host-only and happens before any device
 *    work; a call that returns an error has enqueued nothing and written
 *    nothing.  Device faults surface as SNERG_ERR_HIP at a later call or
 *    at stream synchronisation.  No C++ exception crosses this ABI.
 *  - Calls on one handle must not run concurrently from several host
 *    threads.  Different handles are independent.
 *
 * Geometry (what every entry point computes)
 * ------------------------------------------
 *  - The grid covers the world box [-1, 1]^3 with N^3 voxels; voxel i spans
 *    [i, i+1) in voxel units u = (x + 1) N / 2 and its value sits at its
 *    centre.  Macroblocks are B^3 voxels; the indirection grid has
 *    G^3 = (N/B)^3 int32 entries, x fastest ((bz*G + by)*G + bx): -1 marks
 *    an empty macroblock, otherwise the entry is the macroblock's atlas id.
 *  - Canonical atlas arrays (inputs of snerg_pack_grid, shapes of the grid
 *    gradients): dens [n_blocks][B][B][B], rgb [n_blocks][B][B][B][3],
 *    feat [n_blocks][B][B][B][4], voxel (x, y, z) of a block at
 *    (z*B + y)*B + x.  SNERG_U8 values are bytes v with value v/255;
 *    SNERG_F32 values are used as stored.  Density value s gives
 *    sigma = sigma_scale * s (50 in the paper's setting of 8-bit density).
 *  - Rays: pixel (i, j) of a W x H camera (column i, row j from the top)
 *    has x = (i + 1/2 - W/2)/focal, y = (j + 1/2 - H/2)/focal and
 *    direction d = D/|D|, D = fwd + x right - y up, computed in FP64 with
 *    this exact operation order and no fused multiply-add.  Samples lie on
 *    an integer lattice in Q16 fixed point from the camera centre:
 *    o = rint(((eye + 1) (N/2)) 2^16), s = rint(d 2^15) (half a voxel),
 *    P_k = o + k s for k = 0, 1, ...; a sample is inside the grid when
 *    0 <= P_k < N 2^16 on every axis and is skipped when its macroblock
 *    floor(P_k / (B 2^16)) is empty.
 *  - Sampling: trilinear over the virtual dense grid (corner voxels outside
 *    the grid or in empty macroblocks read 0), with Q = P_k - 2^15,
 *    i0 = floor(Q / 2^16), f = (Q mod 2^16) / 2^16.  A sample is composited
 *    only if some corner has non-zero density and non-zero weight.
 *  - Compositing with step delta = 1/N: alpha = 1 - exp(-sigma delta),
 *    w = T alpha, C_d += w c_d, V += w v, T *= 1 - alpha; with early stop
 *    the march ends after the sample that brings T below t_stop.
 *  - Deferred MLP (when mlp_on and at least one sample was composited):
 *    x = [C_d(3), V(4), d(3), PE(d)(24)], PE octave l = 0..3:
 *    sin(2^l pi d_xyz), cos(2^l pi d_xyz); R = sigmoid(W3 relu(W2 relu(W1 x
 *    + b1) + b2) + b3).  Output rgb = C_d + T bg + R, alpha = 1 - T.
 *  - Ray ids: cameras in order, rows from the top, columns left to right;
 *    ray r of camera c has id offset_c + j W_c + i.
 */
#ifndef SNERG_H
#define SNERG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define SNERG_OK 0
#define SNERG_ERR_INVALID_ARG (-1) /* null pointer, bad size, NaN/Inf, non-orthonormal camera */
#define SNERG_ERR_UNSUPPORTED (-2) /* B not a power of two, N % B != 0, unknown dtype/flag */
#define SNERG_ERR_RANGE (-3)       /* lattice out of range: N > 16384 or an eye coordinate beyond +-1000 */
#define SNERG_ERR_HIP (-4)         /* a HIP runtime call failed; see snerg_last_error() */
#define SNERG_ERR_WORKSPACE (-5)   /* a caller-provided buffer is too small */

/* -------------------------------------------------------------- grid types */
#define SNERG_U8 0  /* 8-bit values (Section 5.4: all values quantised to 8 bits) */
#define SNERG_F32 1 /* float32 values: the trainable shadow used by the backward pass */

/* ------------------------------------------------------------- option flags */
#define SNERG_FLAG_MLP_FP16 (1u << 0)   /* deferred MLP on FP16 MFMA tiles, FP32 accumulation */
#define SNERG_FLAG_PERSISTENT (1u << 1) /* one persistent launch over a global tile queue */
#define SNERG_FLAG_GRAPH (1u << 2)      /* replay the launch from a captured HIP graph */
#define SNERG_FLAG_MLP_GRAD_ONLY (1u << 3) /* backward: MLP gradient only (any grid dtype) */
/* Render variants of the paper's own viewer (they change the image):
 * NN_GATE composites a sample only if the voxel nearest to it (voxel floor(x)
 * in voxel units) has non-zero density, the in-block test of the WebGL
 * renderer (Appendix A), instead of the exact "some corner with non-zero
 * density and weight"; UNPREMULTIPLY scales C_d, V and alpha by
 * min(1, 1.5 alpha) / alpha after compositing (Eq. 9, forward-facing scenes),
 * before the deferred MLP; forward only. */
#define SNERG_FLAG_NN_GATE (1u << 4)
#define SNERG_FLAG_UNPREMULTIPLY (1u << 5)
/* Not deferred (the performance ablation of Section 7.1): the view network
 * runs on every composited sample, on that sample's colour and features and
 * the ray direction, its residual added to the sample's colour before
 * compositing; nothing runs per pixel.  Forward only, without aux; with
 * SNERG_FLAG_MLP_FP16 the per-sample network runs on FP16 MFMA tiles. */
#define SNERG_FLAG_PER_SAMPLE_MLP (1u << 6)
/* Backward with a ray list that comes in aligned groups of 64 neighbouring
 * rays (8x8 pixel patches, as the fine-tuning patch sampler draws them):
 * each wavefront's rays share voxels, so their gradients are summed per
 * voxel in LDS before the device atomics, as for whole views.  Without it a
 * ray list's gradients pass through an LDS log (no summing; faster when
 * rays share little).  Results are the same up to float summation order
 * either way. */
#define SNERG_FLAG_PATCH_RAYS (1u << 7)
/* Backward: add the gradients into grad_mlp, grad_dens, grad_rgb and
 * grad_feat instead of overwriting them (gradient accumulation over
 * minibatches; the caller zeroes the arrays when it starts a sum).  Skips
 * the pass that clears the grid-gradient arrays, which for a small
 * minibatch on a large grid costs more than the minibatch itself. */
#define SNERG_FLAG_ACCUMULATE (1u << 8)
/* Backward: the grid gradients go to one device array, grad_dens, of
 * [n_voxels][8] float32 per voxel in canonical atlas order (density, R, G,
 * B, features 0..3); grad_rgb and grad_feat must be NULL.  The same sums as
 * the three separate arrays, up to float summation order.  gfx950 serves
 * device float atomics per 64-byte cache line, and a voxel's eight sums then
 * share one line instead of three, which speeds up ray lists whose rays
 * share few voxels (1.2x to 1.6x on scattered minibatches). */
#define SNERG_FLAG_GRAD_PACKED (1u << 9)

#define SNERG_MLP_PARAMS 883 /* W1[16][34] b1[16] W2[16][16] b2[16] W3[3][16] b3[3], [out][in] */

typedef struct snerg_handle snerg_handle;

/* A packed grid as the render kernels read it. */
typedef struct {
    int32_t N;                  /* voxels per axis, 1 <= N <= 16384 */
    int32_t B;                  /* macroblock edge, power of two, 2 <= B <= 64, N % B == 0 */
    int32_t n_blocks;           /* atlas macroblocks (>= 0) */
    int32_t dtype;              /* SNERG_U8 or SNERG_F32 (of the packed values) */
    const int32_t *indirection; /* device, (N/B)^3 entries as described above */
    const void *packed;         /* device, written by snerg_pack_grid for the same N, B, n_blocks, dtype */
    float sigma_scale;          /* sigma = sigma_scale * density value (50) */
    int32_t reserved;
} snerg_grid;

/* Pinhole camera; fwd, right, up must be orthonormal (|.| within 1e-6). */
typedef struct {
    double eye[3], fwd[3], right[3], up[3];
    int32_t W, H;  /* image size, >= 1 */
    double focal;  /* focal length in pixels, > 0 */
} snerg_camera;

typedef struct {
    float bg[3];        /* background colour added with weight T */
    float t_stop;       /* early-stop threshold on T (1e-3) */
    int32_t early_stop; /* 0/1 */
    int32_t mlp_on;     /* 0/1: 0 renders the diffuse colour only */
    uint32_t flags;     /* SNERG_FLAG_* */
    int32_t reserved;
} snerg_opts;

/* Launch shape used by the forward kernels (chosen by snerg_autotune). */
typedef struct {
    int32_t tile_w, tile_h;   /* pixels per wavefront tile, tile_w * tile_h == 64 */
    int32_t waves_per_group;  /* wavefronts per workgroup: 1, 2 or 4 */
    int32_t groups_per_cu;    /* persistent launch: resident workgroups per compute unit, 1..16 */
} snerg_tuning;

/* ---------------------------------------------------------------- handles */

/* Creates a handle on the current HIP device.  It owns small device buffers
 * (camera table, tile counter, the render's tile-order scratch, the backward
 * pass's MLP partial sums and per-ray dL/dC_d, dL/dV scratch, the baking
 * scratch), a cached HIP graph, timing events and the tuning; nothing the
 * caller passes in.  The buffers are allocated on first use and grown (by
 * half again as much as the call needs) when a call needs more; the growing
 * call first waits for the work queued on its stream, so a call made inside
 * a caller's stream capture must have been made once outside it with the
 * same sizes, and snerg_render_noalloc needs no buffer at all.  Calls on one handle should use one stream (or the
 * caller orders the streams). */
int snerg_create(snerg_handle **out);
int snerg_destroy(snerg_handle *h);

/* Static description of a status code; never NULL. */
const char *snerg_status_string(int status);
/* Message of the last failure on this host thread ("" if none). */
const char *snerg_last_error(void);

/* ---------------------------------------------------------------- packing */

/* Bytes of the packed grid for the given shape (Section 5.1 data structure
 * re-laid out for the GPU: per macroblock a copy of its B^3 voxels with a
 * one-voxel apron taken from the neighbouring macroblocks, channels
 * interleaved per voxel, plus a per-cell occupancy bitmask). */
int snerg_packed_size(int32_t N, int32_t B, int32_t n_blocks, int32_t dtype, size_t *bytes);

/* Builds the packed grid from canonical arrays.  indirection, dens, rgb,
 * feat: device, canonical layout, element type given by dtype (uint8 or
 * float32).  packed: device, at least snerg_packed_size() bytes. */
int snerg_pack_grid(snerg_handle *h, int32_t N, int32_t B, int32_t n_blocks, int32_t dtype,
                    const int32_t *indirection, const void *dens, const void *rgb, const void *feat,
                    void *packed, size_t packed_bytes, void *stream);

/* ------------------------------------------------------------- rendering */

/*
 * Renders rays (Section 5.2, Eq. 5-7).  cams: host, n_cams >= 1.  ray_ids:
 * device int64 [n_rays] or NULL for every ray of every camera (then n_rays
 * must equal the total pixel count).  mlp: device float32 [883] (may be
 * NULL when opts->mlp_on == 0).  out_rgba: device float32 [n_rays][4].
 * aux: device float32 [n_rays][8] or NULL; receives C_d[3], V[4] and T,
 * with T replaced by -1 when no sample was composited (then T = 1).  The
 * backward pass consumes aux.
 */
int snerg_render(snerg_handle *h, const snerg_grid *grid, const float *mlp, const snerg_camera *cams,
                 int32_t n_cams, const int64_t *ray_ids, int64_t n_rays, const snerg_opts *opts,
                 float *out_rgba, float *aux, void *stream);

/*
 * Gradient of L = sum_r grad_rgba[r] . rgba[r] (Eq. 3 fine-tuning, Section
 * 5.5) with respect to the 883 MLP parameters and the float32 grid values,
 * holding the set of composited samples and the stopping sample fixed.
 * grid->dtype must be SNERG_F32.  Rays are re-marched (nothing per sample
 * is stored); aux must come from snerg_render of the same rays, grid, MLP,
 * cameras and options.  grad_rgba: device [n_rays][4].  Outputs (device,
 * overwritten, or added to with SNERG_FLAG_ACCUMULATE): grad_mlp [883],
 * grad_dens, grad_rgb, grad_feat in canonical atlas layout (or all eight
 * channels in grad_dens with SNERG_FLAG_GRAD_PACKED).  Gradient sums
 * use float32 atomics, so their rounding depends on scheduling; where a
 * wavefront's rays are summed per voxel in LDS first (whole views, and ray
 * lists with SNERG_FLAG_PATCH_RAYS) the colour and feature sums are 32-bit
 * fixed point, each hand-over rounded to within 2^-24 of the wavefront's
 * largest |dL/dC_d|, |dL/dV|.  A ray list of at most 2^18 rays runs in two
 * phases whose per-ray sample lists (up to 8 KB per ray) live in
 * handle-owned device memory, kept for later calls.  With SNERG_FLAG_MLP_FP16 the MLP
 * backward runs on FP16 MFMA tiles with FP32 accumulation (as the forward).
 * With SNERG_FLAG_MLP_GRAD_ONLY only grad_mlp is computed (the fine-tuning
 * of Section 5.5 optimises the deferred network alone): no ray is
 * re-marched, the grid may be SNERG_U8 and grad_dens/rgb/feat may be NULL.
 */
int snerg_render_backward(snerg_handle *h, const snerg_grid *grid, const float *mlp,
                          const snerg_camera *cams, int32_t n_cams, const int64_t *ray_ids,
                          int64_t n_rays, const snerg_opts *opts, const float *aux,
                          const float *grad_rgba, float *grad_mlp, float *grad_dens,
                          float *grad_rgb, float *grad_feat, void *stream);

/*
 * snerg_render for callers that cannot allocate device memory (code under
 * HIP stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, with every scratch buffer (camera table,
 * tile order, tile counter) in a fixed 16 MiB device array that the library
 * holds on each GPU it runs on until the process ends; it calls no
 * allocating routine.  Limits: at most 1024 cameras and, without ray_ids, at
 * most 3,327,488 tiles of 64 pixels (about 212 M rays) per call, else
 * SNERG_ERR_WORKSPACE; SNERG_FLAG_GRAPH is SNERG_ERR_UNSUPPORTED (graph
 * instantiation allocates).  All calls on one GPU share the array: calls
 * whose work overlaps on that GPU (other streams, other host threads) race
 * and must be ordered by the caller.  Arguments and results as snerg_render;
 * the handle supplies the launch shape.
 */
int snerg_render_noalloc(snerg_handle *h, const snerg_grid *grid, const float *mlp, const snerg_camera *cams,
                         int32_t n_cams, const int64_t *ray_ids, int64_t n_rays, const snerg_opts *opts,
                         float *out_rgba, float *aux, void *stream);

/*
 * snerg_render that also reports, per ray, what the render kernel's own
 * march did (the samples of Section 5.2 and the per-sample accounting of
 * Appendix A), for verification and measurement: the same kernel code and
 * launch modes, compiled with counting.  counters: device int32
 * [n_rays][7] = macroblocks entered, occupied macroblocks among them,
 * samples inside occupied macroblocks (up to and including the stopping
 * sample), composited samples, the stopping k (-1 if none), and the sums of
 * the composited samples' k and k^2 modulo 2^32 (as int32 bits).  Other
 * arguments and results as snerg_render; SNERG_FLAG_PER_SAMPLE_MLP is
 * SNERG_ERR_UNSUPPORTED.
 */
int snerg_render_counted(snerg_handle *h, const snerg_grid *grid, const float *mlp, const snerg_camera *cams,
                         int32_t n_cams, const int64_t *ray_ids, int64_t n_rays, const snerg_opts *opts,
                         float *out_rgba, float *aux, int32_t *counters, void *stream);

/*
 * Occupied macroblocks each ray visits in order (linear indirection index,
 * consecutive repeats collapsed), up to max_visits per ray, with the same
 * march and stopping rule as snerg_render.  visits: device int32
 * [n_rays][max_visits] (unused slots untouched; may be NULL when
 * max_visits == 0); counts: device int32 [n_rays] (full count, may exceed
 * max_visits); counters: device int32 [n_rays][5] or NULL = macroblocks
 * traversed, occupied macroblocks visited, samples inside occupied
 * macroblocks, composited samples, stopping k (-1 if none).
 */
int snerg_trace_visits(snerg_handle *h, const snerg_grid *grid, const snerg_camera *cams,
                       int32_t n_cams, const int64_t *ray_ids, int64_t n_rays, const snerg_opts *opts,
                       int32_t max_visits, int32_t *visits, int32_t *counts, int32_t *counters,
                       void *stream);

/* ----------------------------------------------------------- fine-tuning */

/*
 * Squared error of rendered against observed pixels, the loss of the
 * fine-tuning in Section 5.5: loss = (1 / 3n) sum over rays and RGB of
 * (rgba - target)^2, and its gradient grad_rgba = (2 / 3n) (rgba - target)
 * for RGB, 0 for alpha (the observed images carry no alpha).  rgba,
 * grad_rgba: device float32 [n][4]; target: device float32 [rows][4], row i
 * of rgba compared with row target_ids[i] (device int64 [n], each in
 * [0, rows), unchecked) or, with target_ids NULL, row i; loss: device
 * float32 [1] (overwritten).  n may be 0 (loss 0).
 */
int snerg_loss_mse(snerg_handle *h, const float *rgba, const float *target, const int64_t *target_ids,
                   int64_t n, float *grad_rgba, float *loss, void *stream);

typedef struct {
    float lr;     /* Section 5.5 uses 3e-4 */
    float beta1;  /* 0.9 */
    float beta2;  /* 0.999 */
    float eps;    /* 1e-8 */
    int32_t step; /* t >= 1: this update's index, for the bias corrections */
    int32_t reserved;
} snerg_adam;

/*
 * One Adam update (Kingma and Ba, Algorithm 1), the optimiser of Section
 * 5.5, applied elementwise: m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
 * p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).  param, m, v
 * (updated in place) and grad: device float32 [n]; m and v start at zero.
 */
int snerg_adam_step(snerg_handle *h, float *param, const float *grad, float *m, float *v, int64_t n,
                    const snerg_adam *cfg, void *stream);

/* ---------------------------------------------------------------- baking */

/* Thresholds of the baking culls (Section 5.3) and the density scale of the
 * 8-bit quantisation (Section 5.4). */
typedef struct {
    float tau_alpha;   /* empty-space cull: keep a macroblock whose largest voxel alpha is >= this (0.005) */
    float tau_vis;     /* visibility cull: keep a macroblock whose largest voxel visibility is >= this (0.01) */
    float sigma_scale; /* density byte = rint(sigma * (255 / sigma_scale)); the grid's sigma_scale (50) */
    int32_t reserved;
} snerg_bake_opts;

/*
 * Macroblock culling of a densely evaluated field (Section 5.3): a
 * macroblock is stored only if it is both non-empty and visible from at
 * least one training view.
 *  - sigma: device float32 [N^3] (x fastest), the density of every voxel
 *    per unit length of the world box (finite, >= 0).  N and B obey the
 *    limits of the grid struct above (N/B <= 64).
 *  - Opacity of a voxel: alpha = 1 - exp(-sigma v), v = 1/N.  A macroblock
 *    passes the empty-space cull when its largest alpha is >= tau_alpha.
 *  - Visibility of a voxel: the largest transmittance between it and any
 *    training camera.  Every pixel ray of `cams` (host, the training views)
 *    is marched on the render's sample lattice (geometry above, step
 *    delta = 1/N); sample k lies in voxel floor(P_k / 2^16), reads that
 *    voxel's density and sees T_k = exp(-delta * S_k), S_k the sum of the
 *    densities of the ray's earlier samples inside the grid (summed in
 *    float64 in sample order).  A macroblock passes the visibility cull
 *    when some sample inside it has T_k >= tau_vis.  Both tests are decided
 *    on the exact equivalents max sigma >= -N log(1 - tau_alpha) and
 *    min S_k <= -N log(tau_vis), in float64.
 *  - Outputs (device): indirection int32 [(N/B)^3], -1 for a culled
 *    macroblock, else its atlas id, kept blocks numbered 0, 1, ... in
 *    indirection order; block_alpha and block_vis (nullable) float32
 *    [(N/B)^3], the largest voxel alpha and the largest visibility (0 when
 *    below tau_vis).  *n_blocks (host) receives the number of kept blocks.
 * Synchronises `stream` (the count is read back).
 */
int snerg_bake_cull(snerg_handle *h, int32_t N, int32_t B, const float *sigma, const snerg_camera *cams,
                    int32_t n_cams, const snerg_bake_opts *opts, float *block_alpha, float *block_vis,
                    int32_t *indirection, int32_t *n_blocks, void *stream);

/*
 * 8-bit canonical atlas of the kept macroblocks (Section 5.4: every baked
 * value is stored in 8 bits): density byte rint(sigma * k) with
 * k = 255 / sigma_scale, colour and feature bytes rint(255 c), each a single
 * float32 multiplication rounded half to even and clamped to [0, 255] (NaN
 * to 0).  sigma [N^3], rgb [N^3][3], feat [N^3][4]: device float32, x
 * fastest.  indirection: device int32 [(N/B)^3] with atlas ids in
 * [0, n_blocks), each at most once (as written by snerg_bake_cull); an atlas
 * block no entry names is written as zeros.  dens8 [n_blocks][B][B][B],
 * rgb8 [n_blocks][B][B][B][3], feat8 [n_blocks][B][B][B][4]: device, the
 * canonical layout snerg_pack_grid takes with SNERG_U8.
 */
int snerg_bake_quantize(snerg_handle *h, int32_t N, int32_t B, const float *sigma, const float *rgb,
                        const float *feat, const int32_t *indirection, int32_t n_blocks,
                        const snerg_bake_opts *opts, uint8_t *dens8, uint8_t *rgb8, uint8_t *feat8,
                        void *stream);

/* ---------------------------------------------------------------- tuning */

int snerg_set_tuning(snerg_handle *h, const snerg_tuning *t);
int snerg_get_tuning(snerg_handle *h, snerg_tuning *t);

/*
 * Times each candidate launch shape (HIP events, `reps` renders after one
 * warm-up) for the given render call and keeps the fastest in the handle.
 * candidates: host [n_candidates] or NULL for the built-in search space
 * (tiles 8x8, 16x4, 4x16 and 32x2; 1, 2 or 4 wavefronts per workgroup; with
 * SNERG_FLAG_PERSISTENT also 2, 3, 4, 6 or 8 resident workgroups per CU).
 * The launch mode itself (tiles or persistent) is the one opts selects.
 * out_rgba receives the last render.  best (host, nullable) receives the
 * winner and best_ms its time per render.  The winner becomes the handle's
 * tuning and is recorded for this workload (snerg_tuning_lookup).
 * Synchronises `stream`.
 */
int snerg_autotune(snerg_handle *h, const snerg_grid *grid, const float *mlp,
                   const snerg_camera *cams, int32_t n_cams, const snerg_opts *opts,
                   const snerg_tuning *candidates, int32_t n_candidates, int32_t reps,
                   float *out_rgba, snerg_tuning *best, float *best_ms, void *stream);

/*
 * Launch shapes by workload.  snerg_autotune also records its winner under
 * the call's workload signature (a hash of the grid's N, B, block count and
 * value type, every camera's image size, the kernel-selecting option flags,
 * mlp_on and early_stop); snerg_render, snerg_render_counted and
 * snerg_render_noalloc then use the recorded shape for a matching workload
 * and the handle's tuning (snerg_set_tuning) otherwise.
 * snerg_tuning_lookup writes the shape a render of this workload would use
 * to *t and whether it was recorded (*found = 1) or is the handle's (0).
 * snerg_tuning_save writes the recorded shapes to a text file (one line per
 * workload: hexadecimal signature, tile_w, tile_h, waves_per_group,
 * groups_per_cu) and snerg_tuning_load adds a file's entries to the handle
 * (SNERG_ERR_INVALID_ARG, and nothing added, for an unreadable file, a
 * malformed line or an invalid shape).  Host only.
 */
int snerg_tuning_lookup(snerg_handle *h, const snerg_grid *grid, const snerg_camera *cams, int32_t n_cams,
                        const snerg_opts *opts, snerg_tuning *t, int32_t *found);
int snerg_tuning_save(snerg_handle *h, const char *path);
int snerg_tuning_load(snerg_handle *h, const char *path);

/* ----------------------------------------------------------- measurement */

/*
 * Kernel timing for measurement.  While enabled, every on-th snerg_render
 * call (on = 1: every call; the first call after enabling is timed)
 * records a pair of HIP events on its stream around its render kernel
 * alone (after the tile-order pre-pass; around the whole replay in graph
 * mode) into a ring that keeps the last 256 timed renders.  Each event
 * pair costs the stream some microseconds, so timing a sample of the calls
 * disturbs a run of back-to-back renders less.  snerg_timing_enable with
 * on >= 1 empties the ring; on = 0 stops recording; on < 0 is
 * SNERG_ERR_INVALID_ARG.
 * snerg_timing_read synchronises the recorded events and writes up to
 * `max` kernel times in milliseconds, oldest first, to ms (host), and the
 * number written to *n.
 */
int snerg_timing_enable(snerg_handle *h, int32_t on);
int snerg_timing_read(snerg_handle *h, float *ms, int32_t max, int32_t *n);

#ifdef __cplusplus
}
#endif

#endif /* SNERG_H */
