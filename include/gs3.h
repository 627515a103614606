/*
 * gs3 — 3DGStream Stage-1 hot path on MI355X (gfx950): C ABI.
 *
 * One Stage-1 iteration of 3DGStream (arXiv 2403.01444, Sec. 4.1): query the
 * Neural Transformation Cache (NTC) at every Gaussian mean (Eq. 5),
 * transform the Gaussians (mu' = mu + dmu, q' = norm(q) x norm(dq), SH
 * rotation), render a view with a tile-based differentiable rasterizer
 * (Sec. 3.2, Eq. 2-4), evaluate the loss of Eq. 6, backpropagate, and step
 * Adam on the NTC parameters.
 *
 * Conventions for every call:
 *  - Array arguments are caller-owned DEVICE memory (contiguous float32,
 *    structure of arrays) unless a comment says "host".  The library never
 *    frees them and never keeps them beyond what a comment states.
 *  - Calls are asynchronous on the context's stream (gs3_set_stream) unless
 *    a comment says they synchronise.  Kernel-side conditions (pair-list
 *    overflow, non-finite loss) raise device flags, reported by
 *    gs3_debug_counts / gs3_check_flags as GS3_ECAPACITY / GS3_ENONFINITE.
 *  - Every call returns a gs3_status and never aborts the process; the text
 *    of the last error of a context is returned by gs3_last_error.
 *  - Gradient outputs ACCUMULATE (+=); the caller zeroes them.  Any gradient
 *    pointer may be NULL to skip that output.
 *  - Quaternions are (w, x, y, z); the identity is (1, 0, 0, 0) (Sec. 4.2).
 *  - Images are planar 3 x H x W float32 (channel, row, column).
 */
#ifndef GS3_H
#define GS3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GS3_OK = 0,
    GS3_EINVAL = -1,      /* bad argument (NULL, size out of range, bad slot) */
    GS3_ENOMEM = -2,      /* device allocation failed */
    GS3_EHIP = -3,        /* a HIP runtime call failed */
    GS3_ECAPACITY = -4,   /* more (Gaussian, tile) pairs than max_pairs */
    GS3_ENONFINITE = -5,  /* the loss was NaN or infinite */
    GS3_ESTATE = -6       /* call out of order (e.g. backward before render) */
} gs3_status;

enum { GS3_F32 = 0, GS3_F16 = 1, GS3_BF16 = 2 };            /* NTC storage precision */
enum { GS3_SORT_DEPTH_FIRST = 0, GS3_SORT_RADIX64 = 1 };    /* pair-ordering method */

#define GS3_MAX_LEVELS 16
#define GS3_TILE 16          /* tiles are 16 x 16 pixels */
#define GS3_MAX_TILES 16384  /* ceil(W/16) * ceil(H/16) must not exceed this */
#define GS3_MAX_WIDTH 4096   /* widest image (256 tile columns) */

/* NTC shape (Sec. 4.1, Suppl. Sec. A): L levels of a multi-resolution hash
 * grid with F = 2 features per entry and 2^log2_T entries per hashed level,
 * then an MLP (L*F) -> 64 -> 64 -> 7 with ReLU hidden layers, no biases. */
typedef struct {
    int32_t levels;                  /* L, 1..16; L*F must be 32 */
    int32_t feats;                   /* F, must be 2 */
    int32_t log2_T;                  /* 10..22 */
    int32_t hidden;                  /* must be 64 */
    int32_t precision;               /* GS3_F32 | GS3_F16 | GS3_BF16 */
    int32_t res[GS3_MAX_LEVELS];     /* grid resolution N_l per level, 1..65535 */
    float aabb_min[3];               /* scene AABB corner */
    float inv_extent[3];             /* 1 / (aabb_max - aabb_min), per axis */
} gs3_ntc_config;

typedef struct {
    int64_t max_gaussians;           /* capacity in Gaussians, >= 1 */
    int64_t max_pairs;               /* capacity in (Gaussian, tile) pairs per slot */
    int32_t max_width, max_height;   /* largest image; max_width <= GS3_MAX_WIDTH */
    int32_t num_slots;               /* renders whose state is kept for backward, 1..8 */
    int32_t sort_mode;               /* GS3_SORT_DEPTH_FIRST (default) | GS3_SORT_RADIX64 */
    int32_t enable_ntc;              /* 0: rasterizer only */
    int32_t grad_record_log2;        /* 0: the backward blend accumulates per-Gaussian gradients
                                        with atomics (fastest).  k > 0: deterministic mode, each
                                        walked (tile, Gaussian) pair writes its sums to a record
                                        buffer of 2^k pairs, gathered per Gaussian in a fixed order;
                                        pairs past the buffer fall back to atomics */
    gs3_ntc_config ntc;
} gs3_config;

/* Frozen Gaussians (Sec. 3.1): n means (n x 3), quaternions (n x 4),
 * log-scales (n x 3), opacity logits (n), SH coefficients
 * (n x (sh_degree+1)^2 x 3, coefficient-major, channel-minor), sh_degree 0..3.
 * Real orthonormal SH basis with the Condon-Shortley phase; colour =
 * max(0, sum_k sh_k Y_k(d) + 0.5). */
typedef struct {
    int64_t n;
    int32_t sh_degree;
    int32_t reserved;
    const float* means;
    const float* quats;
    const float* log_scales;
    const float* opacity_logits;
    const float* sh;
} gs3_gaussians;

/* Pinhole camera: pixel (x, y) is evaluated at integer coordinates; a
 * camera-space point t maps to (fx t_x / t_z + cx, fy t_y / t_z + cy).
 * world_to_cam is the row-major 3 x 4 [R | t]; cam_pos its centre;
 * near_z the cull plane (t_z <= near_z is culled); bg the background. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy, near_z;
    float world_to_cam[12];
    float cam_pos[3];
    float bg[3];
} gs3_camera;

/* Gradient outputs of gs3_render_backward (all accumulate, any may be NULL).
 * Stage 1 trains only the NTC, so only d_dmu and d_dq are needed there;
 * the others give the full adjoint.  d_uv, d_conic, d_opacity, d_rgb are the
 * per-Gaussian 2D accumulators (image-space mean, conic (A, B, C) with
 * power = -(A dx^2 + C dy^2)/2 - B dx dy, activated opacity, colour). */
typedef struct {
    float* d_means;          /* n x 3 */
    float* d_quats;          /* n x 4 */
    float* d_log_scales;     /* n x 3 */
    float* d_opacity_logits; /* n */
    float* d_sh;             /* n x (deg+1)^2 x 3 */
    float* d_dmu;            /* n x 3 */
    float* d_dq;             /* n x 4 */
    float* d_uv;             /* n x 2 */
    float* d_conic;          /* n x 3 */
    float* d_opacity;        /* n */
    float* d_rgb;            /* n x 3 */
    /* Stage 2 bookkeeping (Sec. 4.2), both accumulated, both or neither:
     * vspace_grad[i] += |(dL/du W/2, dL/dv H/2)|, the norm of the gradient
     * with respect to the Gaussian's mean in normalised device coordinates;
     * vspace_count[i] += 1 when the Gaussian is visible in the view. */
    float* vspace_grad;      /* n */
    float* vspace_count;     /* n */
} gs3_grads;

typedef struct gs3_ctx gs3_ctx;

/* Create a context on the current HIP device: allocates every workspace
 * (pair lists sized by max_pairs, per-slot render state, NTC parameters and
 * Adam state).  Synchronises.  Returns GS3_EINVAL for out-of-range fields,
 * GS3_ENOMEM when an allocation fails. */
gs3_status gs3_create(const gs3_config* cfg, gs3_ctx** out);

/* Free a context and everything it allocated.  Synchronises.  NULL is a no-op. */
void gs3_destroy(gs3_ctx* ctx);

/* Text of the last error on this context (static storage owned by ctx). */
const char* gs3_last_error(const gs3_ctx* ctx);

/* Launch all further work of this context on `hip_stream` (a hipStream_t;
 * NULL = the default stream). */
gs3_status gs3_set_stream(gs3_ctx* ctx, void* hip_stream);

/* ---- Per-frame setup ------------------------------------------------------ */

/* Spatial order of n means: perm (n u32, DEVICE) lists the indices sorted
 * by the 30-bit Morton code of (mean - aabb_min) * inv_extent (clamped to
 * [0, 1], 10 bits per axis), ties by index.  Stage 1 keeps the Gaussians
 * frozen for the whole frame (Sec. 4.1), so reordering them once per frame
 * is free to choose; neighbouring Gaussians then share hash-grid cells and
 * cache lines. */
gs3_status gs3_morton_order(gs3_ctx* ctx, const float* means, int64_t n, const float aabb_min[3],
                            const float inv_extent[3], uint32_t* perm);

/* dst[i, :] = src[perm[i], :] for n rows of row_floats floats (DEVICE;
 * dst must not alias src; every perm[i] must index a row of src, which may
 * hold more rows than dst). */
gs3_status gs3_gather_rows(gs3_ctx* ctx, const float* src, const uint32_t* perm, int64_t n, int32_t row_floats,
                           float* dst);

/* ---- Neural Transformation Cache (Sec. 4.1, Eq. 5) ----------------------- */

/* Number of float32 NTC parameters: table (sum_l min((N_l+1)^3, T) x F)
 * followed by W1 (64 x L*F), W2 (64 x 64), W3 (7 x 64), row-major [out][in]. */
gs3_status gs3_ntc_num_params(const gs3_ctx* ctx, int64_t* n);

/* Load the float32 master parameters from HOST memory (layout above), reset
 * the Adam moments, the step counter and the accumulated gradients.
 * Synchronises. */
gs3_status gs3_ntc_load(gs3_ctx* ctx, const float* host_params, int64_t n);

/* Copy the float32 master parameters to HOST memory (cap >= num_params).
 * Synchronises. */
gs3_status gs3_ntc_save(gs3_ctx* ctx, float* host_params, int64_t cap);

/* Initialise the NTC parameters on the device (Suppl. Sec. A gives the
 * architecture, not the initialisation; the instant-NGP encoding it follows
 * starts its table near zero): table entries U(-1e-4, 1e-4), each weight
 * matrix Kaiming-uniform U(-sqrt(6 / fan_in), +sqrt(6 / fan_in)) (fan-in 32
 * for W1, 64 for W2 and W3).  Parameter i is b * (2u - 1), u = (top 24 bits
 * of output i of SplitMix64 seeded with `seed`) / 2^24, where output i is
 * the SplitMix64 mixing function applied to seed + (i + 1) *
 * 0x9E3779B97F4A7C15 (Steele, Lea and Flood 2014); float32 arithmetic, one
 * rounding.  Resets the gradients, Adam moments and step counter like
 * gs3_ntc_load.  Synchronises. */
gs3_status gs3_ntc_init(gs3_ctx* ctx, uint64_t seed);

/* Checkpoint of the whole NTC training state: a fixed header (magic
 * "GS3NTC1", parameter count, Adam step, NTC shape and AABB), then the
 * float32 parameters and the first and second Adam moments (num_params
 * each), all in HOST memory.  gs3_ntc_state_bytes gives the size;
 * gs3_ntc_save_state writes it (cap >= that size, *used = the size, may be
 * NULL); gs3_ntc_load_state restores parameters, moments and step (the
 * gradients are zeroed) and returns GS3_EINVAL when n or the saved shape or
 * AABB differ from this context's.  The storage precision may differ (the
 * working copy is rebuilt from the float32 parameters).  Both synchronise. */
gs3_status gs3_ntc_state_bytes(const gs3_ctx* ctx, size_t* bytes);
gs3_status gs3_ntc_save_state(gs3_ctx* ctx, void* host, size_t cap, size_t* used);
gs3_status gs3_ntc_load_state(gs3_ctx* ctx, const void* host, size_t n);

/* (dmu, dq) = MLP(h(mu)) for n means (n x 3) -> dmu (n x 3), dq (n x 4).
 * Means outside the AABB get the identity (0, (1,0,0,0)) (Suppl. Sec. A).
 * token: 0, or the token of the last gs3_ntc_prepare, whose means and n
 * these must be (GS3_ESTATE for a stale token, GS3_EINVAL for other means).
 * With a token the context also keeps each point's encoding h(mu) for the
 * next gs3_ntc_backward with that token. */
gs3_status gs3_ntc_forward(gs3_ctx* ctx, const float* means, int64_t n, uint64_t token, float* dmu, float* dq);

/* Accumulate into the context's float32 gradient buffers the gradient of
 * <d_dmu, dmu> + <d_dq, dq> for the same means (adjoint of Eq. 5: MLP
 * backward, then the hash-table scatter-add).  token as for
 * gs3_ntc_forward: with a token the table gradient is the per-entry sum over
 * the prepared contribution lists (no atomics, fixed order) and the encoding
 * of the last forward with that token is reused when no gs3_ntc_step,
 * gs3_ntc_init or load came in between; with 0 the table gradient is
 * scattered with atomics. */
gs3_status gs3_ntc_backward(gs3_ctx* ctx, const float* means, int64_t n, uint64_t token,
                            const float* d_dmu, const float* d_dq);

/* Per-frame setup for gs3_ntc_backward on frozen means (Stage 1 keeps the
 * previous frame's Gaussians frozen, Sec. 4.1): for every (mean, level,
 * corner) the table entry and trilinear weight are computed once and the
 * contributions are sorted by entry.  *token receives a new nonzero token
 * that names this preparation; forward and backward calls pass it to use
 * the prepared lists.  The caller guarantees that the contents of `means`
 * do not change while the token is in use; a later gs3_ntc_prepare makes
 * the previous token stale.  Allocates device memory on first use or growth
 * (about 3.3 KB per mean) and synchronises. */
gs3_status gs3_ntc_prepare(gs3_ctx* ctx, const float* means, int64_t n, uint64_t* token);

/* One Adam step on the NTC parameters with the accumulated gradients,
 * then zero the gradients and refresh the FP16/BF16 working copy. */
gs3_status gs3_ntc_step(gs3_ctx* ctx, float lr, float beta1, float beta2, float eps);

/* Copy the accumulated float32 gradients (num_params) to DEVICE memory. */
gs3_status gs3_ntc_grads(gs3_ctx* ctx, float* dev_out, int64_t cap);

/* Zero the accumulated gradients. */
gs3_status gs3_ntc_zero_grads(gs3_ctx* ctx);

/* Warm-up loss (Eq. 7) averaged over n points: mean ||dmu||_1 -
 * mean (dq_w / ||dq||)^2.  Writes the loss to loss_dev[0] (device float)
 * and OVERWRITES d_dmu (n x 3), d_dq (n x 4) with its gradient. */
gs3_status gs3_warmup_loss(gs3_ctx* ctx, const float* dmu, const float* dq, int64_t n,
                           float* loss_dev, float* d_dmu, float* d_dq);

/* ---- Rasterizer (Sec. 3.2, Eq. 2-4) -------------------------------------- */

/* Transform (mu' = mu + dmu, q' = norm(q) x norm(dq), SH evaluated at the
 * direction rotated back by R(q') R(norm q)^T) and render one view into
 * `image` (3 x H x W).  dmu (n x 3) and dq (n x 4) may be NULL (no
 * translation / no rotation).  The slot keeps this render's state for
 * gs3_render_backward, INCLUDING the pointers g->*, dmu and dq: they must
 * stay valid and unchanged until the slot's backward has run. */
gs3_status gs3_render(gs3_ctx* ctx, int32_t slot, const gs3_gaussians* g, const float* dmu,
                      const float* dq, const gs3_camera* cam, float* image);

/* Adjoint of the slot's last gs3_render for dL/dimage (3 x H x W); gradients
 * accumulate into `out`.  Per-pixel transmittance is recomputed from the
 * final transmittance, not stored. */
gs3_status gs3_render_backward(gs3_ctx* ctx, int32_t slot, const float* d_image, const gs3_grads* out);

/* Frame carry-over (Sec. 4.1: the transformed Gaussians are carried into the
 * next frame): means_out = mu + dmu (n x 3), quats_out = norm(q) x norm(dq)
 * (n x 4), sh_out = the SH coefficients turned with the Gaussian
 * (n x (deg+1)^2 x 3): band l >= 1 multiplied by M_l(dR), dR = R(q')
 * R(norm q)^T, M_l = [P_l(dR N_k)] A_l^{-1} over 2l+1 fixed directions N_k
 * (Suppl. Sec. B; the paper uses band 1 with N = e_x, e_y, e_z).  Rendering
 * the outputs without a transform gives the image gs3_render gives for the
 * inputs with (dmu, dq).  dmu / dq may be NULL.  Outputs must not alias the
 * inputs. */
gs3_status gs3_transform_bake(gs3_ctx* ctx, const gs3_gaussians* g, const float* dmu, const float* dq,
                              float* means_out, float* quats_out, float* sh_out);

/* ---- Stage 2: adaptive 3DG addition (Sec. 4.2) ---------------------------- */

/* Indices (ascending, written to idx, capacity n) of the elements that pass a
 * threshold; their number goes to *count (host memory; the call waits for
 * the stream).  With den != NULL: den[i] > 0 and num[i] / den[i] > threshold
 * (the average view-space gradient above tau_grad); with den == NULL:
 * num[i] >= threshold (pruning: opacity logits at or above logit(tau_alpha)).
 * n may not exceed max_gaussians. */
gs3_status gs3_select(gs3_ctx* ctx, const float* num, const float* den, int64_t n, float threshold,
                      uint32_t* idx, int64_t* count);

#define GS3_SPAWN 0   /* new Gaussian: identity rotation, opacity 0.1, source scale and SH */
#define GS3_SPLIT 1   /* quantity control: source rotation, opacity and SH, 80% of the scale */
/* Additional Gaussians around the sources src[idx[k]], k < m: mean
 * mu + sqrt(2) R S z_k, a draw of N(mu, 2 Sigma) for z_k ~ N(0, I) given in
 * z (m x 3, device); the other attributes by mode.  Outputs (device, m rows
 * each) follow the gs3_gaussians layout and must not alias the sources. */
gs3_status gs3_spawn(gs3_ctx* ctx, const gs3_gaussians* src, const uint32_t* idx, int64_t m, const float* z,
                     int32_t mode, float* means, float* quats, float* log_scales, float* opacity_logits,
                     float* sh);

/* ---- Loss (Eq. 6) and optimiser ------------------------------------------ */

/* L = (1 - lambda) L1 + lambda (1 - SSIM) over 3 x H x W images (11x11
 * Gaussian window, sigma 1.5, zero padding); lambda = 0 gives plain L1.
 * Writes L to loss_dev[0] and OVERWRITES d_image with dL/dimage. */
gs3_status gs3_loss(gs3_ctx* ctx, const float* image, const float* target, int32_t height,
                    int32_t width, float lambda_dssim, float* loss_dev, float* d_image);

/* gs3_loss for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): no
 * context, no allocation of any kind.  The kernels' scratch (SSIM partial
 * maps, per-block partial sums) lives in a static device array of the
 * library, about 76 MB, that every GPU the library runs on holds until the
 * process ends.  Same arguments and results as gs3_loss, launched on
 * `hip_stream` (a hipStream_t; NULL = the default stream) on the current
 * device.  Limits: 1 <= height, width <= 4096 and height x width <=
 * 2,097,152 (1920 x 1080 fits); larger images, NULL pointers or lambda
 * outside [0, 1] return GS3_EINVAL, a failed HIP call GS3_EHIP.  All calls
 * on one GPU share the array: calls that overlap on one GPU (other streams,
 * other host threads) race and must be serialised by the caller.  A
 * non-finite loss is written as computed; no flag is raised. */
gs3_status gs3_loss_noalloc(const float* image, const float* target, int32_t height, int32_t width,
                            float lambda_dssim, float* loss_dev, float* d_image, void* hip_stream);

/* In-place Adam on n float32 parameters (bias correction with `step` >= 1);
 * used by the direct per-Gaussian optimisation comparator. */
gs3_status gs3_adam(gs3_ctx* ctx, float* param, const float* grad, float* m, float* v, int64_t n,
                    int32_t step, float lr, float beta1, float beta2, float eps);

/* Set n floats of DEVICE memory to zero with a fill kernel on the context
 * stream (no memset node, so it is safe inside captured graphs); used to
 * clear gradient outputs between iterations. */
gs3_status gs3_zero(gs3_ctx* ctx, float* dev, int64_t n);

/* ---- Inspection (parity tests, benchmarks) ------------------------------- */

/* Counts of the slot's last render (any pointer may be NULL): the number of
 * (Gaussian, tile) pairs K, the sum over pixels of n_contrib (the tile-list
 * entries each pixel walked up to its last contributor of Eq. 4), the sum
 * over tiles of the longest such walk in the tile (the entries the blend
 * kernels evaluate for the whole tile), and the overflow flag.  The sums
 * are -1 when the slot holds no render.  Synchronises.  Returns
 * GS3_ECAPACITY when the pair list overflowed. */
gs3_status gs3_debug_counts(gs3_ctx* ctx, int32_t slot, int64_t* num_pairs, int64_t* sum_contrib,
                            int64_t* walked, int32_t* overflow);

/* Sorted pairs of the slot's last render into DEVICE buffers: keys
 * (tile << 32 | float bits of view-space z) and Gaussian indices; cap >=
 * num_pairs. */
gs3_status gs3_debug_pairs(gs3_ctx* ctx, int32_t slot, uint64_t* keys, uint32_t* vals, int64_t cap);

/* Per-tile [start, end) into the sorted pairs, (tiles x 2) u32, DEVICE. */
gs3_status gs3_debug_ranges(gs3_ctx* ctx, int32_t slot, uint32_t* ranges);

/* Per-Gaussian decisions of the slot's last render into DEVICE buffers (any
 * may be NULL): depth key bits (0xFFFFFFFF when culled), pixel box
 * (n x 4 int32: x0, y0, x1, y1), 2D record (n x 9 float: u, v, A, B, C,
 * opacity, r, g, b). */
gs3_status gs3_debug_gaussians(gs3_ctx* ctx, int32_t slot, uint32_t* key, int32_t* box, float* rec);

/* Per-pixel final transmittance (H x W float) and number of tile-list
 * entries walked up to the last contributor (H x W int32), DEVICE. */
gs3_status gs3_debug_pixels(gs3_ctx* ctx, int32_t slot, float* T_final, int32_t* last);

/* Device memory the context holds (workspaces sized at gs3_create plus the
 * per-frame NTC contribution lists), in bytes.  Per-pixel render state is
 * 8 bytes (final transmittance and last walked entry): transmittance is
 * recomputed in the backward, never stored per contributor (Eq. 4). */
gs3_status gs3_workspace_bytes(const gs3_ctx* ctx, int64_t* bytes);

/* Check the device flags raised since the last check (overflow of any slot,
 * non-finite loss) and clear them.  Synchronises. */
gs3_status gs3_check_flags(gs3_ctx* ctx);

/* ---- Profiling ----------------------------------------------------------- */

/* When on, every kernel launch is bracketed by HIP events on the context
 * stream; gs3_profile_query returns the summed device time (ms) and launch
 * count of one kernel by name, synchronising first.  gs3_profile_only
 * restricts the timing to the launches of one kernel (NULL or "": all), so
 * that a timed loop carries two events per launch of that kernel only. */
gs3_status gs3_profile_enable(gs3_ctx* ctx, int32_t on);
gs3_status gs3_profile_only(gs3_ctx* ctx, const char* kernel);
gs3_status gs3_profile_reset(gs3_ctx* ctx);
gs3_status gs3_profile_query(gs3_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* GS3_H */
