/*
 * gs.h -- C ABI of the MI355X (gfx950) differentiable Gaussian-splatting
 * rasterizer: projection, tile binning and sort, front-to-back compositing
 * of colour and depth, the analytic backward, and a continuous-batching
 * render server.
 *
 * What is computed (paper, §3.1 "Preliminary"):
 *   Eq. 1  each 3D Gaussian G(x) = exp(-1/2 (x - mu)^T Sigma^-1 (x - mu)),
 *          Sigma = R S S^T R^T from a rotation (unit quaternion) and scales;
 *   text   the Gaussians are projected onto the image plane as 2D Gaussians
 *          G' (EWA linearisation of the perspective map) and "processed in
 *          depth order";
 *   Eq. 2  C(x_p) = sum_i c_i o_i G'_i(x_p) prod_{j<i} (1 - o_j G'_j(x_p)).
 * Anti-aliasing (§3.5.4): the 2D covariance is dilated by `dilation` px^2
 * and, with aa_compensate, the opacity is scaled by sqrt(det / det_dilated).
 * Depth regulariser (§3.5.3): the accumulated depth sum_i z_i a_i T_i is
 * rendered beside the colour; expected depth = depth / alpha.
 * Densification statistics (§3.1, and AbsGS in §3.5.4): the backward
 * returns |dL/d mean2d| per view and, optionally, the per-pixel absolute
 * accumulation of dL/d mean2d.
 * Level of detail (§3.4.2): the server picks a level per render-time
 * partition from the partition-camera distance under a Gaussian budget.
 *
 * Rules the paper leaves open, fixed here: alpha = min(0.99, o' G');
 * entries with alpha < 1/255 are skipped; a pixel stops before an entry
 * that would take its transmittance below 1e-4; pixel centres at
 * integer + 0.5; 16x16 tiles; a Gaussian covers the tiles of the square
 * [floor(m) - r, floor(m) + r], r = ceil(3 sqrt(lambda_max)); ties in depth
 * are broken by input order; colour = max(0, sum_lm sh_lm Y_lm(d) + 0.5)
 * with real SH of degree <= 3 (m = -l..l order, Condon-Shortley phase).
 *
 * Conventions for every call:
 *   - Array pointers are DEVICE pointers owned by the caller, contiguous,
 *     float32 unless stated.  The library allocates no device memory in
 *     these calls; scratch comes from a caller-provided workspace whose
 *     size the matching *_workspace_size function returns (256-byte
 *     aligned pointers required).
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *     asynchronously; no call of the rendering path synchronises it.
 *   - Return value 0 (GS_OK) or a negative GS_ERR_* code; nothing throws.
 *     gs_last_error() returns the calling thread's last message.
 *   - Gaussian parameters over n Gaussians: means [3][n], scales [3][n]
 *     (positive), quats [4][n] as (w, x, y, z) (normalised inside) and
 *     opacities [n] in (0, 1) are structure-of-arrays; sh [n][16][3]
 *     (Gaussian, coefficient, channel) keeps each Gaussian's 48 colour
 *     coefficients in one 192-byte row, so that the few Gaussians a view
 *     sees read whole rows (16-byte aligned base pointer required).
 *   - Several views of the same Gaussians are rendered in one launch per
 *     stage (at most GS_MAX_VIEWS).  A "slot" is (view, Gaussian) with index
 *     view * n + gaussian.  Tiles of all views share one numbering (view
 *     tile offsets are the running sums of ceil(W/16) * ceil(H/16)); pixels
 *     likewise (running sums of W * H), each view stored row-major.
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_OK 0
#define GS_ERR_INVALID_ARG (-1)
#define GS_ERR_CAPACITY (-2)
#define GS_ERR_HIP (-3)
#define GS_ERR_BUDGET (-4)
#define GS_EAGAIN (-5)
#define GS_ERR_INTERNAL (-6)

#define GS_MAX_VIEWS 16
#define GS_TILE 16
#define GS_REC_FLOATS 16
#define GS_GRAD2D_FLOATS 12

/* Pinhole camera.  viewmat is the row-major world-to-camera matrix
 * [R | t; 0 0 0 1] with OpenCV axes (x right, y down, z forward).
 * Gaussians with view depth outside [near_plane, far_plane] are culled. */
typedef struct gs_camera {
    float fx, fy, cx, cy;
    float viewmat[16];
    int32_t width, height;
    float near_plane, far_plane;
} gs_camera;

typedef struct gs_options {
    int32_t sh_degree;      /* 0..3: SH bands used for colour */
    float dilation;         /* px^2 added to the 2D covariance diagonal (0.3) */
    int32_t aa_compensate;  /* 1: opacity *= sqrt(det(S2D) / det(S2D + dilation I)) */
    float bg[3];            /* background colour added as T_final * bg */
} gs_options;

/* app (nullable): appearance offsets [n][4] = (dc_r, dc_g, dc_b, do) from
 * gs_appearance_fwd (§3.5.1).  When set, the colour constant 1/2 becomes dc
 * (colour = max(0, sum_lm sh_lm Y_lm(d) + dc)) and the opacity becomes
 * o (1 - do); dc = 1/2, do = 0 is the plain rasterizer.  16-byte aligned. */
typedef struct gs_gaussians {
    const float *means, *scales, *quats, *opacities, *sh;
    int64_t n;
    const float *app;
} gs_gaussians;

/* Parameter gradients, same layouts as gs_gaussians; written (not added to),
 * summed over the views of the call.  d_app [n][4] (nullable; used only when
 * gs_gaussians.app is set) receives the gradient with respect to the
 * appearance offsets. */
typedef struct gs_gaussians_grad {
    float *d_means, *d_scales, *d_quats, *d_opacities, *d_sh;
    float *d_app;
} gs_gaussians_grad;

/* Projected per-slot records (n_views * n slots).
 *   rec  [slots][16] float: floor(mean2d x), floor(mean2d y); qa, qb;
 *        qc, opacity', depth, frac(mean2d x); r, g, b, frac(mean2d y);
 *        hx, hy, 0, 0.
 *        The mean is split into an exact integer part and a fraction so
 *        compositing can form tile-relative coordinates without the rounding
 *        of large pixel coordinates.  (qa, qb, qc) = -log2(e) (A/2, B, C/2)
 *        for the conic (A, B, C) of the dilated 2D covariance, so that
 *        G' = exp2(qa dx^2 + qb dx dy + qc dy^2).  (hx, hy) are half-widths
 *        of a box around the mean outside which opacity' G' < 1/255 at every
 *        pixel centre (with a margin over float32 rounding; negative when
 *        opacity' < 1/255): compositing skips entries whose box misses its
 *        pixels, which leaves every result unchanged.
 *   rect [slots][2] uint32: global id of the first tile of the rectangle;
 *        rectangle width in tiles | (tiles per image row << 16).
 *   tiles[slots] uint32: tiles covered, 0 if culled.
 *   depth_key[slots] uint32: bit pattern of the float32 view depth
 *        (0xFFFFFFFF if culled); the primary sort key inside a tile.
 *   tile_order [tiles of all views] uint32, optional (NULL = tile index
 *        order): gs_bin_sort writes a launch order of the tiles, longest
 *        lists first, and the compositing calls launch their workgroups in
 *        that order.  Scheduling only: results do not depend on it.
 *   tile_mask [slots] uint64, optional (NULL = every tile of the
 *        rectangle): exact tile culling.  For rectangles of at most 64
 *        tiles, bit (ty - y0) * width + (tx - x0) is set for the tiles whose
 *        pixel centres the alpha ellipse d^T Sigma'^-1 d <= 2 tau reaches
 *        (its minimum over the tile's pixel-centre rectangle widened by
 *        1e-3 px, within 2 tau (1 + 4e-6)); tiles counts those, and binning
 *        emits only them.  0 for larger rectangles (all tiles kept);
 *        unwritten for culled slots.
 * Records of culled slots are left unwritten. */
typedef struct gs_projected {
    float *rec;
    uint32_t *rect;
    uint32_t *tiles;
    uint32_t *depth_key;
    uint32_t *tile_order;
    uint64_t *tile_mask;
} gs_projected;

const char *gs_last_error(void);
const char *gs_version(void);

/* Total tiles and pixels of a list of views. */
int gs_views_extent(const gs_camera *cams, int32_t n_views, int64_t *n_tiles, int64_t *n_pixels);

/* Projection and colour (§3.1 text after Eq. 1; §3.5.4 anti-aliasing).
 * One thread per Gaussian handles every view, reading its parameters once.
 * Errors: GS_ERR_INVALID_ARG for n <= 0 or n_views outside 1..GS_MAX_VIEWS,
 * null pointers, image sizes outside 1..16384 or sh_degree outside 0..3. */
int gs_project(const gs_gaussians *g, const gs_camera *cams, int32_t n_views, const gs_options *opt,
               const gs_projected *out, void *stream);

/* Scratch bytes needed by gs_bin_sort for n_slots slots and room for
 * pair_capacity (tile, Gaussian) pairs. */
size_t gs_bin_workspace_size(int64_t n_slots, int64_t pair_capacity);

/* Tile binning and depth order ("processed in depth order", §3.1).
 * Sorts the visible slots by depth key (stable, so ties keep slot order),
 * expands each into one pair per covered tile, stably sorts the pairs by
 * global tile id, and writes
 *   pair_vals[P]          slot of each pair, tile-major, depth order inside;
 *   tile_ranges[T][2]     [start, end) of every global tile in pair_vals.
 * Asynchronous, with no host read-back: the pair count P is written to the
 * DEVICE int64 *n_pairs_dev (8-byte aligned) on the stream, and every launch
 * after the count is sized by slots or pair_capacity and reads the counts on
 * the device.  If P > pair_capacity (or P > 2^32 - 256), pair_vals is left
 * unwritten and every tile range is empty (compositing then sees no
 * Gaussians): the caller reads *n_pairs_dev after the stream and, when it
 * exceeds pair_capacity, grows its buffers and calls again. */
int gs_bin_sort(const gs_projected *proj, const gs_camera *cams, int32_t n_views, int64_t n,
                int64_t pair_capacity, uint32_t *pair_vals, uint32_t *tile_ranges, int64_t *n_pairs_dev,
                void *ws, size_t ws_bytes, void *stream);

/* Front-to-back compositing (Eq. 2), one 256-thread workgroup per 16x16
 * tile.  Outputs over all views' pixels: rgb [pix][3] (C + T_final * bg),
 * depth [pix] (sum z a T), alpha [pix] (1 - T_final), T_final [pix] and
 * last [pix] (1-based position in the tile's list of the last composited
 * entry, 0 if none).  T_final and last feed gs_render_bwd. */
int gs_render_fwd(const gs_projected *proj, const uint32_t *pair_vals, const uint32_t *tile_ranges,
                  const gs_camera *cams, int32_t n_views, const gs_options *opt, float *rgb, float *depth,
                  float *alpha, float *T_final, int32_t *last, void *stream);

/* Measurement only: per pixel, the numbers of list entries compositing has
 * to evaluate, written to n_eval [pix][2]: [0] the forward's -- entries whose
 * (hx, hy) box contains the pixel centre, up to and including the one that
 * stops the pixel; [1] the backward's -- the same entries up to and including
 * the pixel's last composited one.  The units of work behind the compositing
 * throughput figures; not needed to render. */
int gs_render_count(const gs_projected *proj, const uint32_t *pair_vals, const uint32_t *tile_ranges,
                    const gs_camera *cams, int32_t n_views, int32_t *n_eval, void *stream);

/* Workspace of the backward: gs_render_bwd_workspace_size(n_slots) bytes of
 * per-slot 2D gradients, optionally followed (gs_render_bwd) or given
 * separately (gs_composite_bwd's seg_ws) by gs_seg_workspace_size(n_tiles,
 * n_pairs) bytes for the segmented walk: tile lists longer than 512
 * positions are then walked in 512-position segments by separate
 * workgroups, each starting from the transmittance and colour behind it
 * (folded from per-segment states a pre-pass computes), so the longest
 * lists no longer serialise the launch.  A smaller or absent segment area
 * walks every list whole; results agree to float rounding either way. */
size_t gs_render_bwd_workspace_size(int64_t n_slots);
size_t gs_seg_workspace_size(int64_t n_tiles, int64_t n_pairs);

/* Compositing (Eq. 2) with the lists longer than 512 positions split into
 * 512-position segments walked by several workgroups, in the segment area
 * seg_ws (gs_seg_workspace_size(n_tiles, n_pairs) bytes, 256-byte aligned;
 * a smaller area, or one too small for the states, walks every list whole
 * as gs_render_fwd does).  A long list's workgroup walks its first two
 * segments with the stop rule; for the pixels still compositing, one
 * workgroup per later segment keeps the segment's state with T restarted
 * at 1; one thread per such pixel folds the segments (T only decreases, so
 * the pixel stops in segment j exactly when T T_seg_j < 1e-4) and the stop
 * segment is walked again from the pixel's state before it.  Outputs as
 * gs_render_fwd up to the grouping of the products: equal to float
 * rounding, a stop decision moving only where T is within rounding of the
 * threshold.  seg_ws then holds each segment's state (transmittance and
 * colour and depth with T restarted at the segment's start, over the
 * pixel's composited entries) -- the states the segmented backward folds:
 * pass the same seg_ws, unchanged, to gs_composite_bwd with seg_ready = 1,
 * together with these lists, T_final and last. */
int gs_render_fwd_seg(const gs_projected *proj, const uint32_t *pair_vals, const uint32_t *tile_ranges,
                      const gs_camera *cams, int32_t n_views, const gs_options *opt, float *rgb, float *depth,
                      float *alpha, float *T_final, int32_t *last, void *seg_ws, size_t seg_ws_bytes,
                      void *stream);

/* Backward of compositing and projection.  Transmittance is recovered back
 * to front from T_final and last instead of stored per-pixel lists.  Inputs
 * d_rgb [pix][3], d_depth [pix], d_alpha [pix] (any may be NULL = zero).
 * Outputs: parameter gradients summed over views (written, not added);
 * mean2d_grad_norm [n_views][n] = |dL/d mean2d| in pixels per view;
 * absgrad [n_views][n][2] (nullable) = sum over pixels of |dL_p/d mean2d|
 * per axis.  The workspace holds per-slot 2D gradients. */
int gs_render_bwd(const gs_gaussians *g, const gs_camera *cams, int32_t n_views, const gs_options *opt,
                  const gs_projected *proj, const uint32_t *pair_vals, const uint32_t *tile_ranges,
                  const float *T_final, const int32_t *last, const float *d_rgb, const float *d_depth,
                  const float *d_alpha, const gs_gaussians_grad *out, float *mean2d_grad_norm, float *absgrad,
                  void *ws, size_t ws_bytes, void *stream);

/* The two halves of gs_render_bwd, for callers that schedule or time them
 * separately.  gs_composite_bwd overwrites the rows of grad2d [slots][12]
 * (fields as in gs_render_bwd_grad2d) whose slot has tiles > 0 with the
 * compositing backward and leaves the other rows unwritten; the AbsGS sums
 * (fields 10, 11) are accumulated only when abs_sums is nonzero, else they
 * are 0 (gs_render_bwd accumulates them when its absgrad output is given).
 * seg_ready = 1: seg_ws holds the plan and segment states that
 * gs_render_fwd_seg wrote for these lists (no second walk here); 0: they
 * are computed here.  gs_project_bwd chains grad2d to the parameters
 * (outputs as in gs_render_bwd; grads_zeroed = 1: the outputs already hold
 * zeros and only the rows of Gaussians some view sees are written), reading
 * only those rows of grad2d. */
int gs_composite_bwd(const gs_projected *proj, const uint32_t *pair_vals, const uint32_t *tile_ranges,
                     const gs_camera *cams, int32_t n_views, const gs_options *opt, const float *T_final,
                     const int32_t *last, const float *d_rgb, const float *d_depth, const float *d_alpha,
                     int32_t abs_sums, int64_t n_slots, float *grad2d, void *seg_ws, size_t seg_ws_bytes,
                     int32_t seg_ready, void *stream);
int gs_project_bwd(const gs_gaussians *g, const gs_camera *cams, int32_t n_views, const gs_options *opt,
                   const gs_projected *proj, const float *grad2d, const gs_gaussians_grad *out,
                   float *mean2d_grad_norm, float *absgrad, int32_t grads_zeroed, void *stream);
/* Zeroes the parameter-gradient arrays of n Gaussians (d_app too when not
 * NULL), device pointers as in gs_gaussians_grad, with launches of at most
 * 64 workgroups each.  With it, gs_project_bwd's grads_zeroed = 1 writes
 * only the rows of Gaussians some view sees (the others are 84 % of the
 * rows of a large street-level scene): enqueued on a second stream after
 * gs_composite_bwd, which is bound by instruction issue and leaves most of
 * the memory bandwidth free, the fill runs beside it and takes few of its
 * wave slots; the caller orders gs_project_bwd after both (an event).
 * Returns GS_ERR_INVALID_ARG for a NULL array (other than d_app) or n < 0,
 * else the launch status. */
int gs_grads_zero(const gs_gaussians_grad *out, int64_t n, void *stream);

/* Per-slot 2D gradients of the last gs_render_bwd call that used `ws`
 * ([slots][12]: d mean2d x, y; d conic A, B, C; d opacity'; d rgb; d depth;
 * |d mean2d| x, y accumulations; rows of slots with tiles == 0 are
 * unwritten) -- for inspection and tests. */
const float *gs_render_bwd_grad2d(void *ws);

/* Measurement.  While timing is enabled, every launch of the kernels below
 * records a pair of library-owned events around itself on the stream it
 * is launched on (binning: around the whole gs_bin_sort sequence);
 * gs_kernel_timing_read waits for the recorded pairs of one kernel, returns
 * their summed elapsed time and count, and forgets them.  Enabling or
 * disabling forgets every pending pair; disabling also waits for and
 * releases the library's timing events.  For benchmarks: the event records
 * cost about a microsecond per launch. */
#define GS_KERNEL_PROJECT_FWD 0   /* k_project_fwd */
#define GS_KERNEL_BIN_SORT 1      /* the binning launches of one gs_bin_sort */
#define GS_KERNEL_RENDER_FWD 2    /* k_render_fwd */
#define GS_KERNEL_RENDER_BWD 3    /* k_render_bwd */
#define GS_KERNEL_PROJECT_BWD 4   /* k_project_bwd */
#define GS_KERNEL_TIMED 5
int gs_kernel_timing(int32_t enable);
int gs_kernel_timing_read(int32_t kernel, double *total_ms, int64_t *launches);

/* Training loss and its gradient in one pass: the L1 term of Eq. 3 plus the
 * depth regulariser of §3.5.3 on the expected depth,
 *   L = mean_{pix, ch} |rgb - target_rgb|
 *     + lambda_depth * mean_pix |depth / max(alpha, 1e-10) - target_depth|
 * over n_pix pixels (rgb, target_rgb [pix][3]; depth, alpha, target_depth
 * [pix]; target_depth NULL drops the depth term).  Writes loss [1] and the
 * gradients d_rgb [pix][3], d_depth [pix], d_alpha [pix] (sign(x) as the
 * derivative of |x|, 0 at 0; no gradient through the clamp below 1e-10) on
 * the device.  The total is summed in a fixed order (deterministic). */
size_t gs_loss_workspace_size(int64_t n_pix);
int gs_loss_l1_depth(const float *rgb, const float *depth, const float *alpha, const float *target_rgb,
                     const float *target_depth, int64_t n_pix, float lambda_depth, float *loss, float *d_rgb,
                     float *d_depth, float *d_alpha, void *ws, size_t ws_bytes, void *stream);

/* gs_loss_l1_depth without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving or training
 * loops, harnesses that forbid allocation).  Same arguments, kernels and
 * results as gs_loss_l1_depth; its workgroup partials live in a static
 * 256 KiB array of the library, one copy per GPU (held until the process
 * ends), whose address is looked up once per device on the first call.  It
 * allocates nothing and needs no zeroed memory (every partial is written
 * before it is read).  n_pix above 2^26 (67,108,864 pixels) returns
 * GS_ERR_CAPACITY.  Calls that overlap in time on one GPU (different
 * streams or threads) share that array and race: serialise them. */
int gs_loss_l1_depth_noalloc(const float *rgb, const float *depth, const float *alpha, const float *target_rgb,
                             const float *target_depth, int64_t n_pix, float lambda_depth, float *loss,
                             float *d_rgb, float *d_depth, float *d_alpha, void *stream);

/* D-SSIM term of Eq. 3 and its gradient: weight * (1 - mean SSIM) over the
 * 3 width * height values of rgb against target (both [H][W][3] float32),
 * SSIM per pixel and channel with an 11x11 Gaussian window (sigma 1.5,
 * normalised), zero outside the image, C1 = 0.01^2, C2 = 0.03^2.  Writes
 * loss [1] and d_rgb [H][W][3] (the term's gradient) on the device; the
 * mean is summed in a fixed order. */
size_t gs_dssim_workspace_size(int32_t width, int32_t height);
int gs_dssim(const float *rgb, const float *target, int32_t width, int32_t height, float weight, float *loss,
             float *d_rgb, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Appearance transform module (§3.5.1; sizes from the implementation
 * details of the appendix).  Every Gaussian has an embedding (16 values),
 * every image one (32 values); a small MLP maps both to per-Gaussian colour
 * and opacity offsets:
 *   x = (g / max(|g|, 1e-12), e / max(|e|, 1e-12))       (48)
 *   h = ReLU(W1 x + b1)                                   (32)
 *   y = sigmoid(W2 h + b2) = (dc_r, dc_g, dc_b, do)       (4)
 * W1 [32][48] (Gaussian-embedding columns first), b1 [32], W2 [4][32],
 * b2 [4], row-major float32 device arrays.  The offsets y feed the
 * rasterizer through gs_gaussians.app; they only change when the image
 * embedding or the weights do, so rendering reuses them at no cost.
 * The opacity-offset regulariser is reg_weight * mean_i do_i.
 * ---------------------------------------------------------------------- */
#define GS_APP_GAUSS_DIM 16
#define GS_APP_IMAGE_DIM 32
#define GS_APP_HIDDEN 32
#define GS_APP_OUT 4

typedef struct gs_appearance_mlp {
    const float *w1, *b1, *w2, *b2;
} gs_appearance_mlp;

/* Gradients of the MLP's weights and of the image embedding, written (not
 * added to); d_image_emb may be NULL. */
typedef struct gs_appearance_grad {
    float *d_w1, *d_b1, *d_w2, *d_b2, *d_image_emb;
} gs_appearance_grad;

/* Scratch bytes of gs_appearance_fwd / gs_appearance_bwd (about 5.5 MB of
 * workgroup partials, whatever n). */
size_t gs_appearance_workspace_size(int64_t n);

/* Offsets y [n][4] of n Gaussians (gauss_emb [n][16], 16-byte aligned) for
 * one image embedding image_emb [32].  reg_value (nullable, device [1])
 * receives reg_weight * mean do, summed in a fixed order.  n = 0 writes
 * only reg_value = 0.  Errors: GS_ERR_INVALID_ARG for n < 0, null or
 * misaligned pointers, a workspace smaller than the size above. */
int gs_appearance_fwd(const float *gauss_emb, int64_t n, const float *image_emb, const gs_appearance_mlp *mlp,
                      float reg_weight, float *offsets, float *reg_value, void *ws, size_t ws_bytes, void *stream);

/* Backward of gs_appearance_fwd for the upstream gradient d_offsets [n][4]
 * plus, when d_reg (device [1], nullable) is given, d_reg times the
 * regulariser's gradient reg_weight / n on every do.  offsets are the
 * forward's outputs.  Writes d_gauss_emb [n][16] and every pointer of
 * `out`; the weight gradients are sums over all Gaussians, added in a fixed
 * order (deterministic). */
int gs_appearance_bwd(const float *gauss_emb, int64_t n, const float *image_emb, const gs_appearance_mlp *mlp,
                      const float *offsets, const float *d_offsets, const float *d_reg, float reg_weight,
                      float *d_gauss_emb, const gs_appearance_grad *out, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Densification bookkeeping (consumers of the backward's statistics between
 * training steps) and the 3D smoothing filter.
 *   - the statistic 3DGS densification thresholds is a Gaussian's mean
 *     image-space gradient over the views that rasterized it (§3.1, after
 *     Eq. 2); AbsGS (§3.5.4) uses the per-axis absolute sums instead;
 *   - in-partition prioritized densification (§3.3, Eq. 4): Gaussian i is a
 *     candidate only if its mean exceeds
 *       tau_i = tau_min (min(d_i, d_max) / d_max (eta - 1) + 1),
 *     d_i = distance from its mean to the partition's box (0 inside);
 *   - a Gaussian budget B caps the model (§3.4.1, the steerable
 *     densification each detail level trains under): after pruning, at most
 *     B - (n - pruned) candidates grow, those with the largest mean / tau_i
 *     (ties: lower index); a grown Gaussian is split when its largest scale
 *     exceeds split_scale, else cloned;
 *   - the Mip-Splatting 3D smoothing filter (§3.5.4): rate_i = max over the
 *     cameras holding the mean (depth in [near, far], projection inside the
 *     image widened by 15 % per side) of fx / depth; the filter adds
 *     (s_f / rate_i)^2 to every axis of Sigma, i.e. scales become
 *     sqrt(s^2 + (s_f / rate)^2) and the opacity is scaled by prod s / s'
 *     (= sqrt(det Sigma / det Sigma')); rate 0 (unseen) means no filter.
 * ---------------------------------------------------------------------- */
#define GS_DENSIFY_KEEP 0
#define GS_DENSIFY_CLONE 1
#define GS_DENSIFY_SPLIT 2
#define GS_DENSIFY_PRUNE 3

/* Adds one step's views to the running statistic: for every view v and
 * Gaussian i with tiles[v][i] > 0, accum[i] += value * view_scale[v] and
 * count[i] += 1 (views in order), where value = grad_norm[v][i] or, when
 * absgrad ([n_views][n][2]) is given instead, the length of absgrad[v][i].
 * view_scale is a host array [n_views] (NULL: all 1), e.g. (W/2, H/2)-style
 * unit changes folded into one factor.  n_views 1..GS_MAX_VIEWS. */
int gs_densify_accumulate(const uint32_t *tiles, const float *grad_norm, const float *absgrad, int32_t n_views,
                          int64_t n, const float *view_scale, float *accum, int32_t *count, void *stream);

typedef struct gs_densify_params {
    float box_min[3], box_max[3];  /* partition box */
    float tau_min, eta, d_max;     /* Eq. 4 */
    float prune_opacity;           /* opacity below this prunes */
    float split_scale;             /* largest scale above this splits, else clones */
    int64_t budget;                /* Gaussians allowed after this densification */
} gs_densify_params;

size_t gs_densify_workspace_size(int64_t n);

/* Writes action[n] (GS_DENSIFY_*) from the statistic (mean = accum / count
 * in float32, 0 when count is 0) and the parameters (means [3][n], scales
 * [3][n], opacities [n]).  counts (host [4]) receives: candidates, pruned,
 * grown, and the budget's room K.  Synchronises `stream` (the candidate and
 * pruned totals decide the selection).  n < 2^32 - 256. */
int gs_densify_select(const float *accum, const int32_t *count, const float *means, const float *scales,
                      const float *opacities, int64_t n, const gs_densify_params *p, uint8_t *action,
                      int64_t *counts, void *ws, size_t ws_bytes, void *stream);

/* rate[n] of the 3D filter over n_cams cameras (any number; taken 16 per
 * launch). */
int gs_filter3d_rate(const float *means, int64_t n, const gs_camera *cams, int32_t n_cams, float *rate, void *stream);

/* Filtered scales_out [3][n] and opacities_out [n], and the backward that
 * chains their gradients to d_scales [3][n] and d_opacities [n]. */
int gs_filter3d_fwd(const float *scales, const float *opacities, const float *rate, int64_t n, float s_f,
                    float *scales_out, float *opacities_out, void *stream);
int gs_filter3d_bwd(const float *scales, const float *opacities, const float *rate, int64_t n, float s_f,
                    const float *d_scales_out, const float *d_opacities_out, float *d_scales, float *d_opacities,
                    void *stream);

/* ------------------------------------------------------------------------
 * Level-of-detail selection and serving (§3.4.2 "Detail Level Selection",
 * Fig. 3b; distance thresholds as in Tab. 13).
 *
 * A level-of-detail scene holds levels 1 (coarsest) .. L (finest) of every
 * render-time partition.  All levels live in ONE set of parameter arrays
 * (gs_gaussians with n = the sum of all levels' sizes); the Gaussians of
 * (level l, partition p) are the contiguous range
 * [offsets[(l-1) * P + p], + counts[(l-1) * P + p]).
 * ---------------------------------------------------------------------- */
#define GS_MAX_LEVELS 8

typedef struct gs_lod_table {
    int32_t n_levels;            /* L, 1..GS_MAX_LEVELS */
    int32_t n_parts;             /* P >= 1 */
    const float *part_min;       /* [P][3] world AABB of the partition (host memory) */
    const float *part_max;       /* [P][3] */
    const int64_t *offsets;      /* [L][P] first Gaussian of (level, partition) (host memory) */
    const int64_t *counts;       /* [L][P] its number of Gaussians */
    /* thresholds[k]: largest partition-camera distance at which level L - k
     * is used (k = 0 .. L-1, increasing; the last is normally +inf) */
    float thresholds[GS_MAX_LEVELS];
    float margin;                /* metres added on every side of each AABB for the view test */
} gs_lod_table;

/* Host-only.  Chooses a level per partition for one camera:
 *   - a partition is culled (level 0) when its AABB grown by `margin` lies
 *     entirely outside one of the five planes of the view frustum (near
 *     plane, and the four sides through the image border widened by 15 % of
 *     the image size per side, as in the projection's Jacobian clamp);
 *   - otherwise its distance d is the distance from the camera centre to the
 *     nearest point of the (un-grown) AABB, 0 inside, and its level is the
 *     finest level L - k with d <= thresholds[k] (level 1 beyond all);
 *   - budget: while the selected Gaussians exceed `budget`, the farthest
 *     partition among those at the finest level in use above 1 drops one
 *     level (ties: lower partition id first); once every selected partition
 *     is at level 1, the farthest ones are dropped (level 0).
 * Writes level [P] and *total (selected Gaussians).  GS_ERR_BUDGET when the
 * budget cannot hold even the nearest visible partition at level 1;
 * GS_ERR_INVALID_ARG for a malformed table or camera. */
int gs_lod_select(const gs_lod_table *table, const gs_camera *cam, int64_t budget, int32_t *level,
                  int64_t *total);

/* Serving: a native request queue with worker threads (allocated by
 * gs_serve_create, the only allocating call).  Each request is a camera, a
 * Gaussian budget and a device output image [H][W][3] float32 owned by the
 * caller.  Requests wait until their arrival time; a worker takes every
 * arrived request at the head of the queue, in order, while the batch stays
 * within max_views_per_batch, the slot, pixel and tile capacities, and an
 * estimate of its (tile, Gaussian) pairs within pair_capacity (admission by
 * sort-buffer size: a request's estimate is its selected Gaussians times a
 * pairs-per-Gaussian ratio learned per image size from the batches already
 * rendered -- raised at once when a batch needs more, lowered gradually --
 * with 15 % headroom; pairs_per_gaussian seeds sizes not yet seen).  It
 * projects each view's selected segments, bins all views of the batch in one
 * sort and composites them in one multi-view launch, then copies each image
 * to its request's output.  Each worker has two HIP streams and
 * pipeline_depth sets of device buffers: with a depth of 2 the projection
 * and binning of the next batch (one stream) overlap the compositing of the
 * current one (the other), ordered by events, with no host wait in between.
 * A batch whose pairs still overflow pair_capacity is split in halves and
 * re-rendered (counted in split_batches); a single request that overflows
 * completes with GS_ERR_CAPACITY.  The rendered image is the image
 * gs_render_fwd_seg gives for the selected Gaussians alone (with
 * persistent compositing, gs_render_fwd's), whatever the batch or the
 * pipeline depth. */
typedef struct gs_serve_config {
    int32_t max_views_per_batch;   /* 1..GS_MAX_VIEWS; 1 = one request per launch */
    int32_t n_streams;             /* worker threads, 1..8 */
    int64_t slot_capacity;         /* selected Gaussians per batch, summed over its views */
    int64_t pair_capacity;         /* (tile, Gaussian) pairs per batch */
    int64_t pixel_capacity;        /* pixels per batch */
    int32_t queue_capacity;        /* pending requests; gs_serve_submit returns GS_EAGAIN beyond */
    int32_t pipeline_depth;        /* batches in flight per worker (buffer sets), 1..4 */
    int32_t persistent_ctas;       /* 0: lists longer than 512 positions composited in segments
                                      (gs_render_fwd_seg); > 0: persistent compositing, every list walked
                                      whole, by at most this many workgroups taking tiles from a counter */
    double pairs_per_gaussian;     /* admission ratio for image sizes not yet rendered; 0 = 8 */
} gs_serve_config;

typedef struct gs_completion {
    uint64_t ticket;
    int32_t status;                /* GS_OK or a GS_ERR_* code */
    int32_t batch_views;           /* views in the batch that rendered it */
    int64_t n_gaussians;           /* Gaussians selected for the request */
    int64_t n_pairs;               /* pairs of the whole batch */
    double t_arrival, t_start, t_done;   /* seconds on the server clock (gs_serve_now) */
} gs_completion;

typedef struct gs_serve_stats {
    int64_t submitted, completed, failed, batches;
    double mean_batch_views;
    double p50_ms, p99_ms, mean_ms, max_ms;   /* latency = t_done - t_arrival, completed requests */
    double span_s;                 /* first arrival to last completion */
    double req_per_s, mpix_per_s;  /* over span_s */
    int64_t split_batches;         /* batches re-rendered in halves after a pair overflow */
    double est_over_actual;        /* mean over admitted batches of estimated / rendered pairs */
    int64_t rebinned_batches;      /* batches binned again with the whole pair buffer after their
                                      estimate-sized bound (1.5 x estimate + 4096) fell short */
} gs_serve_stats;

typedef struct gs_server gs_server;

/* `scene` and `table` (with the arrays they point to) are copied: device
 * parameter pointers must stay valid until gs_serve_destroy.  Worker
 * threads use device `device`. */
int gs_serve_create(const gs_gaussians *scene, const gs_lod_table *table, const gs_options *opt,
                    const gs_serve_config *cfg, int32_t device, gs_server **out);
/* Seconds since the server was created (the clock of arrival times). */
double gs_serve_now(const gs_server *srv);
/* Queues one request arriving at t_arrival (server clock; it is not started
 * before).  An event is recorded on `stream` (a HIP stream of the server's
 * device; NULL is the null stream) and the worker writes out_rgb only after
 * it, so work the caller queued there before submitting (filling or
 * reusing out_rgb) is ordered before the image.  out_rgb must stay valid
 * until the request's completion is polled.  Selection errors
 * (GS_ERR_BUDGET, GS_ERR_INVALID_ARG) and requests larger than one batch's
 * capacities (GS_ERR_CAPACITY) are returned here; GS_EAGAIN when the queue
 * is full; GS_ERR_HIP when the event cannot be recorded. */
int gs_serve_submit(gs_server *srv, const gs_camera *cam, int64_t budget, float *out_rgb, void *stream,
                    double t_arrival, uint64_t *ticket);
/* Waits up to timeout_us for completions and returns up to max of them. */
int gs_serve_poll(gs_server *srv, gs_completion *done, int32_t max, int32_t timeout_us, int32_t *n_done);
int gs_serve_stats_get(gs_server *srv, gs_serve_stats *out);
/* Stops the workers after their current batch; requests still queued are
 * dropped.  Frees the server's device buffers. */
int gs_serve_destroy(gs_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
