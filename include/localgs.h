/*
 * localgs.h -- C ABI of the MI355X (gfx950) tile-based Gaussian-splatting
 * rasterizer with the Local-GS render stages (arXiv 2606.16566).
 *
 * Pipeline (Sec. II-A, Fig. 2 of the paper):
 *   lgs_project      -> projected 2D splats, depth keys, touched-tile rectangles
 *   lgs_sort         -> (tile, Gaussian) pairs ordered by tile, then depth
 *   lgs_tile_ranges  -> [start, end) of every tile's list
 *   lgs_render       -> RGB image, final transmittance, last-contributor index
 * plus the gradient path (lgs_render_backward, lgs_project_backward,
 * lgs_l1_loss), which the paper does not cover.
 *
 * Conventions shared by every entry point
 *  - Pointer arguments named as device buffers are device pointers owned by the
 *    caller; the library never allocates or frees device memory.  Workspace
 *    sizes come from the *_workspace_size queries.
 *  - Arrays are row-major and contiguous, float32 / int32 / uint32 as typed.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *    enqueues work on that stream; none synchronises the host.
 *  - Arguments are validated on the host before anything is enqueued; a failed
 *    check returns LGS_ERR_INVALID_ARG and enqueues nothing.  A HIP launch
 *    failure returns LGS_ERR_HIP.  lgs_last_error() then holds a message
 *    (per host thread).  No C++ exception crosses this interface.
 *  - Calls on different streams may run concurrently when their output
 *    buffers are disjoint.
 */
#ifndef LOCALGS_H
#define LOCALGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LGS_TILE 16

/*
 * Projected splat record: LGS_SPLAT_FLOATS floats (64 bytes) per Gaussian
 * (per view in a batch), written by lgs_project and read by the sort's exact
 * tile assignment, the render and the backward:
 *   [0..3]   a, b, c, o   conic (inverse 2D covariance, with a 0.3 px^2
 *                         low-pass added to the covariance) and opacity
 *   [4..5]   x, y         projected mean in pixels
 *   [6..8]   r, g, b      view-dependent colour, clamped at 0
 *   [9..15]  unused: never read; lgs_project writes them as zero, so that
 *            every record is written as one whole 64-byte sector
 * Record arrays must be 16-byte aligned; with 64-byte alignment (any
 * hipMalloc'd base) every record is one 64-byte memory sector, so that the
 * render's and the backward's gathers, whose addresses follow the depth
 * order of each tile's list, read one sector per (tile, Gaussian) instead of
 * one per attribute array.
 *
 * Gradient record: LGS_GRAD_FLOATS floats (36 bytes, packed) per element,
 * dL/d (a, b, c, o, x, y, r, g, b) in the order of the splat record's first
 * nine floats.  The backward adds its per-(tile, Gaussian) sums into it with
 * atomics (one or two cache lines per record) after clearing it; packed, the
 * clear writes no padding.  4-byte alignment.
 */
#define LGS_SPLAT_FLOATS 16
#define LGS_GRAD_FLOATS 9

typedef enum {
    LGS_OK = 0,
    LGS_ERR_INVALID_ARG = 1,
    LGS_ERR_CAPACITY = 2,
    LGS_ERR_HIP = 3,
    LGS_ERR_UNSUPPORTED = 4
} lgs_status;

/*
 * Pinhole camera, OpenCV axes (x right, y down, z forward).  Host struct,
 * passed by pointer and copied at the call.
 *   viewmat   world->camera [R | t], row-major 3x4
 *   campos    camera centre in world space (direction of the SH colour)
 *   fx, fy    focal lengths in pixels; cx, cy principal point in pixels.
 *             Pixel (i, j) has its centre at image coordinates (i, j).
 *   tan_fovx, tan_fovy   tangent of half the field of view; the projection
 *             Jacobian is evaluated at points clamped to 1.3x these.
 *   width, height        image size in pixels (>= 1)
 *   znear     Gaussians with camera-space z <= znear are culled
 *   bg        background colour blended behind the last Gaussian
 */
typedef struct lgs_camera {
    float viewmat[12];
    float campos[3];
    float fx, fy, cx, cy;
    float tan_fovx, tan_fovy;
    int32_t width, height;
    float znear;
    float bg[3];
} lgs_camera;

/* Render-kernel variants: the cumulative ablation ladder of the paper
 * (Table "ablation", Sec. IV-C).  By default the exponent of alpha (the
 * hoisted dot product or the plain quadratic) is evaluated in double, which
 * the gfx950 vector ALU issues at the single-precision rate, and alpha, T and
 * the colour are float with the fused update T <- fma(-alpha, T, T) in every
 * variant.  OR with LGS_RENDER_FP32 for the paper's single-precision
 * arithmetic throughout, with LGS_RENDER_Q8 to change the wavefront
 * sub-tile shape of the culling variants, and with LGS_RENDER_VOTE4 to space
 * out the termination vote of LOCAL. */
typedef enum {
    LGS_RENDER_PLAIN = 0,       /* baseline per-pixel loop (Alg. 1, baseline column) */
    LGS_RENDER_HOIST = 1,       /* + tile-local hoisted dot product (Sec. III-B) */
    LGS_RENDER_HOIST_CULL = 2,  /* + wavefront-level tight-box culling (Sec. III-C) */
    LGS_RENDER_LOCAL = 3,       /* + uniform blend, wave-wide termination vote (Sec. III-D) */
    LGS_RENDER_FP32 = 0x10,
    LGS_RENDER_Q8 = 0x20,       /* HOIST_CULL / LOCAL: each wavefront owns an 8x8 quadrant of
                                   the tile instead of a 16x4 row strip (same results) */
    LGS_RENDER_VOTE4 = 0x40,    /* LOCAL: the wave-wide termination vote runs once per 4
                                   Gaussians instead of after each one (same results) */
    LGS_RENDER_GLOBAL = 0x80    /* hoisted variants: the basis [x'^2, x'y', y'^2, x', y', 1]
                                   in image coordinates instead of tile-centre ones (the
                                   paper's global-coordinate precision baseline, Sec.
                                   III-B-4; with LGS_RENDER_FP32 it loses the accuracy the
                                   tile-local origin keeps) */
} lgs_render_variant;

/* Message for the last non-OK status on the calling host thread. */
const char *lgs_last_error(void);
/* Library version string. */
const char *lgs_version(void);

/*
 * lgs_project -- preprocessing of n 3D Gaussians for one camera (Sec. II-A,
 * Fig. 2: projection to a 2D mean and covariance, footprint for tile culling).
 *
 * Inputs (device, raw parameters):
 *   means3d [n,3], log_scales [n,3] (natural log of the per-axis standard
 *   deviation), quats [n,4] (w, x, y, z; normalised inside), opacity_logits
 *   [n] (opacity = sigmoid), sh [n,(sh_degree+1)^2,3] real SH coefficients.
 *   sh_degree in 0..3.
 * Outputs (device):
 *   splats [n,LGS_SPLAT_FLOATS] projected splat records (conic, opacity,
 *                         mean, colour; layout at LGS_SPLAT_FLOATS); culled
 *                         Gaussians get an all-zero record
 *   depth [n]             depth key: the float32 rounding of camera-space z
 *   rect [n,4]            touched tiles [tx0, ty0, tx1, ty1): the tiles
 *                         holding a pixel centre of the alpha >= 1/255 ellipse;
 *                         all zero for culled Gaussians
 * Culled (rect empty, depth = +inf): z <= znear, opacity < 1/255, singular
 * covariance, footprint outside the image, non-finite parameters.
 */
lgs_status lgs_project(const lgs_camera *cam, int64_t n, int32_t sh_degree,
                       const float *means3d, const float *log_scales, const float *quats,
                       const float *opacity_logits, const float *sh,
                       float *splats, float *depth, int32_t *rect, void *stream);

/*
 * lgs_sort -- duplication of every visible Gaussian into one (tile, id) pair
 * per touched tile and a stable sort so that each tile's pairs are in
 * ascending (depth, id) order (Sec. II-A: prefix scan, key duplication,
 * radix sort).  Implemented as a stable radix sort of all n depth keys
 * (culled ones hold +inf and sort last) over only the bits in which the
 * visible keys differ (their range is taken on the device first) and a scan
 * of their tile counts in that order; then, for grids at most 256 tiles wide, a column pass that
 * generates the pairs from the rectangles straight into tile-column order
 * (depth order kept within a column) and a stable radix sort on the tile row,
 * or, for wider grids, duplication in depth order and a stable radix sort on
 * the tile id.  Either way the result equals a stable sort of 64-bit
 * (tile << 32 | depth bits) keys emitted in id order.
 *
 * Inputs: depth [n], rect [n,4] from lgs_project; tiles_x * tiles_y tiles.
 *   A visible Gaussian's depth is positive and finite; a depth whose bit
 *   pattern is at or above +inf's (+inf, NaN, negative values) marks a culled
 *   one, whose rectangle must be empty (lgs_project writes both so).
 * splats [n,LGS_SPLAT_FLOATS] (from lgs_project): NULL to give each
 *   Gaussian every tile of its rectangle, else the exact tile assignment: only the tiles whose pixel-centre square its alpha >= 1/255
 *   ellipse meets (the test is conservative: a float evaluation on a
 *   slightly enlarged ellipse), which removes the rectangle's corner tiles
 *   (about 20% of the pairs of round splats).  Applied on grids at most 256
 *   tiles wide; wider grids keep the rectangles.  Either way every pixel's
 *   contributors are listed, so the rendered image is the same.
 * Outputs (device):
 *   tile_keys [capacity_pairs]  tile id of each pair, ascending
 *   values    [capacity_pairs]  Gaussian id of each pair
 *   num_pairs (device int64)    total pair count P (also when P > capacity)
 *   overflow  (device int32)    set to 1 if P > capacity_pairs, else 0; then
 *                               nothing past capacity_pairs is written and the
 *                               pair lists are invalid (lgs_tile_ranges then
 *                               yields empty tiles).  Grow and call again.
 * workspace: device scratch of at least lgs_sort_workspace_size(...) bytes.
 */
size_t lgs_sort_workspace_size(int64_t n, int64_t capacity_pairs, int32_t num_tiles);
lgs_status lgs_sort(int64_t n, int32_t tiles_x, int32_t tiles_y, const float *depth, const int32_t *rect,
                    const float *splats, uint32_t *tile_keys, uint32_t *values, int64_t capacity_pairs,
                    int64_t *num_pairs, int32_t *overflow, void *workspace, size_t workspace_bytes,
                    void *stream);

/*
 * lgs_sort_noalloc -- lgs_sort for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same sort, same outputs, with the library's own scratch
 * instead of a workspace argument.  The scratch is a static device array of
 * LGS_SORT_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; a call
 * whose lgs_sort_workspace_size(n, capacity_pairs, tiles) exceeds it returns
 * LGS_ERR_INVALID_ARG (with the sizes in lgs_last_error()) and enqueues
 * nothing.  The call allocates nothing (the scratch's address is looked up
 * once per device, on the first call with that device current).  Every call
 * on one GPU shares that GPU's scratch: calls that overlap on one GPU (other
 * streams, other host threads) race; calls in one stream are ordered.  The
 * scratch keeps the last call's contents; each call clears what it needs.
 */
#define LGS_SORT_NOALLOC_SCRATCH_BYTES (64u << 20)
lgs_status lgs_sort_noalloc(int64_t n, int32_t tiles_x, int32_t tiles_y, const float *depth, const int32_t *rect,
                            const float *splats, uint32_t *tile_keys, uint32_t *values, int64_t capacity_pairs,
                            int64_t *num_pairs, int32_t *overflow, void *stream);

/*
 * lgs_tile_ranges -- [start, end) of every tile's run in the sorted pairs
 * (Sec. II-A, "tile ranges").  ranges [num_tiles,2] uint32 (device); tiles
 * without pairs get (0, 0), and so do all tiles if *overflow != 0.
 */
lgs_status lgs_tile_ranges(const uint32_t *tile_keys, const int64_t *num_pairs, const int32_t *overflow,
                           int64_t capacity_pairs, int32_t num_tiles, uint32_t *ranges, void *stream);

/*
 * lgs_render -- front-to-back alpha blending of every 16x16 tile (Sec. II-A
 * render kernel; Local-GS stages of Sec. III).  For each pixel p, over its
 * tile's list in order: alpha = min(0.99, o * exp(-q/2)) with
 * q = a dx^2 + 2 b dx dy + c dy^2, d = p - mean; Gaussians with
 * alpha < 1/255 are skipped; blending stops before the first Gaussian that
 * would take the transmittance T below 1e-4; C += rgb * alpha * T.
 * Inputs: ranges from lgs_tile_ranges, values from lgs_sort, the splat
 * records from lgs_project.  `variant` is an lgs_render_variant.
 * Outputs (device): out_rgb [3,H,W] = C + T * bg; out_T [H,W] final T;
 *   out_ncontrib [H,W] 1-based position, in the tile's list, of the last
 *   blended Gaussian (0 if none).
 * stats: NULL, or device uint64[8] that receives (added) counters:
 *   [0] (wavefront, Gaussian) steps met by live wavefronts,
 *   [1] of those, steps evaluated (not culled), [2] Gaussians staged,
 *   [3] lane evaluations.  Counting runs a separate, slower instantiation.
 */
lgs_status lgs_render(int32_t variant, const lgs_camera *cam, const uint32_t *ranges, const uint32_t *values,
                      const float *splats, float *out_rgb, float *out_T, int32_t *out_ncontrib, uint64_t *stats, void *stream);

/*
 * lgs_render_backward -- gradient of L through the blending, given
 * grad_rgb = dL/d out_rgb [3,H,W] and optionally grad_T = dL/d out_T [H,W]
 * (NULL = 0).  Replays each pixel back to front from its last contributor,
 * recovering T from the stored final T.  Writes (overwrites) the gradient
 * records g_splats [n,LGS_GRAD_FLOATS] (see LGS_GRAD_FLOATS); the clamp at 0.99 and all skip / stop decisions are held fixed.
 * `variant` is LGS_RENDER_PLAIN or LGS_RENDER_LOCAL (hoisted, culled), the
 * latter optionally with LGS_RENDER_Q8 (8x8 wavefront quadrants for the
 * culling), either with LGS_RENDER_FP32 when the forward ran a single-
 * precision variant: the replay then evaluates alpha with that forward's
 * expression (the float hoisted dot product, or the plain o * exp of the
 * float quadratic), so it takes the forward's skip and clamp decisions.
 * and with LGS_RENDER_GLOBAL after a global-coordinate forward.
 * LGS_RENDER_VOTE4 is ignored.  Use PLAIN after a PLAIN forward and LOCAL
 * after any hoisted one (HOIST, HOIST_CULL, LOCAL).  Gradients agree across
 * these choices up to the order of floating-point summation.
 * OR with LGS_BWD_ACCUMULATE to add into the gradient buffers instead of
 * overwriting them (e.g. to sum the gradients of several batches of views).
 */
#define LGS_BWD_ACCUMULATE 0x100
lgs_status lgs_render_backward(int32_t variant, const lgs_camera *cam, int64_t n, const uint32_t *ranges,
                               const uint32_t *values, const float *splats, const float *out_T,
                               const int32_t *out_ncontrib, const float *grad_rgb, const float *grad_T,
                               float *g_splats, void *stream);

/*
 * lgs_project_backward -- chain rule from the projected attributes back to
 * the raw parameters of lgs_project (same inputs, plus its rect output to
 * know which Gaussians were culled), given the gradient records g_splats
 * [n,LGS_GRAD_FLOATS].  Writes (overwrites) d_means3d [n,3],
 * d_log_scales [n,3], d_quats [n,4], d_opacity_logits [n],
 * d_sh [n,(deg+1)^2,3]; culled Gaussians get zero.
 * flags: 0, or LGS_PROJ_BWD_CLEAR to set every nonzero gradient record it
 * reads back to zero, so that the records are all zero afterwards and the
 * next lgs_render_backward can add into them (LGS_BWD_ACCUMULATE) without
 * clearing them first: the clear costs only the records that were written.
 */
#define LGS_PROJ_BWD_CLEAR 0x1
lgs_status lgs_project_backward(const lgs_camera *cam, int64_t n, int32_t sh_degree,
                                const float *means3d, const float *log_scales, const float *quats,
                                const float *opacity_logits, const float *sh, const int32_t *rect,
                                float *g_splats, float *d_means3d, float *d_log_scales,
                                float *d_quats, float *d_opacity_logits, float *d_sh, int32_t flags,
                                void *stream);

/*
 * Multi-view batches.  A batch renders up to LGS_MAX_VIEWS cameras (sizes may
 * differ) of one Gaussian set in single launches, the paper's stages applied
 * to each view unchanged (Sec. II-A, Sec. III).  Layouts:
 *   - per-Gaussian projected arrays are view-major: element e = v * n + i
 *     (splats [V*n,LGS_SPLAT_FLOATS], depth [V*n], rect [V*n,4] and the
 *     gradient records);
 *   - tiles of all views form one global index space: view v owns tiles
 *     [T_v, T_v + tiles_x(v) * tiles_y(v)) with T_v the sum of the tile
 *     counts of the views before it; pair values are element ids e;
 *   - images are packed: view v's out_rgb [3,H_v,W_v] starts at float
 *     3 * P_v and out_T / out_ncontrib [H_v,W_v] at element P_v, where P_v
 *     is the sum of W*H over the views before it.
 * Each *_batch call with num_views = 1 is exactly its single-view form.
 */
#define LGS_MAX_VIEWS 16
#define LGS_QUEUE_WORDS 256   /* size of the persistent render's counter block */

/* lgs_project for num_views cameras; the raw parameters are read once.
 * Outputs [num_views * n, ...], view-major. */
lgs_status lgs_project_batch(const lgs_camera *cams, int32_t num_views, int64_t n, int32_t sh_degree,
                             const float *means3d, const float *log_scales, const float *quats,
                             const float *opacity_logits, const float *sh,
                             float *splats, float *depth, int32_t *rect, void *stream);

/* lgs_sort over num_views * n_per_view elements; tiles_x / tiles_y are host
 * arrays [num_views].  The workspace size is
 * lgs_sort_workspace_size(num_views * n_per_view, capacity_pairs, total tiles). */
lgs_status lgs_sort_batch(int32_t num_views, const int32_t *tiles_x, const int32_t *tiles_y,
                          int64_t n_per_view, const float *depth, const int32_t *rect,
                          const float *splats, uint32_t *tile_keys, uint32_t *values, int64_t capacity_pairs,
                          int64_t *num_pairs, int32_t *overflow, void *workspace, size_t workspace_bytes,
                          void *stream);

/* lgs_render over the global tiles of num_views cameras (ranges [total,2]
 * from lgs_tile_ranges with num_tiles = total tiles).
 * queue: NULL for one workgroup per tile; else LGS_QUEUE_WORDS device
 *   uint32 words of work counters (cleared by the call itself) that turn the
 *   culling variants (HOIST_CULL, LOCAL) into a persistent kernel of
 *   blocks_per_cu workgroups per compute unit (<= 0: 8) whose wavefronts
 *   take wavefront sub-tiles from the counters until none is left.  Other
 *   variants ignore it.  Concurrent calls must not share a queue.
 * tile_order: NULL to hand out tiles in index order (XCD-banded for one
 *   workgroup per tile), else a device permutation [total tiles] (e.g. from
 *   lgs_tile_order) giving the tile of each queue position, or of each
 *   workgroup without a queue.  Outputs do not depend on the order.
 * used_masks: NULL, or device uint64 [used_mask_words] (at least
 *   lgs_used_mask_words(capacity of the pair buffers, total tiles)): the LOCAL
 *   variant then records, per wavefront sub-tile and chunk of 64 list
 *   entries, which entries some pixel of the sub-tile blended (alpha >= 1/255
 *   before its termination), for lgs_render_backward_batch.  Chunks that a
 *   sub-tile never reached (it had terminated) are not written.  Other
 *   variants ignore it. */
lgs_status lgs_render_batch(int32_t variant, const lgs_camera *cams, int32_t num_views,
                            const uint32_t *ranges, const uint32_t *values, const float *splats,
                            float *out_rgb, float *out_T, int32_t *out_ncontrib, uint64_t *stats,
                            uint32_t *queue, const uint32_t *tile_order, int32_t blocks_per_cu,
                            uint64_t *used_masks, int64_t used_mask_words, void *stream);

/* Words of the used-entry masks for pair buffers of capacity_pairs pairs and
 * num_tiles tiles (4 sub-tile planes of capacity_pairs / 64 + num_tiles + 1
 * words each; 0 for invalid arguments). */
int64_t lgs_used_mask_words(int64_t capacity_pairs, int32_t num_tiles);

/* lgs_render_debug -- lgs_render_batch's statistics instantiation (one
 * workgroup per tile, tiles in index order) that also records the culling
 * decisions of the culling variants (Sec. III-C-3, the warp mask): for every
 * list entry j (position in the sorted pairs) that wavefront sub-tile w of
 * the entry's tile tested, masks[j] gets bit w, and bit 4 + w if the test
 * kept it (tight-box test passed).  Sub-tiles: 16x4 row strips (w = row
 * quarter of the tile), or with LGS_RENDER_Q8 8x8 quadrants (w = 2 * row half
 * + column half).  masks: device uint32 [num_pairs], zeroed by the caller;
 * stats: device uint64[8] as for lgs_render.  A verification aid (one atomic
 * per tested entry); the other variants leave masks untouched. */
lgs_status lgs_render_debug(int32_t variant, const lgs_camera *cams, int32_t num_views,
                            const uint32_t *ranges, const uint32_t *values, const float *splats,
                            float *out_rgb, float *out_T, int32_t *out_ncontrib, uint64_t *stats,
                            uint32_t *masks, void *stream);

/* lgs_tile_order -- longest-first work order for the persistent render: a
 * permutation of the tile ids (device uint32 [num_tiles]) by non-increasing
 * list length, lengths compared in classes of 1/8 octave (tiles of one class
 * stay in index order).  Not a step of the paper; it balances the tail of a
 * queue-driven launch.  workspace: 256-byte aligned device scratch of
 * lgs_tile_order_workspace_size(num_tiles) bytes. */
size_t lgs_tile_order_workspace_size(int32_t num_tiles);
lgs_status lgs_tile_order(const uint32_t *ranges, int32_t num_tiles, uint32_t *order, void *workspace,
                          size_t workspace_bytes, void *stream);

/* lgs_render_backward of a batch: n_elem = num_views * n elements of the
 * view-major gradient outputs.
 * tile_order: NULL, or a permutation of the batch's global tile ids (as from
 *   lgs_tile_order), e.g. longest list first so that the longest tiles do not
 *   run last.
 * queue: NULL for one workgroup per tile (in tile_order, if given); else
 *   LGS_QUEUE_WORDS device uint32 words of work counters (cleared by the call
 *   itself) that make the backward one persistent launch of blocks_per_cu
 *   workgroups per compute unit (<= 0: 4), each taking whole tiles in
 *   tile_order from the counters until none is left.  Concurrent calls must
 *   not share a queue.
 * stats: NULL, or device uint64[8] that receives (added) counters:
 *   [0] (wavefront, Gaussian) steps met within the replay range (after
 *   culling), [1] steps replayed (some lane takes the Gaussian), [2] (pixel,
 *   Gaussian) pairs taken, [3] lane evaluations (64 per replayed step).
 *   Counting runs a separate, slower instantiation.
 * used_masks: NULL, or the used-entry masks that the LOCAL forward of these
 *   same pair lists recorded (lgs_render_batch with the same sub-tile shape,
 *   LGS_RENDER_Q8 or not): the replay then visits exactly those entries
 *   instead of testing every entry its culling keeps (the same gradients,
 *   less work).  Requires variant LOCAL.
 * The gradients do not depend on the order or the schedule beyond float
 * summation order. */
lgs_status lgs_render_backward_batch(int32_t variant, const lgs_camera *cams, int32_t num_views, int64_t n_elem,
                                     const uint32_t *ranges, const uint32_t *values, const float *splats,
                                     const float *out_T, const int32_t *out_ncontrib, const float *grad_rgb,
                                     const float *grad_T, float *g_splats, const uint32_t *tile_order,
                                     uint32_t *queue, int32_t blocks_per_cu, uint64_t *stats,
                                     const uint64_t *used_masks, int64_t used_mask_words, void *stream);

/* lgs_project_backward of a batch: the view-major gradients of the projected
 * attributes are summed over the views into the raw-parameter gradients
 * [n, ...] (overwritten); flags as for lgs_project_backward. */
lgs_status lgs_project_backward_batch(const lgs_camera *cams, int32_t num_views, int64_t n, int32_t sh_degree,
                                      const float *means3d, const float *log_scales, const float *quats,
                                      const float *opacity_logits, const float *sh, const int32_t *rect,
                                      float *g_splats, float *d_means3d, float *d_log_scales,
                                      float *d_quats, float *d_opacity_logits, float *d_sh, int32_t flags,
                                      void *stream);

/*
 * Step graphs: lgs_graph_begin starts capturing the calls enqueued on
 * `stream` by this host thread (a created stream, not NULL) instead of
 * running them; lgs_graph_end stops and instantiates them as one HIP graph.
 * lgs_graph_launch replays the whole sequence on a stream with one call, on
 * the same device buffers and arguments as captured.  Every library call is
 * capturable (clears are kernels, never memset nodes) except the host-side
 * read of a pair count, which stays outside: capture a step with a fixed
 * pair capacity and check the overflow flag after replays.
 */
typedef struct lgs_graph lgs_graph;
lgs_status lgs_graph_begin(void *stream);
lgs_status lgs_graph_end(void *stream, lgs_graph **graph);
lgs_status lgs_graph_launch(lgs_graph *graph, void *stream);
lgs_status lgs_graph_destroy(lgs_graph *graph);

/*
 * lgs_l1_loss -- L = mean |image - target| over `count` floats and
 * grad = dL/d image = sign(image - target) / count (0 where equal); the
 * training objective of the differentiable path (not part of the paper).
 * loss: device float (overwritten); grad: device [count].
 * workspace: 8-byte aligned device scratch of lgs_l1_workspace_size() bytes
 * for the per-block partial sums (summed in a fixed order: the loss is
 * deterministic).  Calls with distinct workspaces may run concurrently.
 */
size_t lgs_l1_workspace_size(void);
lgs_status lgs_l1_loss(const float *image, const float *target, int64_t count, float *loss, float *grad,
                       void *workspace, size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LOCALGS_H */
