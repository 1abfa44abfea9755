/*
 * gsup.h -- C ABI of the MI355X (gfx950) implementation of gradient-aware
 * upscaling of 3D Gaussian Splatting images (Niedermayr, Neuhauser,
 * Westermann, arXiv 2503.14171).
 *
 * One camera view goes through four calls:
 *
 *   gs_project          3D Gaussians -> 2D splats: EWA projection of the
 *                       covariance, view-dependent SH colour, depth, and the
 *                       rectangle of screen tiles the splat can reach.
 *   gs_bin_sort         splats -> one front-to-back index list per tile.
 *   gs_raster_grad      tile lists -> low-res colour I and its analytical
 *                       screen-space derivatives dI/dx, dI/dy, d2I/dxdy.
 *   gs_upscale_hermite  low-res colour + derivatives -> high-res image, one
 *                       bicubic Hermite patch per low-res pixel cell.
 *
 * Many views of one scene go through the *_views calls (one launch per step);
 * training goes through gs_raster_grad_views_train and the *_backward_views
 * calls; gs_fd_slopes provides the classical bicubic comparator.
 *
 * Conventions shared by every call
 *   - Array arguments are DEVICE pointers (HBM), owned by the caller, dense
 *     row-major, little-endian, FP32 unless stated.  The library never
 *     allocates, frees or keeps device memory between calls.
 *   - Structs (gs_camera, gs_raster_cfg), camera arrays, size arrays and the
 *     scalar out-parameter n_pairs live in HOST memory; n_pairs_dev is a
 *     DEVICE pointer.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     Every call only enqueues work on that stream and returns, except
 *     gs_bin_sort, which waits on the stream once to read the pair count
 *     (gs_bin_sort_async and gs_bin_sort_views do not wait: the chains they
 *     belong to can be captured in a HIP graph).
 *   - Arguments are validated on the host before anything is enqueued.  On
 *     any error the call returns a non-zero gs_status, enqueues nothing (or
 *     nothing further), and gs_last_error_message() describes the problem.
 *   - Image coordinates: x = column (right), y = row (down); the centre of
 *     pixel (x, y) is the point (x, y); the image spans [-1/2, W-1/2] in x.
 *   - Camera: pinhole with OpenCV axes (+x right, +y down, +z forward).
 *   - Calls are reentrant; concurrent calls on different streams must use
 *     distinct output and workspace buffers.
 */
#ifndef GSUP_H
#define GSUP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Most camera views one batched call takes. */
#define GS_MAX_VIEWS 16

typedef enum gs_status {
  GS_OK = 0,
  GS_ERR_INVALID_ARGUMENT = 1, /* a pointer, size or setting is out of range */
  GS_ERR_CAPACITY = 2,         /* gs_bin_sort: more (tile, splat) pairs than `capacity` */
  GS_ERR_HIP = 3,              /* the HIP runtime reported an error */
  GS_ERR_UNSUPPORTED = 4       /* a setting the library does not implement */
} gs_status;

/* Pinhole camera.  A world point p maps to camera space t = R p + t_W with
 * view = [R | t_W] (row-major 3x4), and to the image point
 * (fx t.x / t.z + cx, fy t.y / t.z + cy). */
typedef struct gs_camera {
  int32_t width, height; /* raster size in pixels, >= 1 */
  float fx, fy;          /* focal lengths in pixels, > 0 */
  float cx, cy;          /* principal point in pixels */
  float view[12];        /* world -> camera [R | t_W], row-major */
  float cam_pos[3];      /* camera centre in world space (SH view direction) */
  float near_plane;      /* Gaussians with camera z <= near_plane are culled, > 0 */
  float far_plane;       /* Gaussians with camera z > far_plane are culled; 0: no far plane.
                            A far plane bounds the depth keys, so gs_bin_sort runs only the
                            radix passes the range [near_plane, far_plane] needs */
} gs_camera;

/* Render settings.  The paper fixes none of these numbers; see each field. */
typedef struct gs_raster_cfg {
  int32_t tile_size; /* square screen tile of the per-tile lists, in pixels: 8, 16, 32 or 64
                        (32x32 and 64x64 lists are rasterized by 16x16 workgroups) */
  int32_t sh_degree; /* degree of the SH colour, 0..3 */
  float dilation;    /* px^2 added to the 2D covariance diagonal (low-pass), >= 0; 3DGS uses 0.3 */
  float alpha_min;   /* fragments with alpha < alpha_min are skipped, in (0, alpha_max) */
  float alpha_max;   /* alpha > alpha_max is clamped to alpha_max (zero screen derivatives), < 1 */
  float t_min;       /* a pixel stops once its transmittance after a blend is < t_min, in (0, 1) */
  float bg[3];       /* background colour behind the last fragment */
  int32_t batch;     /* splats staged per LDS batch in the rasterizer: 0 or tile_size^2 (one per
                        thread), tile_size^2 / 2 or tile_size^2 / 4 (for tile_size 32 and 64
                        these are per list tile, split over its 16x16 workgroups); changes only the
                        speed */
} gs_raster_cfg;

/* A projected Gaussian (48 bytes, 16-byte aligned).  The 2D mean is kept in
 * FP64 so that pixel-relative offsets stay exact at 4K image coordinates. */
typedef struct gs_splat {
  double mean[2];  /* image-plane mean (pixels) */
  float conic[3];  /* (a, b, c): inverse of the dilated 2D covariance [[a, b], [b, c]] */
  float opacity;   /* sigma in [alpha_min, 1] */
  float rgb[3];    /* view-dependent colour, max(0, sum_lm Y_lm k_lm + 1/2) */
  float support;   /* 2 ln(sigma / alpha_min): alpha >= alpha_min <=> d^T Q d <= support */
} gs_splat;

/* Pair count the asynchronous bin sorts report when a finite depth lies
 * outside the cameras' [near_plane, far_plane] (see gs_camera.far_plane). */
#define GS_PAIRS_DEPTH_RANGE (1ll << 62)

/* Number of tiles of a width x height raster: ceil(W/ts) * ceil(H/ts). */
int64_t gs_num_tiles(int32_t width, int32_t height, int32_t tile_size);

/* gs_project -- EWA projection and SH colour of n Gaussians.
 * Follows Sec. "Differentiable 3D Gaussian Splatting" (2D covariance
 * Sigma' = J W Sigma W^T J^T, Gaussians ordered by the depth of their mean,
 * SH view-dependent colour).
 *
 * Inputs (device, FP32):
 *   means [n,3]       world-space centres mu
 *   log_scales [n,3]  per-axis log standard deviations; Sigma = R S S^T R^T, S = diag(exp(.))
 *   quats [n,4]       rotation quaternions (w, x, y, z), normalised here
 *   opacity [n]       sigma in [0, 1] (after the sigmoid)
 *   sh [n,(d+1)^2,3]  SH coefficients, real orthonormal basis ordered l^2+l+m
 *                     (graphics sign convention), d = cfg->sh_degree
 * Outputs (device):
 *   splats [n]        gs_splat records (zeroed for splats that reach no tile)
 *   depth [n]         camera-space z rounded to FP32 (the sort key); +inf when the
 *                     splat reaches no tile (culled or off-screen)
 *   rect [n,4] int16  tile rectangle [tx0, ty0, tx1, ty1) that holds every pixel
 *                     with alpha >= alpha_min; all zero when culled or off-screen
 * A Gaussian is culled when an input is not finite, its camera z <= near_plane,
 * its 2D covariance is not positive definite, or sigma < alpha_min.  The SH
 * coefficients of a Gaussian are read only when its rectangle is not empty.
 * The Jacobian J is evaluated with the mean's direction clamped to 1.3x the
 * half field of view.  n == 0 is a no-op. */
gs_status gs_project(int64_t n, const float* means, const float* log_scales, const float* quats,
                     const float* opacity, const float* sh, const gs_camera* cam,
                     const gs_raster_cfg* cfg, gs_splat* splats, float* depth, int16_t* rect,
                     void* stream);

/* Bytes of device workspace gs_bin_sort needs for n splats and `capacity` pairs. */
size_t gs_bin_sort_workspace_size(int64_t n, int64_t capacity, const gs_camera* cam,
                                  const gs_raster_cfg* cfg);

/* gs_bin_sort -- per-tile front-to-back lists (the depth order of
 * Sec. "Differentiable 3D Gaussian Splatting", restricted to each tile).
 *
 * Inputs (device): depth [n] and rect [n,4] from gs_project (depth must be
 * positive wherever rect is non-empty: its bits are the sort key; a splat
 * with depth +inf reaches no tile and its rect is not read).  With a far
 * plane (cam->far_plane > 0) the finite depths must also lie in
 * [near_plane, far_plane], as gs_project leaves them: only the radix passes
 * that range needs run.  Depths outside it whose keys then span more bits
 * than those passes sort fail the call with GS_ERR_INVALID_ARGUMENT (the
 * asynchronous variants report the pair count GS_PAIRS_DEPTH_RANGE instead
 * and emit nothing); others are still ordered correctly.
 * Outputs:
 *   sorted_ids [capacity] int32  (device) splat indices; tile t's list is
 *                               sorted_ids[tile_ranges[2t] .. tile_ranges[2t+1]),
 *                               ordered by (FP32 depth, index)
 *   tile_ranges [T,2] int32     (device) [start, end) per tile, T = gs_num_tiles(..);
 *                               [0, 0) for a tile no splat reaches
 *   n_pairs                     (HOST) number of (tile, splat) pairs K
 * workspace: device scratch of at least gs_bin_sort_workspace_size(n, capacity, ..)
 * bytes, 256-byte aligned; its contents are undefined after the call.
 * If K > capacity the call returns GS_ERR_CAPACITY with *n_pairs = K and the
 * outputs undefined; the caller grows the buffers and calls again.
 * Waits on `stream` once (to read K).  K must stay below 2^31. */
gs_status gs_bin_sort(int64_t n, const float* depth, const int16_t* rect, const gs_camera* cam,
                      const gs_raster_cfg* cfg, int64_t capacity, int32_t* sorted_ids,
                      int32_t* tile_ranges, int64_t* n_pairs, void* workspace,
                      size_t workspace_bytes, void* stream);

/* gs_bin_sort_async -- gs_bin_sort without the wait: the pair count K is
 * written to n_pairs_dev (DEVICE, one int64, 8-byte aligned) on the stream.
 * When K > capacity (or K >= 2^31) nothing is emitted, every tile range is
 * [0, 0) and sorted_ids is left as it was: the caller reads *n_pairs_dev
 * after the stream has run, grows the buffers and runs the frame again.
 * Never waits on the stream; safe to capture in a HIP graph.  Same inputs,
 * outputs and workspace as gs_bin_sort. */
gs_status gs_bin_sort_async(int64_t n, const float* depth, const int16_t* rect,
                            const gs_camera* cam, const gs_raster_cfg* cfg, int64_t capacity,
                            int32_t* sorted_ids, int32_t* tile_ranges, int64_t* n_pairs_dev,
                            void* workspace, size_t workspace_bytes, void* stream);

/* Bytes of the static device scratch gs_bin_sort_async_static works in. */
#define GS_STATIC_SCRATCH_BYTES (64u << 20)

/* gs_bin_sort_async_static -- gs_bin_sort_async for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): no workspace argument; the library's
 * own static scratch of GS_STATIC_SCRATCH_BYTES per GPU (held from the first
 * call on that GPU to the end of the process) takes its place.  Same inputs,
 * outputs, overflow rule and results as gs_bin_sort_async.  Sizes whose
 * workspace, gs_bin_sort_workspace_size(n, capacity, ..), exceeds the scratch
 * (about 24 bytes per splat and 12 per pair of capacity: 500k splats with a
 * capacity of 4M pairs fit, 1M splats with 4M do not) are rejected with
 * GS_ERR_INVALID_ARGUMENT before anything is enqueued.  The call allocates
 * nothing: the scratch's device address is looked up once per device, on the
 * first call there.  Every call on one GPU shares that scratch, so calls that
 * overlap on one GPU (other streams, other host threads) race and give
 * undefined results; calls on one stream are ordered and safe.  Nothing in
 * the scratch needs to start at zero: every pass writes what it later reads. */
gs_status gs_bin_sort_async_static(int64_t n, const float* depth, const int16_t* rect,
                                   const gs_camera* cam, const gs_raster_cfg* cfg,
                                   int64_t capacity, int32_t* sorted_ids, int32_t* tile_ranges,
                                   int64_t* n_pairs_dev, void* stream);

/* gs_raster_grad -- front-to-back alpha blending of every pixel's tile list,
 * with the analytical screen-space derivatives of the blended colour.
 * Follows Sec. "Image Gradient Based Upscaling" (3DGS image gradients: the
 * derivatives of I = sum_i T_i alpha_i c_i and the iterative transmittance
 * derivatives) and Suppl. "3DGS Gradient Computation - Forward pass".
 * Per fragment alpha = sigma exp(-1/2 d^T Q d), d = pixel - mean; skipped if
 * alpha < alpha_min, clamped (zero derivatives) if alpha > alpha_max; a pixel
 * stops after the blend that takes its transmittance below t_min.
 *
 * Inputs (device): splats [n], sorted_ids, tile_ranges from gs_bin_sort (for
 * the same camera and tile size).
 * Output (device) `out`, per pixel of the cam->width x cam->height raster:
 *   want_grads != 0: [H, W, 12] = (I rgb, dI/dx rgb, dI/dy rgb, d2I/dxdy rgb),
 *                    derivatives per pixel (per pixel^2 for the mixed one)
 *   want_grads == 0: [H, W, 3]  = I rgb (plain 3DGS compositing)
 * n_blend (device, optional, may be NULL): [H, W] int32 blended fragments per pixel. */
gs_status gs_raster_grad(const gs_splat* splats, const int32_t* sorted_ids,
                         const int32_t* tile_ranges, const gs_camera* cam,
                         const gs_raster_cfg* cfg, int32_t want_grads, float* out,
                         int32_t* n_blend, void* stream);

/* gs_upscale_hermite -- bicubic Hermite upscaling from values and derivatives.
 * Follows Sec. "Image Gradient Based Upscaling" (F = C A C^T, patch
 * p(x,y) = [1 x x^2 x^3] A [1 y y^2 y^3]^T, one A per low-res cell) and
 * Suppl. "Spline Image Interpolation".
 * High-res pixel (X, Y) samples the low-res point u = (X + 1/2) w / W - 1/2,
 * v = (Y + 1/2) h / H - 1/2 with the patch of cell (i, j) = (clamp(floor u, 0,
 * w-2), clamp(floor v, 0, h-2)) at local (u - i, v - j) (extrapolated at the
 * border).  Any real factors W/w >= 1, H/h >= 1 (independent per axis).
 *
 * in  [h, w, 12] (device): (I rgb, I_x rgb, I_y rgb, I_xy rgb) as written by
 *     gs_raster_grad, derivatives per low-res pixel; w, h >= 2.
 * out [H, W, 3]  (device): upscaled rgb.  `in` and `out` must not overlap. */
gs_status gs_upscale_hermite(const float* in, int32_t w, int32_t h, float* out, int32_t W,
                             int32_t H, void* stream);

/* gs_fd_slopes -- the classical bicubic comparator: derivative buffers of a
 * plain image estimated by finite differences (Sec. "Image Gradient Based
 * Upscaling", Spline Interpolation: classical bicubic interpolation estimates
 * the gradients with finite differences of neighbouring pixels; Sec.
 * "Motivational Example").  Feeding the result to gs_upscale_hermite gives
 * Catmull-Rom (Keys a = -1/2) bicubic upscaling on interior cells.
 * img [h, w, 3] (device) -> out [h, w, 12] (device, 16-byte aligned, no
 * overlap): values, f_x = (f[x+1] - f[x-1]) / 2, f_y likewise, f_xy = the
 * y-difference of f_x; one-sided differences on the border rows/columns. */
gs_status gs_fd_slopes(const float* img, int32_t w, int32_t h, float* out, void* stream);

/* ---- Batched views --------------------------------------------------------
 * Many cameras of one scene (stereo pairs, training batches) go through the
 * same four steps with one launch per step.  `cams` is a HOST array of
 * n_views (1..GS_MAX_VIEWS) cameras; per-view device arrays are concatenated
 * in view order.  Each view's results equal those of the single-view calls
 * for that camera.  None of these calls waits on the stream. */

/* Tiles of all views: sum over v of gs_num_tiles(cams[v].width, cams[v].height, tile_size). */
int64_t gs_num_tiles_views(int32_t n_views, const gs_camera* cams, int32_t tile_size);

/* gs_project_views -- gs_project for every view, reading each Gaussian's
 * parameters once per batch.  Outputs splats [n_views, n], depth [n_views, n],
 * rect [n_views, n, 4]: record v * n + i is Gaussian i seen by view v, its
 * rect in view v's tile grid.  n * n_views < 2^31. */
gs_status gs_project_views(int64_t n, const float* means, const float* log_scales,
                           const float* quats, const float* opacity, const float* sh,
                           int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                           gs_splat* splats, float* depth, int16_t* rect, void* stream);

/* Bytes of device workspace gs_bin_sort_views needs. */
size_t gs_bin_sort_views_workspace_size(int64_t n, int32_t n_views, const gs_camera* cams,
                                        const gs_raster_cfg* cfg, int64_t capacity);

/* gs_bin_sort_views -- per-tile lists of all views at once.  Tiles are
 * numbered view after view (view v's tile (tx, ty) has the id
 * sum_{u<v} tiles(u) + ty * tiles_x(v) + tx); tile_ranges [T_all, 2]; list
 * entries are splat records v * n + i, ordered by (FP32 depth, i).  The pair
 * count goes to n_pairs_dev as in gs_bin_sort_async (same overflow rule). */
gs_status gs_bin_sort_views(int64_t n, int32_t n_views, const gs_camera* cams,
                            const gs_raster_cfg* cfg, const float* depth, const int16_t* rect,
                            int64_t capacity, int32_t* sorted_ids, int32_t* tile_ranges,
                            int64_t* n_pairs_dev, void* workspace, size_t workspace_bytes,
                            void* stream);

/* gs_raster_grad_views -- one launch over the tiles of all views.  out holds
 * the views' [H_v, W_v, 12] (or [H_v, W_v, 3]) images back to back; n_blend
 * (optional) their [H_v, W_v] counts. */
gs_status gs_raster_grad_views(const gs_splat* splats, const int32_t* sorted_ids,
                               const int32_t* tile_ranges, int32_t n_views,
                               const gs_camera* cams, const gs_raster_cfg* cfg,
                               int32_t want_grads, float* out, int32_t* n_blend, void* stream);

/* gs_raster_fragment_counts -- gs_raster_grad_views (same inputs and `out`)
 * that also reports the rasterizer's work per pixel, for measuring it:
 *   n_eval [sum H W] int32 (device)  list entries the pixel evaluated before
 *                                    it stopped: splats of its tile list whose
 *                                    support reaches its 8x8 pixel block, for
 *                                    each of which d^T Q d is computed and
 *                                    tested against the alpha_min support
 *   n_blend [sum H W] int32 (device) fragments it blended (alpha >= alpha_min)
 * Both are required.  The counters cost the launch a few instructions per
 * fragment; gs_raster_grad_views is the call to time. */
gs_status gs_raster_fragment_counts(const gs_splat* splats, const int32_t* sorted_ids,
                                    const int32_t* tile_ranges, int32_t n_views,
                                    const gs_camera* cams, const gs_raster_cfg* cfg,
                                    int32_t want_grads, float* out, int32_t* n_eval,
                                    int32_t* n_blend, void* stream);

/* gs_upscale_hermite_views -- one launch for all views.  lo_sizes and
 * hi_sizes are HOST arrays [n_views][2] of (width, height); in holds the
 * views' [h_v, w_v, 12] buffers back to back, out their [H_v, W_v, 3] images.
 * band_rows: output rows per workgroup, 4, 8, 16 or 32 (0 = 16); it changes
 * only the speed. */
gs_status gs_upscale_hermite_views(const float* in, int32_t n_views, const int32_t* lo_sizes,
                                   float* out, const int32_t* hi_sizes, int32_t band_rows,
                                   void* stream);

/* ---- Backward pass (training through the upscaler) --------------------------
 * Sec. "Image Gradient Based Upscaling" (Differentiable Image Gradients) and
 * Suppl. "3DGS Gradient Computation - Backward pass" (back-to-front blending,
 * dI/d alpha_k and its screen derivatives, colour gradients, inversion trick).
 * A training step: gs_project_views, gs_bin_sort_views,
 * gs_raster_grad_views_train, gs_upscale_hermite_views; then, with
 * dL/d(upscaled), gs_upscale_hermite_backward_views, gs_raster_grad_backward_views,
 * gs_project_backward_views.  The index set of every pixel (skips, clamps,
 * stop) is the forward's and is held fixed; a clamped fragment has no
 * geometric gradient; a colour clamped at zero has none either. */

/* Forward with gradients (as gs_raster_grad_views with want_grads = 1) that
 * also saves, per low-res pixel, state [pix, 4] = final (T, T_x, T_y, T_xy)
 * (device, 16-byte aligned) and last [pix] (int32) = the position in
 * sorted_ids after the pixel's last blended fragment.  Both feed
 * gs_raster_grad_backward_views. */
gs_status gs_raster_grad_views_train(const gs_splat* splats, const int32_t* sorted_ids,
                                     const int32_t* tile_ranges, int32_t n_views,
                                     const gs_camera* cams, const gs_raster_cfg* cfg, float* out,
                                     float* state, int32_t* last, void* stream);

/* Adjoint of gs_upscale_hermite_views: d_out [sum H W, 3] = dL/d(upscaled) ->
 * d_in [sum h w, 12] = dL/d(low-res values and derivatives), overwritten.
 * Deterministic (no atomics).  d_in 16-byte aligned, no overlap. */
gs_status gs_upscale_hermite_backward_views(const float* d_out, int32_t n_views,
                                            const int32_t* lo_sizes, float* d_in,
                                            const int32_t* hi_sizes, void* stream);

/* d_lowres [sum h w, 12] = dL/d(I, I_x, I_y, I_xy) -> d_splats [n_views * n, 9]
 * (overwritten) = dL/d(mean x, mean y, conic a, b, c, opacity, r, g, b) of every
 * splat record, from the buffers of the matching forward (same splats, lists,
 * state and last).  The state before each fragment is recovered by inverting
 * the blend; contributions are summed with atomics (order not fixed, so the
 * last bits may vary between runs). */
gs_status gs_raster_grad_backward_views(const gs_splat* splats, const int32_t* sorted_ids,
                                        const int32_t* tile_ranges, int32_t n_views,
                                        const gs_camera* cams, const gs_raster_cfg* cfg,
                                        const float* state, const int32_t* last,
                                        const float* d_lowres, int64_t n, float* d_splats,
                                        void* stream);

/* d_splats [n_views * n, 9] -> dL/d(means [n,3], log_scales [n,3], quats [n,4]
 * (16-byte aligned), opacity [n], sh [n,(d+1)^2,3]), summed over the views,
 * overwritten.  Records with an all-zero gradient are skipped. */
gs_status gs_project_backward_views(int64_t n, const float* means, const float* log_scales,
                                    const float* quats, const float* opacity, const float* sh,
                                    int32_t n_views, const gs_camera* cams,
                                    const gs_raster_cfg* cfg, const float* d_splats,
                                    float* d_means, float* d_log_scales, float* d_quats,
                                    float* d_opacity, float* d_sh, void* stream);

/* Message of the last failed call on this host thread ("" if none). */
const char* gs_last_error_message(void);

/* Library version string. */
const char* gs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GSUP_H */
