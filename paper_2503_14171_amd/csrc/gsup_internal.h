// Internal declarations shared by the HIP translation units of libgsup.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "gsup.h"

namespace gsup {

// ---- error reporting (api.hip) --------------------------------------------
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
gs_status fail(gs_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
gs_status check_hip(hipError_t e, const char* what);

// ---- small helpers -----------------------------------------------------------
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with its own L2.  Launching 8 * ceil(n/8) workgroups and renumbering them
// this way gives every XCD one contiguous range of logical blocks, so
// neighbouring tiles share an L2.  Logical ids >= n are idle.
constexpr int kNumXcd = 8;
inline int64_t xcd_grid(int64_t n) { return kNumXcd * ceil_div(n, kNumXcd); }
__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t grid) {
  const int64_t per = grid / kNumXcd;
  return (bid % kNumXcd) * per + bid / kNumXcd;
}

// ---- projection (project.hip) ------------------------------------------------
// Views v of a batch write splats / depth / rect at offset v * n.
hipError_t launch_project(int64_t n, const float* means, const float* log_scales,
                          const float* quats, const float* opacity, const float* sh, int32_t nv,
                          const gs_camera* cams, const gs_raster_cfg& cfg, gs_splat* splats,
                          float* depth, int16_t* rect, hipStream_t stream);

hipError_t launch_project_backward(int64_t n, const float* means, const float* log_scales,
                                   const float* quats, const float* opacity, const float* sh,
                                   int32_t nv, const gs_camera* cams, const gs_raster_cfg& cfg,
                                   const float* dsplat, float* d_means, float* d_log_scales,
                                   float* d_quats, float* d_opacity, float* d_sh,
                                   hipStream_t stream);

// ---- binning and sorting (binsort.hip) --------------------------------------
// Tile grids of the views of a batch; view v's tiles have the global ids
// tile_off[v] .. tile_off[v+1) (row-major inside the view).
struct ViewTiles {
  int32_t nv = 1;
  int64_t n = 0;  // splats per view
  int32_t tiles_x[GS_MAX_VIEWS], tiles_y[GS_MAX_VIEWS];
  uint32_t tile_off[GS_MAX_VIEWS + 1];
  // FP32 bits of the smallest near plane and the largest far plane of the
  // views; bounded: every view has a far plane, so every finite depth key
  // lies in [key_lo, key_hi]
  uint32_t key_lo = 0, key_hi = 0;
  bool bounded = false;
};
ViewTiles make_view_tiles(int32_t nv, const gs_camera* cams, int32_t tile_size, int64_t n);

struct BinSortPlan {
  int64_t n = 0;          // splat records (all views)
  int64_t capacity = 0;   // pair capacity
  int64_t tiles = 0;      // tiles of all views
  int tile_bits = 0;      // bits of the tile id key
  // workspace layout (byte offsets)
  size_t off_gkey[2], off_gval[2];  // depth keys / splat ids, ping-pong [n]
  size_t off_bsum;                  // pairs of a count block before each of its emit blocks
  size_t off_bblk;                  // pairs per count block of splats
  size_t off_prect[2];              // packed clipped tile rectangles, ping-pong with the ids [n]
  size_t off_pkey[2];               // pair tile keys, ping-pong [capacity]
  size_t off_pval;                  // pair ids, second buffer [capacity]
  size_t off_hist;                  // radix digit counts [2^digit bits * max blocks]
  size_t off_totals;                // per-digit totals
  size_t off_total;                 // 1 x uint64 pair total
  size_t off_dinfo;                 // depth keys: min, max, last buffer (4 x u32), kept count (u64)
  size_t off_bstat;                 // depth keys: per-block min, max, count of the first pass
  size_t bytes = 0;
};
BinSortPlan make_bin_sort_plan(int64_t n, int64_t capacity, int64_t tiles);
// Host-count mode (n_pairs_dev == NULL): reads K to *n_pairs, waits once and
// fails with GS_ERR_CAPACITY when it does not fit.  Device-count mode: never
// waits; K goes to *n_pairs_dev and an oversized K leaves every range empty.
gs_status run_bin_sort(const BinSortPlan& plan, const ViewTiles& vt, const float* depth,
                       const int16_t* rect, int32_t* sorted_ids, int32_t* tile_ranges,
                       int64_t* n_pairs, int64_t* n_pairs_dev, void* workspace,
                       hipStream_t stream);

// ---- rasterization (raster.hip) -----------------------------------------------
// One launch over the tiles of all views; view v's pixels go to
// out + (sum of earlier views' pixels) * channels, likewise n_blend / n_eval
// (optional: fragments blended / evaluated per pixel).
// state / last (optional): final T, T_x, T_y, T_xy per pixel and the end of
// its walked list, for the backward pass.
hipError_t launch_raster(const gs_splat* splats, const int32_t* sorted_ids,
                         const int32_t* tile_ranges, int32_t nv, const gs_camera* cams,
                         const gs_raster_cfg& cfg, bool grads, float* out, int32_t* n_blend,
                         int32_t* n_eval, float* state, int32_t* last, hipStream_t stream);
// dsplat [n_records, 9] (zeroed here): mean x, mean y, conic a, b, c, opacity, rgb.
hipError_t launch_raster_backward(const gs_splat* splats, const int32_t* sorted_ids,
                                  const int32_t* tile_ranges, int32_t nv, const gs_camera* cams,
                                  const gs_raster_cfg& cfg, const float* state, const int32_t* last,
                                  const float* dout, int64_t n_records, float* dsplat,
                                  hipStream_t stream);

// ---- upscaling (upscale.hip) ---------------------------------------------------
// Views are concatenated in both buffers; sizes are host arrays [nv][2].
hipError_t launch_upscale(const float* in, int32_t nv, const int32_t* lo_sizes, float* out,
                          const int32_t* hi_sizes, int32_t band_rows, hipStream_t stream);
hipError_t launch_upscale_backward(const float* d_out, int32_t nv, const int32_t* lo_sizes,
                                   float* d_in, const int32_t* hi_sizes, hipStream_t stream);
hipError_t launch_fd_slopes(const float* img, int32_t w, int32_t h, float* out,
                            hipStream_t stream);

}  // namespace gsup
