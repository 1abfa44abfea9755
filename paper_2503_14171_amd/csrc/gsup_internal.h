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
hipError_t launch_project(int64_t n, const float* means, const float* log_scales,
                          const float* quats, const float* opacity, const float* sh,
                          const gs_camera& cam, const gs_raster_cfg& cfg, gs_splat* splats,
                          float* depth, int32_t* rect, hipStream_t stream);

// ---- binning and sorting (binsort.hip) --------------------------------------
struct BinSortPlan {
  int64_t n = 0;          // splats
  int64_t capacity = 0;   // pair capacity
  int64_t tiles_x = 0, tiles_y = 0, tiles = 0;
  int tile_bits = 0;      // bits of the tile id key
  // workspace layout (byte offsets)
  size_t off_gkey[2], off_gval[2];  // depth keys / splat ids, ping-pong [n]
  size_t off_bsum;                  // tile-count sums per block of splats -> pair offsets
  size_t off_srect;                 // clipped tile rectangles in depth order [n]
  size_t off_pkey[2];               // pair tile keys, ping-pong [capacity]
  size_t off_pval;                  // pair ids, second buffer [capacity]
  size_t off_hist;                  // radix digit counts [2^11 * max blocks]
  size_t off_totals;                // per-digit totals [2^11]
  size_t off_total;                 // 1 x uint64 pair total
  size_t bytes = 0;
};
BinSortPlan make_bin_sort_plan(int64_t n, int64_t capacity, int32_t width, int32_t height,
                               int32_t tile_size);
gs_status run_bin_sort(const BinSortPlan& plan, const float* depth, const int32_t* rect,
                       int32_t* sorted_ids, int32_t* tile_ranges, int64_t* n_pairs,
                       void* workspace, hipStream_t stream);

// ---- rasterization (raster.hip) -----------------------------------------------
hipError_t launch_raster(const gs_splat* splats, const int32_t* sorted_ids,
                         const int32_t* tile_ranges, const gs_camera& cam,
                         const gs_raster_cfg& cfg, bool grads, float* out, int32_t* n_blend,
                         hipStream_t stream);

// ---- upscaling (upscale.hip) ---------------------------------------------------
hipError_t launch_upscale(const float* in, int32_t w, int32_t h, float* out, int32_t W,
                          int32_t H, hipStream_t stream);
hipError_t launch_fd_slopes(const float* img, int32_t w, int32_t h, float* out,
                            hipStream_t stream);

}  // namespace gsup
