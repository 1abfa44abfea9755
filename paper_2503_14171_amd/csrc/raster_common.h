// Shared by the forward (raster.hip) and backward (raster_bwd.hip)
// rasterizers: per-view launch parameters and the culling margin.  Both
// kernels derive every pixel's FP32 offsets from these in the same way, so
// the backward pass recomputes exactly the forward's decisions.
#pragma once

#include "gsup_internal.h"

namespace gsup {
namespace raster_detail {

// One view of a batch: its raster, its first global tile id and the offset
// of its first pixel in the concatenated outputs.
struct RasterView {
  int32_t width, height, tiles_x;
  uint32_t tile_off;
  int64_t pix_off;
};

struct RasterParams {
  int32_t nv;
  int64_t tiles;  // all views
  float alpha_max, t_min;
  float bg[3];
  RasterView view[GS_MAX_VIEWS];
};

// Workgroup -> (list tile, sub-tile).  MI355X deals consecutive workgroups
// round-robin to its 8 XCDs.  The SUB2 workgroups of one list tile share an
// XCD (they stage the same list through its L2), and list tiles go to the
// XCDs in turn, so every XCD gets dense and sparse screen regions alike: a
// contiguous band of tiles per XCD leaves the XCDs holding the dense centre
// of a frame working long after the others.  The grid is tile_grid(); tiles
// at or beyond the real count are idle.
inline int64_t tile_grid(int64_t tiles, int sub2) {
  return (int64_t)kNumXcd * ceil_div(tiles, kNumXcd) * sub2;
}
__device__ __forceinline__ void tile_block(int64_t bid, int sub2, int64_t& tile, int& sub) {
  const int64_t i = bid / kNumXcd;
  tile = (i / sub2) * kNumXcd + bid % kNumXcd;
  sub = (int)(i % sub2);
}

// Widening, in pixels, of a splat's support box in the per-wave culling test
// (covers FP32 rounding of the box and of the per-pixel alpha test).
constexpr float kCullMargin = 0.25f;

// Staging-time bounds (the box and the quadrant test below) only have to
// keep every quadrant with a pixel above alpha_min: they use the hardware
// reciprocal and square root (about 1 ulp) instead of the correctly rounded
// sequences.  The box half-extents' relative error of a few 1e-7 is far
// inside the kCullMargin widening, and an approximate 1/a or 1/c only moves
// the minimiser along an edge, which changes the edge minimum to second
// order.  Opacities are normal numbers (>= alpha_min),
// so the hardware log2 equals log2f for them.
__device__ __forceinline__ float stage_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float stage_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float opacity_log2(float x) { return __builtin_amdgcn_logf(x); }

// Quadrants [k0, k1] along one axis (quadrant k holds the pixel centres
// 8k .. 8k+7 of the workgroup) that the box [m - r, m + r] meets; empty when
// k0 > k1.  Clamped in float before the conversion, since converting a float
// outside the int range is undefined.
template <int QX>
__device__ __forceinline__ void quad_span(float m, float r, int& k0, int& k1) {
  k0 = (int)fminf(fmaxf(ceilf((m - r - 7.f) * 0.125f), 0.f), (float)QX);
  k1 = (int)fminf(fmaxf(floorf((m + r) * 0.125f), -1.f), (float)(QX - 1));
}

// Whether the ellipse {d^T Q d <= S} around (mx, my) reaches the 8x8 pixel
// centres [x0, x0 + 7] x [y0, y0 + 7] widened by kCullMargin: the minimum of
// the quadratic over that rectangle (zero if it holds the centre, else on an
// edge, where the quadratic in the free coordinate has its minimum clamped to
// the edge) against S.  ia = 1/a, ic = 1/c (a, c > 0).
__device__ __forceinline__ bool quad_reaches(float mx, float my, float a, float b, float c, float ia,
                                             float ic, float S, float x0, float y0) {
  const float lx = x0 - kCullMargin - mx, hx = x0 + 7.f + kCullMargin - mx;
  const float ly = y0 - kCullMargin - my, hy = y0 + 7.f + kCullMargin - my;
  if (lx <= 0.f && hx >= 0.f && ly <= 0.f && hy >= 0.f) return true;
  float best = INFINITY;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const float X = e ? hx : lx;  // edge x = const, free y
    const float ty = fminf(fmaxf(-b * X * ic, ly), hy);
    best = fminf(best, fmaf(a * X, X, fmaf(2.f * b * X, ty, c * ty * ty)));
    const float Y = e ? hy : ly;  // edge y = const, free x
    const float tx = fminf(fmaxf(-b * Y * ia, lx), hx);
    best = fminf(best, fmaf(c * Y, Y, fmaf(2.f * b * Y, tx, a * tx * tx)));
  }
  return best <= S;
}

inline RasterParams make_params(int32_t nv, const gs_camera* cams, const gs_raster_cfg& cfg) {
  RasterParams p{};
  p.nv = nv;
  int64_t tiles = 0, pix = 0;
  for (int v = 0; v < nv; ++v) {
    RasterView& rv = p.view[v];
    rv.width = cams[v].width;
    rv.height = cams[v].height;
    rv.tiles_x = (int32_t)ceil_div(cams[v].width, cfg.tile_size);
    rv.tile_off = (uint32_t)tiles;
    rv.pix_off = pix;
    tiles += (int64_t)rv.tiles_x * ceil_div(cams[v].height, cfg.tile_size);
    pix += (int64_t)cams[v].width * cams[v].height;
  }
  p.tiles = tiles;
  p.alpha_max = cfg.alpha_max;
  p.t_min = cfg.t_min;
  for (int k = 0; k < 3; ++k) p.bg[k] = cfg.bg[k];
  return p;
}

}  // namespace raster_detail
}  // namespace gsup
