// Shared by the upscaler (upscale.hip) and its adjoint (upscale_bwd.hip):
// the cubic Hermite basis, the exact output-to-cell mapping and the per-view
// launch parameters, so that both use the same cells and weights.
#pragma once

#include "gsup_internal.h"

namespace gsup {
namespace upscale_detail {

constexpr int kThreads = 256;

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

__device__ __forceinline__ void hermite(float t, float& h0, float& h1, float& h2, float& h3) {
  const float t2 = t * t;
  h1 = t2 * fmaf(-2.f, t, 3.f);
  h0 = 1.f - h1;
  h2 = t * fmaf(t, t - 2.f, 1.f);
  h3 = t2 * (t - 1.f);
}

// Cell index and local coordinate of output index X on an axis of n_lo -> n_hi:
// u = (X + 1/2) n_lo / n_hi - 1/2 = ((2X+1) n_lo - n_hi) / (2 n_hi), computed
// exactly in integers; the local coordinate is rounded once.
__device__ __forceinline__ void axis_map(int X, int n_lo, int n_hi, int& cell, float& t) {
  const int64_t num = (int64_t)(2 * X + 1) * n_lo - n_hi;
  const int64_t den = 2 * (int64_t)n_hi;
  int64_t i = floor_div(num, den);
  i = i < 0 ? 0 : (i > n_lo - 2 ? n_lo - 2 : i);
  cell = (int)i;
  t = (float)(num - i * den) / (float)den;
}

// One view of a batch: sizes, offsets (in pixels) into the concatenated
// buffers, and its first logical block.
struct UpView {
  int32_t w, h, W, H, strips;
  int64_t in_off, out_off, blk_off;
};

struct UpParams {
  int32_t nv;
  int64_t blocks;  // logical blocks of all views
  UpView view[GS_MAX_VIEWS];
};

inline UpParams make_up_params(int32_t nv, const int32_t* lo_sizes, const int32_t* hi_sizes,
                        int32_t band_rows, int64_t* lo_total) {
  UpParams p{};
  p.nv = nv;
  int64_t blocks = 0, in_off = 0, out_off = 0;
  for (int v = 0; v < nv; ++v) {
    UpView& u = p.view[v];
    u.w = lo_sizes[2 * v];
    u.h = lo_sizes[2 * v + 1];
    u.W = hi_sizes[2 * v];
    u.H = hi_sizes[2 * v + 1];
    u.strips = (int32_t)ceil_div(u.W, kThreads);
    u.in_off = in_off;
    u.out_off = out_off;
    u.blk_off = blocks;
    blocks += (int64_t)u.strips * ceil_div(u.H, band_rows);
    in_off += (int64_t)u.w * u.h;
    out_off += (int64_t)u.W * u.H;
  }
  p.blocks = blocks;
  if (lo_total) *lo_total = in_off;
  return p;
}

}  // namespace upscale_detail
}  // namespace gsup
