// gs_upscale_hermite_backward_views: the adjoint of the Hermite upscaler
// (Sec. "Image Gradient Based Upscaling", Differentiable Image Gradients:
// the upscaled image is a fixed linear map of the low-res values and
// derivatives, so its gradient is the transposed map).
#include "upscale_common.h"

namespace gsup {

using namespace upscale_detail;

namespace {

// ---------------------------------------------------------------------------
// Adjoint of the upscaler: dL/d(low-res values and derivatives) from
// dL/d(upscaled image).  Every output pixel is a fixed linear combination of
// the 16 F entries of its cell, weight h_k(t_x) h_l(t_y), so the adjoint of
// node (i, j) gathers, over the output pixels of the (up to) four cells that
// have the node as a corner, g times the node's weights: h0 (value) / h2
// (derivative) where the node is the left/top corner, h1 / h3 where it is the
// right/bottom one.  One lane per node, no atomics, deterministic.
// ---------------------------------------------------------------------------
// Local coordinate of output index X inside cell `cell` (the cell axis_map
// gives X); no division by the cell count: the adjoint loops over the output
// indices of known cells.
__device__ __forceinline__ float local_coord(int X, int n_lo, int n_hi, int cell) {
  const int64_t den = 2 * (int64_t)n_hi;
  const int64_t r = (int64_t)(2 * X + 1) * n_lo - n_hi - (int64_t)cell * den;
  return (float)r / (float)den;
}

// First output index whose cell (clamped) is >= c on an axis n_lo -> n_hi.
__device__ __forceinline__ int cell_start(int c, int n_lo, int n_hi) {
  if (c <= 0) return 0;
  if (c >= n_lo - 1) return n_hi;
  // smallest X with (2X + 1) n_lo - n_hi >= 2 c n_hi
  const int64_t num = 2 * (int64_t)c * n_hi + n_hi - n_lo;
  const int64_t den = 2 * (int64_t)n_lo;
  int64_t X = num >= 0 ? (num + den - 1) / den : 0;
  return (int)(X < n_hi ? X : n_hi);
}

__global__ __launch_bounds__(kThreads) void upscale_bwd_kernel(UpParams p,
                                                               const float* __restrict__ g_all,
                                                               float* __restrict__ d_all,
                                                               int64_t lo_total) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;  // node over all views
  if (e >= lo_total) return;
  int vi = 0;
  while (vi + 1 < p.nv && e >= p.view[vi + 1].in_off) ++vi;
  const int w = p.view[vi].w, h = p.view[vi].h, W = p.view[vi].W, H = p.view[vi].H;
  const int64_t node = e - p.view[vi].in_off;
  const int i = (int)(node % w), j = (int)(node / w);
  const float* __restrict__ g = g_all + p.view[vi].out_off * 3;
  float acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.f;
  // the node is corner 1 (right / bottom) of cell i-1 and corner 0 of cell i;
  // output columns of those two cells (the same for every output row)
  int xs[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) xs[k] = cell_start(i - 1 + k, w, W);
  for (int cy = j - 1; cy <= j; ++cy) {
    if (cy < 0 || cy > h - 2) continue;
    const int ry = cy == j ? 0 : 1;
    const int Y0 = cell_start(cy, h, H), Y1 = cell_start(cy + 1, h, H);
    for (int Y = Y0; Y < Y1; ++Y) {
      const float ty = local_coord(Y, h, H, cy);  // Y lies in cell cy
      float hy0, hy1, hy2, hy3;
      hermite(ty, hy0, hy1, hy2, hy3);
      const float wyV = ry ? hy1 : hy0, wyD = ry ? hy3 : hy2;
      float sV[3] = {0.f, 0.f, 0.f}, sD[3] = {0.f, 0.f, 0.f};  // x-weighted row sums
      for (int cx = i - 1; cx <= i; ++cx) {
        if (cx < 0 || cx > w - 2) continue;
        const int rx = cx == i ? 0 : 1;
        const int X0 = xs[cx - i + 1], X1 = xs[cx - i + 2];
        for (int X = X0; X < X1; ++X) {
          const float tx = local_coord(X, w, W, cx);  // X lies in cell cx
          float hx0, hx1, hx2, hx3;
          hermite(tx, hx0, hx1, hx2, hx3);
          const float wxV = rx ? hx1 : hx0, wxD = rx ? hx3 : hx2;
          const float* gp = g + ((int64_t)Y * W + X) * 3;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            sV[c] = fmaf(wxV, gp[c], sV[c]);
            sD[c] = fmaf(wxD, gp[c], sD[c]);
          }
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[c] = fmaf(wyV, sV[c], acc[c]);          // value
        acc[3 + c] = fmaf(wyV, sD[c], acc[3 + c]);  // x derivative
        acc[6 + c] = fmaf(wyD, sV[c], acc[6 + c]);  // y derivative
        acc[9 + c] = fmaf(wyD, sD[c], acc[9 + c]);  // xy derivative
      }
    }
  }
  float4* d = reinterpret_cast<float4*>(d_all + e * 12);
  d[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
  d[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
  d[2] = make_float4(acc[8], acc[9], acc[10], acc[11]);
}

}  // namespace

hipError_t launch_upscale_backward(const float* d_out, int32_t nv, const int32_t* lo_sizes,
                                   float* d_in, const int32_t* hi_sizes, hipStream_t stream) {
  int64_t lo_total = 0;
  const UpParams p = make_up_params(nv, lo_sizes, hi_sizes, 16, &lo_total);
  if (lo_total == 0) return hipSuccess;
  upscale_bwd_kernel<<<(unsigned)ceil_div(lo_total, kThreads), kThreads, 0, stream>>>(p, d_out, d_in,
                                                                                    lo_total);
  return hipGetLastError();
}

}  // namespace gsup
