// gs_upscale_hermite: bicubic Hermite upscaling from image values and
// analytical derivatives.
//
// Sec. "Image Gradient Based Upscaling" and Suppl. "Spline Image
// Interpolation" of arXiv 2503.14171: each low-res cell gets the bicubic
// p(x,y) = [1 x x^2 x^3] A [1 y y^2 y^3]^T with F = C A C^T, F holding the
// values and the x, y, xy derivatives at the cell's four corners.  Written in
// the cubic Hermite basis h(t) = C^-T [1 t t^2 t^3]^T,
//     h0 = 2t^3 - 3t^2 + 1, h1 = -2t^3 + 3t^2, h2 = t^3 - 2t^2 + t, h3 = t^3 - t^2,
// the patch is p(x,y) = h(x)^T F h(y), which separates: on a low-res row r
//     V_r(x) = h0 f(i,r) + h1 f(i+1,r) + h2 f_x(i,r) + h3 f_x(i+1,r)
//     D_r(x) = h0 f_y(i,r) + h1 f_y(i+1,r) + h2 f_xy(i,r) + h3 f_xy(i+1,r)
// and p = h0(y) V_j + h1(y) V_j+1 + h2(y) D_j + h3(y) D_j+1.
//
// The kernel is HBM-bound (48 B read per low-res pixel, 12 B written per
// high-res pixel).  One lane owns one output column and walks a band of
// output rows; V and D of a low-res row are computed once per lane and reused
// for every output row of the cell and for the next cell (which shares the
// row), so a lane reads each low-res row once and spends 12 FMAs per output
// pixel plus 24 per low-res row.  A wave stores 64 consecutive 12-byte pixels
// (768 contiguous bytes) per output row, with non-temporal stores (measured
// 24 us instead of 37 us for 960x540 -> 3840x2160 on MI355X).
#include "gsup_internal.h"

namespace gsup {
namespace {

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

// Local coordinate of output index X inside cell `cell` (the cell axis_map
// gives X); no division by the cell count: the adjoint loops over the output
// indices of known cells.
__device__ __forceinline__ float local_coord(int X, int n_lo, int n_hi, int cell) {
  const int64_t den = 2 * (int64_t)n_hi;
  const int64_t r = (int64_t)(2 * X + 1) * n_lo - n_hi - (int64_t)cell * den;
  return (float)r / (float)den;
}

// V (values) and D (y-derivatives) of low-res row r along x at the lane's column.
__device__ __forceinline__ void row_terms(const float* __restrict__ in, int w, int r, int i, float h0,
                                          float h1, float h2, float h3, float (&V)[3],
                                          float (&D)[3]) {
  const float4* a = reinterpret_cast<const float4*>(in + ((int64_t)r * w + i) * 12);
  const float4 a0 = a[0], a1 = a[1], a2 = a[2];  // node i:   f rgb, fx r | fx gb, fy rg | fy b, fxy rgb
  const float4 b0 = a[3], b1 = a[4], b2 = a[5];  // node i+1
  V[0] = fmaf(h0, a0.x, fmaf(h1, b0.x, fmaf(h2, a0.w, h3 * b0.w)));
  V[1] = fmaf(h0, a0.y, fmaf(h1, b0.y, fmaf(h2, a1.x, h3 * b1.x)));
  V[2] = fmaf(h0, a0.z, fmaf(h1, b0.z, fmaf(h2, a1.y, h3 * b1.y)));
  D[0] = fmaf(h0, a1.z, fmaf(h1, b1.z, fmaf(h2, a2.y, h3 * b2.y)));
  D[1] = fmaf(h0, a1.w, fmaf(h1, b1.w, fmaf(h2, a2.z, h3 * b2.z)));
  D[2] = fmaf(h0, a2.x, fmaf(h1, b2.x, fmaf(h2, a2.w, h3 * b2.w)));
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

template <int ROWS>
__global__ __launch_bounds__(kThreads) void upscale_kernel(UpParams p,
                                                           const float* __restrict__ in_all,
                                                           float* __restrict__ out_all) {
  // bands of one XCD are contiguous, so the low-res row two bands share is
  // fetched into one L2
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  if (blk >= p.blocks) return;
  int vi = 0;  // uniform over the block
  while (vi + 1 < p.nv && blk >= p.view[vi + 1].blk_off) ++vi;
  const int w = p.view[vi].w, h = p.view[vi].h, W = p.view[vi].W, H = p.view[vi].H;
  const int strips = p.view[vi].strips;
  const int64_t local = blk - p.view[vi].blk_off;
  const float* __restrict__ in = in_all + p.view[vi].in_off * 12;
  float* __restrict__ out = out_all + p.view[vi].out_off * 3;
  const int bx = (int)(local % strips), by = (int)(local / strips);
  const int X = bx * kThreads + threadIdx.x;
  const int Y0 = by * ROWS;
  if (X >= W || Y0 >= H) return;
  const int Y1 = min(Y0 + ROWS, H);
  int i;
  float tx;
  axis_map(X, w, W, i, tx);
  float hx0, hx1, hx2, hx3;
  hermite(tx, hx0, hx1, hx2, hx3);

  float V0[3], D0[3], V1[3], D1[3];
  int jcur = -2;
  float* o = out + ((int64_t)Y0 * W + X) * 3;
  for (int Y = Y0; Y < Y1; ++Y, o += (int64_t)W * 3) {
    int j;
    float ty;
    axis_map(Y, h, H, j, ty);
    if (j != jcur) {
      if (j == jcur + 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          V0[c] = V1[c];
          D0[c] = D1[c];
        }
      } else {
        row_terms(in, w, j, i, hx0, hx1, hx2, hx3, V0, D0);
      }
      row_terms(in, w, j + 1, i, hx0, hx1, hx2, hx3, V1, D1);
      jcur = j;
    }
    float hy0, hy1, hy2, hy3;
    hermite(ty, hy0, hy1, hy2, hy3);
    // streaming output: non-temporal stores keep it from displacing the input in L2/MALL
#pragma unroll
    for (int c = 0; c < 3; ++c)
      __builtin_nontemporal_store(fmaf(hy0, V0[c], fmaf(hy1, V1[c], fmaf(hy2, D0[c], hy3 * D1[c]))),
                                  o + c);
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the upscaler: dL/d(low-res values and derivatives) from
// dL/d(upscaled image).  Every output pixel is a fixed linear combination of
// the 16 F entries of its cell, weight h_k(t_x) h_l(t_y), so the adjoint of
// node (i, j) gathers, over the output pixels of the (up to) four cells that
// have the node as a corner, g times the node's weights: h0 (value) / h2
// (derivative) where the node is the left/top corner, h1 / h3 where it is the
// right/bottom one.  One lane per node, no atomics, deterministic.
// ---------------------------------------------------------------------------
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

UpParams make_up_params(int32_t nv, const int32_t* lo_sizes, const int32_t* hi_sizes,
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

}  // namespace

hipError_t launch_upscale(const float* in, int32_t nv, const int32_t* lo_sizes, float* out,
                          const int32_t* hi_sizes, int32_t band_rows, hipStream_t stream) {
  if (band_rows <= 0) band_rows = 8;
  const UpParams p = make_up_params(nv, lo_sizes, hi_sizes, band_rows, nullptr);
  const int64_t blocks = p.blocks;
  const unsigned grid = (unsigned)xcd_grid(blocks);
  switch (band_rows) {
    case 4: upscale_kernel<4><<<grid, kThreads, 0, stream>>>(p, in, out); break;
    case 8: upscale_kernel<8><<<grid, kThreads, 0, stream>>>(p, in, out); break;
    case 16: upscale_kernel<16><<<grid, kThreads, 0, stream>>>(p, in, out); break;
    case 32: upscale_kernel<32><<<grid, kThreads, 0, stream>>>(p, in, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gsup

namespace gsup {
namespace {

// Classical bicubic comparator: central-difference slopes of a plain image.
// f_x = (f[i+1] - f[i-1]) / 2 inside, one-sided differences on the border
// columns; f_y likewise on rows; f_xy = the y-difference of f_x.
__device__ __forceinline__ float diff(const float* __restrict__ img, int64_t stride_px, int i, int n,
                                      int64_t base, int c) {
  const int lo = i > 0 ? i - 1 : 0, hi = i < n - 1 ? i + 1 : n - 1;
  const float sc = (hi - lo == 2) ? 0.5f : 1.f;
  return sc * (img[(base + (int64_t)hi * stride_px) * 3 + c] - img[(base + (int64_t)lo * stride_px) * 3 + c]);
}

__global__ __launch_bounds__(kThreads) void fd_slopes_kernel(const float* __restrict__ img, int w,
                                                             int h, float* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= (int64_t)w * h) return;
  const int x = (int)(p % w), y = (int)(p / w);
  const int y0 = y > 0 ? y - 1 : 0, y1 = y < h - 1 ? y + 1 : h - 1;
  const float sy = (y1 - y0 == 2) ? 0.5f : 1.f;
  float o[12];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    o[c] = img[p * 3 + c];
    o[3 + c] = diff(img, 1, x, w, (int64_t)y * w, c);
    o[6 + c] = diff(img, w, y, h, x, c);
    o[9 + c] = sy * (diff(img, 1, x, w, (int64_t)y1 * w, c) - diff(img, 1, x, w, (int64_t)y0 * w, c));
  }
  float4* d = reinterpret_cast<float4*>(out + p * 12);
  d[0] = make_float4(o[0], o[1], o[2], o[3]);
  d[1] = make_float4(o[4], o[5], o[6], o[7]);
  d[2] = make_float4(o[8], o[9], o[10], o[11]);
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

hipError_t launch_fd_slopes(const float* img, int32_t w, int32_t h, float* out, hipStream_t stream) {
  const int64_t n = (int64_t)w * h;
  fd_slopes_kernel<<<(unsigned)ceil_div(n, kThreads), kThreads, 0, stream>>>(img, w, h, out);
  return hipGetLastError();
}

}  // namespace gsup
