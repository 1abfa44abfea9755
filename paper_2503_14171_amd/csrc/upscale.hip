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
// pixel plus 24 per low-res row; each row's cell index and Hermite weights
// are computed once per block (no division per row and lane).  A wave
// stores 64 consecutive 12-byte pixels (768 contiguous bytes) per output row,
// with non-temporal stores (they keep the output from displacing the input
// in L2 and the MALL).
#include "upscale_common.h"

namespace gsup {

using namespace upscale_detail;

namespace {


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
  if (Y0 >= H) return;  // uniform over the block
  const int Y1 = min(Y0 + ROWS, H);
  // The band's rows, once per block: each row's cell index and Hermite
  // weights are the same for every lane, so ROWS threads compute them into
  // LDS and the row loop reads them.  Computing them per lane and row (a
  // 64-bit division for the cell index on the scalar unit the CU's waves
  // share, a float division and the weights on every lane) had bounded the
  // kernel.
  __shared__ float4 s_hy[ROWS];
  __shared__ int s_j[ROWS];
  if ((int)threadIdx.x < Y1 - Y0) {
    int j;
    float ty, a0, a1, a2, a3;
    axis_map(Y0 + (int)threadIdx.x, h, H, j, ty);
    hermite(ty, a0, a1, a2, a3);
    s_hy[threadIdx.x] = make_float4(a0, a1, a2, a3);
    s_j[threadIdx.x] = j;
  }
  __syncthreads();
  if (X >= W) return;
  int i;
  float tx;
  axis_map(X, w, W, i, tx);
  float hx0, hx1, hx2, hx3;
  hermite(tx, hx0, hx1, hx2, hx3);

  float V0[3], D0[3], V1[3], D1[3];
  int jcur = -2;
  float* o = out + ((int64_t)Y0 * W + X) * 3;
  for (int r = 0; r < Y1 - Y0; ++r, o += (int64_t)W * 3) {
    const int j = s_j[r];
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
    const float4 hy = s_hy[r];
    const float hy0 = hy.x, hy1 = hy.y, hy2 = hy.z, hy3 = hy.w;
    // streaming output: non-temporal stores keep it from displacing the input in L2/MALL
#pragma unroll
    for (int c = 0; c < 3; ++c)
      __builtin_nontemporal_store(fmaf(hy0, V0[c], fmaf(hy1, V1[c], fmaf(hy2, D0[c], hy3 * D1[c]))),
                                  o + c);
  }
}

}  // namespace

hipError_t launch_upscale(const float* in, int32_t nv, const int32_t* lo_sizes, float* out,
                          const int32_t* hi_sizes, int32_t band_rows, hipStream_t stream) {
  if (band_rows <= 0) band_rows = 16;  // measured best for one view (960x540 -> 3840x2160: 27 us vs 29 at 8)
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

hipError_t launch_fd_slopes(const float* img, int32_t w, int32_t h, float* out, hipStream_t stream) {
  const int64_t n = (int64_t)w * h;
  fd_slopes_kernel<<<(unsigned)ceil_div(n, kThreads), kThreads, 0, stream>>>(img, w, h, out);
  return hipGetLastError();
}

}  // namespace gsup
