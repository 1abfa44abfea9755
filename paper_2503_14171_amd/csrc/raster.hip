// gs_raster_grad: tile rasterizer that blends each pixel's splats front to
// back and carries the analytical screen-space derivatives of the colour.
//
// Sec. "Image Gradient Based Upscaling" (3DGS image gradients) and Suppl.
// "3DGS Gradient Computation - Forward pass" of arXiv 2503.14171: the image
// I = sum_i T_i alpha_i c_i with alpha_i = sigma_i exp(g_i) is differentiated
// in x and y; the transmittance derivatives follow an iterative recurrence
// that runs inside the blending loop.  With A the accumulated alpha, the
// paper's recurrences for B_i, A_i and their x, y, xy derivatives are carried
// here in terms of T = 1 - A (T_x = -A_x, ...), which keeps T accurate in FP32
// where A approaches one:
//     k    = T alpha                          (weight of this fragment)
//     k_x  = T alpha_x + T_x alpha,   k_y likewise
//     k_xy = T alpha_xy + T_x alpha_y + T_y alpha_x + T_xy alpha
//     B_* += c k_*,   T_* -= k_*       for * in {_, x, y, xy}
// with alpha_x = -alpha u, alpha_y = -alpha v, alpha_xy = alpha (u v - b),
// (u, v) = Q d, d = pixel - mean, Q = [[a, b], [b, c]] the conic.
//
// Work decomposition (gfx950): one workgroup per screen tile of 8x8 or 16x16
// pixels (a 32x32 or 64x64 list tile is rasterized by four or sixteen 16x16
// workgroups that share its list), one pixel per lane, and every wave64 owns one 8x8
// quadrant of the tile.  The tile's splats stream through LDS in batches of up to one
// splat per thread (BATCH = TILE^2, or TILE^2/2, TILE^2/4); while staging, each thread marks the quadrants its splat's
// support ellipse reaches (its box, then the exact minimum of d^T Q d over the
// quadrant: a third of the box hits have no pixel above alpha_min), and each
// wave then compacts the batch (ballot + prefix
// popcount) into its own LDS list of hits in depth order, so a wave only
// evaluates splats that can reach its 64 pixels.  Every lane reads the same
// LDS record (broadcast, no bank conflicts).  A lane whose transmittance
// dropped below t_min blends nothing more (it still takes the loop's uniform
// steps, which costs less than masking it out), the wave leaves the loop once
// every lane is done, and the workgroup stops fetching
// batches once a barrier count shows no live pixel.  Splat means are held in
// FP64 and turned into tile-relative FP32 offsets when staged into LDS, so
// pixel - mean is exact at any image coordinate.  List tiles are dealt to
// the XCDs in turn, the workgroups of one list tile on one XCD (tile_block).
// Several views
// go through one launch: the grid covers the tiles of all views, numbered
// view after view, and each workgroup finds its view from the tile id.
#include "raster_common.h"

namespace gsup {

using namespace raster_detail;

namespace {


// AUX: the per-pixel fragment counts and walk end are kept (n_blend, n_eval
// or state requested); the headline frame needs none of them and saves the
// updates.  n_eval counts the list entries a pixel evaluates (its quadrant's
// hits, alpha test computed) before it stops, n_blend those it blends.
template <int TILE, bool GRAD, int BATCH, int SUB, bool AUX>
__global__ __launch_bounds__(TILE* TILE) void raster_kernel(RasterParams p,
                                                            const gs_splat* __restrict__ splats,
                                                            const int32_t* __restrict__ ids,
                                                            const int2* __restrict__ ranges,
                                                            float* __restrict__ out,
                                                            int32_t* __restrict__ n_blend,
                                                            int32_t* __restrict__ n_eval,
                                                            float4* __restrict__ state,
                                                            int32_t* __restrict__ last) {
  constexpr int NT = TILE * TILE;
  constexpr int NW = NT / 64;   // waves; wave w owns one 8x8 quadrant of the tile
  constexpr int QX = TILE / 8;  // quadrants per tile row
  constexpr float kHalfLog2e = 0.72134752044448170368f;  // log2(e) / 2
  static_assert(BATCH >= 16 && BATCH <= NT, "one splat per staging thread");
  static_assert(BATCH * 16 <= 65536, "the hit lists hold 16-bit byte offsets");
  __shared__ float4 s_a[BATCH];  // mean x, mean y (tile-relative), conic a, conic b
  __shared__ float4 s_b[BATCH];  // conic c, log2 sigma, support, red
  __shared__ float4 s_c[BATCH];  // green, blue (16-byte stride: one LDS address for all three)
  __shared__ uint32_t s_mask[NW > 1 ? BATCH : 1];                // quadrants a staged splat can reach
  __shared__ uint16_t s_list[NW > 1 ? NW : 1][NW > 1 ? BATCH : 1];  // per-wave hits (16 j), batch order

  // a workgroup covers one TILE x TILE part of a (TILE SUB)^2 list tile
  int64_t tile;
  int sub;
  tile_block(blockIdx.x, SUB * SUB, tile, sub);
  if (tile >= p.tiles) return;
  int vi = 0;  // the view this tile belongs to (uniform over the block)
  while (vi + 1 < p.nv && (uint32_t)tile >= p.view[vi + 1].tile_off) ++vi;
  const int width = p.view[vi].width, height = p.view[vi].height, tiles_x = p.view[vi].tiles_x;
  const int64_t local = tile - p.view[vi].tile_off;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int tx = (int)(local % tiles_x), ty = (int)(local / tiles_x);
  const int x0 = tx * TILE * SUB + (sub % SUB) * TILE, y0 = ty * TILE * SUB + (sub / SUB) * TILE;
  const int lx = (wave % QX) * 8 + (lane & 7), ly = (wave / QX) * 8 + (lane >> 3);
  const int px = x0 + lx, py = y0 + ly;
  const bool inside = px < width && py < height;
  const float fx = (float)lx, fy = (float)ly;
  const double ox = (double)x0, oy = (double)y0;
  const int2 rg = ranges[tile];
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));

  bool done = !inside;
  float T = 1.f, Tx = 0.f, Ty = 0.f, Txy = 0.f;
  float B0 = 0.f, B1 = 0.f, B2 = 0.f;
  float Bx0 = 0.f, Bx1 = 0.f, Bx2 = 0.f, By0 = 0.f, By1 = 0.f, By2 = 0.f;
  float Bxy0 = 0.f, Bxy1 = 0.f, Bxy2 = 0.f;
  int nb = 0, ne = 0;
  int lastpos = rg.x;  // list position after the last blended fragment

  for (int base = rg.x; base < rg.y; base += BATCH) {
    if (__syncthreads_count(!done) == 0) break;
    // stage one splat per thread of the first BATCH threads
    const int idx = base + t;
    uint32_t mask = 0;
    if (t < BATCH && idx < rg.y) {
      const float4* s = reinterpret_cast<const float4*>(splats + ids[idx]);
      const double2 m = *reinterpret_cast<const double2*>(s);
      const float4 q = s[1];  // a, b, c, sigma
      const float4 c = s[2];  // r, g, b, support
      const float mx = (float)(m.x - ox), my = (float)(m.y - oy);
      s_a[t] = make_float4(mx, my, q.x, q.y);
      s_b[t] = make_float4(q.z, opacity_log2(q.w), c.w, c.x);
      s_c[t] = make_float4(c.y, c.z, 0.f, 0.f);
      if (NW > 1) {
        // quadrants met by the box of {d^T Q d <= support}: half extents
        // sqrt(support Sigma'_xx), Sigma'_xx = c / (a c - b^2)
        const float det = q.x * q.z - q.y * q.y;
        if (det > 0.f) {
          const float idet = stage_rcp(det);
          const float rx = stage_sqrt(fmaxf(c.w * q.z * idet, 0.f)) + kCullMargin;
          const float ry = stage_sqrt(fmaxf(c.w * q.x * idet, 0.f)) + kCullMargin;
          int qx0, qx1, qy0, qy1;
          quad_span<QX>(mx, rx, qx0, qx1);
          quad_span<QX>(my, ry, qy0, qy1);
          const bool exact = q.x > 0.f && q.z > 0.f;
          const float ia = exact ? stage_rcp(q.x) : 0.f, ic = exact ? stage_rcp(q.z) : 0.f;
          for (int qy = qy0; qy <= qy1; ++qy)
            for (int qx = qx0; qx <= qx1; ++qx)
              if (!exact || quad_reaches(mx, my, q.x, q.y, q.z, ia, ic, c.w, 8.f * qx, 8.f * qy))
                mask |= 1u << (qy * QX + qx);
        } else {
          mask = (NW >= 32) ? ~0u : ((1u << NW) - 1u);  // degenerate in FP32: keep everywhere
        }
      }
    }
    if (NW > 1 && t < BATCH) s_mask[t] = mask;
    __syncthreads();
    const int cnt = min(BATCH, rg.y - base);
    int nl = cnt;
    if (NW > 1) {
      // this wave's splats of the batch, in batch (= depth) order
      nl = 0;
      if (__ballot(!done) != 0) {
        for (int c0 = 0; c0 < cnt; c0 += 64) {
          const int j = c0 + lane;
          const bool hit = j < cnt && ((s_mask[j] >> wave) & 1u);
          const uint64_t bal = __ballot(hit);
          if (hit) s_list[wave][nl + __popcll(bal & lt)] = (uint16_t)(16 * j);  // byte offset
          nl += __popcll(bal);
        }
      }
      __syncthreads();
    }
    if (!done) {
      for (int k = 0; k < nl; ++k) {
        {
          // staged record j sits at byte offset 16 j of s_a, s_b and s_c
          const int off = NW > 1 ? (int)s_list[wave][k] : 16 * k;
          const int j = off >> 4;
          const float4 ga = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(s_a) + off);
          const float4 gb = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(s_b) + off);
          const float4 gc = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(s_c) + off);
          const float dx = fx - ga.x, dy = fy - ga.y;
          const float u = fmaf(ga.z, dx, ga.w * dy);  // (Q d)_x
          const float v = fmaf(ga.w, dx, gb.x * dy);  // (Q d)_y
          const float q = fmaf(dx, u, dy * v);        // d^T Q d
          // the colour is read with the other fields: left to itself the
          // compiler moves its reads into the blend branch, after the exp,
          // where their latency is not hidden (this empty statement only
          // consumes the registers)
          asm volatile("" ::"v"(gc.x), "v"(gc.y), "v"(gb.w));
          if (AUX && !done) ++ne;
          if (!done && q <= gb.z) {                   // alpha >= alpha_min
            // the exponent is >= log2(alpha_min) > -126: no denormal handling needed
            const float a0 = __builtin_amdgcn_exp2f(fmaf(q, -kHalfLog2e, gb.y));
            // clamped at alpha_max with zero screen derivatives: sa scales them
            const bool clamp = a0 > p.alpha_max;
            const float alpha = clamp ? p.alpha_max : a0;
            const float w = T * alpha;
            if (GRAD) {
              const float sa = clamp ? 0.f : a0;
              const float ax = -sa * u;
              const float ay = -sa * v;
              const float axy = sa * fmaf(u, v, -ga.w);
              const float kx = fmaf(T, ax, Tx * alpha);
              const float ky = fmaf(T, ay, Ty * alpha);
              const float kxy = fmaf(T, axy, fmaf(Tx, ay, fmaf(Ty, ax, Txy * alpha)));
              Bx0 = fmaf(gb.w, kx, Bx0);
              Bx1 = fmaf(gc.x, kx, Bx1);
              Bx2 = fmaf(gc.y, kx, Bx2);
              By0 = fmaf(gb.w, ky, By0);
              By1 = fmaf(gc.x, ky, By1);
              By2 = fmaf(gc.y, ky, By2);
              Bxy0 = fmaf(gb.w, kxy, Bxy0);
              Bxy1 = fmaf(gc.x, kxy, Bxy1);
              Bxy2 = fmaf(gc.y, kxy, Bxy2);
              Tx -= kx;
              Ty -= ky;
              Txy -= kxy;
            }
            B0 = fmaf(gb.w, w, B0);
            B1 = fmaf(gc.x, w, B1);
            B2 = fmaf(gc.y, w, B2);
            T -= w;
            if (AUX) {
              ++nb;
              lastpos = base + j + 1;
            }
            done = T < p.t_min;
          }
        }
        if (__ballot(!done) == 0) break;  // every pixel of the wave is done
      }
    }
  }
  if (!inside) return;
  const int64_t pix = p.view[vi].pix_off + (int64_t)py * width + px;
  if (GRAD) {
    float4* o = reinterpret_cast<float4*>(out + pix * 12);
    o[0] = make_float4(fmaf(T, p.bg[0], B0), fmaf(T, p.bg[1], B1), fmaf(T, p.bg[2], B2),
                       fmaf(Tx, p.bg[0], Bx0));
    o[1] = make_float4(fmaf(Tx, p.bg[1], Bx1), fmaf(Tx, p.bg[2], Bx2), fmaf(Ty, p.bg[0], By0),
                       fmaf(Ty, p.bg[1], By1));
    o[2] = make_float4(fmaf(Ty, p.bg[2], By2), fmaf(Txy, p.bg[0], Bxy0),
                       fmaf(Txy, p.bg[1], Bxy1), fmaf(Txy, p.bg[2], Bxy2));
  } else {
    float* o = out + pix * 3;
    o[0] = fmaf(T, p.bg[0], B0);
    o[1] = fmaf(T, p.bg[1], B1);
    o[2] = fmaf(T, p.bg[2], B2);
  }
  if (AUX && n_blend) n_blend[pix] = nb;
  if (AUX && n_eval) n_eval[pix] = ne;
  if (AUX && state) {  // for the backward pass: final T and derivatives, end of the walked list
    state[pix] = make_float4(T, Tx, Ty, Txy);
    last[pix] = lastpos;
  }
}

struct RasterOut {
  float* out;
  int32_t* n_blend;
  int32_t* n_eval;
  float4* state;
  int32_t* last;
};

template <int TILE, bool GRAD, int BATCH, int SUB>
void launch(const RasterParams& p, const gs_splat* splats, const int32_t* ids, const int2* ranges,
            const RasterOut& o, hipStream_t stream) {
  const unsigned grid = (unsigned)tile_grid(p.tiles, SUB * SUB);
  if (o.n_blend || o.n_eval || o.state)
    raster_kernel<TILE, GRAD, BATCH, SUB, true><<<grid, TILE * TILE, 0, stream>>>(
        p, splats, ids, ranges, o.out, o.n_blend, o.n_eval, o.state, o.last);
  else
    raster_kernel<TILE, GRAD, BATCH, SUB, false><<<grid, TILE * TILE, 0, stream>>>(
        p, splats, ids, ranges, o.out, o.n_blend, o.n_eval, o.state, o.last);
}

// List tiles of edge TILE * SUB, workgroups of TILE x TILE pixels.  batch
// (relative to the list tile, as in gs_raster_cfg): its area -> one splat per
// thread; a half or a quarter of it -> that fraction of the threads stage.
template <int TILE, bool GRAD, int SUB>
void launch_batch(int batch, const RasterParams& p, const gs_splat* splats, const int32_t* ids,
                  const int2* ranges, const RasterOut& o, hipStream_t stream) {
  constexpr int NT = TILE * TILE, LT = NT * SUB * SUB;
  if (batch == LT / 4) launch<TILE, GRAD, NT / 4, SUB>(p, splats, ids, ranges, o, stream);
  else if (batch == LT / 2) launch<TILE, GRAD, NT / 2, SUB>(p, splats, ids, ranges, o, stream);
  else launch<TILE, GRAD, NT, SUB>(p, splats, ids, ranges, o, stream);
}

}  // namespace

hipError_t launch_raster(const gs_splat* splats, const int32_t* sorted_ids,
                         const int32_t* tile_ranges, int32_t nv, const gs_camera* cams,
                         const gs_raster_cfg& cfg, bool grads, float* out, int32_t* n_blend,
                         int32_t* n_eval, float* state, int32_t* last, hipStream_t stream) {
  const RasterParams p = make_params(nv, cams, cfg);
  const RasterOut o{out, n_blend, n_eval, reinterpret_cast<float4*>(state), last};
  const int2* r2 = reinterpret_cast<const int2*>(tile_ranges);
  if (cfg.tile_size == 8) {
    if (grads) launch_batch<8, true, 1>(cfg.batch, p, splats, sorted_ids, r2, o, stream);
    else launch_batch<8, false, 1>(cfg.batch, p, splats, sorted_ids, r2, o, stream);
  } else if (cfg.tile_size == 16) {
    if (grads) launch_batch<16, true, 1>(cfg.batch, p, splats, sorted_ids, r2, o, stream);
    else launch_batch<16, false, 1>(cfg.batch, p, splats, sorted_ids, r2, o, stream);
  } else if (cfg.tile_size == 32) {
    // 32x32 list tiles, rasterized by 16x16 workgroups (four per list tile)
    if (grads) launch_batch<16, true, 2>(cfg.batch, p, splats, sorted_ids, r2, o, stream);
    else launch_batch<16, false, 2>(cfg.batch, p, splats, sorted_ids, r2, o, stream);
  } else {
    // 64x64 list tiles, sixteen 16x16 workgroups each
    if (grads) launch_batch<16, true, 4>(cfg.batch, p, splats, sorted_ids, r2, o, stream);
    else launch_batch<16, false, 4>(cfg.batch, p, splats, sorted_ids, r2, o, stream);
  }
  return hipGetLastError();
}

}  // namespace gsup
