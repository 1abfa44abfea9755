// gs_raster_grad_backward_views: the backward pass of the gradient-aware
// rasterizer (see the comment below for the method).
#include "raster_common.h"

namespace gsup {

using namespace raster_detail;

namespace {


// ---------------------------------------------------------------------------
// Backward pass (Suppl. "3DGS Gradient Computation - Backward pass").
//
// Given dL/d(I, I_x, I_y, I_xy) per pixel, every pixel walks its blended
// fragments back to front.  The forward saved the final T, T_x, T_y, T_xy and
// the end of the walked list; the state before each fragment is recovered by
// inverting the blend (the inversion trick, in the T form used here, with the
// reading that the state before fragment k is T_k = 1 - A_{k-1}):
//     T = T' / (1 - a),  T_x = (T_x' + T a_x) / (1 - a),  T_y likewise,
//     T_xy = (T_xy' + T a_xy + T_x a_y + T_y a_x) / (1 - a),
// with a <= alpha_max < 1.  Reverse-mode differentiation of the forward
// recurrence (k_* the weights, B_* += c k_*, T_* -= k_*) with the adjoint
// lambda of (T, T_x, T_y, T_xy) gives, with K_* = G_* . c - lambda'_*:
//     dL/dc      += G_0 k + G_x k_x + G_y k_y + G_xy k_xy
//     dL/dalpha   = K T + K_x T_x + K_y T_y + K_xy T_xy
//     dL/dalpha_x = K_x T + K_xy T_y,  dL/dalpha_y = K_y T + K_xy T_x,
//     dL/dalpha_xy = K_xy T
//     lambda_T   = lambda'_T + K a + K_x a_x + K_y a_y + K_xy a_xy,
//     lambda_Tx  = lambda'_Tx + K_x a + K_xy a_y, lambda_Ty likewise,
//     lambda_Txy = lambda'_Txy + K_xy a
// starting from lambda_* = G_* . bg (I_* = B_* + T_* bg).  The alpha
// adjoints go to the splat's mean, conic and opacity through
// a = sigma exp(-q/2), a_x = -a u, a_y = -a v, a_xy = a (u v - b).
// Every wave reduces a splat's contributions over its 64 pixels and adds them
// to the splat's gradient record with one atomic per field (nine lanes, one
// instruction).
// ---------------------------------------------------------------------------
// Sums nine per-lane values over the wave with a transposing butterfly: at
// each of the first four steps a lane keeps half of its (padded to 16)
// partial sums, hands the other half to its partner and adds what it
// receives (8 + 4 + 2 + 1 exchanges instead of 9 x 6); two more steps finish
// the sums.  Afterwards lane L with L % 4 == 0 holds the total of component
// comp = 8 b5 + 4 b4 + 2 b3 + b2 (b_k the bits of L).  The partners at lane
// distance 32 and 16 are reached with gfx950's permlane swaps: swapping the
// upper half-wave (odd rows) of register a with the lower half-wave (even
// rows) of register b leaves every lane holding its own kept value in one
// register and its partner's in the other, so one swap and one add serve a
// pair of components with no lane selects.  The steps inside a row of 16
// lanes pair lanes by DPP (mirror images in the row, the half-row, then the
// quad), which also differ in the bit that decides the kept half.
__device__ __forceinline__ float add_swapped32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float add_swapped16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// A lane's copy of another lane's value by a DPP operand modifier (a VALU
// move, no LDS round trip as for ds_bpermute); CTRL is the GFX9 dpp_ctrl.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}

// Partner lanes by DPP within a row of 16: row_mirror (0x140) pairs i with
// 15 - i (different bit 3), row_half_mirror (0x141) pairs i with 7 - i
// (different bit 2); both keep bits 4 and 5.
template <int N, int CTRL>
__device__ __forceinline__ void half_exchange(float (&v)[16], int lane, int bit) {
  const bool hi = (lane >> bit) & 1;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const float send = hi ? v[i] : v[i + N];
    const float keep = hi ? v[i + N] : v[i];
    v[i] = keep + dpp_mov<CTRL>(send);
  }
}

__device__ __forceinline__ float wave_reduce9(const float (&g)[9], int lane, int& comp) {
  float v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = i < 9 ? g[i] : 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = add_swapped32(v[i], v[i + 8]);  // lane distance 32
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = add_swapped16(v[i], v[i + 4]);  // lane distance 16
  half_exchange<2, 0x140>(v, lane, 3);
  half_exchange<1, 0x141>(v, lane, 2);
  float r = v[0];
  r += dpp_mov<0x4E>(r);  // quad_perm [2, 3, 0, 1]
  r += dpp_mov<0xB1>(r);  // quad_perm [1, 0, 3, 2]
  comp = (((lane >> 5) & 1) << 3) | (((lane >> 4) & 1) << 2) | (((lane >> 3) & 1) << 1) |
         ((lane >> 2) & 1);
  return r;
}

template <int TILE, int BATCH, int SUB>
__global__ __launch_bounds__(TILE* TILE) void raster_bwd_kernel(
    RasterParams p, const gs_splat* __restrict__ splats, const int32_t* __restrict__ ids,
    const int2* __restrict__ ranges, const float4* __restrict__ state,
    const int32_t* __restrict__ last, const float* __restrict__ dout, float* __restrict__ dsplat) {
  constexpr int NT = TILE * TILE;
  constexpr int NW = NT / 64;
  constexpr int QX = TILE / 8;
  constexpr float kHalfLog2e = 0.72134752044448170368f;
  __shared__ float4 s_a[BATCH];   // mean x, mean y (tile-relative), conic a, conic b
  __shared__ float4 s_b[BATCH];   // conic c, log2 sigma, support, red
  __shared__ float4 s_c[BATCH];   // green, blue, 1 / sigma, -
  __shared__ int32_t s_id[BATCH];
  __shared__ uint32_t s_mask[NW > 1 ? BATCH : 1];
  __shared__ uint16_t s_list[NW > 1 ? NW : 1][NW > 1 ? BATCH : 1];
  __shared__ float s_acc[BATCH * 9];  // the batch's splat gradients, summed over the block's waves
  __shared__ int s_end;

  // the same workgroup-to-pixel layout as the forward (identical FP32 offsets)
  int64_t tile;
  int sub;
  tile_block(blockIdx.x, SUB * SUB, tile, sub);
  if (tile >= p.tiles) return;
  int vi = 0;
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
  const int64_t pix = p.view[vi].pix_off + (int64_t)py * width + px;

  float T = 1.f, Tx = 0.f, Ty = 0.f, Txy = 0.f;
  float G[12];
  int lst = rg.x;
  if (inside) {
    const float4 st = state[pix];
    T = st.x;
    Tx = st.y;
    Ty = st.z;
    Txy = st.w;
    lst = last[pix];
    const float4* g4 = reinterpret_cast<const float4*>(dout + pix * 12);
    const float4 a = g4[0], b = g4[1], c = g4[2];
    G[0] = a.x; G[1] = a.y; G[2] = a.z; G[3] = a.w; G[4] = b.x; G[5] = b.y;
    G[6] = b.z; G[7] = b.w; G[8] = c.x; G[9] = c.y; G[10] = c.z; G[11] = c.w;
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) G[k] = 0.f;
  }
  // adjoint of the state after the last fragment: I_* = B_* + T_* bg
  float lT = G[0] * p.bg[0] + G[1] * p.bg[1] + G[2] * p.bg[2];
  float lTx = G[3] * p.bg[0] + G[4] * p.bg[1] + G[5] * p.bg[2];
  float lTy = G[6] * p.bg[0] + G[7] * p.bg[1] + G[8] * p.bg[2];
  float lTxy = G[9] * p.bg[0] + G[10] * p.bg[1] + G[11] * p.bg[2];

  if (t == 0) s_end = rg.x;
  __syncthreads();
  if (lst > rg.x) atomicMax(&s_end, lst);
  __syncthreads();
  const int end = s_end;

  for (int top = end; top > rg.x; top -= BATCH) {
    const int base = max(rg.x, top - BATCH);
    const int cnt = top - base;
    __syncthreads();  // the previous batch's LDS is no longer read
    uint32_t mask = 0;
    if (t < cnt) {
      const int id = ids[base + t];
      const float4* sp = reinterpret_cast<const float4*>(splats + id);
      const double2 m = *reinterpret_cast<const double2*>(sp);
      const float4 q = sp[1];
      const float4 c = sp[2];
      const float mx = (float)(m.x - ox), my = (float)(m.y - oy);
      s_a[t] = make_float4(mx, my, q.x, q.y);
      s_b[t] = make_float4(q.z, opacity_log2(q.w), c.w, c.x);
      s_c[t] = make_float4(c.y, c.z, 1.f / q.w, 0.f);
      s_id[t] = id;
#pragma unroll
      for (int f = 0; f < 9; ++f) s_acc[t * 9 + f] = 0.f;
      if (NW > 1) {
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
          mask = (NW >= 32) ? ~0u : ((1u << NW) - 1u);
        }
        s_mask[t] = mask;
      }
    }
    __syncthreads();
    int nl = cnt;
    if (NW > 1) {
      nl = 0;
      for (int c0 = 0; c0 < cnt; c0 += 64) {
        const int j = c0 + lane;
        const bool hit = j < cnt && ((s_mask[j] >> wave) & 1u);
        const uint64_t bal = __ballot(hit);
        if (hit) s_list[wave][nl + __popcll(bal & lt)] = (uint16_t)j;
        nl += __popcll(bal);
      }
    }
    // this wave's splats of the batch, back to front
    for (int k = nl - 1; k >= 0; --k) {
      const int j = NW > 1 ? (int)s_list[wave][k] : k;
      const int idx = base + j;
      const float4 ga = s_a[j];
      const float4 gb = s_b[j];
      const float dx = fx - ga.x, dy = fy - ga.y;
      const float u = fmaf(ga.z, dx, ga.w * dy);
      const float v = fmaf(ga.w, dx, gb.x * dy);
      const float q = fmaf(dx, u, dy * v);
      // exactly the forward's decisions: blended iff before the pixel's end and above alpha_min
      const bool act = inside && idx < lst && q <= gb.z;
      float g[9];
#pragma unroll
      for (int f = 0; f < 9; ++f) g[f] = 0.f;
      if (act) {
        const float4 gc = s_c[j];
        const float cr = gb.w, cg = gc.x, cb = gc.y, inv_sig = gc.z;
        const float a0 = __builtin_amdgcn_exp2f(fmaf(q, -kHalfLog2e, gb.y));
        // the forward's clamp: alpha_max with zero screen derivatives
        const bool clamp = a0 > p.alpha_max;
        const float alpha = fminf(a0, p.alpha_max);
        const float sa = clamp ? 0.f : a0;
        const float ax = -sa * u;
        const float ay = -sa * v;
        const float axy = sa * fmaf(u, v, -ga.w);
        // state before this fragment (1 / (1 - alpha) by the hardware reciprocal:
        // 1 ulp, and 1 - alpha >= 1 - alpha_max is far from zero)
        const float om = __builtin_amdgcn_rcpf(1.f - alpha);
        T = T * om;
        Tx = fmaf(T, ax, Tx) * om;
        Ty = fmaf(T, ay, Ty) * om;
        Txy = fmaf(T, axy, fmaf(Tx, ay, fmaf(Ty, ax, Txy))) * om;
        const float k0 = T * alpha;
        const float kx = fmaf(T, ax, Tx * alpha);
        const float ky = fmaf(T, ay, Ty * alpha);
        const float kxy = fmaf(T, axy, fmaf(Tx, ay, fmaf(Ty, ax, Txy * alpha)));
        // colour
        g[6] = fmaf(G[0], k0, fmaf(G[3], kx, fmaf(G[6], ky, G[9] * kxy)));
        g[7] = fmaf(G[1], k0, fmaf(G[4], kx, fmaf(G[7], ky, G[10] * kxy)));
        g[8] = fmaf(G[2], k0, fmaf(G[5], kx, fmaf(G[8], ky, G[11] * kxy)));
        const float K0 = fmaf(G[0], cr, fmaf(G[1], cg, G[2] * cb)) - lT;
        const float Kx = fmaf(G[3], cr, fmaf(G[4], cg, G[5] * cb)) - lTx;
        const float Ky = fmaf(G[6], cr, fmaf(G[7], cg, G[8] * cb)) - lTy;
        const float Kxy = fmaf(G[9], cr, fmaf(G[10], cg, G[11] * cb)) - lTxy;
        const float dA = fmaf(K0, T, fmaf(Kx, Tx, fmaf(Ky, Ty, Kxy * Txy)));
        const float dAx = fmaf(Kx, T, Kxy * Ty);
        const float dAy = fmaf(Ky, T, Kxy * Tx);
        const float dAxy = Kxy * T;
        lT = fmaf(K0, alpha, fmaf(Kx, ax, fmaf(Ky, ay, fmaf(Kxy, axy, lT))));
        lTx = fmaf(Kx, alpha, fmaf(Kxy, ay, lTx));
        lTy = fmaf(Ky, alpha, fmaf(Kxy, ax, lTy));
        lTxy = fmaf(Kxy, alpha, lTxy);
        if (!clamp) {
          // g_theta = alpha'_theta E + F_u u'_theta + F_v v'_theta + F_b b'_theta
          const float E = dA - dAx * u - dAy * v + dAxy * fmaf(u, v, -ga.w);
          const float Fu = alpha * fmaf(dAxy, v, -dAx);
          const float Fv = alpha * fmaf(dAxy, u, -dAy);
          const float aE = alpha * E;
          const float a_ = ga.z, b_ = ga.w, c_ = gb.x;
          g[0] = aE * u - a_ * Fu - b_ * Fv;                         // mean x
          g[1] = aE * v - b_ * Fu - c_ * Fv;                         // mean y
          g[2] = fmaf(-0.5f * aE, dx * dx, dx * Fu);                 // conic a
          g[3] = fmaf(-aE, dx * dy, fmaf(dy, Fu, fmaf(dx, Fv, -alpha * dAxy)));  // conic b
          g[4] = fmaf(-0.5f * aE, dy * dy, dy * Fv);                 // conic c
          g[5] = aE * inv_sig;                                       // opacity
        }
      }
      if (__ballot(act) != 0) {
        int comp;
        const float r = wave_reduce9(g, lane, comp);
        if ((lane & 3) == 0 && comp < 9) atomicAdd(&s_acc[j * 9 + comp], r);
      }
    }
    // one global add per (splat, field) the block touched
    __syncthreads();
    for (int e = t; e < cnt * 9; e += NT) {
      const float v = s_acc[e];
      if (v != 0.f) atomicAdd(dsplat + (int64_t)s_id[e / 9] * 9 + e % 9, v);
    }
  }
}

template <int TILE, int SUB>
void launch_bwd(int batch, const RasterParams& p, const gs_splat* splats, const int32_t* ids,
                const int2* ranges, const float4* state, const int32_t* last, const float* dout,
                float* dsplat, hipStream_t stream) {
  constexpr int NT = TILE * TILE, LT = NT * SUB * SUB;
  const unsigned grid = (unsigned)tile_grid(p.tiles, SUB * SUB);
  if (batch == LT / 4)
    raster_bwd_kernel<TILE, NT / 4, SUB><<<grid, NT, 0, stream>>>(p, splats, ids, ranges, state, last, dout, dsplat);
  else if (batch == LT / 2)
    raster_bwd_kernel<TILE, NT / 2, SUB><<<grid, NT, 0, stream>>>(p, splats, ids, ranges, state, last, dout, dsplat);
  else
    raster_bwd_kernel<TILE, NT, SUB><<<grid, NT, 0, stream>>>(p, splats, ids, ranges, state, last, dout, dsplat);
}

__global__ void zero_f32_kernel(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

}  // namespace

hipError_t launch_raster_backward(const gs_splat* splats, const int32_t* sorted_ids,
                                  const int32_t* tile_ranges, int32_t nv, const gs_camera* cams,
                                  const gs_raster_cfg& cfg, const float* state, const int32_t* last,
                                  const float* dout, int64_t n_records, float* dsplat,
                                  hipStream_t stream) {
  const int64_t nz = n_records * 9;
  if (nz > 0) zero_f32_kernel<<<(unsigned)ceil_div(nz, 256), 256, 0, stream>>>(dsplat, nz);
  const RasterParams p = make_params(nv, cams, cfg);
  const int2* r2 = reinterpret_cast<const int2*>(tile_ranges);
  const float4* s4 = reinterpret_cast<const float4*>(state);
  if (cfg.tile_size == 8) launch_bwd<8, 1>(cfg.batch, p, splats, sorted_ids, r2, s4, last, dout, dsplat, stream);
  else if (cfg.tile_size == 16) launch_bwd<16, 1>(cfg.batch, p, splats, sorted_ids, r2, s4, last, dout, dsplat, stream);
  else if (cfg.tile_size == 32) launch_bwd<16, 2>(cfg.batch, p, splats, sorted_ids, r2, s4, last, dout, dsplat, stream);
  else launch_bwd<16, 4>(cfg.batch, p, splats, sorted_ids, r2, s4, last, dout, dsplat, stream);
  return hipGetLastError();
}

}  // namespace gsup
