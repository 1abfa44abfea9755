// gs_bin_sort: per-tile front-to-back splat lists.
//
// The paper blends Gaussians sorted by the depth of their mean
// (Sec. "Differentiable 3D Gaussian Splatting").  A tiled rasterizer needs
// that order restricted to the splats that can reach each tile.  Instead of
// sorting one 64-bit (tile, depth) key per pair, this implementation
//   1. sorts the n splats once by their FP32 depth bits (32-bit LSD radix,
//      4 passes over n elements, stable, so equal depths keep index order),
//   2. counts the tiles of every splat in that order and scans the counts,
//   3. emits (tile, splat) pairs in depth order, and
//   4. stably sorts the pairs by tile id only (ceil(log2 T) bits, 2-3 passes),
// which yields each tile's list in (depth, index) order while moving the
// large pair array only 2-3 times with 8-byte records.
//
// The radix sort is a reduce-then-scan LSD sort with 8-bit digits: an
// upsweep kernel histograms each 4096-element block, a device-wide scan turns
// the digit-major histogram into per-(digit, block) output bases, and a
// downsweep kernel ranks each block's elements stably (wave64 ballot match
// plus per-wave counts in LDS), reorders them in LDS and writes every digit
// run contiguously.
#include <algorithm>

#include "gsup_internal.h"

namespace gsup {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;  // elements per sort / scan block
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kWaves = kThreads / 64;

// ----------------------------------------------------------------------------
// fill
// ----------------------------------------------------------------------------
__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ----------------------------------------------------------------------------
// device-wide exclusive scan (reduce-then-scan), T = uint32_t or uint64_t
// ----------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// Exclusive scan of one value per thread over the block; returns the block total.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* excl, T* s_w) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const T inc = wave_inclusive_scan(v);
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  T wbase = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const T s = s_w[w];
    if (w < wave) wbase += s;
    total += s;
  }
  __syncthreads();
  *excl = wbase + inc - v;
  return total;
}

template <typename T>
__device__ __forceinline__ void load_blocked(const T* in, int64_t m, int64_t base, T (&v)[kItems]) {
  const int64_t s = base + (int64_t)threadIdx.x * kItems;
#pragma unroll
  for (int k = 0; k < kItems; ++k) v[k] = (s + k < m) ? in[s + k] : T(0);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const T* __restrict__ in, int64_t m,
                                                               uint64_t* __restrict__ partials) {
  __shared__ T s_w[kWaves];
  T v[kItems];
  load_blocked(in, m, (int64_t)blockIdx.x * kTile, v);
  T sum = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) sum += v[k];
  T excl;
  const T total = block_exclusive_scan(sum, &excl, s_w);
  if (threadIdx.x == 0) partials[blockIdx.x] = (uint64_t)total;
}

// Scans `in` (m elements) into `out` (may alias) adding bases[blockIdx.x];
// with bases == nullptr the block base is 0.  If total != nullptr the block
// with the last element writes the grand total there.
template <typename T>
__global__ __launch_bounds__(kThreads) void scan_down_kernel(const T* in, T* out, int64_t m,
                                                             const uint64_t* __restrict__ bases,
                                                             uint64_t* __restrict__ total) {
  __shared__ T s_w[kWaves];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  T v[kItems];
  load_blocked(in, m, base, v);
  T sum = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) sum += v[k];
  T excl;
  const T btotal = block_exclusive_scan(sum, &excl, s_w);
  const T off = bases ? (T)bases[blockIdx.x] : T(0);
  T run = off + excl;
  const int64_t s = base + (int64_t)threadIdx.x * kItems;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    if (s + k < m) out[s + k] = run;
    run += v[k];
  }
  if (total && threadIdx.x == 0 && base + kTile >= m) *total = (uint64_t)(off + btotal);
}

// partial-sum storage needed to scan m elements (all recursion levels)
size_t scan_partials_elems(int64_t m) {
  size_t s = 0;
  while (m > kTile) {
    m = ceil_div(m, kTile);
    s += (size_t)m;
  }
  return s + 1;
}

// Exclusive scan of m elements of `data` in place.  partials: uint64 scratch of
// scan_partials_elems(m) elements.  total (optional): device uint64 grand total.
template <typename T>
hipError_t device_exclusive_scan(T* data, int64_t m, uint64_t* partials, uint64_t* total,
                                 hipStream_t stream) {
  if (m <= 0) return hipSuccess;
  const int64_t nb = ceil_div(m, kTile);
  if (nb == 1) {
    scan_down_kernel<T><<<1, kThreads, 0, stream>>>(data, data, m, nullptr, total);
    return hipGetLastError();
  }
  scan_reduce_kernel<T><<<(unsigned)nb, kThreads, 0, stream>>>(data, m, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // scan the block partials (uint64) recursively; their total is the grand total
  e = device_exclusive_scan<uint64_t>(partials, nb, partials + nb, total, stream);
  if (e != hipSuccess) return e;
  scan_down_kernel<T><<<(unsigned)nb, kThreads, 0, stream>>>(data, data, m, partials, nullptr);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// LSD radix sort pass on (uint32 key, uint32 value), BITS-bit digits
//
// Every block owns kTile consecutive elements; wave w of the block owns the
// contiguous quarter [w * kSeg, (w + 1) * kSeg) and walks it 64 elements at a
// time.  Lanes holding the same digit are found with BITS ballots (wave64
// match); the lowest such lane updates the wave's private digit counter in
// LDS.  No block barrier is needed while ranking, and equal digits keep
// their input order (wave-major, then round, then lane).
// ----------------------------------------------------------------------------
constexpr int kSeg = kTile / kWaves;   // elements per wave
constexpr int kRounds = kSeg / 64;     // 64-element rounds per wave

template <int BITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t same = __ballot(valid);
#pragma unroll
  for (int b = 0; b < BITS; ++b) {
    const uint64_t bal = __ballot((d >> b) & 1u);
    same &= ((d >> b) & 1u) ? bal : ~bal;
  }
  return same;
}

__device__ __forceinline__ uint64_t lanes_below(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

template <int BITS>
__global__ __launch_bounds__(kThreads) void radix_upsweep_kernel(const uint32_t* __restrict__ keys,
                                                                 int64_t m, int shift,
                                                                 uint32_t* __restrict__ hist,
                                                                 int64_t nblocks) {
  constexpr uint32_t R = 1u << BITS;
  __shared__ uint32_t s_h[kWaves][kRadix];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) s_h[w][t] = 0;
  __syncthreads();
  const uint64_t lt = lanes_below(lane);
  const int64_t seg = (int64_t)blockIdx.x * kTile + wave * kSeg;
  for (int r = 0; r < kRounds; ++r) {
    const int64_t e = seg + r * 64 + lane;
    const bool valid = e < m;
    const uint32_t d = valid ? (keys[e] >> shift) & (R - 1) : 0u;
    const uint64_t same = match_digit<BITS>(d, valid);
    if (valid && (same & lt) == 0) s_h[wave][d] += (uint32_t)__popcll(same);
  }
  __syncthreads();
  if (t < (int)R) {
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) c += s_h[w][t];
    hist[(int64_t)t * nblocks + blockIdx.x] = c;
  }
}

template <int BITS>
__global__ __launch_bounds__(kThreads) void radix_downsweep_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out, int64_t m, int shift,
    const uint32_t* __restrict__ hist, int64_t nblocks) {
  constexpr uint32_t R = 1u << BITS;
  __shared__ uint32_t s_keys[kTile];
  __shared__ uint32_t s_vals[kTile];
  __shared__ uint32_t s_wh[kWaves][kRadix];  // per-wave digit counts, then per-wave bases
  __shared__ uint32_t s_gbase[kRadix];
  __shared__ uint32_t s_lstart[kRadix];
  __shared__ uint32_t s_w[kWaves];

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t base = (int64_t)blockIdx.x * kTile;
  const int64_t seg = base + wave * kSeg;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) s_wh[w][t] = 0;
  s_gbase[t] = t < (int)R ? hist[(int64_t)t * nblocks + blockIdx.x] : 0u;
  __syncthreads();

  // 1. rank within the wave's segment
  const uint64_t lt = lanes_below(lane);
  uint32_t key[kRounds], val[kRounds], rank[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t e = seg + r * 64 + lane;
    const bool valid = e < m;
    key[r] = valid ? keys_in[e] : 0u;
    val[r] = valid ? vals_in[e] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const bool valid = seg + r * 64 + lane < m;
    const uint32_t d = (key[r] >> shift) & (R - 1);
    const uint64_t same = match_digit<BITS>(d, valid);
    const uint32_t below = (uint32_t)__popcll(same & lt);
    const uint32_t old = s_wh[wave][d];
    if (valid && below == 0) s_wh[wave][d] = old + (uint32_t)__popcll(same);
    rank[r] = old + below;
  }
  __syncthreads();

  // 2. per digit: wave bases inside the block, digit starts of the block
  {
    uint32_t c[kWaves], tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      c[w] = s_wh[w][t];
      tot += c[w];
    }
    uint32_t excl;
    block_exclusive_scan<uint32_t>(tot, &excl, s_w);
    s_lstart[t] = excl;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      s_wh[w][t] = excl;
      excl += c[w];
    }
  }
  __syncthreads();

  // 3. reorder the block in LDS by digit
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    if (seg + r * 64 + lane < m) {
      const uint32_t d = (key[r] >> shift) & (R - 1);
      const uint32_t pos = s_wh[wave][d] + rank[r];
      s_keys[pos] = key[r];
      s_vals[pos] = val[r];
    }
  }
  __syncthreads();

  // 4. digit runs are contiguous: consecutive threads write consecutive addresses
  const int count = (m - base < kTile) ? (int)(m - base) : kTile;
  for (int i = t; i < count; i += kThreads) {
    const uint32_t k = s_keys[i];
    const uint32_t d = (k >> shift) & (R - 1);
    const uint32_t dst = s_gbase[d] + (uint32_t)i - s_lstart[d];
    keys_out[dst] = k;
    vals_out[dst] = s_vals[i];
  }
}

template <int BITS>
hipError_t radix_pass_bits(const uint32_t* kin, const uint32_t* vin, uint32_t* kout,
                           uint32_t* vout, int64_t m, int shift, uint32_t* hist,
                           uint64_t* partials, hipStream_t stream) {
  const int64_t nb = ceil_div(m, kTile);
  radix_upsweep_kernel<BITS><<<(unsigned)nb, kThreads, 0, stream>>>(kin, m, shift, hist, nb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = device_exclusive_scan<uint32_t>(hist, (int64_t)(1 << BITS) * nb, partials, nullptr, stream);
  if (e != hipSuccess) return e;
  radix_downsweep_kernel<BITS><<<(unsigned)nb, kThreads, 0, stream>>>(kin, vin, kout, vout, m,
                                                                       shift, hist, nb);
  return hipGetLastError();
}

// One stable pass over `bits` (1..8) bits starting at `shift`.
hipError_t radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                      int64_t m, int shift, int bits, uint32_t* hist, uint64_t* partials,
                      hipStream_t stream) {
  switch (bits) {
    case 1: return radix_pass_bits<1>(kin, vin, kout, vout, m, shift, hist, partials, stream);
    case 2: return radix_pass_bits<2>(kin, vin, kout, vout, m, shift, hist, partials, stream);
    case 3: return radix_pass_bits<3>(kin, vin, kout, vout, m, shift, hist, partials, stream);
    case 4: return radix_pass_bits<4>(kin, vin, kout, vout, m, shift, hist, partials, stream);
    case 5: return radix_pass_bits<5>(kin, vin, kout, vout, m, shift, hist, partials, stream);
    case 6: return radix_pass_bits<6>(kin, vin, kout, vout, m, shift, hist, partials, stream);
    case 7: return radix_pass_bits<7>(kin, vin, kout, vout, m, shift, hist, partials, stream);
    default: return radix_pass_bits<8>(kin, vin, kout, vout, m, shift, hist, partials, stream);
  }
}

// ----------------------------------------------------------------------------
// binning kernels
// ----------------------------------------------------------------------------
// Tile rectangle clipped to the tile grid (so no tile id can leave it).
__device__ __forceinline__ int4 clip_rect(int4 r, int32_t tiles_x, int32_t tiles_y) {
  return make_int4(max(r.x, 0), max(r.y, 0), min(r.z, tiles_x), min(r.w, tiles_y));
}

__device__ __forceinline__ uint32_t rect_tiles(int4 r) {
  return (uint32_t)(max(r.z - r.x, 0) * max(r.w - r.y, 0));
}

// depth key of splat i: FP32 bits (monotone for depth > 0); splats that reach
// no tile sort last.
__global__ void depth_key_kernel(int64_t n, const float* __restrict__ depth,
                                 const int4* __restrict__ rect, int32_t tiles_x, int32_t tiles_y,
                                 uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int4 r = clip_rect(rect[i], tiles_x, tiles_y);
  keys[i] = rect_tiles(r) ? __float_as_uint(depth[i]) : 0xFFFFFFFFu;
  vals[i] = (uint32_t)i;
}

// rectangles in depth order (clipped) and their tile counts
__global__ void gather_rect_kernel(int64_t n, const uint32_t* __restrict__ order,
                                   const int4* __restrict__ rect, int32_t tiles_x,
                                   int32_t tiles_y, int4* __restrict__ srect,
                                   uint64_t* __restrict__ cnt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int4 r = clip_rect(rect[order[p]], tiles_x, tiles_y);
  srect[p] = r;
  cnt[p] = rect_tiles(r);
}

// Pair emission, load-balanced: a block takes 256 consecutive splats (depth
// order), whose pairs form one contiguous range; every thread writes one pair
// per step, finding its splat by binary search over the block's offsets in
// LDS, so the writes are coalesced whatever the splats' tile counts.
constexpr int kEmit = 256;
__global__ __launch_bounds__(kEmit) void emit_kernel(int64_t n, const uint32_t* __restrict__ order,
                                                     const int4* __restrict__ srect,
                                                     const uint64_t* __restrict__ offs,
                                                     const uint64_t* __restrict__ total,
                                                     int32_t tiles_x, uint32_t* __restrict__ tkeys,
                                                     uint32_t* __restrict__ tvals) {
  __shared__ uint32_t s_off[kEmit + 1];
  __shared__ int4 s_rect[kEmit];
  __shared__ uint32_t s_gid[kEmit];
  const int t = threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.x * kEmit;
  const int nb = (int)((n - p0 < kEmit) ? (n - p0) : kEmit);
  const uint64_t base = offs[p0];
  if (t < nb) {
    s_off[t] = (uint32_t)(offs[p0 + t] - base);
    s_rect[t] = srect[p0 + t];
    s_gid[t] = order[p0 + t];
  }
  if (t == 0) s_off[nb] = (uint32_t)(((p0 + kEmit < n) ? offs[p0 + kEmit] : *total) - base);
  __syncthreads();
  const uint32_t end = s_off[nb];
  for (uint32_t k = t; k < end; k += kEmit) {
    // owner: the last j with s_off[j] <= k (splats without tiles have s_off[j] == s_off[j+1])
    int lo = 0, hi = nb;  // invariant: s_off[lo] <= k < s_off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_off[mid] <= k) lo = mid;
      else hi = mid;
    }
    const int4 r = s_rect[lo];
    const uint32_t li = k - s_off[lo];
    const uint32_t w = (uint32_t)(r.z - r.x);
    // row / column inside the rectangle; the float quotient is exact to +-1
    int dy = (int)(((float)li + 0.5f) / (float)w);
    int dx = (int)li - dy * (int)w;
    if (dx < 0) {
      --dy;
      dx += (int)w;
    } else if (dx >= (int)w) {
      ++dy;
      dx -= (int)w;
    }
    tkeys[base + k] = (uint32_t)(r.y + dy) * (uint32_t)tiles_x + (uint32_t)(r.x + dx);
    tvals[base + k] = s_gid[lo];
  }
}

__global__ void tile_range_kernel(int64_t K, const uint32_t* __restrict__ tkeys,
                                  int32_t* __restrict__ ranges) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= K) return;
  const uint32_t t = tkeys[p];
  if (p == 0 || tkeys[p - 1] != t) ranges[2 * (int64_t)t] = (int32_t)p;
  if (p == K - 1 || tkeys[p + 1] != t) ranges[2 * (int64_t)t + 1] = (int32_t)(p + 1);
}

inline unsigned grid1d(int64_t n, int threads) { return (unsigned)ceil_div(n, threads); }

}  // namespace

BinSortPlan make_bin_sort_plan(int64_t n, int64_t capacity, int32_t width, int32_t height,
                               int32_t tile_size) {
  BinSortPlan p;
  p.n = n;
  p.capacity = capacity;
  p.tiles_x = ceil_div(width, tile_size);
  p.tiles_y = ceil_div(height, tile_size);
  p.tiles = p.tiles_x * p.tiles_y;
  int bits = 1;
  while ((int64_t(1) << bits) < p.tiles) ++bits;
  p.tile_bits = bits;
  const size_t A = 256;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, A);
    return o;
  };
  const size_t n4 = sizeof(uint32_t) * (size_t)std::max<int64_t>(n, 1);
  const size_t c4 = sizeof(uint32_t) * (size_t)std::max<int64_t>(capacity, 1);
  p.off_gkey[0] = take(n4);
  p.off_gkey[1] = take(n4);
  p.off_gval[0] = take(n4);
  p.off_gval[1] = take(n4);
  p.off_cnt = take(sizeof(uint64_t) * (size_t)(n + 1));
  p.off_srect = take(sizeof(int32_t) * 4 * (size_t)std::max<int64_t>(n, 1));
  p.off_pkey[0] = take(c4);
  p.off_pkey[1] = take(c4);
  p.off_pval = take(c4);
  const int64_t max_blocks = std::max<int64_t>(ceil_div(std::max<int64_t>(n, 1), kTile),
                                               ceil_div(std::max<int64_t>(capacity, 1), kTile));
  const int64_t hist_elems = (int64_t)kRadix * max_blocks;
  p.off_hist = take(sizeof(uint32_t) * (size_t)hist_elems);
  const size_t part = std::max(scan_partials_elems(hist_elems), scan_partials_elems(n + 1));
  p.off_scan = take(sizeof(uint64_t) * part);
  p.off_total = take(sizeof(uint64_t));
  p.bytes = off;
  return p;
}

gs_status run_bin_sort(const BinSortPlan& p, const float* depth, const int32_t* rect,
                       int32_t* sorted_ids, int32_t* tile_ranges, int64_t* n_pairs,
                       void* workspace, hipStream_t stream) {
  char* ws = static_cast<char*>(workspace);
  auto u32 = [&](size_t o) { return reinterpret_cast<uint32_t*>(ws + o); };
  uint64_t* cnt = reinterpret_cast<uint64_t*>(ws + p.off_cnt);
  uint32_t* hist = u32(p.off_hist);
  uint64_t* partials = reinterpret_cast<uint64_t*>(ws + p.off_scan);
  uint64_t* total = reinterpret_cast<uint64_t*>(ws + p.off_total);
  const int4* r4 = reinterpret_cast<const int4*>(rect);
  const int64_t n = p.n;
  hipError_t e;
#define GS_TRY(expr, what)                         \
  do {                                             \
    e = (expr);                                    \
    if (e != hipSuccess) return check_hip(e, what); \
  } while (0)

  if (n == 0) {
    *n_pairs = 0;
    fill_i32_kernel<<<grid1d(2 * p.tiles, 256), 256, 0, stream>>>(tile_ranges, 2 * p.tiles, 0);
    return check_hip(hipGetLastError(), "fill_i32_kernel");
  }
  // 1. depth order of all splats (4 stable 8-bit passes over the FP32 bits)
  const int32_t tx = (int32_t)p.tiles_x, ty = (int32_t)p.tiles_y;
  depth_key_kernel<<<grid1d(n, 256), 256, 0, stream>>>(n, depth, r4, tx, ty, u32(p.off_gkey[0]),
                                                        u32(p.off_gval[0]));
  GS_TRY(hipGetLastError(), "depth_key_kernel");
  int cur = 0;
  for (int shift = 0; shift < 32; shift += kRadixBits) {
    GS_TRY(radix_pass(u32(p.off_gkey[cur]), u32(p.off_gval[cur]), u32(p.off_gkey[cur ^ 1]),
                      u32(p.off_gval[cur ^ 1]), n, shift, kRadixBits, hist, partials, stream),
           "depth radix pass");
    cur ^= 1;
  }
  const uint32_t* order = u32(p.off_gval[cur]);

  // 2. tiles per splat in depth order -> pair offsets and the total K
  int4* srect = reinterpret_cast<int4*>(ws + p.off_srect);
  gather_rect_kernel<<<grid1d(n, 256), 256, 0, stream>>>(n, order, r4, tx, ty, srect, cnt);
  GS_TRY(hipGetLastError(), "gather_rect_kernel");
  GS_TRY(device_exclusive_scan<uint64_t>(cnt, n, partials, total, stream), "pair offset scan");
  uint64_t K = 0;
  GS_TRY(hipMemcpyAsync(&K, total, sizeof(K), hipMemcpyDeviceToHost, stream), "pair count copy");
  GS_TRY(hipStreamSynchronize(stream), "pair count sync");
  *n_pairs = (int64_t)K;
  if (K >= (uint64_t(1) << 31))
    return fail(GS_ERR_CAPACITY, "gs_bin_sort: %llu pairs exceed the 2^31 index limit",
                (unsigned long long)K);
  if ((int64_t)K > p.capacity)
    return fail(GS_ERR_CAPACITY, "gs_bin_sort: %llu pairs exceed capacity %lld",
                (unsigned long long)K, (long long)p.capacity);

  // 3. empty ranges, then pairs in depth order
  fill_i32_kernel<<<grid1d(2 * p.tiles, 256), 256, 0, stream>>>(tile_ranges, 2 * p.tiles, 0);
  GS_TRY(hipGetLastError(), "fill_i32_kernel");
  if (K == 0) return GS_OK;
  const int passes = (p.tile_bits + kRadixBits - 1) / kRadixBits;
  // values end in sorted_ids after `passes` ping-pong steps
  uint32_t* vbuf[2];
  vbuf[0] = (passes % 2 == 0) ? reinterpret_cast<uint32_t*>(sorted_ids) : u32(p.off_pval);
  vbuf[1] = (passes % 2 == 0) ? u32(p.off_pval) : reinterpret_cast<uint32_t*>(sorted_ids);
  uint32_t* kbuf[2] = {u32(p.off_pkey[0]), u32(p.off_pkey[1])};
  emit_kernel<<<grid1d(n, kEmit), kEmit, 0, stream>>>(n, order, srect, cnt, total, tx, kbuf[0],
                                                       vbuf[0]);
  GS_TRY(hipGetLastError(), "emit_kernel");

  // 4. stable sort of the pairs by tile id
  cur = 0;
  for (int k = 0; k < passes; ++k) {
    const int shift = k * kRadixBits;
    const int bits = std::min(kRadixBits, p.tile_bits - shift);
    GS_TRY(radix_pass(kbuf[cur], vbuf[cur], kbuf[cur ^ 1], vbuf[cur ^ 1], (int64_t)K, shift, bits,
                      hist, partials, stream),
           "tile radix pass");
    cur ^= 1;
  }
  tile_range_kernel<<<grid1d((int64_t)K, 256), 256, 0, stream>>>((int64_t)K, kbuf[cur],
                                                                  tile_ranges);
  GS_TRY(hipGetLastError(), "tile_range_kernel");
#undef GS_TRY
  return GS_OK;
}

}  // namespace gsup
