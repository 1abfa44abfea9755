// gs_bin_sort: per-tile front-to-back splat lists.
//
// The paper blends Gaussians sorted by the depth of their mean
// (Sec. "Differentiable 3D Gaussian Splatting").  A tiled rasterizer needs
// that order restricted to the splats that can reach each tile.  Instead of
// sorting one 64-bit (tile, depth) key per pair, this implementation
//   1. sorts the splats that reach a tile (finite depth) once by their FP32
//      depth bits (stable LSD radix sort, so equal depths keep index order;
//      the first pass drops the +inf depths of splats without tiles and the
//      top pass runs only for depth ranges wider than 8 binades),
//   2. sums the splats' tile counts per block of 4096 splats in that order
//      (their clipped rectangles travel through the sort packed in 32 bits),
//   3. emits (tile, splat) pairs in depth order, one thread per pair, every
//      block of 256 splats finding its first pair and the total K from those
//      sums itself (no separate scan launch), and
//   4. stably sorts the pairs by tile id only (ceil(log2 T) bits; with one
//      pass, its digit counts are the tile ranges),
// which yields each tile's list in (depth, index) order while moving the
// large pair array only once or twice with 8-byte records.
//
// Radix passes use digits of up to GSUP_MAX_DIGIT_BITS bits (default 8; the
// key bits are split evenly over the fewest passes; on MI355X 11-bit digits
// measured slower: their LDS footprint allows one block per CU): an upsweep
// kernel counts each 4096-element block's digits (LDS atomic adds into
// wave-private counts), one workgroup per digit scans that digit's counts
// over the blocks, and a downsweep kernel ranks each block's elements stably
// (each lane finds the lanes of its wave holding its digit, then the lowest
// of them advances the wave's private counter in LDS), reorders them in LDS
// and writes every digit run contiguously.
#include <algorithm>
#include <cstring>

#include "gsup_internal.h"

namespace gsup {
namespace {

constexpr int kThreads = 256;
#ifndef GSUP_SORT_ITEMS
#define GSUP_SORT_ITEMS 16
#endif
constexpr int kItems = GSUP_SORT_ITEMS;  // elements per thread of a sort / scan block
constexpr int kTile = kThreads * kItems;  // elements per sort / scan block
constexpr int kWaves = kThreads / 64;

// Pair count reported when the depth keys span more than the launched depth
// passes sort (a depth outside the views' [near_plane, far_plane]).
constexpr uint64_t kDepthRangeError = uint64_t(GS_PAIRS_DEPTH_RANGE);

// Pair count a device-count pass works on: the emitted total when it fits the
// capacity (and the int32 index range), else 0 so that every later pass and
// the tile ranges see an empty pair list.
__device__ __forceinline__ int64_t eff_count(const uint64_t* total, int64_t cap) {
  const uint64_t k = *total;
  return (k <= (uint64_t)cap && k < (uint64_t(1) << 31)) ? (int64_t)k : 0;
}

// ----------------------------------------------------------------------------
// fill
// ----------------------------------------------------------------------------
__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ----------------------------------------------------------------------------
// block-level scans (wave64 shuffles + one LDS slot per wave)
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

// Exclusive scan of one value per thread over a block of NT threads; returns
// the block total.  s_w: NT / 64 slots of LDS.
template <typename T, int NT = kThreads>
__device__ __forceinline__ T block_exclusive_scan(T v, T* excl, T* s_w) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const T inc = wave_inclusive_scan(v);
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  T wbase = 0, total = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const T s = s_w[w];
    if (w < wave) wbase += s;
    total += s;
  }
  __syncthreads();
  *excl = wbase + inc - v;
  return total;
}

// Exclusive scan, in place, of m elements by one workgroup of NT threads;
// returns the total.  Rounds of NT * kItems elements: thread t loads
// elements t, t + NT, ... of the round (coalesced: a wave reads 64
// consecutive elements per load), then the stripes are scanned across the
// block one after the other with a running carry.
template <typename T, int NT>
__device__ __forceinline__ T block_scan_inplace(T* __restrict__ data, int64_t m, T* s_w) {
  T carry = 0;
  for (int64_t base = 0; base < m; base += (int64_t)NT * kItems) {
    T v[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int64_t i = base + (int64_t)k * NT + threadIdx.x;
      v[k] = i < m ? data[i] : T(0);
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      if (base + (int64_t)k * NT >= m) break;  // uniform over the block
      const int64_t i = base + (int64_t)k * NT + threadIdx.x;
      T excl;
      const T tot = block_exclusive_scan<T, NT>(v[k], &excl, s_w);
      if (i < m) data[i] = carry + excl;
      carry += tot;
    }
  }
  return carry;
}

// ----------------------------------------------------------------------------
// tile rectangles
// ----------------------------------------------------------------------------
// Tile rectangle clipped to the tile grid (so no tile id can leave it).
__device__ __forceinline__ int4 clip_rect(short4 r, int32_t tiles_x, int32_t tiles_y) {
  return make_int4(max((int)r.x, 0), max((int)r.y, 0), min((int)r.z, tiles_x), min((int)r.w, tiles_y));
}

__device__ __forceinline__ uint32_t rect_tiles(int4 r) {
  return (uint32_t)(max(r.z - r.x, 0) * max(r.w - r.y, 0));
}

// View of splat record e: splats of view v are e in [v n, (v + 1) n).
__device__ __forceinline__ int view_of(const ViewTiles& vt, uint32_t e) {
  return vt.nv > 1 ? (int)(e / (uint32_t)vt.n) : 0;
}

// A clipped rectangle in 32 bits (x0: 10, y0: 10, width: 6, height: 6 bits)
// travels with its splat through the depth sort, so that the pair count and
// emission read it in depth order without a random 16-byte gather (which
// costs a whole cache line per splat).  Rectangles that do not fit get the
// escape code and are read from the projection's array instead.
constexpr uint32_t kRectEscape = 0xFFFFFFFFu;
__device__ __forceinline__ uint32_t pack_rect(int4 r) {
  const int w = max(r.z - r.x, 0), h = max(r.w - r.y, 0);
  if (r.x > 1022 || r.y > 1023 || w > 63 || h > 63) return kRectEscape;  // x0 = 1023: escape only
  return (uint32_t)r.x | ((uint32_t)r.y << 10) | ((uint32_t)w << 20) | ((uint32_t)h << 26);
}

__device__ __forceinline__ int4 unpack_rect(uint32_t c) {
  const int x = (int)(c & 1023u), y = (int)((c >> 10) & 1023u);
  return make_int4(x, y, x + (int)((c >> 20) & 63u), y + (int)(c >> 26));
}

// Clipped rectangle of splat record e from its packed code (or, escaped,
// from the projection's rectangles).
__device__ __forceinline__ int4 splat_rect(uint32_t code, uint32_t e, const short4* __restrict__ rect,
                                           const ViewTiles& vt) {
  if (code != kRectEscape) return unpack_rect(code);
  const int v = view_of(vt, e);
  return clip_rect(rect[e], vt.tiles_x[v], vt.tiles_y[v]);
}

// 32-bit payload a downsweep moves with each element (to == nullptr: none):
// the packed rectangle, built from `rect` in the first depth pass (where
// the value is the splat record's index) and read from `from` in later ones.
struct Payload {
  const uint32_t* from = nullptr;
  const short4* rect = nullptr;
  ViewTiles vt;
  uint32_t* to = nullptr;
};

// ----------------------------------------------------------------------------
// LSD radix sort pass on (uint32 key, uint32 value), BITS-bit digits (1..11)
//
// upsweep    per-block digit histogram -> hist[digit][block]
// hist_scan  one workgroup per digit: exclusive scan of that digit's row over
//            the blocks, plus the digit's total
// downsweep  per block: digit starts from the totals, stable local ranks,
//            reorder in LDS, contiguous writes of every digit run
//
// Every block owns kTile consecutive elements; wave w of the block owns the
// contiguous quarter [w * kSeg, (w + 1) * kSeg) and walks it 64 elements at a
// time.  In the downsweep, the lanes holding the same digit are found through
// a 64-bit LDS mask word per digit (9-bit digits) or BITS ballots (narrower
// ones); the lowest such lane updates the wave's private digit counter in
// LDS.  No block barrier is needed while ranking, and equal digits keep
// their input order (wave-major, then round, then lane).  The upsweep needs
// only counts: one LDS atomic add per element.
// ----------------------------------------------------------------------------
constexpr int kSeg = kTile / kWaves;   // elements per wave
constexpr int kRounds = kSeg / 64;     // 64-element rounds per wave
#ifndef GSUP_MAX_DIGIT_BITS
#define GSUP_MAX_DIGIT_BITS 8
#endif
constexpr int kMaxDigitBits = GSUP_MAX_DIGIT_BITS;
static_assert(kMaxDigitBits >= 1 && kMaxDigitBits <= 11, "digit width");
// Widest digit of the pair (tile id) sort: up to 2^kMaxTileDigitBits list
// tiles sort in a single pass, whose digit counts are then the tile ranges.
#ifndef GSUP_MAX_TILE_DIGIT_BITS
#define GSUP_MAX_TILE_DIGIT_BITS 9
#endif
constexpr int kMaxTileDigitBits = GSUP_MAX_TILE_DIGIT_BITS;
constexpr int kMaxAnyDigitBits = kMaxDigitBits > kMaxTileDigitBits ? kMaxDigitBits : kMaxTileDigitBits;
static_assert(kMaxTileDigitBits >= 1 && kMaxTileDigitBits <= 11, "tile digit width");

// Tile ranges from per-tile pair counts (tiles <= 2^kMaxAnyDigitBits): an
// exclusive scan by one workgroup; a tile without pairs gets [0, 0).  Run by
// block 0 of a single-pass tile sort's downsweep, whose digit counts are the
// list lengths.
struct RangesOut {
  int32_t* ranges = nullptr;
  int64_t tiles = 0;
};

__device__ __forceinline__ void ranges_from_counts(const uint32_t* __restrict__ counts,
                                                   const RangesOut& ro, uint32_t* s_w) {
  constexpr int R = 1 << kMaxAnyDigitBits;
  constexpr int DPT = R > kThreads ? R / kThreads : 1;
  uint32_t v[DPT], sum = 0;
#pragma unroll
  for (int k = 0; k < DPT; ++k) {
    const int64_t t = (int64_t)threadIdx.x * DPT + k;
    v[k] = t < ro.tiles ? counts[t] : 0u;
    sum += v[k];
  }
  uint32_t excl;
  block_exclusive_scan<uint32_t>(sum, &excl, s_w);
#pragma unroll
  for (int k = 0; k < DPT; ++k) {
    const int64_t t = (int64_t)threadIdx.x * DPT + k;
    if (t < ro.tiles) {
      ro.ranges[2 * t] = v[k] ? (int32_t)excl : 0;
      ro.ranges[2 * t + 1] = v[k] ? (int32_t)(excl + v[k]) : 0;
    }
    excl += v[k];
  }
}


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

// Depth-key passes.  A splat without tiles has the depth +inf; the first
// pass drops those keys (they would only travel to the end of the order)
// and records the min, max and count of the others.  Later passes sort
// key - base, base = min with the first pass's digit bits cleared (so the
// first pass's digit of key and of key - base agree); a pass whose digit is
// zero for every key - base (its shift is at or above the bit length of
// max - base) does nothing.  With the depth plan's widths (8, 9, 9, 6) that
// skips the top pass whenever max - base < 2^26, which any set of depths
// within a factor of 128 of each other satisfies, without the host reading
// the range.  With info == nullptr a pass sorts plain keys.
struct DepthKeys {
  uint32_t* info = nullptr;  // device: [0] min kept key, [1] max kept key, [2] buffer of the last pass run
  uint64_t* kept = nullptr;  // device: keys kept by the first pass
  uint32_t* bstat = nullptr;  // device: first pass, per block (min, max, count, -) of its kept keys
  uint32_t low_mask = 0;     // (1 << first pass width) - 1
  int first = 0;             // this is the first pass
  int out_index = 0;         // ping-pong buffer this pass writes (recorded in info[2])
};
constexpr uint32_t kInfBits = 0x7F800000u;

__device__ __forceinline__ uint32_t depth_base(const DepthKeys& dk) {
  return (dk.info && !dk.first) ? (dk.info[0] & ~dk.low_mask) : 0u;
}

__device__ __forceinline__ bool pass_is_identity(const DepthKeys& dk, int shift) {
  if (!dk.info || dk.first) return false;
  const uint32_t base = depth_base(dk), hi = dk.info[1];
  const int bits = hi > base ? 32 - __clz(hi - base) : 0;
  return shift >= bits;
}

__device__ __forceinline__ bool key_kept(const DepthKeys& dk, uint32_t key) {
  return !dk.first || key != kInfBits;
}

// Min, max and count of a block's kept keys (first pass) to bstat[block];
// the pass's scan reduces them.  No atomics: thousands of them on one
// address serialise in L2.
__device__ __forceinline__ void record_kept_keys(const DepthKeys& dk, uint32_t lo, uint32_t hi,
                                                 uint32_t count, uint4* s_stat) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, d, 64));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, d, 64));
    count += (uint32_t)__shfl_xor((int)count, d, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) s_stat[wave] = make_uint4(lo, hi, count, 0u);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint4 r = s_stat[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) {
      r.x = min(r.x, s_stat[w].x);
      r.y = max(r.y, s_stat[w].y);
      r.z += s_stat[w].z;
    }
    reinterpret_cast<uint4*>(dk.bstat)[blockIdx.x] = r;
  }
}

// First pass: min, max and count over the blocks' records into info / kept.
__device__ __forceinline__ void reduce_kept_keys(const DepthKeys& dk, int64_t nblocks) {
  __shared__ uint32_t s_lo[kWaves], s_hi[kWaves];
  __shared__ uint64_t s_n[kWaves];
  uint32_t lo = 0xFFFFFFFFu, hi = 0u;
  uint64_t cnt = 0;
  for (int64_t b = threadIdx.x; b < nblocks; b += kThreads) {
    const uint4 r = reinterpret_cast<const uint4*>(dk.bstat)[b];
    lo = min(lo, r.x);
    hi = max(hi, r.y);
    cnt += r.z;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, d, 64));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, d, 64));
    cnt += __shfl_xor(cnt, d, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    s_lo[wave] = lo;
    s_hi[wave] = hi;
    s_n[wave] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 1; w < kWaves; ++w) {
      lo = min(lo, s_lo[w]);
      hi = max(hi, s_hi[w]);
      cnt += s_n[w];
    }
    dk.info[0] = lo;
    dk.info[1] = hi;
    dk.info[2] = 0u;
    dk.kept[0] = cnt;
  }
}

template <int BITS>
__global__ __launch_bounds__(kThreads) void radix_upsweep_kernel(const uint32_t* __restrict__ keys,
                                                                 int64_t m, const uint64_t* m_dev,
                                                                 int64_t cap, int shift,
                                                                 uint32_t* __restrict__ hist,
                                                                 int64_t nblocks, DepthKeys dk) {
  constexpr int R = 1 << BITS;
  __shared__ uint32_t s_h[kWaves][R];
  __shared__ uint4 s_stat[kWaves];
  if (pass_is_identity(dk, shift)) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (m_dev) m = eff_count(m_dev, cap);
  if ((int64_t)blockIdx.x * kTile >= m) {  // past the data: an empty column
    for (int d = t; d < R; d += kThreads) hist[(int64_t)d * nblocks + blockIdx.x] = 0u;
    if (dk.first && t == 0)
      reinterpret_cast<uint4*>(dk.bstat)[blockIdx.x] = make_uint4(0xFFFFFFFFu, 0u, 0u, 0u);
    return;
  }
  for (int k = t; k < kWaves * R; k += kThreads) (&s_h[0][0])[k] = 0;
  const int64_t seg = (int64_t)blockIdx.x * kTile + wave * kSeg;
  uint32_t key[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t e = seg + r * 64 + lane;
    key[r] = e < m ? keys[e] : 0u;
  }
  __syncthreads();
  const uint32_t base = depth_base(dk);
  uint32_t lo = 0xFFFFFFFFu, hi = 0u, kept = 0u;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const bool valid = seg + r * 64 + lane < m && key_kept(dk, key[r]);
    const uint32_t d = ((key[r] - base) >> shift) & (R - 1);
    // counts only (no ranks here): one LDS atomic add per key
    if (valid) atomicAdd(&s_h[wave][d], 1u);
    if (valid) {
      lo = min(lo, key[r]);
      hi = max(hi, key[r]);
      ++kept;
    }
  }
  if (dk.first) record_kept_keys(dk, lo, hi, kept, s_stat);
  __syncthreads();
  for (int d = t; d < R; d += kThreads) {
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) c += s_h[w][d];
    hist[(int64_t)d * nblocks + blockIdx.x] = c;
  }
}

// Block d scans row d of hist (nblocks entries) in place and writes its total.
__global__ __launch_bounds__(kThreads) void hist_scan_kernel(uint32_t* __restrict__ hist,
                                                             int64_t nblocks,
                                                             uint32_t* __restrict__ totals,
                                                             DepthKeys dk, int shift) {
  __shared__ uint32_t s_w[kWaves];
  if (pass_is_identity(dk, shift)) return;
  if (dk.first && blockIdx.x == 0) reduce_kept_keys(dk, nblocks);
  uint32_t* row = hist + (int64_t)blockIdx.x * nblocks;
  const uint32_t carry = block_scan_inplace<uint32_t, kThreads>(row, nblocks, s_w);
  if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Depth-pass downsweep blocks are numbered so that every XCD owns one
// contiguous range of blocks (xcd_block): the digit runs of neighbouring
// blocks are adjacent in the output and share cache lines, which then meet
// in one L2 before they are written back instead of leaving several XCDs as
// partial lines.  The pair (tile id) passes keep the plain numbering, which
// measured faster for them on MI355X.
template <int BITS>
__global__ __launch_bounds__(kThreads) void radix_downsweep_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in /* null: index */,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out, int64_t m,
    const uint64_t* m_dev, int64_t cap, int shift, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ totals, int64_t nblocks, DepthKeys dk, Payload pl,
    RangesOut ro) {
  constexpr int R = 1 << BITS;
  __shared__ uint32_t s_w[kWaves];
  if (pass_is_identity(dk, shift)) return;
  const int64_t blk = dk.info ? xcd_block(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
  if (blk >= nblocks) return;
  // a single-pass tile sort: its digit counts are the list lengths (written
  // also when the pair list is empty)
  if (ro.ranges && blk == 0) ranges_from_counts(totals, ro, s_w);
  if (m_dev) m = eff_count(m_dev, cap);
  if (blk * kTile >= m) return;
  if (dk.info && blk == 0 && threadIdx.x == 0) dk.info[2] = (uint32_t)dk.out_index;
  constexpr int DPT = R > kThreads ? R / kThreads : 1;  // digits per thread in the digit phases
  // s_keys also holds, while ranking, each wave's R 64-bit lane masks
  __shared__ __align__(16) uint32_t s_keys[kTile];
  __shared__ uint32_t s_vals[kTile];
  __shared__ uint32_t s_wh[kWaves][R];  // per-wave digit counts, then per-wave bases
  __shared__ uint32_t s_gbase[R];
  __shared__ uint32_t s_count;

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const uint32_t kbase = depth_base(dk);
  const int64_t base = blk * kTile;
  const int64_t seg = base + wave * kSeg;
  for (int k = t; k < kWaves * R; k += kThreads) (&s_wh[0][0])[k] = 0;

  uint32_t key[kRounds], val[kRounds], rank[kRounds], pay[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t e = seg + r * 64 + lane;
    const bool valid = e < m;
    key[r] = valid ? keys_in[e] : 0u;
    val[r] = valid ? (vals_in ? vals_in[e] : (uint32_t)e) : 0u;
  }
  // the payload is loaded with the keys and values, so its latency overlaps
  // the ranking (the first pass builds it from the projection's rectangles)
  if (pl.to) {
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const int64_t e = seg + r * 64 + lane;
      pay[r] = 0u;
      if (e < m && key_kept(dk, key[r])) {
        if (pl.from) {
          pay[r] = pl.from[e];
        } else {
          const int v = view_of(pl.vt, val[r]);
          pay[r] = pack_rect(clip_rect(pl.rect[e], pl.vt.tiles_x[v], pl.vt.tiles_y[v]));
        }
      }
    }
  }
  // global digit starts (exclusive scan of the totals) + this block's prefix
  {
    uint32_t tv[DPT], sum = 0;
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
      const int d = t * DPT + k;
      tv[k] = d < R ? totals[d] : 0u;
      sum += tv[k];
    }
    uint32_t excl;
    block_exclusive_scan<uint32_t>(sum, &excl, s_w);
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
      const int d = t * DPT + k;
      if (d < R) s_gbase[d] = excl + hist[(int64_t)d * nblocks + blk];
      excl += tv[k];
    }
  }
  __syncthreads();

  // 1. rank within the wave's segment (dropped keys take no rank).  With
  // 9-bit digits the lanes holding digit d are found by each OR-ing its bit
  // into the wave's mask word for d in LDS, reading the word back and
  // clearing it: a wave's LDS operations take effect in issue order, so
  // every lane reads the mask of all lanes with its digit (three LDS
  // operations instead of nine ballots and their mask arithmetic).  The
  // words live in s_keys, which is not used until step 3.  Narrower digits
  // use the ballot match (fewer ballots, and more lanes share a word).
  constexpr bool kMaskWords = BITS >= 9 && (int64_t)kWaves * R * 8 <= (int64_t)kTile * 4;
  uint64_t* const words = reinterpret_cast<uint64_t*>(s_keys) + (kMaskWords ? wave * R : 0);
  if (kMaskWords)
    for (int k = lane; k < R; k += 64) words[k] = 0ull;
  const uint64_t lt = lanes_below(lane);
  bool kept[kRounds];
  uint32_t dig[kRounds];  // each element's digit, kept for steps 3 and 5
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const bool valid = seg + r * 64 + lane < m && key_kept(dk, key[r]);
    kept[r] = valid;
    const uint32_t d = ((key[r] - kbase) >> shift) & (R - 1);
    dig[r] = d;
    uint64_t same;
    if constexpr (kMaskWords) {
      if (valid) atomicOr(&words[d], 1ull << lane);
      same = valid ? words[d] : 0ull;
      if (valid) words[d] = 0ull;
    } else {
      same = match_digit<BITS>(d, valid);
    }
    const uint32_t below = (uint32_t)__popcll(same & lt);
    const uint32_t old = s_wh[wave][d];
    if (valid && below == 0) s_wh[wave][d] = old + (uint32_t)__popcll(same);
    rank[r] = old + below;
  }
  __syncthreads();

  // 2. per digit: wave bases inside the block, digit starts of the block
  {
    uint32_t c[DPT][kWaves], tot[DPT], sum = 0;
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
      const int d = t * DPT + k;
      tot[k] = 0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        c[k][w] = d < R ? s_wh[w][d] : 0u;
        tot[k] += c[k][w];
      }
      sum += tot[k];
    }
    uint32_t excl;
    const uint32_t kept_total = block_exclusive_scan<uint32_t>(sum, &excl, s_w);
    if (t == 0) s_count = kept_total;
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
      const int d = t * DPT + k;
      if (d < R) {
        s_gbase[d] -= excl;  // global start minus block-local start: dst = s_gbase[d] + i
        uint32_t run = excl;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
          s_wh[w][d] = run;
          run += c[k][w];
        }
      }
      excl += tot[k];
    }
  }
  __syncthreads();

  // 3. reorder the block in LDS by digit (rank becomes the block position).
  // A pass that writes no keys stores each element's output index in the
  // key slot instead, so steps 4 and 5 need no digit lookup.
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    if (kept[r]) {
      const uint32_t pos = s_wh[wave][dig[r]] + rank[r];
      rank[r] = pos;
      s_keys[pos] = keys_out ? key[r] : s_gbase[dig[r]] + pos;
      s_vals[pos] = val[r];
    }
  }
  __syncthreads();

  // 4. digit runs are contiguous: consecutive threads write consecutive addresses
  const int count = (int)s_count;
  for (int i = t; i < count; i += kThreads) {
    const uint32_t k = s_keys[i];
    if (keys_out) {
      const uint32_t dst = s_gbase[((k - kbase) >> shift) & (R - 1)] + (uint32_t)i;
      keys_out[dst] = k;
      vals_out[dst] = s_vals[i];
    } else {  // values only (no later pass reads the keys)
      vals_out[k] = s_vals[i];
    }
  }

  // 5. the payload, through the value slots of LDS: same positions, same runs
  if (pl.to) {
    __syncthreads();  // step 4 has read s_vals
#pragma unroll
    for (int r = 0; r < kRounds; ++r)
      if (kept[r]) s_vals[rank[r]] = pay[r];
    __syncthreads();
    for (int i = t; i < count; i += kThreads) {
      const uint32_t k = s_keys[i];
      const uint32_t dst =
          keys_out ? s_gbase[((k - kbase) >> shift) & (R - 1)] + (uint32_t)i : k;
      pl.to[dst] = s_vals[i];
    }
  }
}

// A pass over m elements, or, with m_dev set, over the device-side count
// eff_count(m_dev, m) with m (the capacity) sizing the grid.
template <int BITS>
hipError_t radix_pass_bits(const uint32_t* kin, const uint32_t* vin, uint32_t* kout,
                           uint32_t* vout, int64_t m, const uint64_t* m_dev, int shift,
                           uint32_t* hist, uint32_t* totals, const DepthKeys& dk,
                           const Payload& pl, const RangesOut& ro, hipStream_t stream) {
  const int64_t nb = std::max<int64_t>(ceil_div(m, kTile), 1);
  radix_upsweep_kernel<BITS><<<(unsigned)nb, kThreads, 0, stream>>>(kin, m, m_dev, m, shift, hist,
                                                                     nb, dk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hist_scan_kernel<<<1u << BITS, kThreads, 0, stream>>>(hist, nb, totals, dk, shift);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t grid = dk.info ? xcd_grid(nb) : nb;  // depth passes: XCD-numbered blocks
  radix_downsweep_kernel<BITS><<<(unsigned)grid, kThreads, 0, stream>>>(
      kin, vin, kout, vout, m, m_dev, m, shift, hist, totals, nb, dk, pl, ro);
  return hipGetLastError();
}

// One stable pass over `bits` (1..kMaxAnyDigitBits) bits starting at `shift`.
hipError_t radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                      int64_t m, const uint64_t* m_dev, int shift, int bits, uint32_t* hist,
                      uint32_t* totals, const DepthKeys& dk, const Payload& pl,
                      const RangesOut& ro, hipStream_t stream) {
  switch (bits) {
#define GS_RADIX_CASE(B)                                                                  \
  case B:                                                                                 \
    if (B <= kMaxAnyDigitBits)                                                            \
      return radix_pass_bits<(B <= kMaxAnyDigitBits ? B : 1)>(kin, vin, kout, vout, m, m_dev, \
                                                           shift, hist, totals, dk, pl, ro, stream); \
    break;
    GS_RADIX_CASE(1)
    GS_RADIX_CASE(2)
    GS_RADIX_CASE(3)
    GS_RADIX_CASE(4)
    GS_RADIX_CASE(5)
    GS_RADIX_CASE(6)
    GS_RADIX_CASE(7)
    GS_RADIX_CASE(8)
    GS_RADIX_CASE(9)
    GS_RADIX_CASE(10)
    GS_RADIX_CASE(11)
#undef GS_RADIX_CASE
    default: break;
  }
  return hipErrorInvalidValue;
}

// Splits `bits` key bits into the fewest passes of at most max_bits,
// as evenly as possible; returns the pass count and fills widths[].
int radix_plan(int bits, int widths[8], int max_bits = kMaxDigitBits) {
  const int passes = (bits + max_bits - 1) / max_bits;
  for (int k = 0; k < passes; ++k) widths[k] = bits / passes + (k < bits % passes ? 1 : 0);
  return passes;
}

// Digit widths of the depth sort and how many passes to launch.  Without a
// far plane on every view: passes of 8, 9, 9 and 6 bits, the top one
// skipping itself on the device when the keys span fewer than 2^26 ulps
// (depths within a factor of 128).  With far planes the key range
// [near, far] is known on the host and only the passes it needs are
// launched: 8 + 9 + 9 bits when it spans at most 2^26 ulps above the first
// pass's base, else 9 + 9 + 9 when 2^27 (a depth ratio of 65536) suffice
// (on MI355X a 9-bit first pass over every splat costs about 5 us more than
// an 8-bit one, a skipped top pass about 6 us).  *covered: key bits above
// the base the launched passes sort, 32 when all four run.
int depth_plan(const ViewTiles& vt, int widths[8], int* covered) {
  static_assert(kMaxAnyDigitBits >= 9, "depth plan needs 9-bit digits");
  *covered = 32;
  if (vt.bounded && vt.key_hi > vt.key_lo) {
    const auto span_bits = [&](int first) {
      const uint32_t range = vt.key_hi - (vt.key_lo & ~((1u << first) - 1u));
      return 32 - __builtin_clz(range);
    };
    if (span_bits(8) <= 26) {
      widths[0] = 8;
      widths[1] = widths[2] = 9;
      *covered = 26;
      return 3;
    }
    if (span_bits(9) <= 27) {
      widths[0] = widths[1] = widths[2] = 9;
      *covered = 27;
      return 3;
    }
  }
  widths[0] = 8;
  widths[1] = widths[2] = 9;
  widths[3] = 6;
  return 4;
}

// ----------------------------------------------------------------------------
// binning kernels
// ----------------------------------------------------------------------------
#ifndef GSUP_EMIT_BLOCK
#define GSUP_EMIT_BLOCK 256
#endif
constexpr int kEmit = GSUP_EMIT_BLOCK;  // splats per count / emit block

#ifndef GSUP_COUNT_PER_THREAD
#define GSUP_COUNT_PER_THREAD 16
#endif
constexpr int kCountPer = GSUP_COUNT_PER_THREAD;  // splats per thread of the count kernel
constexpr int kCount = kEmit * kCountPer;     // splats per count block
constexpr int kSubs = kCount / kEmit;         // emit blocks per count block
static_assert(kCount % kEmit == 0 && kCountPer % 4 == 0, "count / emit blocking");
static_assert((kEmit & (kEmit - 1)) == 0, "the owner search halves kEmit");

// Tile count of depth-order position p (the depth sort left only the splats
// with a finite depth, kept[0] of them, in the order and packed-rectangle
// buffers its last pass wrote).
__device__ __forceinline__ uint32_t pair_count_at(int64_t p, uint32_t code,
                                                  const uint32_t* __restrict__ order,
                                                  const short4* __restrict__ rect,
                                                  const ViewTiles& vt) {
  const uint32_t e = code == kRectEscape ? order[p] : 0u;
  return rect_tiles(splat_rect(code, e, rect, vt));
}

// Pair counts in depth order, per block of kCount splats (thread t sums
// kCountPer consecutive ones): sub[16 b + k] = pairs of this block before its
// k-th run of kEmit splats (an emit block), blk[b] = the block's pairs.
__global__ __launch_bounds__(kEmit) void pair_count_kernel(int64_t n,
                                                           const uint32_t* __restrict__ order0,
                                                           const uint32_t* __restrict__ order1,
                                                           const uint32_t* __restrict__ prect0,
                                                           const uint32_t* __restrict__ prect1,
                                                           const uint32_t* __restrict__ dinfo,
                                                           const uint64_t* kept,
                                                           const short4* __restrict__ rect,
                                                           ViewTiles vt,
                                                           uint64_t* __restrict__ sub,
                                                           uint64_t* __restrict__ blk) {
  __shared__ uint64_t s_w[kEmit / 64];
  const int64_t nk = eff_count(kept, n);
  const bool second = dinfo[2] != 0u;
  const uint32_t* __restrict__ order = second ? order1 : order0;
  const uint32_t* __restrict__ prect = second ? prect1 : prect0;
  const int64_t p0 = (int64_t)blockIdx.x * kCount + (int64_t)threadIdx.x * kCountPer;
  uint64_t c = 0;
  if (p0 + kCountPer <= nk) {  // whole run: 16-byte loads (p0 is a multiple of 16)
    const uint4* q = reinterpret_cast<const uint4*>(prect + p0);
#pragma unroll
    for (int k = 0; k < kCountPer / 4; ++k) {
      const uint4 v = q[k];
      c += pair_count_at(p0 + 4 * k, v.x, order, rect, vt);
      c += pair_count_at(p0 + 4 * k + 1, v.y, order, rect, vt);
      c += pair_count_at(p0 + 4 * k + 2, v.z, order, rect, vt);
      c += pair_count_at(p0 + 4 * k + 3, v.w, order, rect, vt);
    }
  } else {
    for (int k = 0; k < kCountPer; ++k)
      if (p0 + k < nk) c += pair_count_at(p0 + k, prect[p0 + k], order, rect, vt);
  }
  uint64_t excl;
  const uint64_t tot = block_exclusive_scan<uint64_t, kEmit>(c, &excl, s_w);
  constexpr int kThreadsPerSub = kEmit / kSubs;
  if (threadIdx.x % kThreadsPerSub == 0)
    sub[(int64_t)blockIdx.x * kSubs + threadIdx.x / kThreadsPerSub] = excl;
  if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

// Pair emission, load-balanced: a block takes kEmit consecutive splats (depth
// order), whose pairs form one contiguous range; it finds where that range
// starts (and the total K) from the count kernel's sums itself, scans its
// splats' tile counts in LDS, then every thread writes one pair per step,
// finding its splat by binary search over those offsets, so the writes are
// coalesced whatever the splats' tile counts.  Tile keys are global: view
// v's tiles are numbered from tile_off[v].  Block 0 writes K to `total`;
// nothing is written when K exceeds `cap` (or the int32 index range).
__global__ __launch_bounds__(kEmit) void emit_kernel(int64_t n, const uint32_t* __restrict__ order0,
                                                     const uint32_t* __restrict__ order1,
                                                     const uint32_t* __restrict__ prect0,
                                                     const uint32_t* __restrict__ prect1,
                                                     const uint32_t* __restrict__ dinfo,
                                                     const uint64_t* kept,
                                                     const short4* __restrict__ rect,
                                                     const uint64_t* __restrict__ sub,
                                                     const uint64_t* __restrict__ blk,
                                                     int64_t nblk, ViewTiles vt,
                                                     uint64_t* __restrict__ total, int64_t cap,
                                                     int covered, uint32_t low_mask,
                                                     uint32_t* __restrict__ tkeys,
                                                     uint32_t* __restrict__ tvals) {
  __shared__ uint32_t s_off[kEmit + 1];
  __shared__ int4 s_rect[kEmit];
  __shared__ uint32_t s_gid[kEmit];
  __shared__ uint32_t s_w[kEmit / 64];
  __shared__ uint64_t s_a[kEmit / 64], s_p[kEmit / 64];
  const int t = threadIdx.x;
  const int64_t nk = eff_count(kept, n);
  const int64_t p0 = (int64_t)blockIdx.x * kEmit;
  if (p0 >= nk && blockIdx.x != 0) return;  // no splats here (block 0 still reports K)
  // K and this block's first pair: sums over the count blocks
  const int64_t cb = (int64_t)blockIdx.x / kSubs;
  uint64_t all = 0, pre = 0;
  for (int64_t b = t; b < nblk; b += kEmit) {
    const uint64_t v = blk[b];
    all += v;
    pre += b < cb ? v : 0;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    all += __shfl_xor(all, d, 64);
    pre += __shfl_xor(pre, d, 64);
  }
  if ((t & 63) == 0) {
    s_a[t >> 6] = all;
    s_p[t >> 6] = pre;
  }
  __syncthreads();
  all = 0;
  pre = 0;
#pragma unroll
  for (int w = 0; w < kEmit / 64; ++w) {
    all += s_a[w];
    pre += s_p[w];
  }
  // the depth passes launched sort `covered` bits above the base: a key
  // range wider than that (a depth outside [near_plane, far_plane]) has not
  // been ordered, so nothing is emitted and K reports the error
  if (covered < 32 && nk > 0 && (uint64_t)(dinfo[1] - (dinfo[0] & ~low_mask)) >> covered != 0)
    all = kDepthRangeError;
  if (blockIdx.x == 0 && t == 0) *total = all;
  if (all > (uint64_t)cap || all >= (uint64_t(1) << 31)) return;  // uniform over the block
  const uint64_t base = pre + sub[blockIdx.x];
  const bool second = dinfo[2] != 0u;
  const uint32_t* __restrict__ order = second ? order1 : order0;
  const uint32_t* __restrict__ prect = second ? prect1 : prect0;
  const int64_t left = nk - p0;
  const int nb = left <= 0 ? 0 : (left < kEmit ? (int)left : kEmit);
  uint32_t c = 0;
  if (t < nb) {
    const uint32_t gid = order[p0 + t];
    const int4 r = splat_rect(prect[p0 + t], gid, rect, vt);
    s_rect[t] = r;
    s_gid[t] = gid;
    c = rect_tiles(r);
  }
  uint32_t excl;
  const uint32_t tot = block_exclusive_scan<uint32_t, kEmit>(c, &excl, s_w);
  s_off[t] = excl;
  if (t == 0) s_off[nb] = tot;
  __syncthreads();
  for (uint32_t k = t; k < tot; k += kEmit) {
    // owner: the last j with s_off[j] <= k (splats without tiles have
    // s_off[j] == s_off[j+1]); a fixed-step search over all kEmit entries:
    // those from nb on hold tot > k (their threads had no splat)
    int lo = 0;
#pragma unroll
    for (int step = kEmit / 2; step >= 1; step >>= 1)
      if (s_off[lo + step] <= k) lo += step;
    const int4 r = s_rect[lo];
    const uint32_t gid = s_gid[lo];
    const int v = view_of(vt, gid);
    const uint32_t li = k - s_off[lo];
    const uint32_t w = (uint32_t)(r.z - r.x);
    // row / column inside the rectangle: li < w h with h at most 4096 tiles
    // (32768-pixel images, 8-pixel tiles), so the quotient is below 4097 and
    // the hardware reciprocal's error is far inside the +-1 correction
    int dy = (int)(((float)li + 0.5f) * __builtin_amdgcn_rcpf((float)w));
    int dx = (int)li - dy * (int)w;
    if (dx < 0) {
      --dy;
      dx += (int)w;
    } else if (dx >= (int)w) {
      ++dy;
      dx -= (int)w;
    }
    tkeys[base + k] =
        vt.tile_off[v] + (uint32_t)(r.y + dy) * (uint32_t)vt.tiles_x[v] + (uint32_t)(r.x + dx);
    tvals[base + k] = gid;
  }
}

// Tile ranges from the tile-sorted keys: a block stages kTile keys plus one
// neighbour on each side in LDS and marks where the tile id changes.
__global__ __launch_bounds__(kThreads) void tile_range_kernel(int64_t K, const uint64_t* K_dev,
                                                              const uint32_t* __restrict__ tkeys,
                                                              int32_t* __restrict__ ranges) {
  __shared__ uint32_t s_k[kTile + 2];
  if (K_dev) K = eff_count(K_dev, K);
  const int64_t base = (int64_t)blockIdx.x * kTile;
  if (base >= K) return;
  for (int i = threadIdx.x; i < kTile + 2; i += kThreads) {
    const int64_t p = base + i - 1;
    s_k[i] = (p >= 0 && p < K) ? tkeys[p] : 0xFFFFFFFFu;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kTile; i += kThreads) {
    const int64_t p = base + i;
    if (p >= K) break;
    const uint32_t t = s_k[i + 1];
    if (p == 0 || s_k[i] != t) ranges[2 * (int64_t)t] = (int32_t)p;
    if (p == K - 1 || s_k[i + 2] != t) ranges[2 * (int64_t)t + 1] = (int32_t)(p + 1);
  }
}

inline unsigned grid1d(int64_t n, int threads) { return (unsigned)ceil_div(n, threads); }

}  // namespace

ViewTiles make_view_tiles(int32_t nv, const gs_camera* cams, int32_t tile_size, int64_t n) {
  ViewTiles vt{};
  vt.nv = nv;
  vt.n = n;
  uint32_t off = 0;
  for (int v = 0; v < nv; ++v) {
    vt.tiles_x[v] = (int32_t)ceil_div(cams[v].width, tile_size);
    vt.tiles_y[v] = (int32_t)ceil_div(cams[v].height, tile_size);
    vt.tile_off[v] = off;
    off += (uint32_t)vt.tiles_x[v] * (uint32_t)vt.tiles_y[v];
  }
  vt.tile_off[nv] = off;
  vt.bounded = true;
  vt.key_lo = 0xFFFFFFFFu;
  vt.key_hi = 0u;
  for (int v = 0; v < nv; ++v) {
    uint32_t lo, hi;
    std::memcpy(&lo, &cams[v].near_plane, 4);
    std::memcpy(&hi, &cams[v].far_plane, 4);
    vt.key_lo = std::min(vt.key_lo, lo);
    vt.key_hi = std::max(vt.key_hi, hi);
    vt.bounded = vt.bounded && cams[v].far_plane > 0.f;
  }
  return vt;
}

BinSortPlan make_bin_sort_plan(int64_t n, int64_t capacity, int64_t tiles) {
  BinSortPlan p;
  p.n = n;
  p.capacity = capacity;
  p.tiles = tiles;
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
  const int64_t n1 = std::max<int64_t>(n, 1);
  const size_t n4 = sizeof(uint32_t) * (size_t)n1;
  const size_t c4 = sizeof(uint32_t) * (size_t)std::max<int64_t>(capacity, 1);
  p.off_gkey[0] = take(n4);
  p.off_gkey[1] = take(n4);
  p.off_gval[0] = take(n4);
  p.off_gval[1] = take(n4);
  p.off_bsum = take(sizeof(uint64_t) * (size_t)ceil_div(n1, kCount) * kSubs);
  p.off_bblk = take(sizeof(uint64_t) * (size_t)ceil_div(n1, kCount));
  p.off_prect[0] = take(n4);
  p.off_prect[1] = take(n4);
  p.off_pkey[0] = take(c4);
  p.off_pkey[1] = take(c4);
  p.off_pval = take(c4);
  const int64_t max_blocks = std::max<int64_t>(ceil_div(n1, kTile),
                                               ceil_div(std::max<int64_t>(capacity, 1), kTile));
  p.off_hist = take(sizeof(uint32_t) * (size_t)((int64_t(1) << kMaxAnyDigitBits) * max_blocks));
  p.off_totals = take(sizeof(uint32_t) * (size_t)(1 << kMaxAnyDigitBits));
  p.off_total = take(sizeof(uint64_t));
  p.off_dinfo = take(4 * sizeof(uint32_t) + sizeof(uint64_t));
  p.off_bstat = take(4 * sizeof(uint32_t) * (size_t)ceil_div(n1, kTile));
  p.bytes = off;
  return p;
}

gs_status run_bin_sort(const BinSortPlan& p, const ViewTiles& vt, const float* depth,
                       const int16_t* rect, int32_t* sorted_ids, int32_t* tile_ranges,
                       int64_t* n_pairs, int64_t* n_pairs_dev, void* workspace,
                       hipStream_t stream) {
  char* ws = static_cast<char*>(workspace);
  auto u32 = [&](size_t o) { return reinterpret_cast<uint32_t*>(ws + o); };
  uint64_t* bsum = reinterpret_cast<uint64_t*>(ws + p.off_bsum);
  uint64_t* bblk = reinterpret_cast<uint64_t*>(ws + p.off_bblk);
  uint32_t* hist = u32(p.off_hist);
  uint32_t* totals = u32(p.off_totals);
  // device-count mode: the total goes straight to the caller's counter
  const bool dev = n_pairs_dev != nullptr;
  uint64_t* total = dev ? reinterpret_cast<uint64_t*>(n_pairs_dev)
                        : reinterpret_cast<uint64_t*>(ws + p.off_total);
  const short4* r4 = reinterpret_cast<const short4*>(rect);
  const int64_t n = p.n;
  hipError_t e;
#define GS_TRY(expr, what)                         \
  do {                                             \
    e = (expr);                                    \
    if (e != hipSuccess) return check_hip(e, what); \
  } while (0)

  if (n == 0) {
    if (n_pairs) *n_pairs = 0;
    if (dev) fill_i32_kernel<<<1, 64, 0, stream>>>(reinterpret_cast<int32_t*>(total), 2, 0);
    fill_i32_kernel<<<grid1d(2 * p.tiles, 256), 256, 0, stream>>>(tile_ranges, 2 * p.tiles, 0);
    return check_hip(hipGetLastError(), "fill_i32_kernel");
  }
  // 1. depth order of the splats with tiles: stable LSD radix sort of the
  //    FP32 depth bits (positive floats order like their bits; +inf marks
  //    splats without tiles, which the first pass drops); the first pass
  //    reads the depths in place and numbers them, the later ones sort
  //    depth - base and skip themselves where the depth range is narrower
  //    than their digit (DepthKeys).  Several views sort together: a tile
  //    only ever holds splats of one view, so the global order restricted to
  //    a tile is that view's order.
  uint32_t* dinfo = u32(p.off_dinfo);
  uint64_t* kept = reinterpret_cast<uint64_t*>(ws + p.off_dinfo + 16);
  const uint64_t* kept_count = kept;
  int widths[8];
  int covered = 32;
  const int passes_depth = depth_plan(vt, widths, &covered);
  const uint32_t low_mask = (1u << widths[0]) - 1u;
  int cur = 0, shift = 0;
  for (int k = 0; k < passes_depth; ++k) {
    const uint32_t* kin = k == 0 ? reinterpret_cast<const uint32_t*>(depth) : u32(p.off_gkey[cur]);
    const uint32_t* vin = k == 0 ? nullptr : u32(p.off_gval[cur]);
    DepthKeys dk;
    dk.info = dinfo;
    dk.kept = kept;
    dk.bstat = u32(p.off_bstat);
    dk.low_mask = low_mask;
    dk.first = k == 0;
    dk.out_index = cur ^ 1;
    // the packed rectangles travel in the same ping-pong order as the ids
    Payload pl;
    pl.from = k == 0 ? nullptr : u32(p.off_prect[cur]);
    pl.rect = r4;
    pl.vt = vt;
    pl.to = u32(p.off_prect[cur ^ 1]);
    // the keys of the last pass are not read again when no pass can follow it
    uint32_t* kout = (k + 1 == passes_depth && covered < 32) ? nullptr : u32(p.off_gkey[cur ^ 1]);
    GS_TRY(radix_pass(kin, vin, kout, u32(p.off_gval[cur ^ 1]), n,
                      k == 0 ? nullptr : kept_count, shift, widths[k], hist, totals, dk, pl,
                      RangesOut{}, stream),
           "depth radix pass");
    shift += widths[k];
    cur ^= 1;
  }
  const uint32_t* order0 = u32(p.off_gval[0]);
  const uint32_t* order1 = u32(p.off_gval[1]);
  const uint32_t* prect0 = u32(p.off_prect[0]);
  const uint32_t* prect1 = u32(p.off_prect[1]);

  // 2. tile counts in depth order per block of splats; 3. pairs in depth
  //    order, each emit block finding its offset and the total K from those
  //    sums (K goes to the caller's counter in device-count mode); nothing is
  //    emitted when K exceeds the capacity
  const int64_t nbc = ceil_div(n, kCount);
  const int64_t nbe = nbc * kSubs;
  pair_count_kernel<<<(unsigned)nbc, kEmit, 0, stream>>>(n, order0, order1, prect0, prect1, dinfo,
                                                          kept_count, r4, vt, bsum, bblk);
  GS_TRY(hipGetLastError(), "pair_count_kernel");
  const int passes = radix_plan(p.tile_bits, widths, kMaxTileDigitBits);
  // values end in sorted_ids after `passes` ping-pong steps
  uint32_t* vbuf[2];
  vbuf[0] = (passes % 2 == 0) ? reinterpret_cast<uint32_t*>(sorted_ids) : u32(p.off_pval);
  vbuf[1] = (passes % 2 == 0) ? u32(p.off_pval) : reinterpret_cast<uint32_t*>(sorted_ids);
  uint32_t* kbuf[2] = {u32(p.off_pkey[0]), u32(p.off_pkey[1])};
  emit_kernel<<<(unsigned)nbe, kEmit, 0, stream>>>(n, order0, order1, prect0, prect1, dinfo,
                                                   kept_count, r4, bsum, bblk, nbc, vt, total,
                                                   p.capacity, covered, low_mask, kbuf[0], vbuf[0]);
  GS_TRY(hipGetLastError(), "emit_kernel");
  int64_t m = p.capacity;  // device-count mode: grids sized by the capacity
  if (!dev) {
    uint64_t K = 0;
    GS_TRY(hipMemcpyAsync(&K, total, sizeof(K), hipMemcpyDeviceToHost, stream), "pair count copy");
    GS_TRY(hipStreamSynchronize(stream), "pair count sync");
    if (K == kDepthRangeError)
      return fail(GS_ERR_INVALID_ARGUMENT,
                  "gs_bin_sort: a finite depth lies outside the cameras' [near_plane, far_plane]");
    *n_pairs = (int64_t)K;
    if (K >= (uint64_t(1) << 31))
      return fail(GS_ERR_CAPACITY, "gs_bin_sort: %llu pairs exceed the 2^31 index limit",
                  (unsigned long long)K);
    if ((int64_t)K > p.capacity)
      return fail(GS_ERR_CAPACITY, "gs_bin_sort: %llu pairs exceed capacity %lld",
                  (unsigned long long)K, (long long)p.capacity);
    m = (int64_t)K;
  }
  const uint64_t* m_dev = dev ? total : nullptr;
  // the ranges start empty unless a single tile pass writes every tile's
  // range from its digit counts anyway
  if (m == 0 || passes > 1) {
    fill_i32_kernel<<<grid1d(2 * p.tiles, 256), 256, 0, stream>>>(tile_ranges, 2 * p.tiles, 0);
    GS_TRY(hipGetLastError(), "fill_i32_kernel");
  }
  if (m == 0) return GS_OK;

  // 4. stable sort of the pairs by tile id
  cur = 0;
  shift = 0;
  for (int k = 0; k < passes; ++k) {
    // the keys of the last pass are only needed by tile_range_kernel
    uint32_t* kout = (k + 1 == passes && passes == 1) ? nullptr : kbuf[cur ^ 1];
    // one pass: the digit of every pair is its whole tile id, so the pass's
    // digit counts are the list lengths and their running sum the starts
    RangesOut ro;
    if (passes == 1) {
      ro.ranges = tile_ranges;
      ro.tiles = p.tiles;
    }
    GS_TRY(radix_pass(kbuf[cur], vbuf[cur], kout, vbuf[cur ^ 1], m, m_dev, shift,
                      widths[k], hist, totals, DepthKeys{}, Payload{}, ro, stream),
           "tile radix pass");
    shift += widths[k];
    cur ^= 1;
  }
  if (passes > 1) {
    tile_range_kernel<<<(unsigned)ceil_div(m, kTile), kThreads, 0, stream>>>(m, m_dev, kbuf[cur],
                                                                             tile_ranges);
    GS_TRY(hipGetLastError(), "tile_range_kernel");
  }
#undef GS_TRY
  return GS_OK;
}

}  // namespace gsup
