// C ABI entry points of libgsup: host-side validation, error reporting and
// kernel launches.  See include/gsup.h for the contract of every call.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "gsup_internal.h"

namespace gsup {

#define GS_CHECK_INNER(x)        \
  do {                           \
    const gs_status s_ = (x);    \
    if (s_ != GS_OK) return s_;  \
  } while (0)

namespace {
thread_local char g_msg[1024] = "";

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

bool finite(float v) { return std::isfinite(v); }

constexpr int32_t kMaxSide = 32768;

gs_status check_camera(const char* fn, const gs_camera* cam) {
  if (!cam) return fail(GS_ERR_INVALID_ARGUMENT, "%s: cam is NULL", fn);
  if (cam->width < 1 || cam->height < 1 || cam->width > kMaxSide || cam->height > kMaxSide)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: raster %d x %d outside [1, %d]", fn, cam->width,
                cam->height, kMaxSide);
  if (!(cam->fx > 0.f) || !(cam->fy > 0.f) || !finite(cam->fx) || !finite(cam->fy))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: focal lengths must be finite and > 0", fn);
  if (!finite(cam->cx) || !finite(cam->cy))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: principal point not finite", fn);
  for (int k = 0; k < 12; ++k)
    if (!finite(cam->view[k])) return fail(GS_ERR_INVALID_ARGUMENT, "%s: view not finite", fn);
  for (int k = 0; k < 3; ++k)
    if (!finite(cam->cam_pos[k]))
      return fail(GS_ERR_INVALID_ARGUMENT, "%s: cam_pos not finite", fn);
  if (!(cam->near_plane > 0.f) || !finite(cam->near_plane))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: near_plane must be finite and > 0", fn);
  if (!finite(cam->far_plane) || cam->far_plane < 0.f ||
      (cam->far_plane > 0.f && !(cam->far_plane > cam->near_plane)))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: far_plane must be 0 or finite and > near_plane", fn);
  return GS_OK;
}

gs_status check_cfg(const char* fn, const gs_raster_cfg* cfg) {
  if (!cfg) return fail(GS_ERR_INVALID_ARGUMENT, "%s: cfg is NULL", fn);
  if (cfg->tile_size != 8 && cfg->tile_size != 16 && cfg->tile_size != 32 && cfg->tile_size != 64)
    return fail(GS_ERR_UNSUPPORTED, "%s: tile_size %d (supported: 8, 16, 32, 64)", fn,
                cfg->tile_size);
  if (cfg->sh_degree < 0 || cfg->sh_degree > 3)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: sh_degree %d outside [0, 3]", fn, cfg->sh_degree);
  if (!(cfg->dilation >= 0.f) || !finite(cfg->dilation))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: dilation must be finite and >= 0", fn);
  if (!(cfg->alpha_min > 0.f) || !(cfg->alpha_min < cfg->alpha_max) || !(cfg->alpha_max < 1.f))
    return fail(GS_ERR_INVALID_ARGUMENT,
                "%s: need 0 < alpha_min < alpha_max < 1 (got %g, %g)", fn, cfg->alpha_min,
                cfg->alpha_max);
  if (!(cfg->t_min > 0.f) || !(cfg->t_min < 1.f))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: need 0 < t_min < 1 (got %g)", fn, cfg->t_min);
  for (int k = 0; k < 3; ++k)
    if (!finite(cfg->bg[k])) return fail(GS_ERR_INVALID_ARGUMENT, "%s: bg not finite", fn);
  const int32_t nt = cfg->tile_size * cfg->tile_size;
  if (cfg->batch != 0 && cfg->batch != nt && cfg->batch != nt / 2 && cfg->batch != nt / 4)
    return fail(GS_ERR_UNSUPPORTED, "%s: batch %d (supported: 0, %d, %d, %d)", fn, cfg->batch, nt,
                nt / 2, nt / 4);
  return GS_OK;
}

gs_status check_views(const char* fn, int32_t nv, const gs_camera* cams) {
  if (nv < 1 || nv > GS_MAX_VIEWS)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: n_views %d outside [1, %d]", fn, nv, GS_MAX_VIEWS);
  if (!cams) return fail(GS_ERR_INVALID_ARGUMENT, "%s: cams is NULL", fn);
  for (int v = 0; v < nv; ++v) GS_CHECK_INNER(check_camera(fn, cams + v));
  return GS_OK;
}

int64_t total_tiles(int32_t nv, const gs_camera* cams, int32_t tile) {
  int64_t t = 0;
  for (int v = 0; v < nv; ++v) t += ceil_div(cams[v].width, tile) * ceil_div(cams[v].height, tile);
  return t;
}

// Bin/sort scratch of gs_bin_sort_async_static: a device array that every
// GPU the library runs on holds from the code object's load to the end of
// the process.  Host code never uses the array's name as an address (on the
// host it is only a stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
__device__ __align__(256) unsigned char scratch[GS_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

gs_status static_scratch(const char* fn, void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return check_hip(e, fn);
  if (dev < 0 || dev >= kMaxDevices)
    return fail(GS_ERR_UNSUPPORTED, "%s: device %d beyond the %d the library tracks", fn, dev,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return check_hip(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(GS_ERR_HIP, "%s: no device address for the static scratch", fn);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GS_OK;
}

}  // namespace

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
  va_end(ap);
}

gs_status fail(gs_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
  va_end(ap);
  return code;
}

gs_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return GS_OK;
  return fail(GS_ERR_HIP, "%s: HIP error %d (%s)", what, (int)e, hipGetErrorString(e));
}

}  // namespace gsup

using namespace gsup;

#define GS_CHECK(x)              \
  do {                           \
    const gs_status s_ = (x);    \
    if (s_ != GS_OK) return s_;  \
  } while (0)

namespace {

gs_status project_impl(const char* fn, int64_t n, const float* means, const float* log_scales,
                       const float* quats, const float* opacity, const float* sh, int32_t nv,
                       const gs_camera* cams, const gs_raster_cfg* cfg, gs_splat* splats,
                       float* depth, int16_t* rect, void* stream) {
  GS_CHECK(check_views(fn, nv, cams));
  GS_CHECK(check_cfg(fn, cfg));
  if (n < 0 || n * nv >= (int64_t(1) << 31))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: n * n_views = %lld * %d outside [0, 2^31)", fn,
                (long long)n, nv);
  if (n == 0) return GS_OK;
  if (!means || !log_scales || !quats || !opacity || !sh || !splats || !depth || !rect)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: NULL array argument", fn);
  if (!aligned(quats, 16) || !aligned(sh, 16) || !aligned(splats, 16) || !aligned(rect, 8) ||
      !aligned(means, 4) || !aligned(log_scales, 4) || !aligned(opacity, 4) || !aligned(depth, 4))
    return fail(GS_ERR_INVALID_ARGUMENT,
                "%s: quats, sh and splats must be 16-byte aligned, rect 8-byte (others 4-byte)", fn);
  return check_hip(launch_project(n, means, log_scales, quats, opacity, sh, nv, cams, *cfg, splats,
                                  depth, rect, static_cast<hipStream_t>(stream)),
                   "projection launch");
}

size_t bin_sort_ws(int64_t n, int32_t nv, const gs_camera* cams, const gs_raster_cfg* cfg,
                   int64_t capacity) {
  if (!cams || !cfg || nv < 1 || nv > GS_MAX_VIEWS || n < 0 || capacity < 0 ||
      (cfg->tile_size != 8 && cfg->tile_size != 16 && cfg->tile_size != 32 &&
       cfg->tile_size != 64))
    return 0;
  for (int v = 0; v < nv; ++v)
    if (cams[v].width < 1 || cams[v].height < 1) return 0;
  return make_bin_sort_plan(n * nv, capacity, total_tiles(nv, cams, cfg->tile_size)).bytes;
}

gs_status bin_sort_impl(const char* fn, int64_t n, int32_t nv, const gs_camera* cams,
                        const gs_raster_cfg* cfg, const float* depth, const int16_t* rect,
                        int64_t capacity, int32_t* sorted_ids, int32_t* tile_ranges,
                        int64_t* n_pairs, int64_t* n_pairs_dev, void* workspace,
                        size_t workspace_bytes, void* stream) {
  GS_CHECK(check_views(fn, nv, cams));
  GS_CHECK(check_cfg(fn, cfg));
  if (n < 0 || n * nv >= (int64_t(1) << 31))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: n * n_views = %lld * %d outside [0, 2^31)", fn,
                (long long)n, nv);
  if (capacity < 0 || capacity >= (int64_t(1) << 31))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: capacity %lld outside [0, 2^31)", fn,
                (long long)capacity);
  if ((!n_pairs && !n_pairs_dev) || !tile_ranges || !workspace || (n > 0 && (!depth || !rect)) ||
      (capacity > 0 && !sorted_ids))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: NULL argument", fn);
  if ((n > 0 && !aligned(rect, 8)) || !aligned(workspace, 256) || !aligned(tile_ranges, 8) ||
      (n_pairs_dev && !aligned(n_pairs_dev, 8)))
    return fail(GS_ERR_INVALID_ARGUMENT,
                "%s: rect, tile_ranges and n_pairs must be 8-byte, workspace 256-byte "
                "aligned", fn);
  const int64_t tiles = total_tiles(nv, cams, cfg->tile_size);
  if (tiles >= (int64_t(1) << 31))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: %lld tiles exceed 2^31", fn, (long long)tiles);
  const BinSortPlan plan = make_bin_sort_plan(n * nv, capacity, tiles);
  if (workspace_bytes < plan.bytes)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: workspace of %zu bytes, %zu needed", fn,
                workspace_bytes, plan.bytes);
  const ViewTiles vt = make_view_tiles(nv, cams, cfg->tile_size, n);
  return run_bin_sort(plan, vt, depth, rect, sorted_ids, tile_ranges, n_pairs, n_pairs_dev,
                      workspace, static_cast<hipStream_t>(stream));
}

gs_status raster_impl(const char* fn, const gs_splat* splats, const int32_t* sorted_ids,
                      const int32_t* tile_ranges, int32_t nv, const gs_camera* cams,
                      const gs_raster_cfg* cfg, int32_t want_grads, float* out, int32_t* n_blend,
                      int32_t* n_eval, void* stream) {
  GS_CHECK(check_views(fn, nv, cams));
  GS_CHECK(check_cfg(fn, cfg));
  if (!splats || !sorted_ids || !tile_ranges || !out)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: NULL argument", fn);
  if (!aligned(splats, 16) || !aligned(tile_ranges, 8) || !aligned(out, want_grads ? 16 : 4) ||
      !aligned(sorted_ids, 4) || (n_blend && !aligned(n_blend, 4)) ||
      (n_eval && !aligned(n_eval, 4)))
    return fail(GS_ERR_INVALID_ARGUMENT,
                "%s: splats (and out with gradients) must be 16-byte aligned", fn);
  if (total_tiles(nv, cams, cfg->tile_size) >= (int64_t(1) << 31))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: too many tiles", fn);
  return check_hip(launch_raster(splats, sorted_ids, tile_ranges, nv, cams, *cfg, want_grads != 0,
                                 out, n_blend, n_eval, nullptr, nullptr,
                                 static_cast<hipStream_t>(stream)),
                   "raster launch");
}

gs_status upscale_impl(const char* fn, const float* in, int32_t nv, const int32_t* lo,
                       float* out, const int32_t* hi, int32_t band_rows, void* stream) {
  if (!in || !out || !lo || !hi) return fail(GS_ERR_INVALID_ARGUMENT, "%s: NULL argument", fn);
  if (nv < 1 || nv > GS_MAX_VIEWS)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: n_views %d outside [1, %d]", fn, nv, GS_MAX_VIEWS);
  if (band_rows != 0 && band_rows != 4 && band_rows != 8 && band_rows != 16 && band_rows != 32)
    return fail(GS_ERR_UNSUPPORTED, "%s: band_rows %d (supported: 0, 4, 8, 16, 32)", fn,
                band_rows);
  int64_t in_px = 0, out_px = 0;
  for (int v = 0; v < nv; ++v) {
    const int32_t w = lo[2 * v], h = lo[2 * v + 1], W = hi[2 * v], H = hi[2 * v + 1];
    if (w < 2 || h < 2 || w > kMaxSide || h > kMaxSide)
      return fail(GS_ERR_INVALID_ARGUMENT, "%s: low-res %d x %d outside [2, %d]", fn, w, h,
                  kMaxSide);
    if (W < w || H < h || W > 4 * kMaxSide || H > 4 * kMaxSide)
      return fail(GS_ERR_INVALID_ARGUMENT,
                  "%s: high-res %d x %d must be >= low-res %d x %d and <= %d", fn, W, H, w, h,
                  4 * kMaxSide);
    in_px += (int64_t)w * h;
    out_px += (int64_t)W * H;
  }
  if (!aligned(in, 16) || !aligned(out, 4))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: in must be 16-byte aligned", fn);
  const char* ib = reinterpret_cast<const char*>(in);
  const char* ie = ib + (size_t)in_px * 12 * sizeof(float);
  const char* ob = reinterpret_cast<const char*>(out);
  const char* oe = ob + (size_t)out_px * 3 * sizeof(float);
  if (ib < oe && ob < ie) return fail(GS_ERR_INVALID_ARGUMENT, "%s: in and out overlap", fn);
  return check_hip(launch_upscale(in, nv, lo, out, hi, band_rows, static_cast<hipStream_t>(stream)),
                   "upscale launch");
}

}  // namespace

extern "C" {

int64_t gs_num_tiles(int32_t width, int32_t height, int32_t tile_size) {
  if (width < 1 || height < 1 || tile_size < 1) return 0;
  return ceil_div(width, tile_size) * ceil_div(height, tile_size);
}

const char* gs_last_error_message(void) { return g_msg; }

const char* gs_version(void) { return "gsup 0.1 (gfx950)"; }


gs_status gs_project(int64_t n, const float* means, const float* log_scales, const float* quats,
                     const float* opacity, const float* sh, const gs_camera* cam,
                     const gs_raster_cfg* cfg, gs_splat* splats, float* depth, int16_t* rect,
                     void* stream) {
  g_msg[0] = 0;
  return project_impl("gs_project", n, means, log_scales, quats, opacity, sh, 1, cam, cfg, splats,
                      depth, rect, stream);
}

size_t gs_bin_sort_workspace_size(int64_t n, int64_t capacity, const gs_camera* cam,
                                  const gs_raster_cfg* cfg) {
  return bin_sort_ws(n, 1, cam, cfg, capacity);
}

gs_status gs_bin_sort(int64_t n, const float* depth, const int16_t* rect, const gs_camera* cam,
                      const gs_raster_cfg* cfg, int64_t capacity, int32_t* sorted_ids,
                      int32_t* tile_ranges, int64_t* n_pairs, void* workspace,
                      size_t workspace_bytes, void* stream) {
  g_msg[0] = 0;
  if (!n_pairs) return fail(GS_ERR_INVALID_ARGUMENT, "gs_bin_sort: n_pairs is NULL");
  return bin_sort_impl("gs_bin_sort", n, 1, cam, cfg, depth, rect, capacity, sorted_ids,
                       tile_ranges, n_pairs, nullptr, workspace, workspace_bytes, stream);
}

gs_status gs_bin_sort_async(int64_t n, const float* depth, const int16_t* rect,
                            const gs_camera* cam, const gs_raster_cfg* cfg, int64_t capacity,
                            int32_t* sorted_ids, int32_t* tile_ranges, int64_t* n_pairs_dev,
                            void* workspace, size_t workspace_bytes, void* stream) {
  g_msg[0] = 0;
  if (!n_pairs_dev) return fail(GS_ERR_INVALID_ARGUMENT, "gs_bin_sort_async: n_pairs_dev is NULL");
  return bin_sort_impl("gs_bin_sort_async", n, 1, cam, cfg, depth, rect, capacity, sorted_ids,
                       tile_ranges, nullptr, n_pairs_dev, workspace, workspace_bytes, stream);
}

gs_status gs_bin_sort_async_static(int64_t n, const float* depth, const int16_t* rect,
                                   const gs_camera* cam, const gs_raster_cfg* cfg,
                                   int64_t capacity, int32_t* sorted_ids, int32_t* tile_ranges,
                                   int64_t* n_pairs_dev, void* stream) {
  g_msg[0] = 0;
  const char* fn = "gs_bin_sort_async_static";
  if (!n_pairs_dev) return fail(GS_ERR_INVALID_ARGUMENT, "%s: n_pairs_dev is NULL", fn);
  // sizes first, on the host (0: the settings are invalid, which the common
  // validation below reports)
  const size_t need = bin_sort_ws(n, 1, cam, cfg, capacity);
  if (need > (size_t)GS_STATIC_SCRATCH_BYTES)
    return fail(GS_ERR_INVALID_ARGUMENT,
                "%s: %lld splats and capacity %lld need %zu bytes of scratch; the static scratch "
                "holds %zu (gs_bin_sort_async takes a workspace of any size)",
                fn, (long long)n, (long long)capacity, need, (size_t)GS_STATIC_SCRATCH_BYTES);
  void* ws = nullptr;
  if (need > 0) GS_CHECK(static_scratch(fn, &ws));
  return bin_sort_impl(fn, n, 1, cam, cfg, depth, rect, capacity, sorted_ids, tile_ranges,
                       nullptr, n_pairs_dev, ws, (size_t)GS_STATIC_SCRATCH_BYTES, stream);
}

gs_status gs_raster_grad(const gs_splat* splats, const int32_t* sorted_ids,
                         const int32_t* tile_ranges, const gs_camera* cam,
                         const gs_raster_cfg* cfg, int32_t want_grads, float* out,
                         int32_t* n_blend, void* stream) {
  g_msg[0] = 0;
  return raster_impl("gs_raster_grad", splats, sorted_ids, tile_ranges, 1, cam, cfg, want_grads,
                     out, n_blend, nullptr, stream);
}

gs_status gs_upscale_hermite(const float* in, int32_t w, int32_t h, float* out, int32_t W,
                             int32_t H, void* stream) {
  g_msg[0] = 0;
  const int32_t lo[2] = {w, h}, hi[2] = {W, H};
  return upscale_impl("gs_upscale_hermite", in, 1, lo, out, hi, 0, stream);
}

int64_t gs_num_tiles_views(int32_t n_views, const gs_camera* cams, int32_t tile_size) {
  if (n_views < 1 || n_views > GS_MAX_VIEWS || !cams || tile_size < 1) return 0;
  for (int v = 0; v < n_views; ++v)
    if (cams[v].width < 1 || cams[v].height < 1) return 0;
  return total_tiles(n_views, cams, tile_size);
}

gs_status gs_project_views(int64_t n, const float* means, const float* log_scales,
                           const float* quats, const float* opacity, const float* sh,
                           int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                           gs_splat* splats, float* depth, int16_t* rect, void* stream) {
  g_msg[0] = 0;
  return project_impl("gs_project_views", n, means, log_scales, quats, opacity, sh, n_views, cams,
                      cfg, splats, depth, rect, stream);
}

size_t gs_bin_sort_views_workspace_size(int64_t n, int32_t n_views, const gs_camera* cams,
                                        const gs_raster_cfg* cfg, int64_t capacity) {
  return bin_sort_ws(n, n_views, cams, cfg, capacity);
}

gs_status gs_bin_sort_views(int64_t n, int32_t n_views, const gs_camera* cams,
                            const gs_raster_cfg* cfg, const float* depth, const int16_t* rect,
                            int64_t capacity, int32_t* sorted_ids, int32_t* tile_ranges,
                            int64_t* n_pairs_dev, void* workspace, size_t workspace_bytes,
                            void* stream) {
  g_msg[0] = 0;
  if (!n_pairs_dev) return fail(GS_ERR_INVALID_ARGUMENT, "gs_bin_sort_views: n_pairs_dev is NULL");
  return bin_sort_impl("gs_bin_sort_views", n, n_views, cams, cfg, depth, rect, capacity,
                       sorted_ids, tile_ranges, nullptr, n_pairs_dev, workspace, workspace_bytes,
                       stream);
}

gs_status gs_raster_grad_views(const gs_splat* splats, const int32_t* sorted_ids,
                               const int32_t* tile_ranges, int32_t n_views,
                               const gs_camera* cams, const gs_raster_cfg* cfg,
                               int32_t want_grads, float* out, int32_t* n_blend, void* stream) {
  g_msg[0] = 0;
  return raster_impl("gs_raster_grad_views", splats, sorted_ids, tile_ranges, n_views, cams, cfg,
                     want_grads, out, n_blend, nullptr, stream);
}

gs_status gs_raster_fragment_counts(const gs_splat* splats, const int32_t* sorted_ids,
                                    const int32_t* tile_ranges, int32_t n_views,
                                    const gs_camera* cams, const gs_raster_cfg* cfg,
                                    int32_t want_grads, float* out, int32_t* n_eval,
                                    int32_t* n_blend, void* stream) {
  g_msg[0] = 0;
  if (!n_eval || !n_blend)
    return fail(GS_ERR_INVALID_ARGUMENT, "gs_raster_fragment_counts: NULL count buffer");
  return raster_impl("gs_raster_fragment_counts", splats, sorted_ids, tile_ranges, n_views, cams,
                     cfg, want_grads, out, n_blend, n_eval, stream);
}

gs_status gs_upscale_hermite_views(const float* in, int32_t n_views, const int32_t* lo_sizes,
                                   float* out, const int32_t* hi_sizes, int32_t band_rows,
                                   void* stream) {
  g_msg[0] = 0;
  return upscale_impl("gs_upscale_hermite_views", in, n_views, lo_sizes, out, hi_sizes, band_rows,
                      stream);
}

gs_status gs_fd_slopes(const float* img, int32_t w, int32_t h, float* out, void* stream) {
  g_msg[0] = 0;
  const char* fn = "gs_fd_slopes";
  if (!img || !out) return fail(GS_ERR_INVALID_ARGUMENT, "%s: NULL argument", fn);
  if (w < 2 || h < 2 || w > kMaxSide || h > kMaxSide)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: image %d x %d outside [2, %d]", fn, w, h, kMaxSide);
  if (!aligned(img, 4) || !aligned(out, 16))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: out must be 16-byte aligned", fn);
  const char* ib = reinterpret_cast<const char*>(img);
  const char* ie = ib + (size_t)w * h * 3 * sizeof(float);
  const char* ob = reinterpret_cast<const char*>(out);
  const char* oe = ob + (size_t)w * h * 12 * sizeof(float);
  if (ib < oe && ob < ie) return fail(GS_ERR_INVALID_ARGUMENT, "%s: img and out overlap", fn);
  return check_hip(launch_fd_slopes(img, w, h, out, static_cast<hipStream_t>(stream)),
                   "gs_fd_slopes launch");
}

// ---- backward ----------------------------------------------------------------

gs_status gs_raster_grad_views_train(const gs_splat* splats, const int32_t* sorted_ids,
                                     const int32_t* tile_ranges, int32_t n_views,
                                     const gs_camera* cams, const gs_raster_cfg* cfg, float* out,
                                     float* state, int32_t* last, void* stream) {
  g_msg[0] = 0;
  const char* fn = "gs_raster_grad_views_train";
  GS_CHECK(check_views(fn, n_views, cams));
  GS_CHECK(check_cfg(fn, cfg));
  if (!splats || !sorted_ids || !tile_ranges || !out || !state || !last)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: NULL argument", fn);
  if (!aligned(splats, 16) || !aligned(tile_ranges, 8) || !aligned(out, 16) ||
      !aligned(state, 16) || !aligned(last, 4) || !aligned(sorted_ids, 4))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: splats, out and state must be 16-byte aligned", fn);
  return check_hip(launch_raster(splats, sorted_ids, tile_ranges, n_views, cams, *cfg, true, out,
                                 nullptr, nullptr, state, last, static_cast<hipStream_t>(stream)),
                   "raster launch");
}

gs_status gs_upscale_hermite_backward_views(const float* d_out, int32_t n_views,
                                            const int32_t* lo_sizes, float* d_in,
                                            const int32_t* hi_sizes, void* stream) {
  g_msg[0] = 0;
  const char* fn = "gs_upscale_hermite_backward_views";
  if (!d_out || !d_in || !lo_sizes || !hi_sizes)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: NULL argument", fn);
  if (n_views < 1 || n_views > GS_MAX_VIEWS)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: n_views %d outside [1, %d]", fn, n_views,
                GS_MAX_VIEWS);
  int64_t in_px = 0, out_px = 0;
  for (int v = 0; v < n_views; ++v) {
    const int32_t w = lo_sizes[2 * v], h = lo_sizes[2 * v + 1];
    const int32_t W = hi_sizes[2 * v], H = hi_sizes[2 * v + 1];
    if (w < 2 || h < 2 || w > kMaxSide || h > kMaxSide || W < w || H < h || W > 4 * kMaxSide ||
        H > 4 * kMaxSide)
      return fail(GS_ERR_INVALID_ARGUMENT, "%s: view %d sizes %d x %d -> %d x %d invalid", fn, v,
                  w, h, W, H);
    in_px += (int64_t)w * h;
    out_px += (int64_t)W * H;
  }
  if (!aligned(d_in, 16) || !aligned(d_out, 4))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: d_in must be 16-byte aligned", fn);
  const char* ib = reinterpret_cast<const char*>(d_in);
  const char* ie = ib + (size_t)in_px * 12 * sizeof(float);
  const char* ob = reinterpret_cast<const char*>(d_out);
  const char* oe = ob + (size_t)out_px * 3 * sizeof(float);
  if (ib < oe && ob < ie) return fail(GS_ERR_INVALID_ARGUMENT, "%s: d_in and d_out overlap", fn);
  return check_hip(launch_upscale_backward(d_out, n_views, lo_sizes, d_in, hi_sizes,
                                           static_cast<hipStream_t>(stream)),
                   "upscale backward launch");
}

gs_status gs_raster_grad_backward_views(const gs_splat* splats, const int32_t* sorted_ids,
                                        const int32_t* tile_ranges, int32_t n_views,
                                        const gs_camera* cams, const gs_raster_cfg* cfg,
                                        const float* state, const int32_t* last,
                                        const float* d_lowres, int64_t n, float* d_splats,
                                        void* stream) {
  g_msg[0] = 0;
  const char* fn = "gs_raster_grad_backward_views";
  GS_CHECK(check_views(fn, n_views, cams));
  GS_CHECK(check_cfg(fn, cfg));
  if (n < 0 || n * n_views >= (int64_t(1) << 31))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: n * n_views outside [0, 2^31)", fn);
  if (!splats || !sorted_ids || !tile_ranges || !state || !last || !d_lowres || !d_splats)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: NULL argument", fn);
  if (!aligned(splats, 16) || !aligned(tile_ranges, 8) || !aligned(state, 16) ||
      !aligned(d_lowres, 16) || !aligned(d_splats, 4) || !aligned(last, 4))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: splats, state and d_lowres must be 16-byte aligned",
                fn);
  return check_hip(launch_raster_backward(splats, sorted_ids, tile_ranges, n_views, cams, *cfg,
                                          state, last, d_lowres, n * n_views, d_splats,
                                          static_cast<hipStream_t>(stream)),
                   "raster backward launch");
}

gs_status gs_project_backward_views(int64_t n, const float* means, const float* log_scales,
                                    const float* quats, const float* opacity, const float* sh,
                                    int32_t n_views, const gs_camera* cams,
                                    const gs_raster_cfg* cfg, const float* d_splats,
                                    float* d_means, float* d_log_scales, float* d_quats,
                                    float* d_opacity, float* d_sh, void* stream) {
  g_msg[0] = 0;
  const char* fn = "gs_project_backward_views";
  GS_CHECK(check_views(fn, n_views, cams));
  GS_CHECK(check_cfg(fn, cfg));
  if (n < 0 || n * n_views >= (int64_t(1) << 31))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: n * n_views outside [0, 2^31)", fn);
  if (n == 0) return GS_OK;
  if (!means || !log_scales || !quats || !opacity || !sh || !d_splats || !d_means ||
      !d_log_scales || !d_quats || !d_opacity || !d_sh)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: NULL argument", fn);
  if (!aligned(quats, 16) || !aligned(d_quats, 16))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: quats and d_quats must be 16-byte aligned", fn);
  return check_hip(launch_project_backward(n, means, log_scales, quats, opacity, sh, n_views, cams,
                                           *cfg, d_splats, d_means, d_log_scales, d_quats,
                                           d_opacity, d_sh, static_cast<hipStream_t>(stream)),
                   "projection backward launch");
}

}  // extern "C"
