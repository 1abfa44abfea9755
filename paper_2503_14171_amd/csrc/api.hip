// C ABI entry points of libgsup: host-side validation, error reporting and
// kernel launches.  See include/gsup.h for the contract of every call.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "gsup_internal.h"

namespace gsup {

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
  return GS_OK;
}

gs_status check_cfg(const char* fn, const gs_raster_cfg* cfg) {
  if (!cfg) return fail(GS_ERR_INVALID_ARGUMENT, "%s: cfg is NULL", fn);
  if (cfg->tile_size != 8 && cfg->tile_size != 16 && cfg->tile_size != 32)
    return fail(GS_ERR_UNSUPPORTED, "%s: tile_size %d (supported: 8, 16, 32)", fn, cfg->tile_size);
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

extern "C" {

int64_t gs_num_tiles(int32_t width, int32_t height, int32_t tile_size) {
  if (width < 1 || height < 1 || tile_size < 1) return 0;
  return ceil_div(width, tile_size) * ceil_div(height, tile_size);
}

const char* gs_last_error_message(void) { return g_msg; }

const char* gs_version(void) { return "gsup 0.1 (gfx950)"; }

gs_status gs_project(int64_t n, const float* means, const float* log_scales, const float* quats,
                     const float* opacity, const float* sh, const gs_camera* cam,
                     const gs_raster_cfg* cfg, gs_splat* splats, float* depth, int32_t* rect,
                     void* stream) {
  g_msg[0] = 0;
  const char* fn = "gs_project";
  GS_CHECK(check_camera(fn, cam));
  GS_CHECK(check_cfg(fn, cfg));
  if (n < 0 || n >= (int64_t(1) << 31))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: n = %lld outside [0, 2^31)", fn, (long long)n);
  if (n == 0) return GS_OK;
  if (!means || !log_scales || !quats || !opacity || !sh || !splats || !depth || !rect)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: NULL array argument", fn);
  if (!aligned(quats, 16) || !aligned(sh, 16) || !aligned(splats, 16) || !aligned(rect, 16) ||
      !aligned(means, 4) || !aligned(log_scales, 4) || !aligned(opacity, 4) || !aligned(depth, 4))
    return fail(GS_ERR_INVALID_ARGUMENT,
                "%s: quats, sh, splats and rect must be 16-byte aligned (others 4-byte)", fn);
  return check_hip(launch_project(n, means, log_scales, quats, opacity, sh, *cam, *cfg, splats,
                                  depth, rect, static_cast<hipStream_t>(stream)),
                   "gs_project launch");
}

size_t gs_bin_sort_workspace_size(int64_t n, int64_t capacity, const gs_camera* cam,
                                  const gs_raster_cfg* cfg) {
  if (!cam || !cfg || n < 0 || capacity < 0 || cam->width < 1 || cam->height < 1 ||
      (cfg->tile_size != 8 && cfg->tile_size != 16 && cfg->tile_size != 32))
    return 0;
  return make_bin_sort_plan(n, capacity, cam->width, cam->height, cfg->tile_size).bytes;
}

gs_status gs_bin_sort(int64_t n, const float* depth, const int32_t* rect, const gs_camera* cam,
                      const gs_raster_cfg* cfg, int64_t capacity, int32_t* sorted_ids,
                      int32_t* tile_ranges, int64_t* n_pairs, void* workspace,
                      size_t workspace_bytes, void* stream) {
  g_msg[0] = 0;
  const char* fn = "gs_bin_sort";
  GS_CHECK(check_camera(fn, cam));
  GS_CHECK(check_cfg(fn, cfg));
  if (n < 0 || n >= (int64_t(1) << 31))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: n = %lld outside [0, 2^31)", fn, (long long)n);
  if (capacity < 0 || capacity >= (int64_t(1) << 31))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: capacity %lld outside [0, 2^31)", fn,
                (long long)capacity);
  if (!n_pairs || !tile_ranges || !workspace || (n > 0 && (!depth || !rect)) ||
      (capacity > 0 && !sorted_ids))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: NULL argument", fn);
  if ((n > 0 && !aligned(rect, 16)) || !aligned(workspace, 256) || !aligned(tile_ranges, 8))
    return fail(GS_ERR_INVALID_ARGUMENT,
                "%s: rect must be 16-byte, tile_ranges 8-byte, workspace 256-byte aligned", fn);
  const BinSortPlan plan = make_bin_sort_plan(n, capacity, cam->width, cam->height, cfg->tile_size);
  if (workspace_bytes < plan.bytes)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: workspace of %zu bytes, %zu needed", fn,
                workspace_bytes, plan.bytes);
  return run_bin_sort(plan, depth, rect, sorted_ids, tile_ranges, n_pairs, workspace,
                      static_cast<hipStream_t>(stream));
}

gs_status gs_raster_grad(const gs_splat* splats, const int32_t* sorted_ids,
                         const int32_t* tile_ranges, const gs_camera* cam,
                         const gs_raster_cfg* cfg, int32_t want_grads, float* out,
                         int32_t* n_blend, void* stream) {
  g_msg[0] = 0;
  const char* fn = "gs_raster_grad";
  GS_CHECK(check_camera(fn, cam));
  GS_CHECK(check_cfg(fn, cfg));
  if (!splats || !sorted_ids || !tile_ranges || !out)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: NULL argument", fn);
  if (!aligned(splats, 16) || !aligned(tile_ranges, 8) || !aligned(out, want_grads ? 16 : 4) ||
      !aligned(sorted_ids, 4) || (n_blend && !aligned(n_blend, 4)))
    return fail(GS_ERR_INVALID_ARGUMENT,
                "%s: splats (and out with gradients) must be 16-byte aligned", fn);
  return check_hip(launch_raster(splats, sorted_ids, tile_ranges, *cam, *cfg, want_grads != 0, out,
                                 n_blend, static_cast<hipStream_t>(stream)),
                   "gs_raster_grad launch");
}

gs_status gs_upscale_hermite(const float* in, int32_t w, int32_t h, float* out, int32_t W,
                             int32_t H, void* stream) {
  g_msg[0] = 0;
  const char* fn = "gs_upscale_hermite";
  if (!in || !out) return fail(GS_ERR_INVALID_ARGUMENT, "%s: NULL argument", fn);
  if (w < 2 || h < 2 || w > kMaxSide || h > kMaxSide)
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: low-res %d x %d outside [2, %d]", fn, w, h, kMaxSide);
  if (W < w || H < h || W > 4 * kMaxSide || H > 4 * kMaxSide)
    return fail(GS_ERR_INVALID_ARGUMENT,
                "%s: high-res %d x %d must be >= low-res %d x %d and <= %d", fn, W, H, w, h,
                4 * kMaxSide);
  if (!aligned(in, 16) || !aligned(out, 4))
    return fail(GS_ERR_INVALID_ARGUMENT, "%s: in must be 16-byte aligned", fn);
  const char* ib = reinterpret_cast<const char*>(in);
  const char* ie = ib + (size_t)w * h * 12 * sizeof(float);
  const char* ob = reinterpret_cast<const char*>(out);
  const char* oe = ob + (size_t)W * H * 3 * sizeof(float);
  if (ib < oe && ob < ie) return fail(GS_ERR_INVALID_ARGUMENT, "%s: in and out overlap", fn);
  return check_hip(launch_upscale(in, w, h, out, W, H, static_cast<hipStream_t>(stream)),
                   "gs_upscale_hermite launch");
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

}  // extern "C"
