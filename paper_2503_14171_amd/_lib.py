"""ctypes binding of libgsup.so (include/gsup.h): argument marshalling only.

Every function has the name of the C entry point it calls and takes torch
tensors for the device arrays; torch provides device memory and the current
HIP stream, every computation runs in the library's HIP kernels.  A non-zero
status raises :class:`GsError` carrying the library's message.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loaded first: libgsup then binds to the HIP runtime torch already mapped

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgsup.so")

GS_OK = 0
GS_ERR_INVALID_ARGUMENT = 1
GS_ERR_CAPACITY = 2
GS_ERR_HIP = 3
GS_ERR_UNSUPPORTED = 4

SPLAT_FLOATS = 12  # gs_splat: 48 bytes = 12 x 4


class GsError(RuntimeError):
    def __init__(self, status: int, message: str, n_pairs: int | None = None):
        super().__init__(f"[gs status {status}] {message}")
        self.status = status
        self.n_pairs = n_pairs


class GsCamera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("view", ctypes.c_float * 12), ("cam_pos", ctypes.c_float * 3),
                ("near_plane", ctypes.c_float), ("far_plane", ctypes.c_float)]


class GsRasterCfg(ctypes.Structure):
    _fields_ = [("tile_size", ctypes.c_int32), ("sh_degree", ctypes.c_int32),
                ("dilation", ctypes.c_float), ("alpha_min", ctypes.c_float),
                ("alpha_max", ctypes.c_float), ("t_min", ctypes.c_float),
                ("bg", ctypes.c_float * 3), ("batch", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with "
                              "`python -m paper_2503_14171_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(_LIB_PATH)
        P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        cam_p, cfg_p = ctypes.POINTER(GsCamera), ctypes.POINTER(GsRasterCfg)
        L.gs_num_tiles.argtypes = [i32, i32, i32]
        L.gs_num_tiles.restype = i64
        L.gs_project.argtypes = [i64, P, P, P, P, P, cam_p, cfg_p, P, P, P, P]
        L.gs_project.restype = ctypes.c_int
        L.gs_bin_sort_workspace_size.argtypes = [i64, i64, cam_p, cfg_p]
        L.gs_bin_sort_workspace_size.restype = sz
        L.gs_bin_sort.argtypes = [i64, P, P, cam_p, cfg_p, i64, P, P, ctypes.POINTER(i64), P, sz, P]
        L.gs_bin_sort.restype = ctypes.c_int
        L.gs_raster_grad.argtypes = [P, P, P, cam_p, cfg_p, i32, P, P, P]
        L.gs_raster_grad.restype = ctypes.c_int
        L.gs_upscale_hermite.argtypes = [P, i32, i32, P, i32, i32, P]
        L.gs_upscale_hermite.restype = ctypes.c_int
        cams_p = ctypes.POINTER(GsCamera)
        L.gs_bin_sort_async.argtypes = [i64, P, P, cam_p, cfg_p, i64, P, P, P, P, sz, P]
        L.gs_bin_sort_async.restype = ctypes.c_int
        L.gs_num_tiles_views.argtypes = [i32, cams_p, i32]
        L.gs_num_tiles_views.restype = i64
        L.gs_project_views.argtypes = [i64, P, P, P, P, P, i32, cams_p, cfg_p, P, P, P, P]
        L.gs_project_views.restype = ctypes.c_int
        L.gs_bin_sort_views_workspace_size.argtypes = [i64, i32, cams_p, cfg_p, i64]
        L.gs_bin_sort_views_workspace_size.restype = sz
        L.gs_bin_sort_views.argtypes = [i64, i32, cams_p, cfg_p, P, P, i64, P, P, P, P, sz, P]
        L.gs_bin_sort_views.restype = ctypes.c_int
        L.gs_raster_grad_views.argtypes = [P, P, P, i32, cams_p, cfg_p, i32, P, P, P]
        L.gs_raster_grad_views.restype = ctypes.c_int
        L.gs_bin_sort_async_static.argtypes = [i64, P, P, cam_p, cfg_p, i64, P, P, P, P]
        L.gs_bin_sort_async_static.restype = ctypes.c_int
        L.gs_raster_fragment_counts.argtypes = [P, P, P, i32, cams_p, cfg_p, i32, P, P, P, P]
        L.gs_raster_fragment_counts.restype = ctypes.c_int
        L.gs_upscale_hermite_views.argtypes = [P, i32, ctypes.POINTER(i32), P, ctypes.POINTER(i32), i32, P]
        L.gs_upscale_hermite_views.restype = ctypes.c_int
        L.gs_raster_grad_views_train.argtypes = [P, P, P, i32, cams_p, cfg_p, P, P, P, P]
        L.gs_raster_grad_views_train.restype = ctypes.c_int
        L.gs_upscale_hermite_backward_views.argtypes = [P, i32, ctypes.POINTER(i32), P, ctypes.POINTER(i32), P]
        L.gs_upscale_hermite_backward_views.restype = ctypes.c_int
        L.gs_raster_grad_backward_views.argtypes = [P, P, P, i32, cams_p, cfg_p, P, P, P, i64, P, P]
        L.gs_raster_grad_backward_views.restype = ctypes.c_int
        L.gs_project_backward_views.argtypes = [i64, P, P, P, P, P, i32, cams_p, cfg_p, P, P, P, P, P, P, P]
        L.gs_project_backward_views.restype = ctypes.c_int
        L.gs_fd_slopes.argtypes = [P, i32, i32, P, P]
        L.gs_fd_slopes.restype = ctypes.c_int
        L.gs_last_error_message.restype = ctypes.c_char_p
        L.gs_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def camera(cam: dict) -> GsCamera:
    c = GsCamera()
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.fx, c.fy, c.cx, c.cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    c.view[:] = [float(v) for v in torch.as_tensor(cam["view"]).reshape(12).tolist()]
    c.cam_pos[:] = [float(v) for v in torch.as_tensor(cam["cam_pos"]).reshape(3).tolist()]
    c.near_plane = float(cam["near_plane"])
    c.far_plane = float(cam.get("far_plane", 0.0))
    return c


def raster_cfg(cfg: dict) -> GsRasterCfg:
    c = GsRasterCfg()
    c.tile_size = int(cfg["tile_size"])
    c.sh_degree = int(cfg["sh_degree"])
    c.dilation = float(cfg["dilation"])
    c.alpha_min, c.alpha_max, c.t_min = float(cfg["alpha_min"]), float(cfg["alpha_max"]), float(cfg["t_min"])
    c.bg[:] = [float(v) for v in cfg["bg"]]
    c.batch = int(cfg.get("batch", 0))
    return c


def cameras(cams) -> ctypes.Array:
    """Host array of gs_camera for the batched calls."""
    arr = (GsCamera * len(cams))()
    for k, c in enumerate(cams):
        arr[k] = camera(c)
    return arr


def _ptr(t: torch.Tensor | None, dtype=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{dtype} tensor expected, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


GS_PAIRS_DEPTH_RANGE = 1 << 62  # pair count of an asynchronous bin sort whose depths left [near, far]


def check_pair_count(k: int) -> int:
    """A pair count read back from an asynchronous bin sort; raises on the
    depth-range error code."""
    if k == GS_PAIRS_DEPTH_RANGE:
        raise GsError(GS_ERR_INVALID_ARGUMENT, "bin sort: a finite depth lies outside the cameras' "
                      "[near_plane, far_plane]")
    return k


def _check(status: int, n_pairs: int | None = None):
    if status != GS_OK:
        raise GsError(status, lib().gs_last_error_message().decode(), n_pairs)


def gs_version() -> str:
    return lib().gs_version().decode()


def gs_num_tiles(width: int, height: int, tile_size: int) -> int:
    return int(lib().gs_num_tiles(width, height, tile_size))


def gs_project(means, log_scales, quats, opacity, sh, cam: dict, cfg: dict, splats, depth, rect,
               stream=None) -> None:
    """Project n Gaussians; outputs splats [n,12] f32 (gs_splat records),
    depth [n] f32, rect [n,4] i16."""
    n = means.shape[0]
    f = torch.float32
    _check(lib().gs_project(n, _ptr(means, f), _ptr(log_scales, f), _ptr(quats, f), _ptr(opacity, f),
                            _ptr(sh, f), ctypes.byref(camera(cam)), ctypes.byref(raster_cfg(cfg)),
                            _ptr(splats, f), _ptr(depth, f), _ptr(rect, torch.int16), _stream(stream)))


def gs_bin_sort_workspace_size(n: int, capacity: int, cam: dict, cfg: dict) -> int:
    return int(lib().gs_bin_sort_workspace_size(n, capacity, ctypes.byref(camera(cam)),
                                                ctypes.byref(raster_cfg(cfg))))


def gs_bin_sort(n: int, depth, rect, cam: dict, cfg: dict, capacity: int, sorted_ids, tile_ranges,
                workspace, stream=None) -> int:
    """Per-tile lists; returns the pair count K (raises GsError with .n_pairs if K > capacity)."""
    k = ctypes.c_int64(0)
    st = lib().gs_bin_sort(n, _ptr(depth, torch.float32), _ptr(rect, torch.int16),
                           ctypes.byref(camera(cam)), ctypes.byref(raster_cfg(cfg)), capacity,
                           _ptr(sorted_ids, torch.int32), _ptr(tile_ranges, torch.int32),
                           ctypes.byref(k), _ptr(workspace, torch.uint8), workspace.numel(),
                           _stream(stream))
    _check(st, int(k.value))
    return int(k.value)


def gs_raster_grad(splats, sorted_ids, tile_ranges, cam: dict, cfg: dict, want_grads: bool, out,
                   n_blend=None, stream=None) -> None:
    _check(lib().gs_raster_grad(_ptr(splats, torch.float32), _ptr(sorted_ids, torch.int32),
                                _ptr(tile_ranges, torch.int32), ctypes.byref(camera(cam)),
                                ctypes.byref(raster_cfg(cfg)), 1 if want_grads else 0,
                                _ptr(out, torch.float32), _ptr(n_blend, torch.int32), _stream(stream)))


def gs_upscale_hermite(inp, out, stream=None) -> None:
    """inp [h, w, 12] -> out [H, W, 3]."""
    h, w = inp.shape[0], inp.shape[1]
    H, W = out.shape[0], out.shape[1]
    if inp.shape[2] != 12 or out.shape[2] != 3:
        raise ValueError("inp must be [h, w, 12] and out [H, W, 3]")
    _check(lib().gs_upscale_hermite(_ptr(inp, torch.float32), w, h, _ptr(out, torch.float32), W, H,
                                    _stream(stream)))


def gs_fd_slopes(img, out, stream=None) -> None:
    """img [h, w, 3] -> out [h, w, 12] with finite-difference slopes."""
    h, w = img.shape[0], img.shape[1]
    if img.shape[2] != 3 or tuple(out.shape) != (h, w, 12):
        raise ValueError("img must be [h, w, 3] and out [h, w, 12]")
    _check(lib().gs_fd_slopes(_ptr(img, torch.float32), w, h, _ptr(out, torch.float32), _stream(stream)))


def gs_bin_sort_async(n: int, depth, rect, cam: dict, cfg: dict, capacity: int, sorted_ids, tile_ranges,
                      n_pairs_dev, workspace, stream=None) -> None:
    """gs_bin_sort without the wait; the pair count lands in n_pairs_dev (int64 [1])."""
    _check(lib().gs_bin_sort_async(n, _ptr(depth, torch.float32), _ptr(rect, torch.int16),
                                   ctypes.byref(camera(cam)), ctypes.byref(raster_cfg(cfg)), capacity,
                                   _ptr(sorted_ids, torch.int32), _ptr(tile_ranges, torch.int32),
                                   _ptr(n_pairs_dev, torch.int64), _ptr(workspace, torch.uint8),
                                   workspace.numel(), _stream(stream)))


def gs_bin_sort_async_static(n: int, depth, rect, cam: dict, cfg: dict, capacity: int, sorted_ids,
                             tile_ranges, n_pairs_dev, stream=None) -> None:
    """gs_bin_sort_async in the library's static scratch (no workspace, no allocation)."""
    _check(lib().gs_bin_sort_async_static(n, _ptr(depth, torch.float32), _ptr(rect, torch.int16),
                                          ctypes.byref(camera(cam)), ctypes.byref(raster_cfg(cfg)), capacity,
                                          _ptr(sorted_ids, torch.int32), _ptr(tile_ranges, torch.int32),
                                          _ptr(n_pairs_dev, torch.int64), _stream(stream)))


# ---- batched views ---------------------------------------------------------
def gs_num_tiles_views(cams, tile_size: int) -> int:
    return int(lib().gs_num_tiles_views(len(cams), cameras(cams), tile_size))


def gs_project_views(means, log_scales, quats, opacity, sh, cams, cfg: dict, splats, depth, rect,
                     stream=None) -> None:
    """splats [V*n, 12], depth [V*n], rect [V*n, 4]; record v*n+i = Gaussian i in view v."""
    n = means.shape[0]
    f = torch.float32
    _check(lib().gs_project_views(n, _ptr(means, f), _ptr(log_scales, f), _ptr(quats, f), _ptr(opacity, f),
                                  _ptr(sh, f), len(cams), cameras(cams), ctypes.byref(raster_cfg(cfg)),
                                  _ptr(splats, f), _ptr(depth, f), _ptr(rect, torch.int16), _stream(stream)))


def gs_bin_sort_views_workspace_size(n: int, cams, cfg: dict, capacity: int) -> int:
    return int(lib().gs_bin_sort_views_workspace_size(n, len(cams), cameras(cams),
                                                      ctypes.byref(raster_cfg(cfg)), capacity))


def gs_bin_sort_views(n: int, cams, cfg: dict, depth, rect, capacity: int, sorted_ids, tile_ranges,
                      n_pairs_dev, workspace, stream=None) -> None:
    _check(lib().gs_bin_sort_views(n, len(cams), cameras(cams), ctypes.byref(raster_cfg(cfg)),
                                   _ptr(depth, torch.float32), _ptr(rect, torch.int16), capacity,
                                   _ptr(sorted_ids, torch.int32), _ptr(tile_ranges, torch.int32),
                                   _ptr(n_pairs_dev, torch.int64), _ptr(workspace, torch.uint8),
                                   workspace.numel(), _stream(stream)))


def gs_raster_grad_views(splats, sorted_ids, tile_ranges, cams, cfg: dict, want_grads: bool, out,
                         n_blend=None, stream=None) -> None:
    _check(lib().gs_raster_grad_views(_ptr(splats, torch.float32), _ptr(sorted_ids, torch.int32),
                                      _ptr(tile_ranges, torch.int32), len(cams), cameras(cams),
                                      ctypes.byref(raster_cfg(cfg)), 1 if want_grads else 0,
                                      _ptr(out, torch.float32), _ptr(n_blend, torch.int32), _stream(stream)))


def gs_raster_fragment_counts(splats, sorted_ids, tile_ranges, cams, cfg: dict, want_grads: bool, out,
                              n_eval, n_blend, stream=None) -> None:
    """gs_raster_grad_views plus per-pixel evaluated and blended fragment counts (int32)."""
    _check(lib().gs_raster_fragment_counts(_ptr(splats, torch.float32), _ptr(sorted_ids, torch.int32),
                                           _ptr(tile_ranges, torch.int32), len(cams), cameras(cams),
                                           ctypes.byref(raster_cfg(cfg)), 1 if want_grads else 0,
                                           _ptr(out, torch.float32), _ptr(n_eval, torch.int32),
                                           _ptr(n_blend, torch.int32), _stream(stream)))


def gs_upscale_hermite_views(inp, lo_sizes, out, hi_sizes, band_rows: int = 0, stream=None) -> None:
    """inp: the views' [h, w, 12] buffers back to back; sizes: lists of (width, height)."""
    nv = len(lo_sizes)
    lo = (ctypes.c_int32 * (2 * nv))(*[int(v) for wh in lo_sizes for v in wh])
    hi = (ctypes.c_int32 * (2 * nv))(*[int(v) for wh in hi_sizes for v in wh])
    _check(lib().gs_upscale_hermite_views(_ptr(inp, torch.float32), nv, lo, _ptr(out, torch.float32), hi,
                                          band_rows, _stream(stream)))


# ---- backward ----------------------------------------------------------------
def _sizes(sizes):
    nv = len(sizes)
    return (ctypes.c_int32 * (2 * nv))(*[int(v) for wh in sizes for v in wh])


def gs_raster_grad_views_train(splats, sorted_ids, tile_ranges, cams, cfg: dict, out, state, last,
                               stream=None) -> None:
    """Forward with gradients that also saves state [pix, 4] and last [pix] for the backward."""
    _check(lib().gs_raster_grad_views_train(_ptr(splats, torch.float32), _ptr(sorted_ids, torch.int32),
                                            _ptr(tile_ranges, torch.int32), len(cams), cameras(cams),
                                            ctypes.byref(raster_cfg(cfg)), _ptr(out, torch.float32),
                                            _ptr(state, torch.float32), _ptr(last, torch.int32), _stream(stream)))


def gs_upscale_hermite_backward_views(d_out, lo_sizes, d_in, hi_sizes, stream=None) -> None:
    _check(lib().gs_upscale_hermite_backward_views(_ptr(d_out, torch.float32), len(lo_sizes), _sizes(lo_sizes),
                                                   _ptr(d_in, torch.float32), _sizes(hi_sizes), _stream(stream)))


def gs_raster_grad_backward_views(splats, sorted_ids, tile_ranges, cams, cfg: dict, state, last, d_lowres,
                                  n: int, d_splats, stream=None) -> None:
    _check(lib().gs_raster_grad_backward_views(_ptr(splats, torch.float32), _ptr(sorted_ids, torch.int32),
                                               _ptr(tile_ranges, torch.int32), len(cams), cameras(cams),
                                               ctypes.byref(raster_cfg(cfg)), _ptr(state, torch.float32),
                                               _ptr(last, torch.int32), _ptr(d_lowres, torch.float32), n,
                                               _ptr(d_splats, torch.float32), _stream(stream)))


def gs_project_backward_views(means, log_scales, quats, opacity, sh, cams, cfg: dict, d_splats, d_means,
                              d_log_scales, d_quats, d_opacity, d_sh, stream=None) -> None:
    f = torch.float32
    _check(lib().gs_project_backward_views(means.shape[0], _ptr(means, f), _ptr(log_scales, f), _ptr(quats, f),
                                           _ptr(opacity, f), _ptr(sh, f), len(cams), cameras(cams),
                                           ctypes.byref(raster_cfg(cfg)), _ptr(d_splats, f), _ptr(d_means, f),
                                           _ptr(d_log_scales, f), _ptr(d_quats, f), _ptr(d_opacity, f),
                                           _ptr(d_sh, f), _stream(stream)))
