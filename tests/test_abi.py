"""The C ABI on the host: the library loads, exports every entry point that
include/gsup.h declares, its struct layouts match the Python binding, and
argument validation rejects bad calls before anything reaches the device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsup.h")


@pytest.fixture(scope="module")
def L():
    from paper_2503_14171_amd import _lib
    if not os.path.exists(_lib._LIB_PATH):
        from paper_2503_14171_amd import build
        build.build()
    return _lib


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(gs_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_entry_point(L):
    names = _declared()
    assert {"gs_project", "gs_bin_sort", "gs_bin_sort_workspace_size", "gs_raster_grad",
            "gs_upscale_hermite", "gs_last_error_message", "gs_num_tiles", "gs_version"} <= set(names)
    lib = ctypes.CDLL(L._LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", L._LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (gs_\w+)", out))
    assert set(names) <= exported


def test_struct_layouts_match_binding(L, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "gsup.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(gs_camera), offsetof(gs_camera, view),
         offsetof(gs_camera, near_plane), sizeof(gs_raster_cfg), offsetof(gs_raster_cfg, bg),
         sizeof(gs_splat), offsetof(gs_camera, far_plane));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(gs_splat, mean), offsetof(gs_splat, conic),
         offsetof(gs_splat, opacity), offsetof(gs_splat, rgb), offsetof(gs_splat, support));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    a, b = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")[:2]
    a = list(map(int, a.split()))
    b = list(map(int, b.split()))
    assert a == [ctypes.sizeof(L.GsCamera), L.GsCamera.view.offset, L.GsCamera.near_plane.offset,
                 ctypes.sizeof(L.GsRasterCfg), L.GsRasterCfg.bg.offset, 4 * L.SPLAT_FLOATS,
                 L.GsCamera.far_plane.offset]
    assert b == [0, 16, 28, 32, 44]


def test_host_helpers(L):
    from paper_2503_14171_amd import scenes
    assert L.gs_num_tiles(960, 540, 16) == 60 * 34
    assert L.gs_num_tiles(3840, 2160, 8) == 480 * 270
    assert L.gs_num_tiles(0, 5, 16) == 0
    cam = scenes.make_camera(960, 540)
    cfg = scenes.render_config(3)
    assert L.gs_bin_sort_workspace_size(1000, 5000, cam, cfg) > 5000 * 12
    assert L.gs_bin_sort_workspace_size(-1, 5000, cam, cfg) == 0
    assert L.gs_bin_sort_workspace_size(10, 10, cam, dict(cfg, tile_size=12)) == 0
    assert "gfx950" in L.gs_version()


def _no_gpu():
    import torch
    return not torch.cuda.is_available()


# The calls below use fake pointers and must be rejected by host-side
# validation; they only run where no GPU is visible.
pytestmark_validation = pytest.mark.skipif("not _no_gpu()", reason="fake-pointer validation runs on GPU-less hosts")


@pytestmark_validation
def test_validation_rejects_bad_calls(L):
    from paper_2503_14171_amd import scenes
    lib = L.lib()
    cam = L.camera(scenes.make_camera(64, 48))
    cfg = L.raster_cfg(scenes.render_config(0))
    F = ctypes.c_void_p(4096)  # never dereferenced: every call below fails validation
    R = ctypes.byref
    bad_tile = L.raster_cfg(scenes.render_config(0, tile_size=12))
    assert lib.gs_project(10, F, F, F, F, F, R(cam), R(bad_tile), F, F, F, None) == L.GS_ERR_UNSUPPORTED
    assert "tile_size" in lib.gs_last_error_message().decode()
    bad_alpha = L.raster_cfg(scenes.render_config(0, alpha_min=0.5, alpha_max=0.4))
    assert lib.gs_project(10, F, F, F, F, F, R(cam), R(bad_alpha), F, F, F, None) == L.GS_ERR_INVALID_ARGUMENT
    bad_sh = L.raster_cfg(scenes.render_config(4))
    assert lib.gs_project(10, F, F, F, F, F, R(cam), R(bad_sh), F, F, F, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_project(-1, F, F, F, F, F, R(cam), R(cfg), F, F, F, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_project(10, None, F, F, F, F, R(cam), R(cfg), F, F, F, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_project(10, F, F, ctypes.c_void_p(4100), F, F, R(cam), R(cfg), F, F, F, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_project(0, None, None, None, None, None, R(cam), R(cfg), None, None, None, None) == L.GS_OK
    assert lib.gs_last_error_message().decode() == ""
    bad_cam = L.camera(dict(scenes.make_camera(64, 48), near_plane=0.0))
    assert lib.gs_project(10, F, F, F, F, F, R(bad_cam), R(cfg), F, F, F, None) == L.GS_ERR_INVALID_ARGUMENT
    for far in (-1.0, 0.1, float("inf")):  # negative, before the near plane, not finite
        bad_far = L.camera(scenes.make_camera(64, 48, far_plane=far))
        assert lib.gs_project(10, F, F, F, F, F, R(bad_far), R(cfg), F, F, F, None) == L.GS_ERR_INVALID_ARGUMENT
        assert "far_plane" in lib.gs_last_error_message().decode()
    zero_cam = L.camera(dict(scenes.make_camera(64, 48), width=0))
    assert lib.gs_raster_grad(F, F, F, R(zero_cam), R(cfg), 1, F, None, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_raster_grad(F, None, F, R(cam), R(cfg), 1, F, None, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_raster_grad(F, F, F, R(cam), R(cfg), 1, ctypes.c_void_p(4104), None, None) == L.GS_ERR_INVALID_ARGUMENT
    k = ctypes.c_int64(0)
    ws = lib.gs_bin_sort_workspace_size(10, 100, R(cam), R(cfg))
    assert lib.gs_bin_sort(10, F, F, R(cam), R(cfg), 100, F, F, R(k), F, ws - 1, None) == L.GS_ERR_INVALID_ARGUMENT
    assert "workspace" in lib.gs_last_error_message().decode()
    assert lib.gs_bin_sort(10, F, F, R(cam), R(cfg), -5, F, F, R(k), F, ws, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_bin_sort(10, F, F, R(cam), R(cfg), 100, F, F, None, F, ws, None) == L.GS_ERR_INVALID_ARGUMENT
    # the scratch-free bin sort: a device counter is required, and sizes beyond
    # its static scratch are refused on the host, before any device call
    assert lib.gs_bin_sort_async_static(10, F, F, R(cam), R(cfg), 100, F, F, None, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_bin_sort_async_static(10, F, F, R(cam), R(cfg), 8_000_000, F, F, F,
                                        None) == L.GS_ERR_INVALID_ARGUMENT
    assert "static scratch" in lib.gs_last_error_message().decode()
    assert lib.gs_upscale_hermite(F, 1, 5, ctypes.c_void_p(1 << 20), 4, 10, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_upscale_hermite(F, 4, 5, ctypes.c_void_p(1 << 20), 3, 10, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_upscale_hermite(F, 4, 5, ctypes.c_void_p(4096 + 64), 8, 10, None) == L.GS_ERR_INVALID_ARGUMENT
    assert "overlap" in lib.gs_last_error_message().decode()
    assert lib.gs_fd_slopes(F, 1, 5, ctypes.c_void_p(1 << 20), None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_fd_slopes(None, 4, 5, ctypes.c_void_p(1 << 20), None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_fd_slopes(F, 4, 5, ctypes.c_void_p((1 << 20) + 4), None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_fd_slopes(F, 4, 5, ctypes.c_void_p(4096 + 32), None) == L.GS_ERR_INVALID_ARGUMENT
    assert "overlap" in lib.gs_last_error_message().decode()


@pytestmark_validation
def test_validation_rejects_bad_batched_and_backward_calls(L):
    from paper_2503_14171_amd import scenes
    lib = L.lib()
    cams = L.cameras([scenes.make_camera(64, 48), scenes.make_camera(32, 40)])
    cfg = L.raster_cfg(scenes.render_config(0))
    R = ctypes.byref
    F = ctypes.c_void_p(4096)  # never dereferenced: every call below fails validation
    I32 = ctypes.c_int32
    # view counts outside [1, GS_MAX_VIEWS] and a missing camera array
    for nv in (0, 17):
        assert lib.gs_project_views(10, F, F, F, F, F, nv, cams, R(cfg), F, F, F, None) == L.GS_ERR_INVALID_ARGUMENT
        assert "n_views" in lib.gs_last_error_message().decode()
    assert lib.gs_raster_grad_views(F, F, F, 2, None, R(cfg), 1, F, None, None) == L.GS_ERR_INVALID_ARGUMENT
    # a bad camera among the views
    bad = L.cameras([scenes.make_camera(64, 48), dict(scenes.make_camera(32, 40), width=0)])
    assert lib.gs_project_views(10, F, F, F, F, F, 2, bad, R(cfg), F, F, F, None) == L.GS_ERR_INVALID_ARGUMENT
    # unsupported LDS batch and tile size
    bad_batch = L.raster_cfg(scenes.render_config(0, tile_size=16, batch=100))
    assert lib.gs_raster_grad_views(F, F, F, 2, cams, R(bad_batch), 1, F, None, None) == L.GS_ERR_UNSUPPORTED
    assert "batch" in lib.gs_last_error_message().decode()
    bad_tile = L.raster_cfg(scenes.render_config(0, tile_size=128))
    assert lib.gs_raster_grad_views(F, F, F, 2, cams, R(bad_tile), 1, F, None, None) == L.GS_ERR_UNSUPPORTED
    # n * n_views beyond the int32 record index
    assert lib.gs_project_views(1 << 30, F, F, F, F, F, 2, cams, R(cfg), F, F, F, None) == L.GS_ERR_INVALID_ARGUMENT
    # the batched bin sort needs a device counter; workspace too small
    ws = lib.gs_bin_sort_views_workspace_size(10, 2, cams, R(cfg), 100)
    assert ws > 0
    assert lib.gs_bin_sort_views(10, 2, cams, R(cfg), F, F, 100, F, F, None, F, ws, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_bin_sort_views(10, 2, cams, R(cfg), F, F, 100, F, F, F, F, ws - 1, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_bin_sort_async(10, F, F, R(L.camera(scenes.make_camera(64, 48))), R(cfg), 100, F, F, None, F,
                                 ws, None) == L.GS_ERR_INVALID_ARGUMENT
    # upscaler views: bad band height, a view smaller than 2x2, overlapping buffers
    lo = (I32 * 4)(16, 8, 4, 4)
    hi = (I32 * 4)(32, 16, 8, 8)
    assert lib.gs_upscale_hermite_views(F, 2, lo, ctypes.c_void_p(1 << 24), hi, 12, None) == L.GS_ERR_UNSUPPORTED
    lo_bad = (I32 * 4)(16, 8, 1, 4)
    assert lib.gs_upscale_hermite_views(F, 2, lo_bad, ctypes.c_void_p(1 << 24), hi, 0, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_upscale_hermite_views(F, 2, lo, ctypes.c_void_p(4096 + 64), hi, 0, None) == L.GS_ERR_INVALID_ARGUMENT
    assert "overlap" in lib.gs_last_error_message().decode()
    # backward entry points: missing buffers, misaligned state, bad sizes
    assert lib.gs_raster_grad_views_train(F, F, F, 2, cams, R(cfg), F, None, F, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_raster_grad_views_train(F, F, F, 2, cams, R(cfg), F, ctypes.c_void_p(4100), F,
                                          None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_raster_grad_backward_views(F, F, F, 2, cams, R(cfg), F, F, F, 10, None, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_raster_grad_backward_views(F, F, F, 2, cams, R(cfg), F, F, F, -1, F, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_project_backward_views(10, F, F, F, F, F, 2, cams, R(cfg), F, F, F, None, F, F,
                                         None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_project_backward_views(10, F, F, F, F, F, 2, cams, R(cfg), F, F, F, ctypes.c_void_p(4104), F, F,
                                         None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_project_backward_views(0, None, None, None, None, None, 2, cams, R(cfg), None, None, None, None,
                                         None, None, None) == L.GS_OK
    assert lib.gs_upscale_hermite_backward_views(F, 2, lo_bad, ctypes.c_void_p(1 << 24), hi, None) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_upscale_hermite_backward_views(F, 2, lo, ctypes.c_void_p(4096 + 32), hi, None) == L.GS_ERR_INVALID_ARGUMENT
    assert "overlap" in lib.gs_last_error_message().decode()
    # sizes on the host
    assert lib.gs_num_tiles_views(2, cams, 16) == 4 * 3 + 2 * 3
    assert lib.gs_num_tiles_views(0, cams, 16) == 0


def test_binding_fails_loudly_without_library(L, monkeypatch):
    import paper_2503_14171_amd._lib as mod
    monkeypatch.setattr(mod, "_lib", None)
    monkeypatch.setattr(mod, "_LIB_PATH", "/nonexistent/libgsup.so")
    with pytest.raises(ImportError):
        mod.lib()
