"""Guard bands around every output buffer of every entry point.

Each output is a slice of a larger allocation whose leading and trailing
bands (256 bytes before, 4 KiB after) hold a sentinel bit pattern; after the
call the bands must be untouched, so no kernel writes outside the buffer it
was given.  Sizes are ragged (images and counts that are not multiples of a
tile, a wave or a workgroup) so that the last block of every grid is partial.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LEAD = 256    # bytes before the buffer (keeps its 256-byte alignment)
TRAIL = 4096  # bytes after it
SENTINEL = 0x7FC0DEAD  # a NaN payload no kernel writes


@pytest.fixture(scope="module")
def gs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_14171_amd import _lib
    _lib.lib()
    return _lib


class Guarded:
    """A device buffer of `shape` and `dtype` inside sentinel bands."""

    def __init__(self, shape, dtype):
        import torch
        self.shape = tuple(int(s) for s in shape)
        self.dtype = dtype
        esz = torch.empty(0, dtype=dtype).element_size()
        n = int(np.prod(self.shape)) if self.shape else 1
        self.lead, self.trail = LEAD // esz, TRAIL // esz
        words = (LEAD + n * esz + TRAIL + 3) // 4
        self.raw = torch.full((words,), SENTINEL, dtype=torch.int32, device="cuda")
        self.bytes = self.raw.view(torch.uint8)
        body = self.bytes[LEAD:LEAD + n * esz].view(dtype)
        self.t = body.view(self.shape) if self.shape else body
        self.n_bytes = n * esz

    def check(self, name):
        import torch
        torch.cuda.synchronize()
        b = self.bytes.cpu().numpy()
        sent = np.frombuffer(np.array([SENTINEL], np.int32).tobytes(), np.uint8)
        lead = b[:LEAD]
        end = LEAD + self.n_bytes
        trail = b[end:end + TRAIL]
        # the bands hold the repeating 4-byte pattern, aligned to the allocation
        exp_lead = np.tile(sent, LEAD // 4)
        off = end % 4
        exp_trail = np.tile(sent, TRAIL // 4 + 2)[off:off + trail.size]
        assert np.array_equal(lead, exp_lead), f"{name}: bytes before the buffer overwritten"
        assert np.array_equal(trail, exp_trail), f"{name}: bytes after the buffer overwritten"


def test_guard_bands_forward_chain(gs):
    import torch
    from paper_2503_14171_amd import scenes
    sc = scenes.make_scene("clusters", 12345, 81, 3)
    cam = scenes.make_camera(203, 117)
    n = sc["means"].shape[0]
    dev = {k: torch.as_tensor(sc[k], device="cuda") for k in ("means", "log_scales", "quats", "opacity", "sh")}
    for tile in (8, 16, 32, 64):
        cfg = scenes.render_config(3, tile_size=tile)
        print(f"guards: forward chain tile={tile}", flush=True)
        splats = Guarded((n, gs.SPLAT_FLOATS), torch.float32)
        depth = Guarded((n,), torch.float32)
        rect = Guarded((n, 4), torch.int16)
        gs.gs_project(dev["means"], dev["log_scales"], dev["quats"], dev["opacity"], dev["sh"], cam, cfg,
                      splats.t, depth.t, rect.t)
        for g, nm in ((splats, "splats"), (depth, "depth"), (rect, "rect")):
            g.check(f"gs_project {nm}")
        tiles = gs.gs_num_tiles(cam["width"], cam["height"], tile)
        cap = 40 * n + 77
        ws = torch.empty(gs.gs_bin_sort_workspace_size(n, cap, cam, cfg), dtype=torch.uint8, device="cuda")
        ids = Guarded((cap,), torch.int32)
        ranges = Guarded((tiles, 2), torch.int32)
        k = gs.gs_bin_sort(n, depth.t, rect.t, cam, cfg, cap, ids.t, ranges.t, ws)
        assert 0 < k <= cap
        ids.check("gs_bin_sort ids")
        ranges.check("gs_bin_sort ranges")
        kd = Guarded((1,), torch.int64)
        ids2 = Guarded((cap,), torch.int32)
        ranges2 = Guarded((tiles, 2), torch.int32)
        gs.gs_bin_sort_async(n, depth.t, rect.t, cam, cfg, cap, ids2.t, ranges2.t, kd.t, ws)
        for g, nm in ((kd, "n_pairs_dev"), (ids2, "ids"), (ranges2, "ranges")):
            g.check(f"gs_bin_sort_async {nm}")
        H, W = cam["height"], cam["width"]
        for grads in (True, False):
            C = 12 if grads else 3
            out = Guarded((H, W, C), torch.float32)
            nbl = Guarded((H, W), torch.int32)
            gs.gs_raster_grad(splats.t, ids.t, ranges.t, cam, cfg, grads, out.t, nbl.t)
            out.check(f"gs_raster_grad out grads={grads}")
            nbl.check(f"gs_raster_grad n_blend grads={grads}")
        out = Guarded((H * W, 12), torch.float32)
        nev = Guarded((H * W,), torch.int32)
        nbl = Guarded((H * W,), torch.int32)
        gs.gs_raster_fragment_counts(splats.t, ids.t, ranges.t, [cam], cfg, True, out.t, nev.t, nbl.t)
        for g, nm in ((out, "out"), (nev, "n_eval"), (nbl, "n_blend")):
            g.check(f"gs_raster_fragment_counts {nm}")
        low = out.t.view(H, W, 12)
        for (Wh, Hh) in ((W, H), (2 * W + 1, 3 * H - 2), (4 * W, 4 * H)):
            up = Guarded((Hh, Wh, 3), torch.float32)
            gs.gs_upscale_hermite(low, up.t)
            up.check(f"gs_upscale_hermite {Wh}x{Hh}")
        fd = Guarded((H, W, 12), torch.float32)
        gs.gs_fd_slopes(low[..., :3].contiguous(), fd.t)
        fd.check("gs_fd_slopes")


def test_guard_bands_views_and_backward(gs):
    import torch
    from paper_2503_14171_amd import scenes
    sc = scenes.make_scene("scene", 5003, 82, 2)
    sc["means"] = sc["means"] * np.float32(0.5)
    cams = [scenes.orbit_camera(61, 45, 10.0, 5.0), scenes.orbit_camera(90, 33, -40.0, -10.0)]
    hi = [(183, 135), (200, 70)]
    cfg = scenes.render_config(2, tile_size=16)
    n, V = sc["means"].shape[0], len(cams)
    dev = {k: torch.as_tensor(sc[k], device="cuda") for k in ("means", "log_scales", "quats", "opacity", "sh")}
    print("guards: views and backward", flush=True)
    splats = Guarded((V * n, gs.SPLAT_FLOATS), torch.float32)
    depth = Guarded((V * n,), torch.float32)
    rect = Guarded((V * n, 4), torch.int16)
    gs.gs_project_views(dev["means"], dev["log_scales"], dev["quats"], dev["opacity"], dev["sh"], cams, cfg,
                        splats.t, depth.t, rect.t)
    for g, nm in ((splats, "splats"), (depth, "depth"), (rect, "rect")):
        g.check(f"gs_project_views {nm}")
    tiles = gs.gs_num_tiles_views(cams, 16)
    cap = 40 * V * n + 99
    ws = torch.empty(gs.gs_bin_sort_views_workspace_size(n, cams, cfg, cap), dtype=torch.uint8, device="cuda")
    ids = Guarded((cap,), torch.int32)
    ranges = Guarded((tiles, 2), torch.int32)
    kd = Guarded((1,), torch.int64)
    gs.gs_bin_sort_views(n, cams, cfg, depth.t, rect.t, cap, ids.t, ranges.t, kd.t, ws)
    for g, nm in ((ids, "ids"), (ranges, "ranges"), (kd, "n_pairs_dev")):
        g.check(f"gs_bin_sort_views {nm}")
    assert 0 < int(kd.t.item()) <= cap
    lo_px = sum(c["width"] * c["height"] for c in cams)
    hi_px = sum(W * H for W, H in hi)
    low = Guarded((lo_px, 12), torch.float32)
    state = Guarded((lo_px, 4), torch.float32)
    last = Guarded((lo_px,), torch.int32)
    gs.gs_raster_grad_views_train(splats.t, ids.t, ranges.t, cams, cfg, low.t, state.t, last.t)
    for g, nm in ((low, "out"), (state, "state"), (last, "last")):
        g.check(f"gs_raster_grad_views_train {nm}")
    lo = [(c["width"], c["height"]) for c in cams]
    for band in (4, 32):
        up = Guarded((hi_px, 3), torch.float32)
        gs.gs_upscale_hermite_views(low.t, lo, up.t, hi, band)
        up.check(f"gs_upscale_hermite_views band={band}")
    d_up = torch.randn((hi_px, 3), device="cuda")
    d_low = Guarded((lo_px, 12), torch.float32)
    gs.gs_upscale_hermite_backward_views(d_up, lo, d_low.t, hi)
    d_low.check("gs_upscale_hermite_backward_views")
    d_splats = Guarded((V * n, 9), torch.float32)
    gs.gs_raster_grad_backward_views(splats.t, ids.t, ranges.t, cams, cfg, state.t, last.t, d_low.t, n,
                                     d_splats.t)
    d_splats.check("gs_raster_grad_backward_views")
    grads = {k: Guarded(tuple(dev[k].shape), torch.float32) for k in dev}
    gs.gs_project_backward_views(dev["means"], dev["log_scales"], dev["quats"], dev["opacity"], dev["sh"], cams,
                                 cfg, d_splats.t, grads["means"].t, grads["log_scales"].t, grads["quats"].t,
                                 grads["opacity"].t, grads["sh"].t)
    for k, g in grads.items():
        g.check(f"gs_project_backward_views d_{k}")
