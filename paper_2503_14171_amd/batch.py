"""Batched views: many cameras of one scene through one launch per step.

:class:`ViewBatch` holds the concatenated per-view buffers of a batch and
enqueues gs_project_views -> gs_bin_sort_views -> gs_raster_grad_views ->
gs_upscale_hermite_views on the current stream.  None of these calls waits,
so the chain is captured once in a HIP graph (through torch's graph API,
which only records the library's kernel launches) and replayed per frame.
The pair count stays on the device; :meth:`ViewBatch.render` checks it after
the frame and, if the pairs did not fit, grows the buffers, captures again
and renders the frame again.
"""
from __future__ import annotations

import torch

from . import _lib as L


class ViewBatch:
    """``direct=True`` is the baseline: the views rendered directly at their
    high-res sizes (plain compositing, no upscaling) into ``up``."""

    def __init__(self, renderer, cams, hi_sizes, cfg: dict, band_rows: int = 0,
                 capacity: int | None = None, direct: bool = False):
        if not 1 <= len(cams) <= 16 or len(cams) != len(hi_sizes):
            raise ValueError("need 1..16 cameras and one high-res size per camera")
        from . import scenes
        self.r = renderer
        self.direct = bool(direct)
        self.hi = [(int(W), int(H)) for (W, H) in hi_sizes]
        self.cams = [scenes.scale_camera(c, W, H) if direct else dict(c)
                     for c, (W, H) in zip(cams, self.hi)]
        self.lo = [(c["width"], c["height"]) for c in self.cams]
        self.cfg = dict(cfg)
        self.band_rows = int(band_rows)
        dev, n, V = renderer.device, max(renderer.n, 1), len(cams)
        self.splats = torch.empty((V * n, L.SPLAT_FLOATS), dtype=torch.float32, device=dev)
        self.depth = torch.empty(V * n, dtype=torch.float32, device=dev)
        self.rect = torch.empty((V * n, 4), dtype=torch.int16, device=dev)
        self.tiles = L.gs_num_tiles_views(self.cams, self.cfg["tile_size"])
        self.ranges = torch.empty((self.tiles, 2), dtype=torch.int32, device=dev)
        self.lo_px = [w * h for (w, h) in self.lo]
        self.hi_px = [W * H for (W, H) in self.hi]
        self.low = None if direct else torch.empty((sum(self.lo_px), 12), dtype=torch.float32, device=dev)
        self.up = torch.empty((sum(self.hi_px), 3), dtype=torch.float32, device=dev)
        self.n_pairs = torch.zeros(1, dtype=torch.int64, device=dev)
        self.capacity = 0
        self._shrink_to = 0
        self._alloc(capacity if capacity is not None else 4 * V * renderer.n + 1024)
        self.graph = None

    def _alloc(self, capacity: int):
        self.capacity = int(capacity)
        self.ids = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=self.r.device)
        ws = L.gs_bin_sort_views_workspace_size(self.r.n, self.cams, self.cfg, self.capacity)
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.r.device)

    # -- the chain -----------------------------------------------------------
    def run(self):
        """Enqueue one frame of all views on the current stream (no waits)."""
        r = self.r
        L.gs_project_views(r.means, r.log_scales, r.quats, r.opacity, r.sh, self.cams, self.cfg,
                           self.splats, self.depth, self.rect)
        L.gs_bin_sort_views(r.n, self.cams, self.cfg, self.depth, self.rect, self.capacity, self.ids,
                            self.ranges, self.n_pairs, self.workspace)
        if self.direct:
            L.gs_raster_grad_views(self.splats, self.ids, self.ranges, self.cams, self.cfg, False, self.up)
            return
        L.gs_raster_grad_views(self.splats, self.ids, self.ranges, self.cams, self.cfg, True, self.low)
        L.gs_upscale_hermite_views(self.low, self.lo, self.up, self.hi, self.band_rows)

    def capture(self):
        """Capture :meth:`run` in a HIP graph (after one eager warm-up run)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.run()
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def launch(self):
        """One frame: graph replay if captured, else the eager chain."""
        if self._shrink_to:
            self._alloc(self._shrink_to)
            self._shrink_to = 0
            if self.graph is not None:
                self.graph = None
                self.capture()
        if self.graph is not None:
            self.graph.replay()
        else:
            self.run()

    def pairs_fit(self) -> bool:
        """Waits for the stream; False (and bigger buffers, graph dropped) if
        the last frame's pairs did not fit.  A capacity far above the count
        is brought down to it plus 25 % before the next frame (the pair
        passes size their grids by the capacity); a captured graph is
        captured again either way."""
        k = L.check_pair_count(int(self.n_pairs.item()))
        if k <= self.capacity:
            if self.capacity > 2 * k + 4096:
                self._shrink_to = int(k * 1.25) + 1024  # before the next frame: ids stay readable
            return True
        if k >= 2 ** 31:
            raise L.GsError(L.GS_ERR_CAPACITY, f"{k} pairs exceed the 2^31 index limit", k)
        self._alloc(int(k * 1.25) + 1024)
        if self.graph is not None:
            self.graph = None
            self.capture()
        return False

    def render(self):
        """One verified frame; returns (low-res buffers, upscaled images) per view."""
        self.launch()
        while not self.pairs_fit():
            self.launch()
        return self.views()

    # -- per-view results ----------------------------------------------------
    def views(self):
        lows, ups, a, b = [], [], 0, 0
        for (w, h), (W, H), pl, ph in zip(self.lo, self.hi, self.lo_px, self.hi_px):
            lows.append(None if self.direct else self.low[a:a + pl].view(h, w, 12))
            ups.append(self.up[b:b + ph].view(H, W, 3))
            a += pl
            b += ph
        return lows, ups
