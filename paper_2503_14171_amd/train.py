"""Differentiable gradient-aware upscaled rendering for training.

:class:`UpscaledRender` is a ``torch.autograd.Function``: its forward runs
gs_project_views -> gs_bin_sort_views -> gs_raster_grad_views_train ->
gs_upscale_hermite_views, its backward gs_upscale_hermite_backward_views ->
gs_raster_grad_backward_views -> gs_project_backward_views, all in the
library's HIP kernels (Suppl. "3DGS Gradient Computation - Backward pass").
The rasterizer's per-pixel state before each fragment is recovered in the
backward pass from the final state the forward saved (inversion trick), so
no per-fragment state is stored.  :class:`TrainViews` holds the buffers of a
fixed set of views between the two passes.
"""
from __future__ import annotations

import torch

from . import _lib as L


class TrainViews:
    def __init__(self, n: int, cams, hi_sizes, cfg: dict, device: str = "cuda"):
        if not 1 <= len(cams) <= 16 or len(cams) != len(hi_sizes):
            raise ValueError("need 1..16 cameras and one high-res size per camera")
        self.n, self.cams, self.cfg, self.device = int(n), [dict(c) for c in cams], dict(cfg), device
        self.hi = [(int(W), int(H)) for (W, H) in hi_sizes]
        self.lo = [(c["width"], c["height"]) for c in self.cams]
        V, n1 = len(cams), max(self.n, 1)
        f, i = torch.float32, torch.int32
        self.splats = torch.empty((V * n1, L.SPLAT_FLOATS), dtype=f, device=device)
        self.depth = torch.empty(V * n1, dtype=f, device=device)
        self.rect = torch.empty((V * n1, 4), dtype=torch.int16, device=device)
        self.tiles = L.gs_num_tiles_views(self.cams, self.cfg["tile_size"])
        self.ranges = torch.empty((self.tiles, 2), dtype=i, device=device)
        self.lo_px = sum(w * h for (w, h) in self.lo)
        self.hi_px = sum(W * H for (W, H) in self.hi)
        self.low = torch.empty((self.lo_px, 12), dtype=f, device=device)
        self.state = torch.empty((self.lo_px, 4), dtype=f, device=device)
        self.last = torch.empty(self.lo_px, dtype=i, device=device)
        self.d_low = torch.empty((self.lo_px, 12), dtype=f, device=device)
        self.d_splats = torch.empty((V * n1, 9), dtype=f, device=device)
        self.n_pairs = torch.zeros(1, dtype=torch.int64, device=device)
        # forwards run so far; the backward of a forward whose saved buffers
        # (lists, final state) a later forward overwrote must not run
        self.generation = 0
        self.capacity = 0
        self._shrink_to = 0
        self._alloc(4 * V * self.n + 1024)

    def _alloc(self, capacity: int):
        self.capacity = int(capacity)
        self.ids = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=self.device)
        ws = L.gs_bin_sort_views_workspace_size(self.n, self.cams, self.cfg, self.capacity)
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.device)

    def forward(self, means, log_scales, quats, opacity, sh) -> torch.Tensor:
        """Upscaled images of all views back to back, [sum W*H, 3]."""
        args = (means, log_scales, quats, opacity, sh)
        if self._shrink_to:  # the last step's lists are no longer needed
            self._alloc(self._shrink_to)
            self._shrink_to = 0
        while True:
            L.gs_project_views(*args, self.cams, self.cfg, self.splats, self.depth, self.rect)
            L.gs_bin_sort_views(self.n, self.cams, self.cfg, self.depth, self.rect, self.capacity, self.ids,
                                self.ranges, self.n_pairs, self.workspace)
            k = L.check_pair_count(int(self.n_pairs.item()))
            if k <= self.capacity:
                # the pair passes size their grids by the capacity: keep it
                # near the count from the next step on
                if self.capacity > 2 * k + 4096:
                    self._shrink_to = int(k * 1.25) + 1024
                break
            if k >= 2 ** 31:
                raise L.GsError(L.GS_ERR_CAPACITY, f"{k} pairs exceed the 2^31 index limit", k)
            self._alloc(int(k * 1.25) + 1024)
        L.gs_raster_grad_views_train(self.splats, self.ids, self.ranges, self.cams, self.cfg, self.low,
                                     self.state, self.last)
        self.generation += 1
        up = torch.empty((self.hi_px, 3), dtype=torch.float32, device=self.device)
        L.gs_upscale_hermite_views(self.low, self.lo, up, self.hi)
        return up

    def backward(self, d_up, means, log_scales, quats, opacity, sh, generation: int | None = None):
        """dL/d(means, log_scales, quats, opacity, sh) for dL/d(upscaled) = d_up.

        Walks the lists and final transmittance state of the latest forward;
        ``generation`` (the value of ``self.generation`` right after the
        forward being differentiated) must name that forward, otherwise a
        RuntimeError is raised: inverting the blend from another forward's
        final state would give wrong gradients silently."""
        if generation is not None and generation != self.generation:
            raise RuntimeError(
                f"TrainViews: backward of forward #{generation}, but forward #{self.generation} has "
                "since overwritten the saved lists and state; run backward before the next forward "
                "on the same TrainViews (or use one TrainViews per pending forward)")
        d_up = d_up.contiguous().to(torch.float32)
        L.gs_upscale_hermite_backward_views(d_up, self.lo, self.d_low, self.hi)
        L.gs_raster_grad_backward_views(self.splats, self.ids, self.ranges, self.cams, self.cfg, self.state,
                                        self.last, self.d_low, self.n, self.d_splats)
        g = [torch.empty_like(t) for t in (means, log_scales, quats, opacity, sh)]
        L.gs_project_backward_views(means, log_scales, quats, opacity, sh, self.cams, self.cfg, self.d_splats,
                                    *g)
        return g

    def split(self, up: torch.Tensor):
        """Per-view [H, W, 3] views of a [sum W*H, 3] tensor."""
        out, a = [], 0
        for (W, H) in self.hi:
            out.append(up[a:a + W * H].view(H, W, 3))
            a += W * H
        return out


class UpscaledRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity, sh, views: TrainViews):
        args = tuple(t.contiguous() for t in (means, log_scales, quats, opacity, sh))
        up = views.forward(*args)
        ctx.views = views
        ctx.generation = views.generation
        ctx.save_for_backward(*args)
        return up

    @staticmethod
    def backward(ctx, d_up):
        grads = ctx.views.backward(d_up, *ctx.saved_tensors, generation=ctx.generation)
        return (*grads, None)


def render_upscaled(params: dict, views: TrainViews) -> torch.Tensor:
    """Differentiable: params holds means, log_scales, quats, opacity, sh tensors."""
    return UpscaledRender.apply(params["means"], params["log_scales"], params["quats"], params["opacity"],
                                params["sh"], views)
