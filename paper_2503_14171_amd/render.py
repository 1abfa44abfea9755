"""Per-view pipeline over the C ABI: project -> bin/sort -> raster -> upscale.

:class:`Renderer` keeps one scene's parameters and the per-view buffers in
device memory and chains the four entry points on the current stream.  It
only allocates buffers and forwards them; every step runs in libgsup's HIP
kernels.  :class:`FramePipeline` keeps several frames in flight, each on a
stream and a set of buffers of its own.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L


class Renderer:
    def __init__(self, scene: dict, device: str = "cuda"):
        t = lambda k: torch.as_tensor(np.ascontiguousarray(scene[k]), dtype=torch.float32, device=device).contiguous()
        self.means, self.log_scales, self.quats = t("means"), t("log_scales"), t("quats")
        self.opacity = t("opacity")
        self.sh = t("sh")
        self.n = self.means.shape[0]
        self.sh_degree = int(scene.get("sh_degree", round(self.sh.shape[1] ** 0.5) - 1))
        self.device = device
        self._bufs: dict = {}

    def sibling(self) -> "Renderer":
        """A renderer over the same scene tensors (shared, read only) with
        per-view buffers of its own, for a frame in flight beside this one's."""
        r = Renderer.__new__(Renderer)
        r.__dict__.update(self.__dict__)
        r._bufs = {}
        return r

    # -- buffers -------------------------------------------------------------
    def _view_bufs(self, cam: dict, cfg: dict):
        key = (cam["width"], cam["height"], cfg["tile_size"])
        b = self._bufs.get(key)
        if b is None:
            dev = self.device
            n = max(self.n, 1)
            tiles = L.gs_num_tiles(cam["width"], cam["height"], cfg["tile_size"])
            b = dict(splats=torch.empty((n, L.SPLAT_FLOATS), dtype=torch.float32, device=dev),
                     depth=torch.empty(n, dtype=torch.float32, device=dev),
                     rect=torch.empty((n, 4), dtype=torch.int16, device=dev),
                     ranges=torch.empty((tiles, 2), dtype=torch.int32, device=dev),
                     capacity=0)
            self._bufs[key] = b
        return b

    def _ensure_capacity(self, b: dict, cam: dict, cfg: dict, capacity: int, shrink: bool = False):
        if capacity <= b["capacity"] and not shrink:
            return
        capacity = int(capacity)
        b["ids"] = torch.empty(max(capacity, 1), dtype=torch.int32, device=self.device)
        ws = L.gs_bin_sort_workspace_size(self.n, capacity, cam, cfg)
        b["workspace"] = torch.empty(ws, dtype=torch.uint8, device=self.device)
        b["capacity"] = capacity

    # -- steps ---------------------------------------------------------------
    def project(self, cam: dict, cfg: dict):
        b = self._view_bufs(cam, cfg)
        L.gs_project(self.means, self.log_scales, self.quats, self.opacity, self.sh, cam, cfg,
                     b["splats"], b["depth"], b["rect"])
        return b

    def bin_sort(self, cam: dict, cfg: dict, b: dict | None = None) -> int:
        b = b or self._view_bufs(cam, cfg)
        if b["capacity"] == 0:
            self._ensure_capacity(b, cam, cfg, 4 * self.n + 1024)
        self._apply_shrink(b, cam, cfg)
        try:
            k = L.gs_bin_sort(self.n, b["depth"], b["rect"], cam, cfg, b["capacity"], b["ids"],
                              b["ranges"], b["workspace"])
        except L.GsError as e:
            if e.status != L.GS_ERR_CAPACITY or e.n_pairs is None or e.n_pairs >= 2 ** 31:
                raise
            self._ensure_capacity(b, cam, cfg, int(e.n_pairs * 1.25) + 1024)
            k = L.gs_bin_sort(self.n, b["depth"], b["rect"], cam, cfg, b["capacity"], b["ids"],
                              b["ranges"], b["workspace"])
        b["n_pairs"] = k
        # the pair passes size their grids by the capacity: bring it near the
        # count (25 % headroom) before the next sort, not now (b["ids"] holds
        # this sort's lists); pairs_fit grows it again when a frame overflows
        if b["capacity"] > 2 * k + 4096:
            b["shrink_to"] = int(k * 1.25) + 1024
        return k

    def _apply_shrink(self, b: dict, cam: dict, cfg: dict):
        cap = b.pop("shrink_to", None)
        if cap is not None and cap < b["capacity"]:
            self._ensure_capacity(b, cam, cfg, cap, shrink=True)

    def bin_sort_async(self, cam: dict, cfg: dict, b: dict | None = None) -> None:
        """gs_bin_sort_async: no wait; the pair count lands in b["n_pairs_dev"].
        Call :meth:`pairs_fit` once the stream has run to see whether the
        frame fitted the buffers."""
        b = b or self._view_bufs(cam, cfg)
        if b["capacity"] == 0:
            self._ensure_capacity(b, cam, cfg, 4 * self.n + 1024)
        self._apply_shrink(b, cam, cfg)
        if "n_pairs_dev" not in b:
            b["n_pairs_dev"] = torch.zeros(1, dtype=torch.int64, device=self.device)
        L.gs_bin_sort_async(self.n, b["depth"], b["rect"], cam, cfg, b["capacity"], b["ids"],
                            b["ranges"], b["n_pairs_dev"], b["workspace"])

    def pairs_fit(self, cam: dict, cfg: dict, b: dict | None = None) -> bool:
        """After gs_bin_sort_async (waits for the stream): True if the pairs fitted;
        otherwise grows the buffers for the next frame and returns False."""
        b = b or self._view_bufs(cam, cfg)
        k = L.check_pair_count(int(b["n_pairs_dev"].item()))
        b["n_pairs"] = k
        if k <= b["capacity"]:
            if b["capacity"] > 2 * k + 4096:
                b["shrink_to"] = int(k * 1.25) + 1024  # applied before the next sort
            return True
        if k >= 2 ** 31:
            raise L.GsError(L.GS_ERR_CAPACITY, f"{k} pairs exceed the 2^31 index limit", k)
        self._ensure_capacity(b, cam, cfg, int(k * 1.25) + 1024)
        return False

    def raster(self, cam: dict, cfg: dict, want_grads: bool = True, out=None, n_blend=None, b=None):
        b = b or self._view_bufs(cam, cfg)
        C = 12 if want_grads else 3
        if out is None:
            out = torch.empty((cam["height"], cam["width"], C), dtype=torch.float32, device=self.device)
        L.gs_raster_grad(b["splats"], b["ids"], b["ranges"], cam, cfg, want_grads, out, n_blend)
        return out

    def render(self, cam: dict, cfg: dict, want_grads: bool = True, out=None, n_blend=None):
        """Low-res colour [H, W, 12] with derivatives (or [H, W, 3] plain)."""
        b = self.project(cam, cfg)
        self.bin_sort(cam, cfg, b)
        return self.raster(cam, cfg, want_grads, out, n_blend, b)

    def render_counts(self, cam: dict, cfg: dict, want_grads: bool, out, n_eval, n_blend):
        """render() through gs_raster_fragment_counts: also the evaluated and
        blended fragments per pixel (int32 [H, W] each)."""
        b = self.project(cam, cfg)
        self.bin_sort(cam, cfg, b)
        L.gs_raster_fragment_counts(b["splats"], b["ids"], b["ranges"], [cam], cfg, want_grads, out, n_eval,
                                    n_blend)
        return out

    @staticmethod
    def upscale(lowres: torch.Tensor, W: int, H: int, out=None):
        if out is None:
            out = torch.empty((H, W, 3), dtype=torch.float32, device=lowres.device)
        L.gs_upscale_hermite(lowres, out)
        return out

    def render_upscaled(self, cam: dict, cfg: dict, W: int, H: int, lowres=None, out=None):
        low = self.render(cam, cfg, True, lowres)
        return self.upscale(low, W, H, out), low


class FramePipeline:
    """Frames in flight on streams of their own.

    One frame is a chain of dependent launches (projection, the depth and tile
    sort passes with their scans, the pair emission, the raster, the
    upscale), and several of them launch far fewer workgroups than the chip
    holds or wait on a single-block scan, so a lone frame leaves compute units
    idle under and between them.  Slot i renders on stream i with buffers of
    its own, so the next frame's projection and sort fill what this frame's
    raster and scans leave.

    ``slots`` is a :class:`Renderer`, to which the pipeline adds ``depth - 1``
    siblings (own pair lists, workspace and counters; the scene tensors are
    shared), or a list of objects that each hold one frame's buffers, such
    as :class:`~paper_2503_14171_amd.batch.ViewBatch` instances over the same
    scene and cameras.

    :meth:`submit` makes the slot's stream wait for the caller's current
    stream first, so inputs written there are seen; :meth:`join` makes the
    caller's stream wait for every slot.  Frames in flight at the same time
    need distinct output buffers, and a buffer a slot writes may be freed or
    reused on another stream only after :meth:`join`.
    """

    def __init__(self, slots, depth: int = 2):
        if isinstance(slots, Renderer):
            if depth < 1:
                raise ValueError("a pipeline needs at least one slot")
            slots = [slots] + [slots.sibling() for _ in range(depth - 1)]
        self.slots = list(slots)
        if not self.slots:
            raise ValueError("a pipeline needs at least one slot")
        self.streams = [torch.cuda.Stream() for _ in self.slots]  # default priority
        self._next = 0

    @property
    def depth(self) -> int:
        return len(self.slots)

    @property
    def next_slot(self) -> int:
        """The slot the next submit() runs on (to pick its output buffers)."""
        return self._next

    def submit(self, frame) -> int:
        """Call ``frame(slot)`` with the next slot's stream current (its
        launches go there); returns the slot index."""
        i = self._next
        self._next = (i + 1) % len(self.slots)
        s = self.streams[i]
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            frame(self.slots[i])
        return i

    def join(self) -> None:
        cur = torch.cuda.current_stream()
        for s in self.streams:
            cur.wait_stream(s)

    def pairs_fit(self, *view) -> bool:
        """join(), then True if every slot's last frame fitted its pairs; a
        slot that overflowed grows its buffers for its next frame.  Renderer
        slots take the view (``cam, cfg``) and check only the slots that
        sorted it; other slots are asked ``slot.pairs_fit(*view)``."""
        self.join()
        ok = True
        for r in self.slots:
            if isinstance(r, Renderer):
                cam, cfg = view
                b = r._bufs.get((cam["width"], cam["height"], cfg["tile_size"]))
                if b is not None and "n_pairs_dev" in b:
                    ok = r.pairs_fit(cam, cfg, b) and ok
            else:
                ok = r.pairs_fit(*view) and ok
        return ok

    def drop_view(self, cam: dict, cfg: dict) -> None:
        """Free every Renderer slot's buffers for this view size (after join())."""
        for r in self.slots:
            if isinstance(r, Renderer):
                r._bufs.pop((cam["width"], cam["height"], cfg["tile_size"]), None)
