"""Autotuner for the batched chain.

For one scene size and one set of views it times, on the GPU, the captured
graph of :class:`~paper_2503_14171_amd.batch.ViewBatch` for every tile size
(8, 16, 32, 64) and LDS batch (tile^2, tile^2/2, tile^2/4), then the upscale band
height (4, 8, 16, 32 output rows per workgroup) for the best of those, and
keeps the fastest setting.  With ``inflight`` > 1 the settings within 3 % of
the fastest (at most three) are timed again the way they will run, that
many frames in flight on streams of their own, and the fastest there wins:
a near tie on one stream can turn either way with frames in flight.  None
of the settings changes the images (the tile size only through the FP32
rounding of tile-relative offsets); they change only the speed.  Results
are cached per (Gaussians, view sizes, SH degree, device, frames in flight).
"""
from __future__ import annotations

import torch

from .batch import ViewBatch
from .render import FramePipeline

_cache: dict = {}


def _time(vb: ViewBatch, reps: int) -> float:
    vb.capture()
    vb.render()                    # verified frame (grows the buffers if needed)
    for _ in range(2):
        vb.launch()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        vb.launch()
    e1.record()
    torch.cuda.synchronize()
    if not vb.pairs_fit():         # cannot happen after a verified frame with the same views
        raise RuntimeError("pair capacity changed while timing")
    return e0.elapsed_time(e1) / reps


def _time_inflight(make, depth: int, reps: int) -> float:
    """ms per frame of `depth` batches (each its own buffers and graph)
    replayed in flight on streams of their own."""
    vbs = [make() for _ in range(depth)]
    for vb in vbs:
        vb.capture()
        vb.render()
    pipe = FramePipeline(vbs)
    for _ in range(2 * depth):
        pipe.submit(lambda vb: vb.launch())
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps * depth):
        pipe.submit(lambda vb: vb.launch())
    pipe.join()
    e1.record()
    torch.cuda.synchronize()
    if not pipe.pairs_fit():
        raise RuntimeError("pair capacity changed while timing")
    return e0.elapsed_time(e1) / (reps * depth)


def tune(renderer, cams, hi_sizes, cfg: dict, tiles=(8, 16, 32, 64), batch_divs=(1, 2, 4),
         band_rows=(4, 8, 16, 32), reps: int = 10, log=None, direct: bool = False,
         inflight: int = 1) -> dict:
    """Fastest (tile_size, batch, band_rows) for these views; returns a dict
    with the setting, its ms per frame and every trial.  ``direct`` tunes the
    direct high-res baseline instead (no band height); ``inflight`` > 1
    settles near ties with that many frames in flight."""
    key = (renderer.n, tuple((c["width"], c["height"]) for c in cams), tuple(map(tuple, hi_sizes)),
           cfg["sh_degree"], torch.cuda.current_device(), bool(direct), int(inflight))
    if key in _cache:
        return _cache[key]
    trials = []
    capacity = None  # each setting starts from the default capacity and grows as needed
    best = None
    for tile in tiles:
        for div in batch_divs:
            c = dict(cfg, tile_size=tile, batch=tile * tile // div)
            vb = ViewBatch(renderer, cams, hi_sizes, c, band_rows=8, capacity=capacity, direct=direct)
            ms = _time(vb, reps)
            trials.append(dict(tile_size=tile, batch=c["batch"], band_rows=8, ms=ms))
            if log:
                log(trials[-1])
            if best is None or ms < best[0]:
                best = (ms, c)
            del vb
    if inflight > 1:
        near = sorted((t for t in trials if t["ms"] <= 1.03 * best[0]), key=lambda t: t["ms"])[:3]
        if len(near) > 1:
            best = None
            for t in near:
                c = dict(cfg, tile_size=t["tile_size"], batch=t["batch"])
                ms = _time_inflight(lambda: ViewBatch(renderer, cams, hi_sizes, c, band_rows=8,
                                                      direct=direct), inflight, reps)
                trials.append(dict(tile_size=t["tile_size"], batch=t["batch"], band_rows=8, ms=ms,
                                   inflight=inflight))
                if log:
                    log(trials[-1])
                if best is None or ms < best[0]:
                    best = (ms, c)
            torch.cuda.synchronize()
    ms0, c = best
    rows_best = (ms0, 8)
    for rows in () if direct else band_rows:
        if rows == 8:
            continue
        vb = ViewBatch(renderer, cams, hi_sizes, c, band_rows=rows)
        ms = _time(vb, reps)
        trials.append(dict(tile_size=c["tile_size"], batch=c["batch"], band_rows=rows, ms=ms))
        if log:
            log(trials[-1])
        if ms < rows_best[0]:
            rows_best = (ms, rows)
        del vb
    res = dict(tile_size=c["tile_size"], batch=c["batch"], band_rows=rows_best[1], ms=rows_best[0],
               trials=trials)
    _cache[key] = res
    return res
