"""Benchmark of the gradient-aware upscaling hot path on one MI355X.

A step is one pass of the whole path over one camera view of a synthetic
scene whose inputs already sit in HBM: gs_project -> gs_bin_sort ->
gs_raster_grad (colour + dI/dx, dI/dy, d2I/dxdy) -> gs_upscale_hermite.
The default workload is the 3M-Gaussian scene (SH degree 3) rendered at
960x540 and upscaled x4 to 3840x2160.  Throughput is high-res output
megapixels per second with four frames in flight (--inflight; the process
gets eight hardware queues, --hw-queues), each on a stream and a set of
buffers of its own; the same frames one at a time give the per-frame
latency, reported beside it.

Beside it the script measures, on the same GPU and with the same number of
frames in flight, the direct full-resolution render (gs_project +
gs_bin_sort + plain gs_raster_grad at 3840x2160), the PSNR of the upscaled
image against it, per-stage HIP-event times on each frame's stream, the
raster kernel's arithmetic roofline and the upscaler's HBM roofline (with a
plain device copy of the same bytes as a reference), both paths from 8 orbit
cameras, and the FP64 CPU oracle on a bounded sample of the same frame plus,
on one thread, the whole tiny frame (rank 0, N = 1).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload scene_x4] [--inflight 4]
                       [--hw-queues 8]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

METRIC = "upscaled output Mpix/s vs direct full-res raster (same GPU) at PSNR gap; BW %"
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
FP32_VALU_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2 (FMA), no packed FP32
VALU_TOPS = 39.32           # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz: VALU lane-operations per second
# FP32 operations of the method per blended fragment (FMA = 2), grad and plain
FLOP_PER_BLEND = {True: 64, False: 25}
# VALU lane-op slots of the rasterizer's work (an exp counts 4 slots): per
# evaluated fragment (offset, quadratic form, support test) and per blended
# fragment on top of that (alpha, its derivatives, the blend), grad / plain
SLOTS_EVAL = 16
SLOTS_BLEND = {True: 35, False: 8}
# Projection bytes per Gaussian: parameters read (means, log-scales,
# quaternion, opacity: 44 B, plus 12 B per SH coefficient) and ~44 B written
PROJ_BYTES_PARAMS, PROJ_BYTES_OUT = 44, 44
# Bin/sort floor per (tile, splat) pair: the pair written once and read once
# (8-byte key/value each way) plus the 4-byte id written and read
BINSORT_BYTES_PER_PAIR = 24
# Bytes the upscaler must move: 48 per low-res pixel read, 12 per output pixel written
UPSCALE_BYTES_LO, UPSCALE_BYTES_HI = 48, 12

PROFILES = os.path.join(ROOT, "profiles", "traffic.json")


def measured_traffic(kernel: str):
    """HBM bytes per dispatch of `kernel` from the committed counter profile,
    or None when one of the kernel's source files has changed since it was
    taken."""
    import hashlib
    try:
        rec = json.load(open(PROFILES))[kernel]
        h = hashlib.sha256()
        for src in rec["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
    except (OSError, KeyError, ValueError):
        return None
    if h.hexdigest() != rec["sha256"]:
        return None
    return int(1024 * (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]))


WORKLOADS = {  # (scene, x factor, y factor); fractional and per-axis factors use the same mapping
    "scene_x4": ("scene", 4, 4), "scene_x3": ("scene", 3, 3), "scene_x2": ("scene", 2, 2),
    "scene_x2.5": ("scene", 2.5, 2.5), "scene_x1.5": ("scene", 1.5, 1.5),
    "scene_x4_x3": ("scene", 4, 3),
    "clusters_x2": ("clusters", 2, 2), "tiny_x2": ("tiny", 2, 2),
    # 1M Gaussians, 8 stereo pairs: 4 at 720x800 -> 1440x1600, 4 at 480x540 -> 1440x1620
    "stereo16": ("batch", None, None),
    # training step: 1M Gaussians, 4 views 480x270 -> 1920x1080, forward + L1 loss + backward
    "train4": ("train", None, None),
}


def _psnr(a, b):
    mse = ((a - b) ** 2).mean().item()
    return 10 * math.log10(1.0 / mse) if mse > 0 else float("inf")


def _events(torch, n):
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def run_gpu(args):
    import torch

    from paper_2503_14171_amd import scenes
    from paper_2503_14171_amd.render import FramePipeline, Renderer

    name, sx, sy = WORKLOADS[args.workload]
    sc = scenes.workload_scene(name)
    cam = scenes.workload_camera(name)
    # a far plane at the scene's depth bound (it culls nothing) tells the
    # depth sort how many digit passes the key range needs
    cam["far_plane"] = scenes.depth_bound(sc, cam)
    cfg = scenes.render_config(sc["sh_degree"], tile_size=args.tile)
    w, h = cam["width"], cam["height"]
    W, H = round(w * sx), round(h * sy)
    s = sx if sx == sy else [sx, sy]
    cam_hi = scenes.scale_camera(cam, W, H)
    torch.cuda.set_device(0)
    rd = Renderer(sc)
    depth = args.inflight

    # Rotating output sets (> 512 MB in total) so that the 256 MB MALL does
    # not absorb the upscaler's reads and writes between steps; slot i of the
    # pipeline only ever uses sets i, i + depth, i + 2 depth, ...
    set_bytes = (w * h * 12 + W * H * 3) * 4
    per_slot = math.ceil(max(2, math.ceil(640e6 / set_bytes)) / depth)
    nsets = per_slot * depth
    lows = [torch.empty((h, w, 12), dtype=torch.float32, device="cuda") for _ in range(nsets)]
    ups = [torch.empty((H, W, 3), dtype=torch.float32, device="cuda") for _ in range(nsets)]

    def frames(d, steps, warmup, with_events, cam=cam):
        """Times `steps` upscaled frames of `cam` with `d` in flight;
        per-stage events on each frame's own stream."""
        pipe = FramePipeline(rd, d)
        used = [0] * d
        last = [0]

        def step(ev=None):
            i = pipe.next_slot
            j = i + d * (used[i] % (nsets // d))
            used[i] += 1
            last[0] = j
            lo, up = lows[j], ups[j]

            def frame(r):
                if ev:
                    ev[0].record()
                b = r.project(cam, cfg)
                if ev:
                    ev[1].record()
                r.bin_sort_async(cam, cfg, b)
                if ev:
                    ev[2].record()
                r.raster(cam, cfg, True, lo, b=b)
                if ev:
                    ev[3].record()
                r.upscale(lo, W, H, up)
                if ev:
                    ev[4].record()
            pipe.submit(frame)

        # pair counts stay on the device: run until every slot's frame fits
        # its buffers, then once more so that capacity changes have landed
        while True:
            for _ in range(d):
                step()
            if pipe.pairs_fit(cam, cfg):
                break
        for _ in range(d + warmup):
            step()
        torch.cuda.synchronize()
        evs = [_events(torch, 5) for _ in range(steps)] if with_events else [None] * steps
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            step(evs[k])
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        assert pipe.pairs_fit(cam, cfg), "pair count changed during the timed frames"
        st = None
        if with_events:
            st = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(4)] for e in evs]).mean(0)
        return ms, st, last[0]

    # the timed frames record no events: an event between two kernels of a
    # stream holds the next kernel back until the previous one has drained
    # (about 5 us per event on MI355X); the stage times come from a second
    # pass of the same frames with events between the stages
    ms_step = frames(depth, args.steps, args.warmup, False)[0]
    st_ms = frames(depth, args.steps, args.warmup, True)[1]
    # one frame at a time: the latency of a frame, and the stages with the GPU
    # to themselves
    # (the output sets then hold that pass's frames: last_set is its last one)
    ms_serial, st_serial = ms_step, st_ms
    if depth > 1:
        ms_serial = frames(1, args.steps, args.warmup, False)[0]
    st_serial, last_set = (lambda r: (r[1], r[2]))(frames(1, args.steps, args.warmup, True))
    # the upscaler's own launch duration: back-to-back launches over the
    # rotating buffer sets between two events on the launch stream
    ue = _events(torch, 2)
    nup = 4 * nsets
    ue[0].record()
    for k in range(nup):
        rd.upscale(lows[k % nsets], W, H, ups[k % nsets])
    ue[1].record()
    torch.cuda.synchronize()
    up_launch_ms = ue[0].elapsed_time(ue[1]) / nup
    # a plain device copy moving the upscaler's bytes (62.2 MB read + 62.2 MB
    # written), back to back over 4 buffer pairs (> 256 MB MALL): the
    # bandwidth a streaming kernel reaches on this GPU
    cbytes = (w * h * UPSCALE_BYTES_LO + W * H * UPSCALE_BYTES_HI) // 2
    csrc = [torch.empty(cbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0) for _ in range(4)]
    cdst = [torch.empty_like(c) for c in csrc]
    for k in range(4):
        cdst[k].copy_(csrc[k])
    ce = _events(torch, 2)
    ce[0].record()
    for k in range(16):
        cdst[k % 4].copy_(csrc[k % 4])
    ce[1].record()
    torch.cuda.synchronize()
    copy_gbs = 2 * cbytes / (ce[0].elapsed_time(ce[1]) / 16 * 1e-3) / 1e9
    del csrc, cdst

    # direct full-resolution render (plain compositing) on the same GPU, with
    # the same number of frames in flight, at the frame's own tile size and at
    # the other tile sizes; the best one is the baseline the speed-up is
    # quoted against
    direct_outs = [torch.empty((H, W, 3), dtype=torch.float32, device="cuda") for _ in range(depth)]

    def time_direct(tile, d, cam_hi=cam_hi, steps=args.steps):
        cfg_d = dict(cfg, tile_size=tile)
        pipe = FramePipeline(rd, d)

        def direct_step(ev=None):
            out = direct_outs[pipe.next_slot]

            def frame(r):
                if ev:
                    ev[0].record()
                b = r.project(cam_hi, cfg_d)
                if ev:
                    ev[1].record()
                r.bin_sort_async(cam_hi, cfg_d, b)
                if ev:
                    ev[2].record()
                r.raster(cam_hi, cfg_d, False, out, b=b)
                if ev:
                    ev[3].record()
            pipe.submit(frame)

        while True:
            for _ in range(d):
                direct_step()
            if pipe.pairs_fit(cam_hi, cfg_d):
                break
        for _ in range(d + max(1, args.warmup)):
            direct_step()
        torch.cuda.synchronize()
        # timed without events (as the upscaled frames), then the stages of
        # the same frames with events between them
        t0 = time.perf_counter()
        for k in range(steps):
            direct_step()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        devs = [_events(torch, 4) for _ in range(steps)]
        for k in range(steps):
            direct_step(devs[k])
        torch.cuda.synchronize()
        assert pipe.pairs_fit(cam_hi, cfg_d)
        st = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(3)] for e in devs]).mean(0)
        if tile != cfg["tile_size"]:
            pipe.drop_view(cam_hi, cfg_d)  # free this tile size's buffers
        else:
            for r in pipe.slots[1:]:
                r._bufs.clear()
        return ms, st

    direct_all = {}
    for tile in sorted({args.tile, 16, 32, 64}):
        direct_all[tile] = time_direct(tile, depth)
    best_tile = min(direct_all, key=lambda t: direct_all[t][0])
    ms_direct, dstage = direct_all[args.tile]
    ms_direct_serial = time_direct(args.tile, 1)[0] if depth > 1 else ms_direct
    torch.cuda.synchronize()
    direct_out = direct_outs[0]
    rd.render(cam_hi, cfg, False, direct_out)  # the reference image for PSNR

    # quality of the upscaled frame against the direct render
    up = ups[last_set].clamp(0, 1)
    ref = direct_out.clamp(0, 1)
    psnr = _psnr(up, ref)

    # comparators on the same low-res colour: classical bicubic (finite-
    # difference slopes through the same Hermite kernel = Catmull-Rom) and
    # torch's bicubic (Keys a = -3/4); quality only, plus the slope kernel's time
    from paper_2503_14171_amd import _lib
    lo_last = lows[last_set]
    rgb_lo = lo_last[..., :3].contiguous()
    fd_in = torch.empty((h, w, 12), dtype=torch.float32, device="cuda")
    fd_up = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    fev = _events(torch, 3)
    _lib.gs_fd_slopes(rgb_lo, fd_in)
    fev[0].record()
    for _ in range(10):
        _lib.gs_fd_slopes(rgb_lo, fd_in)
    fev[1].record()
    for _ in range(10):
        rd.upscale(fd_in, W, H, fd_up)
    fev[2].record()
    torch.cuda.synchronize()
    psnr_fd = _psnr(fd_up.clamp(0, 1), ref)
    tb = torch.nn.functional.interpolate(rgb_lo.permute(2, 0, 1)[None], size=(H, W), mode="bicubic",
                                         align_corners=False)[0].permute(1, 2, 0)
    psnr_torch = _psnr(tb.clamp(0, 1), ref)
    del tb, fd_up
    comparators = dict(psnr_fd_bicubic=psnr_fd, psnr_torch_bicubic=psnr_torch,
                       fd_slopes_ms=fev[0].elapsed_time(fev[1]) / 10,
                       fd_upscale_ms=fev[1].elapsed_time(fev[2]) / 10)

    # algorithmic work of the raster launch: evaluated and blended fragments
    # per pixel (one extra, untimed launch with the per-pixel counters)
    nev = torch.empty((h, w), dtype=torch.int32, device="cuda")
    nbl = torch.empty((h, w), dtype=torch.int32, device="cuda")
    rd.render_counts(cam, cfg, True, lows[0], nev, nbl)
    evals, frags = int(nev.sum().item()), int(nbl.sum().item())
    nev_hi = torch.empty((H, W), dtype=torch.int32, device="cuda")
    nbl_hi = torch.empty((H, W), dtype=torch.int32, device="cuda")
    direct_ref = torch.empty_like(direct_out)
    rd.render_counts(cam_hi, cfg, False, direct_ref, nev_hi, nbl_hi)
    evals_hi, frags_hi = int(nev_hi.sum().item()), int(nbl_hi.sum().item())
    del nev_hi, nbl_hi, direct_ref
    pairs = rd._bufs[(w, h, cfg["tile_size"])]["n_pairs"]
    pairs_hi = rd._bufs[(W, H, cfg["tile_size"])]["n_pairs"]

    ras_ms = st_ms[2]
    ops = SLOTS_EVAL * evals + SLOTS_BLEND[True] * frags
    achieved = ops / (ras_ms * 1e-3) / 1e12
    achieved_serial = ops / (st_serial[2] * 1e-3) / 1e12
    flops_serial = frags * FLOP_PER_BLEND[True] / (st_serial[2] * 1e-3) / 1e12
    proj_bytes = rd.n * (PROJ_BYTES_PARAMS + 12 * (cfg["sh_degree"] + 1) ** 2 + PROJ_BYTES_OUT)
    sort_bytes = BINSORT_BYTES_PER_PAIR * pairs
    up_bytes = w * h * UPSCALE_BYTES_LO + W * H * UPSCALE_BYTES_HI
    up_gbs = up_bytes / (st_ms[3] * 1e-3) / 1e9
    up_gbs_launch = up_bytes / (up_launch_ms * 1e-3) / 1e9
    value = W * H / (ms_step * 1e-3) / 1e6
    direct_value = W * H / (ms_direct * 1e-3) / 1e6
    # the same scene from 8 orbit cameras (radius 3, azimuth k x 45 deg,
    # elevation 15 deg), as the paper averages over test cameras: upscaled
    # frames and the direct render at list tiles 32 and 64 (the better one),
    # same frames in flight; last, since it reuses the frame's buffers
    orbit = None
    if not args.no_orbit:
        # 30 frames per camera: with frames in flight, filling and draining
        # the pipeline weighs more on the shorter upscaled frames
        n_o = max(3, min(args.steps, 30))
        per = []
        for k in range(8):
            cam_o = scenes.orbit_camera(w, h, 45.0 * k, 15.0)
            cam_o["far_plane"] = scenes.depth_bound(sc, cam_o)
            cam_oh = scenes.scale_camera(cam_o, W, H)
            ms_up = frames(depth, n_o, 2, False, cam_o)[0]
            ms_d = min(time_direct(t, depth, cam_oh, n_o)[0] for t in (32, 64))
            per.append((ms_up, ms_d))
        ups_ms = np.array([p[0] for p in per])
        dir_ms = np.array([p[1] for p in per])
        orbit = dict(ms=ups_ms, direct_ms=dir_ms, steps=n_o)

    best = dict(tile=best_tile, ms_per_frame=direct_all[best_tile][0],
                value=W * H / (direct_all[best_tile][0] * 1e-3) / 1e6,
                by_tile={t: round(v[0], 4) for t, v in direct_all.items()})
    return dict(best_direct=best, comparators=comparators, orbit=orbit,
        name=name, s=s, w=w, h=h, W=W, H=H, n=rd.n, cfg=cfg, value=value, ms_step=ms_step,
        stages_ms=dict(project=st_ms[0], bin_sort=st_ms[1], raster_grad=st_ms[2], upscale=st_ms[3]),
        inflight=depth, ms_serial=ms_serial, ms_direct_serial=ms_direct_serial,
        stages_serial=dict(project=st_serial[0], bin_sort=st_serial[1], raster_grad=st_serial[2],
                           upscale=st_serial[3]), achieved_serial=achieved_serial,
        direct=dict(value=direct_value, ms_per_frame=ms_direct,
                    stages_ms=dict(project=dstage[0], bin_sort=dstage[1], raster_plain=dstage[2]),
                    pairs=pairs_hi, blended_fragments=frags_hi, evaluated_fragments=evals_hi),
        psnr=psnr, frags=frags, evals=evals, pairs=pairs, achieved_tops=achieved,
        flops_serial=flops_serial, proj_bytes=proj_bytes, sort_bytes=sort_bytes, up_gbs=up_gbs,
        up_gbs_launch=up_gbs_launch, up_launch_ms=up_launch_ms, copy_gbs=copy_gbs,
        up_bytes=up_bytes, scene=sc, cam=cam)


def run_batch(args):
    """The batched stereo workload: autotuned setting, one captured graph per
    frame for all 16 views, --inflight frames in flight; the direct baseline
    renders the 16 views at their high-res sizes, also batched,
    graph-captured, tuned and with the same number of frames in flight."""
    import torch

    from paper_2503_14171_amd import _lib as L
    from paper_2503_14171_amd import autotune, scenes
    from paper_2503_14171_amd.batch import ViewBatch
    from paper_2503_14171_amd.render import FramePipeline, Renderer

    torch.cuda.set_device(0)
    sc = scenes.workload_scene("batch")
    cams, hi = scenes.stereo_rig()
    cfg0 = scenes.render_config(sc["sh_degree"])
    rd = Renderer(sc)
    t0 = time.perf_counter()
    # near ties on one stream are settled with the benchmark's frames in flight
    tuned = autotune.tune(rd, cams, hi, cfg0, reps=5, inflight=args.inflight)
    tuned_d = autotune.tune(rd, cams, hi, cfg0, reps=3, direct=True, tiles=(16, 32, 64), batch_divs=(1, 2),
                            inflight=args.inflight)
    tune_s = time.perf_counter() - t0
    cfg = dict(cfg0, tile_size=tuned["tile_size"], batch=tuned["batch"])
    cfg_d = dict(cfg0, tile_size=tuned_d["tile_size"], batch=tuned_d["batch"])

    def timed(make, steps, warmup):
        """`steps` frames with args.inflight batches in flight (each its own
        buffers, graph and stream); returns (ms per frame, the batches)."""
        vbs = [make() for _ in range(args.inflight)]
        for vb in vbs:
            vb.capture()
            vb.render()
        pipe = FramePipeline(vbs)
        for _ in range(max(warmup, 1) * len(vbs)):
            pipe.submit(lambda vb: vb.launch())
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            pipe.submit(lambda vb: vb.launch())
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t) / steps
        assert pipe.pairs_fit()
        return ms, vbs

    ms, vbs = timed(lambda: ViewBatch(rd, cams, hi, cfg, band_rows=tuned["band_rows"]), args.steps, args.warmup)
    vb = vbs[0]
    del vbs
    # per-stage times of the same chain, eager, with events between the calls
    r = rd
    ev = _events(torch, 5)
    nrep = 5
    acc = np.zeros(4)
    for _ in range(nrep):
        ev[0].record()
        L.gs_project_views(r.means, r.log_scales, r.quats, r.opacity, r.sh, vb.cams, vb.cfg, vb.splats,
                           vb.depth, vb.rect)
        ev[1].record()
        L.gs_bin_sort_views(r.n, vb.cams, vb.cfg, vb.depth, vb.rect, vb.capacity, vb.ids, vb.ranges,
                            vb.n_pairs, vb.workspace)
        ev[2].record()
        L.gs_raster_grad_views(vb.splats, vb.ids, vb.ranges, vb.cams, vb.cfg, True, vb.low)
        ev[3].record()
        L.gs_upscale_hermite_views(vb.low, vb.lo, vb.up, vb.hi, vb.band_rows)
        ev[4].record()
        torch.cuda.synchronize()
        acc += [ev[i].elapsed_time(ev[i + 1]) for i in range(4)]
    st = acc / nrep
    nbl = torch.empty(sum(vb.lo_px), dtype=torch.int32, device="cuda")
    nev = torch.empty_like(nbl)
    L.gs_raster_fragment_counts(vb.splats, vb.ids, vb.ranges, vb.cams, vb.cfg, True, vb.low, nev, nbl)
    frags, evals = int(nbl.sum().item()), int(nev.sum().item())
    pairs = int(vb.n_pairs.item())
    up_imgs = [u.clone() for u in vb.views()[1]]
    del vb, nbl, nev
    ms_d, vds = timed(lambda: ViewBatch(rd, cams, hi, cfg_d, direct=True), max(3, args.steps // 2), 1)
    vd = vds[0]
    del vds
    psnrs = [_psnr(u.clamp(0, 1), d.clamp(0, 1)) for u, d in zip(up_imgs, vd.views()[1])]
    pairs_d = int(vd.n_pairs.item())
    del vd
    out_px = sum(W * H for (W, H) in hi)
    lo_px = sum(c["width"] * c["height"] for c in cams)
    up_bytes = lo_px * UPSCALE_BYTES_LO + out_px * UPSCALE_BYTES_HI
    return dict(name="batch", n=rd.n, cams=cams, hi=hi, cfg=cfg, tuned=tuned, tuned_direct=tuned_d,
                tune_s=tune_s, ms_step=ms, value=out_px / (ms * 1e-3) / 1e6,
                stages_ms=dict(project=st[0], bin_sort=st[1], raster_grad=st[2], upscale=st[3]),
                direct=dict(value=out_px / (ms_d * 1e-3) / 1e6, ms_per_frame=ms_d, pairs=pairs_d),
                psnr=float(np.mean(psnrs)), psnr_min=float(np.min(psnrs)), frags=frags, evals=evals,
                pairs=pairs,
                achieved_tops=(SLOTS_EVAL * evals + SLOTS_BLEND[True] * frags) / (st[2] * 1e-3) / 1e12,
                up_gbs=up_bytes / (st[3] * 1e-3) / 1e9, up_bytes=up_bytes, out_px=out_px)


def run_train(args):
    """One training step per timed iteration: the differentiable chain's
    forward, an L1 loss against direct 1080p renders of a perturbed copy of
    the scene (means + N(0, 0.01)), and the hand-written backward to every
    Gaussian parameter."""
    import torch

    from paper_2503_14171_amd import _lib as L
    from paper_2503_14171_amd import scenes
    from paper_2503_14171_amd.batch import ViewBatch
    from paper_2503_14171_amd.render import Renderer
    from paper_2503_14171_amd.train import TrainViews, UpscaledRender

    torch.cuda.set_device(0)
    sc = scenes.workload_scene("batch")
    rng = np.random.default_rng(5)
    cams = [scenes.orbit_camera(480, 270, a, e) for a, e in ((0.0, 5.0), (60.0, -10.0), (150.0, 15.0),
                                                             (250.0, -5.0))]
    hi = [(1920, 1080)] * 4
    cfg = scenes.render_config(sc["sh_degree"])
    pert = dict(sc, means=(sc["means"] + rng.normal(0, 0.01, sc["means"].shape)).astype(np.float32))
    tgt = ViewBatch(Renderer(pert), cams, hi, cfg, direct=True)
    tgt.render()
    target = tgt.up.clone()
    del tgt
    rd = Renderer(sc)
    params = {k: getattr(rd, k).clone().requires_grad_(True) for k in
              ("means", "log_scales", "quats", "opacity", "sh")}
    tv = TrainViews(rd.n, cams, hi, cfg)

    def step():
        for p_ in params.values():
            p_.grad = None
        up = UpscaledRender.apply(params["means"], params["log_scales"], params["quats"],
                                  params["opacity"], params["sh"], tv)
        loss = (up - target).abs().mean()
        loss.backward()
        return loss

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss = step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    # stage times of one step, eager with events
    r = {k: v.detach() for k, v in params.items()}
    ev = _events(torch, 8)
    ev[0].record()
    L.gs_project_views(r["means"], r["log_scales"], r["quats"], r["opacity"], r["sh"], tv.cams, tv.cfg,
                       tv.splats, tv.depth, tv.rect)
    ev[1].record()
    L.gs_bin_sort_views(tv.n, tv.cams, tv.cfg, tv.depth, tv.rect, tv.capacity, tv.ids, tv.ranges,
                        tv.n_pairs, tv.workspace)
    ev[2].record()
    L.gs_raster_grad_views_train(tv.splats, tv.ids, tv.ranges, tv.cams, tv.cfg, tv.low, tv.state, tv.last)
    ev[3].record()
    up = torch.empty((tv.hi_px, 3), dtype=torch.float32, device="cuda")
    L.gs_upscale_hermite_views(tv.low, tv.lo, up, tv.hi)
    ev[4].record()
    d_up = torch.sign(up - target) / up.numel()
    ev[5].record()
    L.gs_upscale_hermite_backward_views(d_up, tv.lo, tv.d_low, tv.hi)
    ev[6].record()
    L.gs_raster_grad_backward_views(tv.splats, tv.ids, tv.ranges, tv.cams, tv.cfg, tv.state, tv.last,
                                    tv.d_low, tv.n, tv.d_splats)
    ev[7].record()
    g = [torch.empty_like(t) for t in r.values()]
    e8 = _events(torch, 2)
    e8[0].record()
    L.gs_project_backward_views(r["means"], r["log_scales"], r["quats"], r["opacity"], r["sh"], tv.cams,
                                tv.cfg, tv.d_splats, *g)
    e8[1].record()
    torch.cuda.synchronize()
    st = {"project": ev[0].elapsed_time(ev[1]), "bin_sort": ev[1].elapsed_time(ev[2]),
          "raster_grad_fwd": ev[2].elapsed_time(ev[3]), "upscale_fwd": ev[3].elapsed_time(ev[4]),
          "upscale_bwd": ev[5].elapsed_time(ev[6]), "raster_grad_bwd": ev[6].elapsed_time(ev[7]),
          "project_bwd": e8[0].elapsed_time(e8[1])}
    out_px = sum(W * H for (W, H) in hi)
    return dict(n=rd.n, ms=ms, loss=float(loss.item()), stages=st, out_px=out_px,
                value=out_px / (ms * 1e-3) / 1e6, pairs=int(tv.n_pairs.item()))


def train_line(args, res):
    return {
        "metric": METRIC, "value": round(res["value"], 2), "unit": "Mpix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(res["ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"training step: {res['n']} Gaussians, SH degree 3, 4 views 480x270 rendered "
                               "with gradients and upscaled x4 to 1920x1080, L1 loss against direct 1080p "
                               "renders of the scene with means + N(0, 0.01), backward to all parameters",
                   "gaussians": res["n"], "views": 4, "output_pixels": res["out_px"]},
        "stages_ms": {k: round(v, 4) for k, v in res["stages"].items()},
        "loss": round(res["loss"], 6), "pairs": res["pairs"],
    }


def batch_line(args, res):
    tuned = res["tuned"]
    return {
        "metric": METRIC,
        "value": round(res["value"], 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batch: {res['n']} Gaussians, SH degree 3, 8 stereo pairs (16 views): "
                               "4 pairs 720x800 -> 1440x1600 (x2), 4 pairs 480x540 -> 1440x1620 (x3); "
                               f"one HIP graph per frame, {args.inflight} frames in flight",
                   "gaussians": res["n"], "views": len(res["cams"]), "output_pixels": res["out_px"],
                   "frames_in_flight": args.inflight,
                   "tuned": {k: tuned[k] for k in ("tile_size", "batch", "band_rows")},
                   "tuned_direct": {k: res["tuned_direct"][k] for k in ("tile_size", "batch")}},
        "roofline": {"kernel": "gs_raster_grad_views", "bound": "alu",
                     "achieved": round(res["achieved_tops"], 3), "peak": VALU_TOPS,
                     "unit": "TOP/s (VALU lane-ops)",
                     "frac": round(res["achieved_tops"] / VALU_TOPS, 4), "traffic": None,
                     "units": (f"{SLOTS_EVAL} x {res['evals']} evaluated + {SLOTS_BLEND[True]} x "
                               f"{res['frags']} blended fragments")},
        "upscaler_roofline": {"kernel": "gs_upscale_hermite_views", "bound": "hbm",
                              "achieved": round(res["up_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(res["up_gbs"] / HBM_PEAK_GBS, 4), "bytes": res["up_bytes"],
                              "traffic": None},
        "stages_ms": {k: round(v, 4) for k, v in res["stages_ms"].items()},
        "direct": {"value": round(res["direct"]["value"], 2), "unit": "Mpix/s",
                   "ms_per_frame": round(res["direct"]["ms_per_frame"], 4)},
        "speedup_vs_direct": round(res["value"] / res["direct"]["value"], 3),
        "psnr_vs_direct_db": round(res["psnr"], 2),
        "psnr_vs_direct_min_db": round(res["psnr_min"], 2),
        "pairs": {"lowres": res["pairs"], "direct": res["direct"]["pairs"]},
        "autotune_s": round(res["tune_s"], 1),
        "autotune_trials": [{k: (round(v, 4) if k == "ms" else v) for k, v in t.items()}
                            for t in tuned["trials"]],
    }


def orbit_line(res, W, H):
    o = res["orbit"]
    if o is None:
        return None
    sp = o["direct_ms"] / o["ms"]
    return {"cameras": "orbit radius 3, azimuth 0, 45, ..., 315 deg, elevation 15 deg",
            "steps_per_camera": o["steps"],
            "ms_per_frame": [round(float(v), 4) for v in o["ms"]],
            "direct_best_ms_per_frame": [round(float(v), 4) for v in o["direct_ms"]],
            "median_value": round(float(W * H / (np.median(o["ms"]) * 1e-3) / 1e6), 2),
            "median_speedup_vs_best_direct": round(float(np.median(sp)), 3),
            "min_speedup_vs_best_direct": round(float(sp.min()), 3)}


def cpu_tiny_child():
    """Child process (OMP_NUM_THREADS=1, no GPU): the FP64 oracle on the whole
    tiny frame (10k Gaussians, 128x128 with derivatives, upscaled x2 to
    256x256); prints one JSON line."""
    from oracle import oracle
    from paper_2503_14171_amd import scenes
    sc = scenes.workload_scene("tiny")
    cam = scenes.workload_camera("tiny")
    cfg = scenes.render_config(sc["sh_degree"])
    W, H = 2 * cam["width"], 2 * cam["height"]
    t0 = time.perf_counter()
    img = oracle.render(sc, cam, cfg)["img"]
    oracle.upscale(img, W, H)
    t = time.perf_counter() - t0
    print(json.dumps({"seconds": t, "threads": oracle.num_threads(), "W": W, "H": H}), flush=True)


def cpu_single_thread_tiny():
    """The tiny frame on one host thread, in a CPU-only child process (the
    oracle's OpenMP runtime reads its thread count once per process)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-tiny-child"],
                       capture_output=True, text=True, env=env, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr.strip()[-300:]}
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return {"value": round(d["W"] * d["H"] / d["seconds"] / 1e6, 6), "unit": "Mpix/s",
            "cores": d["threads"], "seconds_per_frame": round(d["seconds"], 2),
            "workload": "tiny: 10k Gaussians, 128x128 with derivatives, upscaled x2 to 256x256, whole frame"}


def cpu_baseline(res, budget_s):
    """The FP64 oracle on a bounded sample of the same frame: projection and
    depth order of every Gaussian, compositing of a random sample of low-res
    pixels, patches of a sample of output pixels; scaled to the whole frame."""
    from oracle import oracle

    sc, cam, cfg = res["scene"], res["cam"], res["cfg"]
    w, h, W, H = res["w"], res["h"], res["W"], res["H"]
    t0 = time.perf_counter()
    proj = oracle.project(sc, cam, cfg)
    order = oracle.depth_order(proj)
    t_setup = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    npx, t_pix = 0, 0.0
    chunk = 16
    while t_pix < budget_s and npx < w * h:
        xs = rng.integers(0, w, chunk)
        ys = rng.integers(0, h, chunk)
        t1 = time.perf_counter()
        oracle.composite(proj, order, cfg, xs, ys)
        t_pix += time.perf_counter() - t1
        npx += chunk
    img = rng.standard_normal((h, w, 12))
    nup = 200000
    X = rng.integers(0, W, nup).astype(np.int32)
    Y = rng.integers(0, H, nup).astype(np.int32)
    t1 = time.perf_counter()
    oracle.upscale(img, W, H, X, Y)
    t_up = time.perf_counter() - t1
    t_frame = t_setup + t_pix * (w * h) / npx + t_up * (W * H) / nup
    return dict(value=W * H / t_frame / 1e6, unit="Mpix/s", cores=oracle.num_threads(), kind="oracle",
                sample=(f"projection + depth order of all {res['n']} Gaussians ({t_setup:.1f} s), "
                        f"{npx} random low-res pixels composited ({t_pix:.1f} s), {nup} output "
                        f"pixels upscaled ({t_up:.1f} s); frame time extrapolated to "
                        f"{w}x{h} -> {W}x{H} = {t_frame:.0f} s"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="scene_x4", choices=sorted(WORKLOADS))
    ap.add_argument("--tile", type=int, default=32)
    ap.add_argument("--inflight", type=int, default=4,
                    help="frames in flight on streams of their own (upscaled and direct paths alike)")
    ap.add_argument("--hw-queues", type=int, default=8,
                    help="hardware queues of the process (GPU_MAX_HW_QUEUES, set before HIP starts); "
                         "with HIP's default of four, four frames' streams and the default stream "
                         "share them")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle compositing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-orbit", action="store_true", help="skip the 8 orbit-camera timings")
    ap.add_argument("--cpu-tiny-child", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.cpu_tiny_child:
        cpu_tiny_child()
        return
    if not 1 <= args.hw_queues <= 16:
        raise SystemExit("--hw-queues must be in [1, 16]")
    os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)  # read when HIP starts (first GPU use)
    # before anything touches the GPU: the single-thread oracle run is a child process
    tiny_1t = None
    if not args.no_cpu_baseline and WORKLOADS[args.workload][0] not in ("batch", "train"):
        tiny_1t = cpu_single_thread_tiny()

    if WORKLOADS[args.workload][0] == "batch":
        res = run_batch(args)
        print(json.dumps(batch_line(args, res)), flush=True)
        return
    if WORKLOADS[args.workload][0] == "train":
        res = run_train(args)
        print(json.dumps(train_line(args, res)), flush=True)
        return
    res = run_gpu(args)
    name, s, w, h, W, H = (res[k] for k in ("name", "s", "w", "h", "W", "H"))
    line = {
        "metric": METRIC,
        "value": round(res["value"], 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{name}: {res['n']} Gaussians, SH degree {res['cfg']['sh_degree']}, "
                               f"{w}x{h} rendered with gradients, upscaled x{s} to {W}x{H}",
                   "gaussians": res["n"], "lowres": [w, h], "highres": [W, H], "scale": s,
                   "tile": args.tile, "frames_in_flight": res["inflight"]},
        # the kernel with the GPU to itself (one frame at a time, events on its
        # stream over the timed frames), as the upscaler's figure below; with
        # frames in flight the launch shares the GPU with other frames' kernels
        "roofline": {"kernel": "gs_raster_grad", "bound": "alu",
                     "achieved": round(res["achieved_serial"], 3), "peak": VALU_TOPS,
                     "unit": "TOP/s (VALU lane-ops)",
                     "frac": round(res["achieved_serial"] / VALU_TOPS, 4),
                     "traffic": measured_traffic("gs_raster_grad") if (args.workload, args.tile) == ("scene_x4", 32) else None,
                     "units": (f"{SLOTS_EVAL} x {res['evals']} evaluated + {SLOTS_BLEND[True]} x "
                               f"{res['frags']} blended fragments"),
                     "ms_per_launch": round(res["stages_serial"]["raster_grad"], 4),
                     "measured": "one frame at a time (the launch alone on the GPU)",
                     "flop_achieved_tflops": round(res["flops_serial"], 3),
                     "flop_frac": round(res["flops_serial"] / FP32_VALU_TFLOPS, 4),
                     "flop_units": f"{res['frags']} blended fragments x {FLOP_PER_BLEND[True]} FLOP "
                                   f"of {FP32_VALU_TFLOPS} TFLOP/s",
                     "in_flight_achieved": round(res["achieved_tops"], 3),
                     "in_flight_frac": round(res["achieved_tops"] / VALU_TOPS, 4),
                     "in_flight_ms_per_launch": round(res["stages_ms"]["raster_grad"], 4)},
        "stage_rooflines": {
            "project": {"bound": "hbm", "bytes": res["proj_bytes"],
                        "units": f"{res['n']} Gaussians x (params + SH read, splat written)",
                        "ms": round(res["stages_serial"]["project"], 4),
                        "achieved": round(res["proj_bytes"] / (res["stages_serial"]["project"] * 1e-3) / 1e9, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(res["proj_bytes"] / (res["stages_serial"]["project"] * 1e-3) / 1e9
                                      / HBM_PEAK_GBS, 4)},
            "bin_sort": {"bound": "hbm", "bytes": res["sort_bytes"],
                         "units": f"{res['pairs']} pairs x {BINSORT_BYTES_PER_PAIR} B",
                         "ms": round(res["stages_serial"]["bin_sort"], 4),
                         "achieved": round(res["sort_bytes"] / (res["stages_serial"]["bin_sort"] * 1e-3) / 1e9, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(res["sort_bytes"] / (res["stages_serial"]["bin_sort"] * 1e-3) / 1e9
                                       / HBM_PEAK_GBS, 4)},
            "measured": "one frame at a time, events on the frame's stream"},
        "upscaler_roofline": {"kernel": "gs_upscale_hermite", "bound": "hbm",
                              "achieved": round(res["up_gbs_launch"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(res["up_gbs_launch"] / HBM_PEAK_GBS, 4),
                              "us_per_launch": round(1e3 * res["up_launch_ms"], 2),
                              "in_frame_achieved": round(res["up_gbs"], 1),
                              "copy_gbs": round(res["copy_gbs"], 1),
                              "frac_of_copy": round(res["up_gbs_launch"] / res["copy_gbs"], 4),
                              "bytes": res["up_bytes"],
                              "traffic": measured_traffic("gs_upscale_hermite") if args.workload == "scene_x4" else None},
        "stages_ms": {k: round(v, 4) for k, v in res["stages_ms"].items()},
        "direct": {"value": round(res["direct"]["value"], 2), "unit": "Mpix/s",
                   "ms_per_frame": round(res["direct"]["ms_per_frame"], 4),
                   "stages_ms": {k: round(v, 4) for k, v in res["direct"]["stages_ms"].items()}},
        "speedup_vs_direct": round(res["value"] / res["direct"]["value"], 3),
        "one_in_flight": {"ms_per_frame": round(res["ms_serial"], 4),
                          "value": round(W * H / (res["ms_serial"] * 1e-3) / 1e6, 2),
                          "stages_ms": {k: round(v, 4) for k, v in res["stages_serial"].items()},
                          "raster_achieved_tops": round(res["achieved_serial"], 3),
                          "raster_frac": round(res["achieved_serial"] / VALU_TOPS, 4),
                          "direct_ms_per_frame": round(res["ms_direct_serial"], 4),
                          "speedup_vs_direct": round(res["ms_direct_serial"] / res["ms_serial"], 3)},
        "direct_best": {"tile": res["best_direct"]["tile"], "value": round(res["best_direct"]["value"], 2),
                        "ms_per_frame": round(res["best_direct"]["ms_per_frame"], 4),
                        "ms_by_tile": res["best_direct"]["by_tile"]},
        "speedup_vs_best_direct": round(res["value"] / res["best_direct"]["value"], 3),
        "psnr_vs_direct_db": round(res["psnr"], 2),
        "orbit_cameras": orbit_line(res, W, H),
        "comparators": {"psnr_fd_bicubic_db": round(res["comparators"]["psnr_fd_bicubic"], 2),
                        "psnr_torch_bicubic_db": round(res["comparators"]["psnr_torch_bicubic"], 2),
                        "fd_slopes_ms": round(res["comparators"]["fd_slopes_ms"], 4),
                        "fd_upscale_ms": round(res["comparators"]["fd_upscale_ms"], 4)},
        "pairs": {"lowres": res["pairs"], "direct": res["direct"]["pairs"]},
        "fragments": {"lowres_evaluated": res["evals"], "lowres_blended": res["frags"],
                      "direct_evaluated": res["direct"]["evaluated_fragments"],
                      "direct_blended": res["direct"]["blended_fragments"]},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(res, args.cpu_budget)
        line["cpu_baseline"]["value"] = round(line["cpu_baseline"]["value"], 6)
        line["cpu_baseline"]["single_thread_tiny"] = tiny_1t
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
