"""Batched views: one launch per step for many cameras of one scene.

Every view of a batch must equal the single-view chain for that camera bit
for bit (the single-view chain is checked against the oracle elsewhere; one
test here also goes to the oracle directly); graph replays must equal the
eager chain; an oversized pair count must leave empty tile lists and be
recovered from; LDS batch and upscale band shape must not change results.
"""
import numpy as np
import pytest

from parity_util import assert_within, best_variant_error, report, summarize

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_14171_amd import _lib
    _lib.lib()
    return torch


def _rig(n_views):
    """Mixed sizes (incl. ragged tiles) around an orbit."""
    from paper_2503_14171_amd import scenes
    sizes = [(200, 120), (96, 160), (130, 77), (64, 64), (250, 90), (33, 47), (160, 160), (120, 200)]
    cams, hi = [], []
    for v in range(n_views):
        w, h = sizes[v % len(sizes)]
        cams.append(scenes.orbit_camera(w, h, 40.0 * v - 70.0, 10.0 * ((v % 5) - 2)))
        s = (2, 3, 2.5, 4)[v % 4]
        hi.append((int(round(w * s)), int(round(h * s))))
    return cams, hi


def _single_view(torch, rd, cam, cfg, hi):
    from paper_2503_14171_amd import _lib as L
    b = rd.project(cam, cfg)
    splats = b["splats"].clone()
    depth = b["depth"].clone()
    rect = b["rect"].clone()
    k = rd.bin_sort(cam, cfg, b)
    low = rd.raster(cam, cfg, True)
    up = torch.empty((hi[1], hi[0], 3), dtype=torch.float32, device="cuda")
    L.gs_upscale_hermite(low, up)
    torch.cuda.synchronize()
    ids = b["ids"][:k].cpu().numpy()
    return dict(splats=splats.cpu().numpy(), depth=depth.cpu().numpy(), rect=rect.cpu().numpy(),
                ranges=b["ranges"].cpu().numpy(), ids=ids, low=low.cpu().numpy(), up=up.cpu().numpy(), k=k)


@pytest.mark.parametrize("n_views,tile", [(1, 16), (3, 8), (5, 16), (16, 32)])
def test_views_equal_single_view_chain(torch_mod, n_views, tile):
    torch = torch_mod
    from paper_2503_14171_amd import _lib as L
    from paper_2503_14171_amd import scenes
    from paper_2503_14171_amd.batch import ViewBatch
    from paper_2503_14171_amd.render import Renderer
    sc = scenes.make_scene("scene", 40000, 41, 3)
    rd = Renderer(sc)
    cams, hi = _rig(n_views)
    cfg = scenes.render_config(3, tile_size=tile)
    print(f"views n_views={n_views} tile={tile}", flush=True)
    vb = ViewBatch(rd, cams, hi, cfg)
    lows, ups = vb.render()
    torch.cuda.synchronize()
    n = rd.n
    K = int(vb.n_pairs.item())
    ranges = vb.ranges.cpu().numpy()
    ids = vb.ids[:K].cpu().numpy()
    splats = vb.splats.cpu().numpy()
    depth = vb.depth.cpu().numpy()
    rect = vb.rect.cpu().numpy()
    toff = 0
    ksum = 0
    for v, (cam, wh) in enumerate(zip(cams, hi)):
        ref = _single_view(torch, rd, cam, cfg, wh)
        sl = slice(v * n, (v + 1) * n)
        np.testing.assert_array_equal(splats[sl], ref["splats"])
        np.testing.assert_array_equal(depth[sl], ref["depth"])
        np.testing.assert_array_equal(rect[sl], ref["rect"])
        T = ref["ranges"].shape[0]
        r = ranges[toff:toff + T]
        # same per-tile lists, shifted to the view's records
        for t in range(T):
            a, b = ref["ranges"][t]
            a2, b2 = r[t]
            assert b2 - a2 == b - a
            np.testing.assert_array_equal(ids[a2:b2], ref["ids"][a:b] + v * n)
        toff += T
        ksum += ref["k"]
        np.testing.assert_array_equal(lows[v].cpu().numpy(), ref["low"])
        np.testing.assert_array_equal(ups[v].cpu().numpy(), ref["up"])
    assert toff == vb.tiles and ksum == K


def test_views_against_oracle(torch_mod, oracle):
    torch = torch_mod
    from paper_2503_14171_amd import scenes
    from paper_2503_14171_amd.batch import ViewBatch
    from paper_2503_14171_amd.render import Renderer
    sc = scenes.make_scene("uniform", 8000, 42, 0)
    cams, hi = _rig(4)
    cfg = scenes.render_config(0)
    print("views vs oracle", flush=True)
    vb = ViewBatch(Renderer(sc), cams, hi, cfg)
    lows, ups = vb.render()
    torch.cuda.synchronize()
    for v, cam in enumerate(cams):
        proj = oracle.project(sc, cam, cfg)
        order = oracle.depth_order(proj)
        rng = np.random.default_rng(v)
        xs = rng.integers(0, cam["width"], 300)
        ys = rng.integers(0, cam["height"], 300)
        ref = oracle.composite(proj, order, cfg, xs.astype(float), ys.astype(float), variants=True)
        err, masked = best_variant_error(lows[v].cpu().numpy()[ys, xs], ref)
        report(f"views_oracle_view{v}", summarize(err, masked, ref["out"]))
        assert_within(err, masked)


@pytest.mark.parametrize("tile", [16, 32])
def test_batch_workload_against_oracle_sampled(torch_mod, oracle, tile):
    """The batched stereo workload at full size (1M Gaussians, 16 views: 720x800
    upscaled x2 and 480x540 upscaled x3, one launch per step) against the oracle
    at sampled low-res and upscaled pixels of four views, one per camera size
    and eye, at list tiles 16 and 32."""
    torch = torch_mod
    from paper_2503_14171_amd import scenes
    from paper_2503_14171_amd.batch import ViewBatch
    from paper_2503_14171_amd.render import Renderer
    from test_gpu_e2e import _check_upscaled_samples
    sc = scenes.workload_scene("batch")
    cams, hi = scenes.stereo_rig()
    cfg = scenes.render_config(sc["sh_degree"], tile_size=tile)
    print(f"batch workload tile {tile}: GPU", flush=True)
    vb = ViewBatch(Renderer(sc), cams, hi, cfg)
    lows, ups = vb.render()
    torch.cuda.synchronize()
    for v in (0, 7, 8, 15):
        cam = cams[v]
        w, h = cam["width"], cam["height"]
        low = lows[v].cpu().numpy()
        up = ups[v].cpu().numpy()
        assert np.isfinite(low).all() and np.isfinite(up).all()
        print(f"batch workload tile {tile}: oracle view {v}", flush=True)
        proj = oracle.project(sc, cam, cfg)
        order = oracle.depth_order(proj)
        rng = np.random.default_rng(100 + v)
        xs = rng.integers(0, w, 200)
        ys = rng.integers(0, h, 200)
        ref = oracle.composite(proj, order, cfg, xs.astype(float), ys.astype(float), variants=True)
        err, masked = best_variant_error(low[ys, xs], ref)
        report(f"batch_t{tile}_view{v}_lowres_sampled", summarize(err, masked, ref["out"]))
        assert_within(err, masked)
        e_up, amb = _check_upscaled_samples(oracle, proj, order, cfg, (w, h), hi[v], up, 60, 200 + v)
        report(f"batch_t{tile}_view{v}_upscaled_sampled", summarize(e_up, amb))
        assert_within(e_up, amb)


def test_graph_replays_match_eager(torch_mod):
    torch = torch_mod
    from paper_2503_14171_amd import scenes
    from paper_2503_14171_amd.batch import ViewBatch
    from paper_2503_14171_amd.render import Renderer
    sc = scenes.make_scene("scene", 60000, 43, 3)
    rd = Renderer(sc)
    cams, hi = _rig(6)
    cfg = scenes.render_config(3)
    print("graph: eager reference", flush=True)
    vb = ViewBatch(rd, cams, hi, cfg)
    vb.render()
    torch.cuda.synchronize()
    low_ref, up_ref = vb.low.cpu().numpy(), vb.up.cpu().numpy()
    print("graph: capture and replays", flush=True)
    vb.capture()
    for rep in range(4):
        vb.low.fill_(float("nan"))
        vb.up.fill_(float("nan"))
        vb.ranges.fill_(-7)
        vb.launch()
        assert vb.pairs_fit()
        # unrelated eager work and a sync between replays
        x = torch.randn(1 << 20, device="cuda")
        float(x.sum().item())
        np.testing.assert_array_equal(vb.low.cpu().numpy(), low_ref)
        np.testing.assert_array_equal(vb.up.cpu().numpy(), up_ref)


def test_graphs_in_flight_match_eager(torch_mod):
    """Two captured batches of different cameras replayed in flight on two
    streams (FramePipeline) give what each gives alone, on every round."""
    torch = torch_mod
    from paper_2503_14171_amd import scenes
    from paper_2503_14171_amd.batch import ViewBatch
    from paper_2503_14171_amd.render import FramePipeline, Renderer
    sc = scenes.make_scene("scene", 60000, 47, 3)
    rd = Renderer(sc)
    cams, hi = _rig(8)
    cfg = scenes.render_config(3)
    vbs = [ViewBatch(rd, cams[:5], hi[:5], cfg), ViewBatch(rd, cams[5:], hi[5:], cfg)]
    refs = []
    for vb in vbs:
        vb.render()
        torch.cuda.synchronize()
        refs.append((vb.low.cpu().numpy(), vb.up.cpu().numpy()))
        vb.capture()
    pipe = FramePipeline(vbs)
    for rnd in range(3):
        print(f"in flight: round {rnd}", flush=True)
        for vb in vbs:
            vb.low.fill_(float("nan"))
            vb.up.fill_(float("nan"))
        for _ in vbs:
            pipe.submit(lambda vb: vb.launch())
        assert pipe.pairs_fit()
        torch.cuda.synchronize()
        for vb, (low_ref, up_ref) in zip(vbs, refs):
            np.testing.assert_array_equal(vb.low.cpu().numpy(), low_ref)
            np.testing.assert_array_equal(vb.up.cpu().numpy(), up_ref)


def test_pair_overflow_is_flagged_and_recovered(torch_mod):
    torch = torch_mod
    from paper_2503_14171_amd import _lib as L
    from paper_2503_14171_amd import scenes
    from paper_2503_14171_amd.batch import ViewBatch
    from paper_2503_14171_amd.render import Renderer
    sc = scenes.make_scene("scene", 30000, 44, 3)
    rd = Renderer(sc)
    cams, hi = _rig(3)
    cfg = scenes.render_config(3)
    print("overflow: reference", flush=True)
    ref = ViewBatch(rd, cams, hi, cfg)
    ref.render()
    K = int(ref.n_pairs.item())
    assert K > 100
    print(f"overflow: capacity {K // 3} < {K}", flush=True)
    vb = ViewBatch(rd, cams, hi, cfg, capacity=K // 3)
    vb.ids.fill_(-5)
    vb.run()
    torch.cuda.synchronize()
    assert int(vb.n_pairs.item()) == K
    assert (vb.ranges.cpu().numpy() == 0).all()          # every list empty
    assert (vb.ids.cpu().numpy() == -5).all()             # nothing emitted
    low = vb.low.cpu().numpy()                            # background only (bg = 0)
    assert (low == 0).all()
    vb.capture()
    vb.render()                                           # grows, re-captures, renders again
    assert vb.capacity >= K
    np.testing.assert_array_equal(vb.up.cpu().numpy(), ref.up.cpu().numpy())
    # the single-view asynchronous call follows the same rule
    cam = cams[0]
    b = rd.project(cam, cfg)
    rd._ensure_capacity(b, cam, cfg, 10)
    b["ranges"].fill_(-3)
    ids_small = b["ids"]
    ids_small.fill_(-5)
    rd.bin_sort_async(cam, cfg, b)
    assert not rd.pairs_fit(cam, cfg, b)  # (and grows b's buffers for the next frame)
    assert (b["ranges"].cpu().numpy() == 0).all() and (ids_small.cpu().numpy() == -5).all()
    b2 = rd.project(cam, cfg)
    rd.bin_sort_async(cam, cfg, b2)
    assert rd.pairs_fit(cam, cfg, b2)


def test_batch_and_band_settings_do_not_change_results(torch_mod):
    torch = torch_mod
    from paper_2503_14171_amd import scenes
    from paper_2503_14171_amd.batch import ViewBatch
    from paper_2503_14171_amd.render import Renderer
    sc = scenes.make_scene("scene", 50000, 45, 3)
    rd = Renderer(sc)
    cams, hi = _rig(4)
    for tile in (8, 16, 32, 64):
        ref = None
        for div, rows in [(1, 16), (2, 4), (4, 32), (1, 8)]:
            cfg = scenes.render_config(3, tile_size=tile, batch=tile * tile // div)
            print(f"settings tile={tile} batch={tile * tile // div} rows={rows}", flush=True)
            vb = ViewBatch(rd, cams, hi, cfg, band_rows=rows)
            vb.render()
            torch.cuda.synchronize()
            got = (vb.low.cpu().numpy(), vb.up.cpu().numpy())
            if ref is None:
                ref = got
            else:
                np.testing.assert_array_equal(got[0], ref[0])
                np.testing.assert_array_equal(got[1], ref[1])


def test_autotuner_picks_a_valid_setting(torch_mod):
    torch = torch_mod
    from paper_2503_14171_amd import autotune, scenes
    from paper_2503_14171_amd.render import Renderer
    sc = scenes.make_scene("scene", 40000, 46, 3)
    rd = Renderer(sc)
    cams, hi = _rig(4)
    print("autotune", flush=True)
    best = autotune.tune(rd, cams, hi, scenes.render_config(3), reps=3)
    assert best["tile_size"] in (8, 16, 32, 64)
    assert best["batch"] in (best["tile_size"] ** 2, best["tile_size"] ** 2 // 2, best["tile_size"] ** 2 // 4)
    assert best["band_rows"] in (4, 8, 16, 32)
    assert best["ms"] > 0 and len(best["trials"]) >= 9
    assert autotune.tune(rd, cams, hi, scenes.render_config(3), reps=3) is best  # cached


def test_views_empty_scene_and_blind_view(torch_mod):
    """No Gaussians at all, and a view that sees none of them: background
    everywhere, no pairs, derivatives zero."""
    torch = torch_mod
    from paper_2503_14171_amd import scenes
    from paper_2503_14171_amd.batch import ViewBatch
    from paper_2503_14171_amd.render import Renderer
    bg = (0.25, 0.5, 0.75)
    cfg = scenes.render_config(3, bg=bg)
    cams, hi = _rig(3)
    empty = scenes.make_scene("scene", 0, 47, 3)
    print("views: empty scene", flush=True)
    vb = ViewBatch(Renderer(empty), cams, hi, cfg)
    lows, ups = vb.render()
    torch.cuda.synchronize()
    assert int(vb.n_pairs.item()) == 0
    for low, up in zip(lows, ups):
        lo = low.cpu().numpy()
        np.testing.assert_array_equal(lo[..., :3], np.broadcast_to(np.float32(bg), lo[..., :3].shape))
        np.testing.assert_array_equal(lo[..., 3:], 0.0)
        np.testing.assert_allclose(up.cpu().numpy(), np.broadcast_to(np.float32(bg), up.shape), atol=1e-6)
    # a camera looking away from the scene next to one that sees it
    sc = scenes.make_scene("scene", 20000, 48, 3)
    away = scenes.make_camera(64, 48, eye=(0.0, 0.0, -3.0), target=(0.0, 0.0, -9.0))
    sc["means"] = (sc["means"] * np.float32(0.3)).astype(np.float32)  # keep the shell out of view
    vb = ViewBatch(Renderer(sc), [away, cams[0]], [(128, 96), hi[0]], cfg)
    lows, ups = vb.render()
    torch.cuda.synchronize()
    lo = lows[0].cpu().numpy()
    np.testing.assert_array_equal(lo[..., :3], np.broadcast_to(np.float32(bg), lo[..., :3].shape))
    assert np.abs(lows[1].cpu().numpy()[..., :3] - np.float32(bg)).max() > 0.05
