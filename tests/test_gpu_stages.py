"""GPU parity of each stage against the FP64 oracle, fed identical inputs.

Each stage is given inputs computed by the oracle (never by another HIP
stage), so a mismatch points at the kernel under test:
  gs_project          vs oracle projection (same FP32 scene)
  gs_bin_sort         vs a plain lexicographic sort of the oracle's rects/depths
  gs_raster_grad      vs oracle compositing of the same FP32-rounded splats
  gs_upscale_hermite  vs oracle patches of the same FP32 low-res buffer
"""
import numpy as np
import pytest

from parity_util import (TOL, assert_within, best_variant_error, report, rounded_proj,
                         splat_records, summarize)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_14171_amd import _lib
    _lib.lib()
    return _lib


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


# ---------------------------------------------------------------------------
# gs_project
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["tiny", "tiny_deg3_orbit", "clusters_subset", "far_plane"])
def test_project_matches_oracle(gs, oracle, case):
    import torch
    from paper_2503_14171_amd import scenes
    if case == "tiny":
        sc = scenes.workload_scene("tiny")
        cam = scenes.workload_camera("tiny")
    elif case == "tiny_deg3_orbit":
        sc = scenes.make_scene("uniform", 20000, 21, 3)
        sc["means"] *= np.float32(2.2)  # near-plane culls and J clamps
        cam = scenes.orbit_camera(200, 120, 40.0, -15.0)
    elif case == "far_plane":  # a far plane through the scene culls its far half
        sc = scenes.make_scene("uniform", 20000, 27, 1)
        cam = scenes.make_camera(320, 240, far_plane=3.0)
    else:
        sc = scenes.make_scene("clusters", 100000, 22, 3)
        cam = scenes.make_camera(960, 540)
    for tile in (8, 16):
        cfg = scenes.render_config(sc["sh_degree"], tile_size=tile)
        print(f"project case={case} tile={tile} n={sc['means'].shape[0]}", flush=True)
        pr = oracle.project(sc, cam, cfg)
        n = sc["means"].shape[0]
        splats = torch.zeros((n, 12), dtype=torch.float32, device="cuda")
        depth = torch.zeros(n, dtype=torch.float32, device="cuda")
        rect = torch.zeros((n, 4), dtype=torch.int16, device="cuda")
        gs.gs_project(_dev(sc["means"]), _dev(sc["log_scales"]), _dev(sc["quats"]),
                      _dev(sc["opacity"]), _dev(sc["sh"]), cam, cfg, splats, depth, rect)
        torch.cuda.synchronize()
        s = splats.cpu().numpy()
        d = depth.cpu().numpy()
        r = rect.cpu().numpy().astype(np.int32)
        ref_rect = oracle.tile_rects(pr, cam["width"], cam["height"], tile)
        np.testing.assert_array_equal(r, ref_rect)
        live = ref_rect[:, 2] > ref_rect[:, 0]
        assert live.sum() > 0.3 * n
        # the sort key is bit-identical: camera z rounded to FP32
        np.testing.assert_array_equal(d[live], pr["depth"][live].astype(np.float32))
        mean = s.view(np.float64)[:, 0:2]
        np.testing.assert_allclose(mean[live], pr["mean2d"][live], rtol=0, atol=1e-9)
        np.testing.assert_allclose(s[live, 4:7], pr["conic"][live], rtol=2e-7, atol=1e-12)
        np.testing.assert_array_equal(s[live, 7], sc["opacity"][live])
        np.testing.assert_allclose(s[live, 8:11], pr["rgb"][live], rtol=0, atol=1e-6)
        amin = float(np.float32(cfg["alpha_min"]))
        np.testing.assert_allclose(s[live, 11], 2 * np.log(pr["opacity"][live] / amin), rtol=2e-7)
        # culled Gaussians: no tiles, zeroed record, infinite depth
        culled = ~pr["valid"]
        assert np.all(r[culled] == 0) and np.all(s[culled] == 0) and np.all(np.isinf(d[culled]))


# ---------------------------------------------------------------------------
# gs_bin_sort
# ---------------------------------------------------------------------------
def _run_bin_sort(gs, depth32, rect, cam, cfg, capacity=None):
    import torch
    n = depth32.shape[0]
    tiles = gs.gs_num_tiles(cam["width"], cam["height"], cfg["tile_size"])
    cnt = np.maximum(rect[:, 2] - rect[:, 0], 0) * np.maximum(rect[:, 3] - rect[:, 1], 0)
    K = int(cnt.sum())
    cap = K if capacity is None else capacity
    ws = torch.empty(gs.gs_bin_sort_workspace_size(n, cap, cam, cfg), dtype=torch.uint8, device="cuda")
    ids = torch.full((max(cap, 1),), -7, dtype=torch.int32, device="cuda")
    ranges = torch.full((tiles, 2), -7, dtype=torch.int32, device="cuda")
    k = gs.gs_bin_sort(n, _dev(depth32), _dev(rect.astype(np.int16)), cam, cfg, cap, ids, ranges, ws)
    torch.cuda.synchronize()
    assert k == K
    return ids.cpu().numpy()[:K], ranges.cpu().numpy()


@pytest.mark.parametrize("tile", [8, 16, 32, 64])
def test_bin_sort_matches_lexsort_oracle_scene(gs, oracle, tile):
    from paper_2503_14171_amd import scenes
    sc = scenes.make_scene("clusters", 60000, 23, 0)
    cam = scenes.make_camera(640, 360)
    cfg = scenes.render_config(0, tile_size=tile)
    pr = oracle.project(sc, cam, cfg)
    rect = oracle.tile_rects(pr, 640, 360, tile)
    d32 = np.where(pr["valid"], pr["depth"], np.inf).astype(np.float32)
    print(f"bin_sort scene tile={tile}", flush=True)
    ids, ranges = _run_bin_sort(gs, d32, rect, cam, cfg)
    ref_ids, ref_ranges = oracle.tile_lists(d32, rect, *_tiles_xy(cam, tile))
    np.testing.assert_array_equal(ranges, ref_ranges)
    np.testing.assert_array_equal(ids, ref_ids)


def _tiles_xy(cam, tile):
    return -(-cam["width"] // tile), -(-cam["height"] // tile)


@pytest.mark.parametrize("seed,tile", [(0, 16), (1, 16), (0, 64), (1, 64)])
def test_bin_sort_stable_under_depth_ties(gs, oracle, seed, tile):
    """Few distinct depths: equal keys must keep index order; many pairs so
    the sort runs several blocks and a two-level scan.  3072 tiles take the
    two-digit pair sort, 192 the single-digit one."""
    from paper_2503_14171_amd import scenes
    rng = np.random.default_rng(seed)
    n = 200000
    cam = scenes.make_camera(1024, 768)
    cfg = scenes.render_config(0, tile_size=tile)
    tx, ty = _tiles_xy(cam, tile)
    x0 = rng.integers(0, tx, n)
    y0 = rng.integers(0, ty, n)
    w = rng.integers(0, 4, n)
    h = rng.integers(1, 4, n)
    rect = np.stack([x0, y0, np.minimum(x0 + w, tx), np.minimum(y0 + h, ty)], 1).astype(np.int32)
    d32 = rng.choice(np.array([0.5, 1.0, 1.0000001, 3.25, 7.0], np.float32), n)
    print(f"bin_sort ties seed={seed} tile={tile}", flush=True)
    ids, ranges = _run_bin_sort(gs, d32, rect, cam, cfg)
    ref_ids, ref_ranges = oracle.tile_lists(d32, rect, tx, ty)
    assert ids.shape[0] > 65536 * 2
    np.testing.assert_array_equal(ranges, ref_ranges)
    np.testing.assert_array_equal(ids, ref_ids)


_DEPTH_KINDS = ["full_range", "narrow", "eight_binades", "just_over_eight_binades", "mostly_culled",
                "one_kept", "all_culled", "all_equal", "denormal_and_huge"]


def _depth_set(kind, rng, n):
    f32 = np.float32
    if kind == "full_range":  # every positive finite float: all four passes
        return rng.integers(1, 0x7F800000, n, dtype=np.uint32).view(f32)
    if kind == "narrow":  # 300 ulps: only the first two digits vary
        return (np.uint32(0x3F800000) + rng.integers(0, 300, n, dtype=np.uint32)).view(f32)
    if kind == "eight_binades":  # [1, 256): max - min < 2^26 ulps, top pass skipped
        return np.exp2(rng.uniform(0.0, 8.0, n)).astype(f32).clip(1.0, np.nextafter(f32(256), f32(0)))
    if kind == "just_over_eight_binades":  # [1, 256]: exactly 2^26 ulps, top pass needed
        d = np.exp2(rng.uniform(0.0, 8.0, n)).astype(f32).clip(1.0, 256.0)
        d[rng.choice(n, 5, replace=False)] = f32(256.0)
        d[rng.choice(n, 5, replace=False)] = f32(1.0)
        return d
    if kind == "mostly_culled":
        d = rng.uniform(0.5, 40.0, n).astype(f32)
        d[rng.random(n) < 0.9] = np.inf
        return d
    if kind == "one_kept":
        d = np.full(n, np.inf, f32)
        d[n // 3] = f32(4.0)
        return d
    if kind == "all_culled":
        return np.full(n, np.inf, f32)
    if kind == "all_equal":
        return np.full(n, 2.5, f32)
    if kind == "denormal_and_huge":
        return rng.choice(np.array([1e-42, 1e-38, 1e-30, 0.25, 3.0, 1e30, 3.4e38], f32), n)
    raise ValueError(kind)


@pytest.mark.parametrize("tile", [16, 32])
@pytest.mark.parametrize("kind", _DEPTH_KINDS)
def test_bin_sort_depth_key_ranges(gs, oracle, kind, tile):
    """Depth sets that need one to four radix passes over their bit range,
    with and without culled (+inf) splats, whose rectangles are empty as the
    projection leaves them: the lists must equal a lexicographic sort (768
    tiles: two-digit pair sort; 192: single-digit)."""
    from paper_2503_14171_amd import scenes
    rng = np.random.default_rng(_DEPTH_KINDS.index(kind) + 40)
    n = 70000
    d32 = _depth_set(kind, rng, n)
    fin = d32[np.isfinite(d32)]
    # depths inside the default camera's [0.2, 100]: the far plane bounds the
    # keys and only the passes that range needs run; otherwise no far plane
    # (every pass may run)
    inside = fin.size == 0 or (fin.min() >= np.float32(0.2) and fin.max() <= np.float32(100.0))
    cam = scenes.make_camera(512, 384, far_plane=100.0 if inside else 0.0)
    cfg = scenes.render_config(0, tile_size=tile)
    tx, ty = _tiles_xy(cam, tile)
    x0 = rng.integers(0, tx, n)
    y0 = rng.integers(0, ty, n)
    w = rng.integers(1, 3, n)
    h = rng.integers(1, 3, n)
    rect = np.stack([x0, y0, np.minimum(x0 + w, tx), np.minimum(y0 + h, ty)], 1).astype(np.int32)
    rect[np.isinf(d32)] = 0
    print(f"bin_sort depth keys kind={kind} tile={tile} far={cam['far_plane']}", flush=True)
    ids, ranges = _run_bin_sort(gs, d32, rect, cam, cfg)
    ref_ids, ref_ranges = oracle.tile_lists(d32, rect, tx, ty)
    np.testing.assert_array_equal(ranges, ref_ranges)
    np.testing.assert_array_equal(ids, ref_ids)


def test_bin_sort_depth_outside_near_far_is_refused(gs, oracle):
    """With a far plane only the depth passes [near, far] needs run (near 0.2,
    far 50: 8 + 9 + 9 bits, sorting 26 key bits above the smallest depth): a
    depth so far beyond it that the keys span more bits makes the synchronous
    sort fail and the asynchronous one report GS_PAIRS_DEPTH_RANGE with empty
    lists; a depth beyond it whose keys still fit is ordered correctly; inside
    it, the lists equal a lexicographic sort."""
    import torch
    from paper_2503_14171_amd import scenes
    rng = np.random.default_rng(93)
    n = 30000
    cam = scenes.make_camera(256, 192, far_plane=50.0)
    cfg = scenes.render_config(0, tile_size=16)
    tx, ty = _tiles_xy(cam, 16)
    x0 = rng.integers(0, tx, n)
    y0 = rng.integers(0, ty, n)
    rect = np.stack([x0, y0, np.minimum(x0 + 2, tx), np.minimum(y0 + 1, ty)], 1).astype(np.int32)
    d32 = rng.uniform(0.25, 50.0, n).astype(np.float32)
    d32[0] = np.float32(50.0)  # on the far plane: inside
    print("bin_sort near/far bounded depths", flush=True)
    ids, ranges = _run_bin_sort(gs, d32, rect, cam, cfg)
    ref_ids, ref_ranges = oracle.tile_lists(d32, rect, tx, ty)
    np.testing.assert_array_equal(ranges, ref_ranges)
    np.testing.assert_array_equal(ids, ref_ids)
    fits = d32.copy()
    fits[n // 3] = np.float32(60.0)  # beyond the far plane, key still within 2^26 ulps of the min
    ids, ranges = _run_bin_sort(gs, fits, rect, cam, cfg)
    ref_ids, ref_ranges = oracle.tile_lists(fits, rect, tx, ty)
    np.testing.assert_array_equal(ranges, ref_ranges)
    np.testing.assert_array_equal(ids, ref_ids)
    bad = d32.copy()
    bad[n // 2] = np.float32(5000.0)  # keys now span more than 2^26 ulps
    with pytest.raises(gs.GsError) as ei:
        _run_bin_sort(gs, bad, rect, cam, cfg)
    assert ei.value.status == gs.GS_ERR_INVALID_ARGUMENT and "far_plane" in str(ei.value)
    K = int(ref_ids.shape[0])
    ws = torch.empty(gs.gs_bin_sort_workspace_size(n, K, cam, cfg), dtype=torch.uint8, device="cuda")
    ids_d = torch.full((K,), -7, dtype=torch.int32, device="cuda")
    rg_d = torch.full((tx * ty, 2), -7, dtype=torch.int32, device="cuda")
    kdev = torch.zeros(1, dtype=torch.int64, device="cuda")
    gs.gs_bin_sort_async(n, _dev(bad), _dev(rect.astype(np.int16)), cam, cfg, K, ids_d, rg_d, kdev, ws)
    torch.cuda.synchronize()
    assert int(kdev.item()) == gs.GS_PAIRS_DEPTH_RANGE
    assert torch.all(rg_d == 0) and torch.all(ids_d == -7)
    with pytest.raises(gs.GsError):
        gs.check_pair_count(int(kdev.item()))


def test_bin_sort_wide_and_far_rectangles(gs, oracle):
    """Rectangles wider or taller than 63 tiles and tiles beyond x = 1022
    (a 1025-tile-wide grid), mixed with ordinary ones and culled splats."""
    from paper_2503_14171_amd import scenes
    rng = np.random.default_rng(77)
    n = 20000
    cam = scenes.make_camera(8200, 600)
    cfg = scenes.render_config(0, tile_size=8)
    tx, ty = _tiles_xy(cam, 8)
    assert tx == 1025
    x0 = rng.integers(0, tx, n)
    y0 = rng.integers(0, ty, n)
    w = rng.integers(1, 4, n)
    h = rng.integers(1, 4, n)
    wide = rng.random(n) < 0.03
    w[wide] = rng.integers(60, 130, wide.sum())
    tall = rng.random(n) < 0.03
    h[tall] = rng.integers(60, 75, tall.sum())
    far = rng.random(n) < 0.1
    x0[far] = rng.integers(1015, tx, far.sum())
    rect = np.stack([x0, y0, np.minimum(x0 + w, tx), np.minimum(y0 + h, ty)], 1).astype(np.int32)
    d32 = rng.uniform(0.5, 30.0, n).astype(np.float32)
    culled = rng.random(n) < 0.2
    d32[culled] = np.inf
    rect[culled] = 0
    print("bin_sort wide and far rectangles", flush=True)
    ids, ranges = _run_bin_sort(gs, d32, rect, cam, cfg)
    ref_ids, ref_ranges = oracle.tile_lists(d32, rect, tx, ty)
    np.testing.assert_array_equal(ranges, ref_ranges)
    np.testing.assert_array_equal(ids, ref_ids)


def test_bin_sort_capacity_error_and_empty(gs, oracle):
    import torch
    from paper_2503_14171_amd import scenes
    cam = scenes.make_camera(64, 48)
    cfg = scenes.render_config(0, tile_size=8)
    rect = np.array([[0, 0, 2, 2], [1, 1, 3, 2], [0, 0, 0, 0]], np.int32)
    d32 = np.array([2.0, 1.0, 3.0], np.float32)
    print("bin_sort capacity", flush=True)
    with pytest.raises(gs.GsError) as ei:
        _run_bin_sort(gs, d32, rect, cam, cfg, capacity=3)
    assert ei.value.status == gs.GS_ERR_CAPACITY and ei.value.n_pairs == 6
    ids, ranges = _run_bin_sort(gs, d32, rect, cam, cfg)
    ref_ids, ref_ranges = oracle.tile_lists(d32, rect, 8, 6)
    np.testing.assert_array_equal(ids, ref_ids)
    np.testing.assert_array_equal(ranges, ref_ranges)
    # no pairs at all: every range empty
    ids, ranges = _run_bin_sort(gs, d32, np.zeros((3, 4), np.int32), cam, cfg)
    assert ids.size == 0 and np.all(ranges == 0)
    # n == 0
    ws = torch.empty(gs.gs_bin_sort_workspace_size(0, 0, cam, cfg), dtype=torch.uint8, device="cuda")
    rg = torch.full((48, 2), -1, dtype=torch.int32, device="cuda")
    ids0 = torch.empty(1, dtype=torch.int32, device="cuda")
    k = gs.gs_bin_sort(0, torch.empty(0, device="cuda"), torch.empty((0, 4), dtype=torch.int16, device="cuda"),
                       cam, cfg, 0, ids0, rg, ws)
    torch.cuda.synchronize()
    assert k == 0 and torch.all(rg == 0)


# ---------------------------------------------------------------------------
# gs_raster_grad (fed the oracle's splats and tile lists)
# ---------------------------------------------------------------------------
def _raster_stage(gs, oracle, sc, cam, cfg, want_grads=True, sample=None, seed=0):
    import torch
    pr = oracle.project(sc, cam, cfg)
    rec = splat_records(pr, cfg)
    rp = rounded_proj(pr)
    tile = cfg["tile_size"]
    rect = oracle.tile_rects(pr, cam["width"], cam["height"], tile)
    d32 = np.where(pr["valid"], pr["depth"], np.inf).astype(np.float32)
    ids, ranges = oracle.tile_lists(d32, rect, *_tiles_xy(cam, tile))
    H, W = cam["height"], cam["width"]
    C = 12 if want_grads else 3
    out = torch.full((H, W, C), np.nan, dtype=torch.float32, device="cuda")
    nbl = torch.full((H, W), -1, dtype=torch.int32, device="cuda")
    gs.gs_raster_grad(_dev(rec), _dev(ids if ids.size else np.zeros(1, np.int32)), _dev(ranges), cam,
                      cfg, want_grads, out, nbl)
    torch.cuda.synchronize()
    g = out.cpu().numpy().reshape(-1, C)
    nb = nbl.cpu().numpy().reshape(-1)
    yy, xx = np.meshgrid(np.arange(H, dtype=float), np.arange(W, dtype=float), indexing="ij")
    px, py = xx.reshape(-1), yy.reshape(-1)
    idx = np.arange(H * W)
    if sample is not None and sample < H * W:
        idx = np.random.default_rng(seed).choice(H * W, sample, replace=False)
    order = oracle.depth_order(rp)
    ref = oracle.composite(rp, order, cfg, px[idx], py[idx], variants=True)
    return g[idx], nb[idx], ref


@pytest.mark.parametrize("tile", [8, 16, 32, 64])
@pytest.mark.parametrize("want_grads", [True, False])
def test_raster_stage_tiny(gs, oracle, tile, want_grads):
    from paper_2503_14171_amd import scenes
    sc = scenes.workload_scene("tiny")
    cam = scenes.workload_camera("tiny")
    cfg = scenes.render_config(0, tile_size=tile)
    print(f"raster stage tiny tile={tile} grads={want_grads}", flush=True)
    g, nb, ref = _raster_stage(gs, oracle, sc, cam, cfg, want_grads)
    err, masked = best_variant_error(g, ref)
    report(f"raster_stage_tiny_t{tile}_g{int(want_grads)}", summarize(err, masked, ref["out"]))
    assert_within(err, masked)
    clean = ref["n_amb"] == 0
    np.testing.assert_array_equal(nb[clean], ref["n_blend"][clean])


@pytest.mark.parametrize("tile", [8, 32])
def test_fragment_counts(gs, oracle, tile):
    """gs_raster_fragment_counts (the benchmark's work counters): the image
    equals gs_raster_grad's bit for bit; the blended count equals the
    oracle's per pixel; every pixel evaluates at least the fragments it
    blends and at most its tile list up to where it stopped."""
    import torch
    from paper_2503_14171_amd import scenes
    sc = scenes.workload_scene("tiny")
    cam = scenes.workload_camera("tiny")
    cfg = scenes.render_config(0, tile_size=tile)
    print(f"fragment counts tile={tile}", flush=True)
    g, nb, ref = _raster_stage(gs, oracle, sc, cam, cfg, True)
    pr = oracle.project(sc, cam, cfg)
    rec = splat_records(pr, cfg)
    rect = oracle.tile_rects(pr, cam["width"], cam["height"], tile)
    d32 = np.where(pr["valid"], pr["depth"], np.inf).astype(np.float32)
    tx, ty = _tiles_xy(cam, tile)
    ids, ranges = oracle.tile_lists(d32, rect, tx, ty)
    H, W = cam["height"], cam["width"]
    out = torch.full((H * W, 12), np.nan, dtype=torch.float32, device="cuda")
    nev = torch.full((H * W,), -1, dtype=torch.int32, device="cuda")
    nbl = torch.full((H * W,), -1, dtype=torch.int32, device="cuda")
    gs.gs_raster_fragment_counts(_dev(rec), _dev(ids), _dev(ranges), [cam], cfg, True, out, nev, nbl)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), g)
    nev, nbl = nev.cpu().numpy(), nbl.cpu().numpy()
    np.testing.assert_array_equal(nbl, nb)
    clean = ref["n_amb"] == 0
    np.testing.assert_array_equal(nbl[clean], ref["n_blend"][clean])
    yy, xx = np.divmod(np.arange(H * W), W)
    t = (yy // tile) * tx + xx // tile
    list_len = ranges[t, 1] - ranges[t, 0]
    assert (nev >= nbl).all() and (nev <= list_len).all()
    assert nev.sum() > nbl.sum() > 0


@pytest.mark.parametrize("tile", [16, 32, 64])
def test_raster_stage_ragged_bg_opaque(gs, oracle, tile):
    """Image size not a multiple of the tile, non-zero background, opaque
    splats (alpha clamp and early termination everywhere)."""
    from paper_2503_14171_amd import scenes
    sc = scenes.make_scene("uniform", 6000, 24, 0)
    sc["opacity"][::2] = np.float32(0.999)
    cam = scenes.make_camera(101, 75)
    cfg = scenes.render_config(0, tile_size=tile, bg=(0.25, 0.5, 1.0))
    print(f"raster stage ragged tile={tile}", flush=True)
    g, nb, ref = _raster_stage(gs, oracle, sc, cam, cfg, True)
    err, masked = best_variant_error(g, ref)
    report(f"raster_stage_ragged_t{tile}", summarize(err, masked, ref["out"]))
    assert_within(err, masked)


@pytest.mark.parametrize("tile", [16, 32])
def test_raster_stage_needles(gs, oracle, tile):
    """Very anisotropic splats (one axis 30x the others) crossing many tiles
    and quadrants: the per-wave culling must keep every reachable splat."""
    from paper_2503_14171_amd import scenes
    sc = scenes.make_scene("uniform", 3000, 26, 0)
    sc["log_scales"][:, 0] += np.float32(3.4)
    sc["log_scales"][:, 1:] -= np.float32(0.5)
    cam = scenes.make_camera(160, 96)
    cfg = scenes.render_config(0, tile_size=tile)
    print(f"raster stage needles tile={tile}", flush=True)
    g, nb, ref = _raster_stage(gs, oracle, sc, cam, cfg, True)
    err, masked = best_variant_error(g, ref)
    report(f"raster_stage_needles_t{tile}", summarize(err, masked, ref["out"]))
    assert_within(err, masked)


def test_raster_stage_clusters_sampled(gs, oracle):
    from paper_2503_14171_amd import scenes
    sc = scenes.make_scene("clusters", 100000, 25, 3)
    cam = scenes.make_camera(480, 270)
    cfg = scenes.render_config(3, tile_size=16)
    print("raster stage clusters sampled", flush=True)
    g, nb, ref = _raster_stage(gs, oracle, sc, cam, cfg, True, sample=3000)
    err, masked = best_variant_error(g, ref)
    report("raster_stage_clusters", summarize(err, masked, ref["out"]))
    assert_within(err, masked)


# ---------------------------------------------------------------------------
# gs_upscale_hermite (fed an oracle-rendered low-res buffer)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def tiny_lowres(oracle):
    from paper_2503_14171_amd import scenes
    sc = scenes.workload_scene("tiny")
    r = oracle.render(sc, scenes.workload_camera("tiny"), scenes.render_config(0))
    return r["img"].astype(np.float32)


@pytest.mark.parametrize("W,H", [(256, 256), (128, 128), (384, 384), (512, 512), (300, 211),
                                 (129, 400), (1000, 129)])
def test_upscale_stage(gs, oracle, tiny_lowres, W, H):
    import torch
    low = tiny_lowres
    out = torch.full((H, W, 3), np.nan, dtype=torch.float32, device="cuda")
    print(f"upscale stage {W}x{H}", flush=True)
    gs.gs_upscale_hermite(_dev(low), out)
    torch.cuda.synchronize()
    ref = oracle.upscale(low.astype(np.float64), W, H)
    err = np.abs(out.cpu().numpy() - ref).reshape(-1, 3)
    report(f"upscale_stage_{W}x{H}", summarize(err, np.zeros(err.shape[0], bool)))
    assert err.max() < 5e-6


def test_upscale_stage_small_and_identity(gs, oracle):
    import torch
    rng = np.random.default_rng(3)
    for (w, h, W, H) in [(2, 2, 2, 2), (2, 2, 7, 5), (3, 5, 3, 5), (17, 9, 51, 27), (5, 4, 640, 4)]:
        low = rng.standard_normal((h, w, 12)).astype(np.float32)
        out = torch.full((H, W, 3), np.nan, dtype=torch.float32, device="cuda")
        print(f"upscale small {w}x{h}->{W}x{H}", flush=True)
        gs.gs_upscale_hermite(_dev(low), out)
        torch.cuda.synchronize()
        ref = oracle.upscale(low.astype(np.float64), W, H)
        np.testing.assert_allclose(out.cpu().numpy(), ref, atol=2e-5, rtol=0)
        if (w, h) == (W, H):
            np.testing.assert_allclose(out.cpu().numpy(), low[..., :3], atol=1e-6)


# ---------------------------------------------------------------------------
# gs_fd_slopes (classical bicubic comparator) and its chain into the upscaler
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("w,h", [(2, 2), (3, 7), (128, 128), (257, 131), (960, 540)])
def test_fd_slopes_stage(gs, oracle, w, h):
    import torch
    rng = np.random.default_rng(w * 1000 + h)
    img = rng.uniform(0, 1, (h, w, 3)).astype(np.float32)
    out = torch.full((h, w, 12), np.nan, dtype=torch.float32, device="cuda")
    print(f"fd_slopes {w}x{h}", flush=True)
    gs.gs_fd_slopes(_dev(img), out)
    torch.cuda.synchronize()
    ref = oracle.fd_slopes(img.astype(np.float64))
    got = out.cpu().numpy()
    np.testing.assert_array_equal(got[..., 0:3], img)
    np.testing.assert_allclose(got, ref, atol=1e-6, rtol=0)


def test_fd_bicubic_chain(gs, oracle, tiny_lowres):
    """gs_fd_slopes then gs_upscale_hermite against the oracle's chain, at an
    integer and two fractional factors."""
    import torch
    low = tiny_lowres
    h, w = low.shape[:2]
    slopes = torch.empty((h, w, 12), dtype=torch.float32, device="cuda")
    gs.gs_fd_slopes(_dev(low[..., :3].copy()), slopes)
    ref_slopes = oracle.fd_slopes(low[..., :3].astype(np.float64))
    for (W, H) in [(4 * w, 4 * h), (int(2.5 * w), int(2.5 * h)), (3 * w // 2, 2 * h)]:
        out = torch.full((H, W, 3), np.nan, dtype=torch.float32, device="cuda")
        print(f"fd bicubic {w}x{h}->{W}x{H}", flush=True)
        gs.gs_upscale_hermite(slopes, out)
        torch.cuda.synchronize()
        ref = oracle.upscale(ref_slopes, W, H)
        np.testing.assert_allclose(out.cpu().numpy(), ref, atol=5e-6, rtol=0)


@pytest.mark.parametrize("sizes", [((8200, 160), (300, 200)), ((600, 40), (120, 64))])
def test_bin_sort_views_matches_per_view_lexsort(gs, oracle, sizes):
    """Two views of different tile grids sorted together, with over-wide
    rectangles (escaped packed rectangles) and culled splats: view after
    view, each view's lists must equal a lexicographic sort of that view's
    records.  The first pair (one grid with tiles beyond x = 1022) takes the
    two-digit pair sort, the second (75x5 + 15x8 = 495 tiles) the
    single-digit one."""
    import torch
    from paper_2503_14171_amd import scenes
    rng = np.random.default_rng(91)
    n = 12000
    cams = [scenes.make_camera(w, h) for w, h in sizes]
    cfg = scenes.render_config(0, tile_size=8)
    depth, rect, refs = [], [], []
    for cam in cams:
        tx, ty = _tiles_xy(cam, 8)
        x0 = rng.integers(0, tx, n)
        y0 = rng.integers(0, ty, n)
        w = rng.integers(1, 4, n)
        wide = rng.random(n) < 0.05
        w[wide] = rng.integers(60, 100, wide.sum())
        h = rng.integers(1, 3, n)
        r = np.stack([x0, y0, np.minimum(x0 + w, tx), np.minimum(y0 + h, ty)], 1).astype(np.int32)
        d = rng.uniform(0.5, 30.0, n).astype(np.float32)
        culled = rng.random(n) < 0.25
        d[culled] = np.inf
        r[culled] = 0
        depth.append(d)
        rect.append(r)
        refs.append(oracle.tile_lists(d, r, tx, ty))
    K = sum(int(ids.shape[0]) for ids, _ in refs)
    tiles = gs.gs_num_tiles_views(cams, 8)
    ws = torch.empty(gs.gs_bin_sort_views_workspace_size(n, cams, cfg, K), dtype=torch.uint8, device="cuda")
    ids = torch.full((K,), -7, dtype=torch.int32, device="cuda")
    ranges = torch.full((tiles, 2), -7, dtype=torch.int32, device="cuda")
    kdev = torch.zeros(1, dtype=torch.int64, device="cuda")
    print(f"bin_sort views with escaped rectangles {sizes}", flush=True)
    gs.gs_bin_sort_views(n, cams, cfg, _dev(np.concatenate(depth)), _dev(np.concatenate(rect).astype(np.int16)), K, ids,
                         ranges, kdev, ws)
    torch.cuda.synchronize()
    assert int(kdev.item()) == K
    got_ids, got_ranges = ids.cpu().numpy(), ranges.cpu().numpy()
    pos, toff = 0, 0
    for v, (ref_ids, ref_ranges) in enumerate(refs):
        k = ref_ids.shape[0]
        np.testing.assert_array_equal(got_ids[pos:pos + k], ref_ids + v * n)
        t = ref_ranges.shape[0]
        want = np.where(ref_ranges[:, 1:2] > ref_ranges[:, 0:1], ref_ranges + pos, 0)
        np.testing.assert_array_equal(got_ranges[toff:toff + t], want)
        pos += k
        toff += t
    assert toff == tiles
