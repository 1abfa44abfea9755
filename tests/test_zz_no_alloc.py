"""gs_bin_sort_async_static (the bin sort in the library's static scratch, for
callers that cannot allocate) against gs_bin_sort_async with a caller
workspace: identical tile lists, ranges and pair counts, on two calls in a
row (the second with fewer splats, so it runs over the first call's leftover
scratch contents), plus the host-side refusal of sizes beyond the scratch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_14171_amd import _lib
    _lib.lib()
    return _lib


def _sort_both(gs, sc, cam, cfg, capacity):
    import torch
    from paper_2503_14171_amd.render import Renderer
    rd = Renderer(sc)
    b = rd.project(cam, cfg)
    n = sc["means"].shape[0]
    tiles = gs.gs_num_tiles(cam["width"], cam["height"], cfg["tile_size"])
    out = []
    for static in (False, True):
        ids = torch.full((capacity,), -7, dtype=torch.int32, device="cuda")
        ranges = torch.full((tiles, 2), -7, dtype=torch.int32, device="cuda")
        k = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        if static:
            gs.gs_bin_sort_async_static(n, b["depth"], b["rect"], cam, cfg, capacity, ids, ranges, k)
        else:
            ws = torch.empty(gs.gs_bin_sort_workspace_size(n, capacity, cam, cfg), dtype=torch.uint8,
                             device="cuda")
            gs.gs_bin_sort_async(n, b["depth"], b["rect"], cam, cfg, capacity, ids, ranges, k, ws)
        torch.cuda.synchronize()
        out.append((ids.cpu().numpy(), ranges.cpu().numpy(), int(k.item())))
    return out


def test_static_scratch_bin_sort_matches_workspace_bin_sort(gs):
    from paper_2503_14171_amd import scenes
    cfg = scenes.render_config(3, tile_size=16)
    cases = [(scenes.make_scene("clusters", 300000, 91, 3), scenes.make_camera(960, 540)),
             (scenes.make_scene("clusters", 20000, 92, 3), scenes.make_camera(333, 177))]
    for i, (sc, cam) in enumerate(cases):
        n = sc["means"].shape[0]
        capacity = 8 * n + 1024
        print(f"static scratch bin sort: call {i}, n={n}, {cam['width']}x{cam['height']}", flush=True)
        (ids_a, rg_a, k_a), (ids_b, rg_b, k_b) = _sort_both(gs, sc, cam, cfg, capacity)
        assert 0 < k_a <= capacity and k_a == k_b
        np.testing.assert_array_equal(rg_a, rg_b)
        np.testing.assert_array_equal(ids_a[:k_a], ids_b[:k_b])


def test_static_scratch_refuses_sizes_beyond_it(gs):
    import torch
    from paper_2503_14171_amd import scenes
    cfg = scenes.render_config(0, tile_size=16)
    cam = scenes.make_camera(64, 48)
    n, capacity = 1000, 8_000_000  # 12 B per pair of capacity alone exceeds 64 MiB
    assert gs.gs_bin_sort_workspace_size(n, capacity, cam, cfg) > 64 << 20
    depth = torch.ones(n, dtype=torch.float32, device="cuda")
    rect = torch.zeros((n, 4), dtype=torch.int16, device="cuda")
    ids = torch.empty(16, dtype=torch.int32, device="cuda")
    ranges = torch.empty((gs.gs_num_tiles(64, 48, 16), 2), dtype=torch.int32, device="cuda")
    k = torch.zeros(1, dtype=torch.int64, device="cuda")
    # rejected on the host before anything is enqueued (ids is far smaller than
    # the capacity claimed, and is never touched)
    with pytest.raises(gs.GsError, match="static scratch"):
        gs.gs_bin_sort_async_static(n, depth, rect, cam, cfg, capacity, ids, ranges, k)
