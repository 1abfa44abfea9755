"""GPU backward pass against the oracle's gradients.

  gs_upscale_hermite_backward_views  vs oracle.upscale_adjoint (same FP32 input gradient)
  gs_raster_grad_backward_views      vs oracle.composite_adjoint of the same FP32 splats
  gs_project_backward_views          vs oracle.project_vjp (FP64 central differences)
  UpscaledRender (the whole chain)   vs oracle.loss_grad and vs FP64 finite differences
                                        of the oracle's forward, 64 Gaussians at 32x32
Gradients are compared element by element with a mixed bound,
|got - ref| <= 1e-3 |ref| + 1e-5 max|ref of the group| (the absolute floor
covers elements whose reference is a cancellation of many contributions that
FP32 atomics sum in another order).
Also: a 1M-Gaussian scene at 480x270 (the training workload's density, and a
near-opaque variant whose lists are walked back through many fragments with
alpha close to 0.99) against the oracle's adjoint on sampled pixels, and the
guard against running backward after a later forward overwrote the saved
state.
"""
import numpy as np
import pytest

from parity_util import report, rounded_proj, splat_records

pytestmark = pytest.mark.gpu

REL = 1e-3
ABS_FLOOR = 1e-5  # of the group's largest reference magnitude


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_14171_amd import _lib
    _lib.lib()
    return torch


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).cuda()


def _rel_err(got, ref):
    """Largest per-element error in units of the mixed bound
    REL |ref| + ABS_FLOOR max|ref| (scaled so that < REL passes)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    floor = ABS_FLOOR * max(np.abs(ref).max(), 1e-30)
    bound = REL * np.abs(ref) + floor
    return float((np.abs(got - ref) / bound).max() * REL)


def test_upscale_backward_matches_oracle(torch_mod):
    torch = torch_mod
    from paper_2503_14171_amd import _lib as L
    from oracle import oracle
    lo = [(17, 9), (40, 31), (5, 4), (64, 48)]
    hi = [(51, 27), (100, 77), (5, 13), (256, 192)]
    rng = np.random.default_rng(1)
    gs = [rng.standard_normal((H, W, 3)).astype(np.float32) for (W, H) in hi]
    d_up = _dev(np.concatenate([g.reshape(-1, 3) for g in gs]))
    d_low = torch.full((sum(w * h for w, h in lo), 12), np.nan, dtype=torch.float32, device="cuda")
    print("upscale backward", flush=True)
    L.gs_upscale_hermite_backward_views(d_up, lo, d_low, hi)
    torch.cuda.synchronize()
    got = d_low.cpu().numpy()
    a = 0
    for (w, h), g in zip(lo, gs):
        ref = oracle.upscale_adjoint(g.astype(np.float64), w, h).reshape(-1, 12)
        report(f"bwd_upscale_{w}x{h}", {"max_abs_err": float(np.abs(got[a:a + w * h] - ref).max()),
                                        "ref_max": float(np.abs(ref).max())})
        np.testing.assert_allclose(got[a:a + w * h], ref, atol=2e-5 * max(1.0, np.abs(ref).max()), rtol=1e-5)
        a += w * h


def _raster_setup(torch, oracle, sc, cam, cfg):
    from paper_2503_14171_amd import _lib as L
    from paper_2503_14171_amd.render import Renderer
    pr = rounded_proj(oracle.project(sc, cam, cfg))
    rec = splat_records(pr, cfg)
    rd = Renderer(sc)
    b = rd.project(cam, cfg)
    # the splat records the stage is fed are the oracle's, so both sides see identical parameters
    b["splats"].copy_(_dev(rec))
    rd.bin_sort(cam, cfg, b)
    w, h = cam["width"], cam["height"]
    low = torch.empty((w * h, 12), dtype=torch.float32, device="cuda")
    state = torch.empty((w * h, 4), dtype=torch.float32, device="cuda")
    last = torch.empty(w * h, dtype=torch.int32, device="cuda")
    L.gs_raster_grad_views_train(b["splats"], b["ids"], b["ranges"], [cam], cfg, low, state, last)
    return pr, b, low, state, last


@pytest.mark.parametrize("tile,bg", [(16, (0.0, 0.0, 0.0)), (8, (0.2, 0.5, 0.9)), (32, (0.0, 0.0, 0.0)),
                                     (64, (0.1, 0.1, 0.1))])
def test_raster_backward_matches_oracle(torch_mod, oracle, tile, bg):
    torch = torch_mod
    from paper_2503_14171_amd import _lib as L
    from paper_2503_14171_amd import scenes
    sc = scenes.make_scene("clusters", 3000, 61, 1)
    sc["log_scales"] = sc["log_scales"] + np.float32(2.0)
    cam = scenes.make_camera(96, 72)
    cfg = scenes.render_config(1, tile_size=tile, bg=bg)
    print(f"raster backward tile={tile}", flush=True)
    pr, b, low, state, last = _raster_setup(torch, oracle, sc, cam, cfg)
    w, h = cam["width"], cam["height"]
    order = oracle.depth_order(pr)
    yy, xx = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64), indexing="ij")
    ref_fwd = oracle.composite(pr, order, cfg, xx.reshape(-1), yy.reshape(-1))
    rng = np.random.default_rng(tile)
    G = rng.standard_normal((w * h, 12))
    G[ref_fwd["n_amb"] > 0] = 0.0   # pixels with a near-tie decision: several correct walks
    n = sc["means"].shape[0]
    d_splats = torch.empty((n, 9), dtype=torch.float32, device="cuda")
    L.gs_raster_grad_backward_views(b["splats"], b["ids"], b["ranges"], [cam], cfg, state, last,
                                    _dev(G.astype(np.float32)), n, d_splats)
    torch.cuda.synchronize()
    got = d_splats.cpu().numpy()
    ref = oracle.composite_adjoint(pr, order, cfg, xx.reshape(-1), yy.reshape(-1), G.astype(np.float32))
    # the training forward writes the same image as the plain forward
    plain = torch.empty((w * h, 12), dtype=torch.float32, device="cuda")
    L.gs_raster_grad(b["splats"], b["ids"], b["ranges"], cam, cfg, True, plain)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(plain.cpu().numpy(), low.cpu().numpy())
    assert (last.cpu().numpy() >= 0).all()
    for f, name in enumerate(oracle.SPLAT_GRAD):
        e = _rel_err(got[:, f], ref[:, f])
        print(f"  {name}: rel err {e:.2e}", flush=True)
        report(f"bwd_raster_t{tile}_bg{int(any(bg))}_{name}", {"mixed_err": e})
        assert e < REL, name


def test_project_backward_matches_oracle(torch_mod, oracle):
    torch = torch_mod
    from paper_2503_14171_amd import _lib as L
    from paper_2503_14171_amd import scenes
    sc = scenes.make_scene("scene", 400, 62, 3)
    sc["means"] = sc["means"] * np.float32(0.5)
    cams = [scenes.orbit_camera(120, 90, 20.0, 10.0), scenes.orbit_camera(64, 80, -50.0, -15.0),
            scenes.orbit_camera(200, 100, 150.0, 5.0)]
    cfg = scenes.render_config(3)
    n = sc["means"].shape[0]
    rng = np.random.default_rng(3)
    d2d = rng.standard_normal((len(cams), n, 9)).astype(np.float32)
    ref = {k: np.zeros(np.shape(sc[k])) for k in oracle.PARAMS}
    for v, cam in enumerate(cams):
        pr = oracle.project(sc, cam, cfg)
        d2d[v][~pr["valid"]] = 0.0          # culled records receive no gradient
        for k, g in oracle.project_vjp(sc, cam, cfg, d2d[v].astype(np.float64)).items():
            ref[k] += g
    t = {k: _dev(sc[k]) for k in oracle.PARAMS}
    out = {k: torch.empty_like(t[k]) for k in oracle.PARAMS}
    print("project backward", flush=True)
    L.gs_project_backward_views(t["means"], t["log_scales"], t["quats"], t["opacity"], t["sh"], cams, cfg,
                                _dev(d2d.reshape(-1, 9)), out["means"], out["log_scales"], out["quats"],
                                out["opacity"], out["sh"])
    torch.cuda.synchronize()
    for k in oracle.PARAMS:
        e = _rel_err(out[k].cpu().numpy(), ref[k])
        print(f"  {k}: rel err {e:.2e}", flush=True)
        report(f"bwd_project_{k}", {"mixed_err": e})
        assert e < REL, k


def _sub_scene():
    from paper_2503_14171_amd import scenes
    sc = scenes.make_scene("scene", 64, 63, 3)
    sc["means"] = sc["means"] * np.float32(0.6)
    sc["log_scales"] = sc["log_scales"] + np.float32(3.0)
    cams = [scenes.orbit_camera(32, 32, 25.0 * v - 30.0, 8.0 * v - 10.0) for v in range(4)]
    hi = [(128, 128)] * 4
    return sc, cams, hi, scenes.render_config(3)


def test_training_chain_matches_oracle_and_finite_differences(torch_mod, oracle):
    """The batched backward (4 views, 64 Gaussians, 32x32 rendered and
    upscaled x4, L1 loss against a perturbed scene's direct render)."""
    torch = torch_mod
    from paper_2503_14171_amd import scenes
    from paper_2503_14171_amd.train import TrainViews, UpscaledRender
    sc, cams, hi, cfg = _sub_scene()
    rng = np.random.default_rng(4)
    target_sc = dict(sc, means=(sc["means"] + rng.normal(0, 0.01, sc["means"].shape)).astype(np.float32))
    targets = []
    for cam, (W, H) in zip(cams, hi):
        r = oracle.render(target_sc, scenes.scale_camera(cam, W, H), cfg)
        targets.append(r["img"][..., :3])
    target = _dev(np.concatenate([t.reshape(-1, 3) for t in targets]).astype(np.float32))
    params = {k: _dev(sc[k]).requires_grad_(True) for k in oracle.PARAMS}
    tv = TrainViews(64, cams, hi, cfg)
    print("training chain: forward + backward", flush=True)
    up = UpscaledRender.apply(params["means"], params["log_scales"], params["quats"], params["opacity"],
                              params["sh"], tv)
    loss = (up - target).abs().mean()
    loss.backward()
    torch.cuda.synchronize()
    g_up = (torch.sign(up - target) / up.numel()).detach().cpu().numpy().astype(np.float64)
    a = 0
    g_views = []
    for (W, H) in hi:
        g_views.append(g_up[a:a + W * H].reshape(H, W, 3))
        a += W * H
    print("training chain: oracle gradient", flush=True)
    ref = oracle.loss_grad(sc, cams, hi, cfg, g_views)
    for k in oracle.PARAMS:
        got = params[k].grad.cpu().numpy()
        e = _rel_err(got, ref[k])
        print(f"  {k}: rel err vs oracle adjoint {e:.2e}", flush=True)
        report(f"bwd_chain_{k}", {"mixed_err": e})
        assert e < REL, k
    # direct FP64 finite differences of the oracle's forward on a few entries
    def lin_loss(s):
        tot = 0.0
        for cam, (W, H), g in zip(cams, hi, g_views):
            img = oracle.render(s, cam, cfg)["img"]
            tot += float((oracle.upscale(img, W, H) * g).sum())
        return tot
    base = {k: np.asarray(sc[k], np.float64) for k in oracle.PARAMS}
    checked = 0
    for k in oracle.PARAMS:  # means, log-scales, quaternions, opacity, SH
        got = params[k].grad.cpu().numpy()
        # the three largest entries of the group
        for flat in np.argsort(-np.abs(ref[k]).reshape(-1))[:3]:
            idx = np.unravel_index(int(flat), ref[k].shape)
            hstep = 1e-6 * max(1.0, abs(base[k][idx]))
            up_s = dict(sc, **base)
            dn_s = dict(sc, **base)
            up_s[k] = base[k].copy()
            dn_s[k] = base[k].copy()
            up_s[k][idx] += hstep
            dn_s[k][idx] -= hstep
            fd = (lin_loss(up_s) - lin_loss(dn_s)) / (2 * hstep)
            print(f"  FD {k}{tuple(int(i) for i in idx)}: gpu {got[idx]:.6e} fd {fd:.6e}", flush=True)
            report(f"bwd_fd_{k}_{checked % 3}", {"rel_err": abs(float(got[idx]) - fd) / max(abs(fd), 1e-12)})
            assert abs(got[idx] - fd) <= REL * max(abs(fd), 1e-12), (k, idx, got[idx], fd)
            checked += 1
    assert checked == 15


def test_backward_of_unseen_scene_is_zero(torch_mod):
    """Every Gaussian behind the cameras: no fragment, no gradient (and no
    NaN from culled records)."""
    torch = torch_mod
    from paper_2503_14171_amd import scenes
    from paper_2503_14171_amd.train import TrainViews, UpscaledRender
    sc = scenes.make_scene("clusters", 500, 64, 2)
    sc["means"] = (sc["means"] * np.float32(0.2) + np.float32([0.0, 0.0, -6.0])).astype(np.float32)
    cams = [scenes.make_camera(40, 30), scenes.make_camera(24, 24)]
    hi = [(80, 60), (48, 48)]
    cfg = scenes.render_config(2)
    params = {k: _dev(sc[k]).requires_grad_(True) for k in ("means", "log_scales", "quats", "opacity", "sh")}
    tv = TrainViews(500, cams, hi, cfg)
    print("backward: unseen scene", flush=True)
    up = UpscaledRender.apply(params["means"], params["log_scales"], params["quats"], params["opacity"],
                              params["sh"], tv)
    (up * up).sum().backward()
    torch.cuda.synchronize()
    assert int(tv.n_pairs.item()) == 0
    for k, p in params.items():
        g = p.grad.cpu().numpy()
        assert np.isfinite(g).all() and (g == 0).all(), k


@pytest.mark.parametrize("opaque", [False, True])
def test_raster_backward_dense_scene_sampled(torch_mod, oracle, opaque):
    """Raster backward on the training workload's density: 1M Gaussians of the
    scene process at 480x270 (and a near-opaque variant, opacity 0.9-0.99,
    whose lists stop after a few fragments with alpha near alpha_max).  The
    loss weights G are non-zero on 240 sampled pixels only, so the oracle's
    adjoint over those pixels is the whole reference.  Checks that recovering
    the state before each fragment from the saved final state (T = T'/(1 -
    alpha) and its derivatives) holds over long, dense lists in FP32."""
    torch = torch_mod
    from paper_2503_14171_amd import _lib as L
    from paper_2503_14171_amd import scenes
    sc = scenes.workload_scene("batch")
    if opaque:
        rng = np.random.default_rng(71)
        sc["opacity"] = rng.uniform(0.9, 0.995, sc["opacity"].shape).astype(np.float32)
    cam = scenes.orbit_camera(480, 270, 30.0, 10.0)
    cfg = scenes.render_config(3, tile_size=16)
    print(f"dense raster backward opaque={opaque}: setup", flush=True)
    pr, b, low, state, last = _raster_setup(torch, oracle, sc, cam, cfg)
    w, h = cam["width"], cam["height"]
    order = oracle.depth_order(pr)
    rng = np.random.default_rng(72 + int(opaque))
    npx = 240
    pix = rng.choice(w * h, npx, replace=False)
    xs, ys = (pix % w).astype(np.float64), (pix // w).astype(np.float64)
    print("dense raster backward: oracle forward at the samples", flush=True)
    fwd = oracle.composite(pr, order, cfg, xs, ys)
    keep = fwd["n_amb"] == 0  # near-tie pixels have several correct walks
    Gs = rng.standard_normal((npx, 12))
    Gs[~keep] = 0.0
    G = np.zeros((w * h, 12), np.float32)
    G[pix] = Gs.astype(np.float32)
    n = sc["means"].shape[0]
    d_splats = torch.empty((n, 9), dtype=torch.float32, device="cuda")
    L.gs_raster_grad_backward_views(b["splats"], b["ids"], b["ranges"], [cam], cfg, state, last,
                                    _dev(G), n, d_splats)
    torch.cuda.synchronize()
    got = d_splats.cpu().numpy()
    print("dense raster backward: oracle adjoint", flush=True)
    ref = oracle.composite_adjoint(pr, order, cfg, xs, ys, Gs.astype(np.float32))
    nb = fwd["n_blend"][keep]
    print(f"  {int(keep.sum())} pixels, blended fragments per pixel: mean {nb.mean():.1f}, max {nb.max()}",
          flush=True)
    # the lists really are walked back through several fragments per pixel
    assert nb.mean() > (1.5 if opaque else 5.0)
    touched = np.abs(ref).sum(1) > 0
    assert touched.sum() > 100
    # records no sampled pixel blends get exactly zero
    assert (got[~touched] == 0).all()
    for f, name in enumerate(oracle.SPLAT_GRAD):
        e = _rel_err(got[:, f], ref[:, f])
        print(f"  {name}: err {e:.2e} (mixed bound, pass < {REL:.0e})", flush=True)
        report(f"bwd_dense_{'opaque' if opaque else 'plain'}_{name}", {"mixed_err": e})
        assert e < REL, name


def test_backward_after_a_later_forward_raises(torch_mod):
    """Two forwards on one TrainViews, then the first one's backward: the
    saved lists and final state belong to the second forward, so backward
    must refuse instead of returning wrong gradients.  The second forward's
    backward still runs."""
    torch = torch_mod
    from paper_2503_14171_amd import scenes
    from paper_2503_14171_amd.train import TrainViews, UpscaledRender
    sc = scenes.make_scene("clusters", 2000, 73, 1)
    cams = [scenes.make_camera(40, 30)]
    cfg = scenes.render_config(1)
    tv = TrainViews(2000, cams, [(80, 60)], cfg)
    params = {k: _dev(sc[k]).requires_grad_(True) for k in ("means", "log_scales", "quats", "opacity", "sh")}
    args = [params[k] for k in ("means", "log_scales", "quats", "opacity", "sh")]
    print("stale backward: two forwards", flush=True)
    up1 = UpscaledRender.apply(*args, tv)
    up2 = UpscaledRender.apply(*args, tv)
    with pytest.raises(RuntimeError, match="overwritten"):
        up1.sum().backward()
    for p in args:
        p.grad = None
    (up2 * up2).sum().backward()
    torch.cuda.synchronize()
    assert all(np.isfinite(p.grad.cpu().numpy()).all() for p in args)
    assert np.abs(params["means"].grad.cpu().numpy()).max() > 0
