"""Pins of the oracle's gradients (Suppl. "3DGS Gradient Computation -
Backward pass").

Checked against: the inner-product identity of a linear map and its adjoint
(upscaler), FP64 central differences of the oracle's own forward compositing
(2D parameters, with and without background), and FP64 central differences
of the whole forward chain project -> composite -> upscale on a tiny scene
(3D parameters).  A plausible slip (a sign in a B-hat recurrence, A_k where
T_k belongs, a dropped cross term in the xy derivative, a transposed
Hermite weight) fails one of them.
"""
import numpy as np
import pytest


@pytest.mark.parametrize("w,h,W,H", [(5, 4, 10, 8), (7, 3, 17, 11), (6, 6, 9, 15), (2, 2, 5, 3)])
def test_upscale_adjoint_inner_product(oracle, w, h, W, H):
    rng = np.random.default_rng(w * 100 + H)
    x = rng.standard_normal((h, w, 12))
    g = rng.standard_normal((H, W, 3))
    lhs = float((oracle.upscale(x, W, H) * g).sum())
    rhs = float((x * oracle.upscale_adjoint(g, w, h)).sum())
    assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(lhs))


def _random_splats(rng, n, size):
    mean2d = rng.uniform(0, size, (n, 2))
    ang = rng.uniform(0, np.pi, n)
    s1 = rng.uniform(1.0, 4.0, n)
    s2 = rng.uniform(1.0, 4.0, n)
    cov = np.zeros((n, 2, 2))
    for i in range(n):
        R = np.array([[np.cos(ang[i]), -np.sin(ang[i])], [np.sin(ang[i]), np.cos(ang[i])]])
        cov[i] = R @ np.diag([s1[i] ** 2, s2[i] ** 2]) @ R.T
    inv = np.linalg.inv(cov)
    conic = np.stack([inv[:, 0, 0], inv[:, 0, 1], inv[:, 1, 1]], 1)
    return dict(mean2d=mean2d, conic=conic, opacity=rng.uniform(0.2, 0.98, n),
                rgb=rng.uniform(0, 1, (n, 3)), valid=np.ones(n, bool))


@pytest.mark.parametrize("bg", [(0.0, 0.0, 0.0), (0.25, 0.5, 0.75)])
def test_composite_adjoint_matches_finite_differences(oracle, bg):
    from paper_2503_14171_amd import scenes
    rng = np.random.default_rng(7)
    n, size = 14, 12.0
    pr = _random_splats(rng, n, size)
    order = np.arange(n, dtype=np.int64)
    cfg = scenes.render_config(0, bg=bg)
    px = rng.uniform(0, size, 25)
    py = rng.uniform(0, size, 25)
    G = rng.standard_normal((25, 12))
    grad = oracle.composite_adjoint(pr, order, cfg, px, py, G)

    def loss(p):
        return float((oracle.composite(p, order, cfg, px, py)["out"] * G).sum())

    fields = [("mean2d", 0), ("mean2d", 1), ("conic", 0), ("conic", 1), ("conic", 2), ("opacity", None),
              ("rgb", 0), ("rgb", 1), ("rgb", 2)]
    h = 1e-6
    for col, (key, j) in enumerate(fields):
        for i in range(n):
            up = {k: np.array(v, copy=True) for k, v in pr.items()}
            dn = {k: np.array(v, copy=True) for k, v in pr.items()}
            if j is None:
                up[key][i] += h
                dn[key][i] -= h
            else:
                up[key][i, j] += h
                dn[key][i, j] -= h
            fd = (loss(up) - loss(dn)) / (2 * h)
            assert abs(fd - grad[i, col]) <= 1e-6 * max(1.0, abs(fd)), (key, j, i, fd, grad[i, col])


def test_composite_adjoint_clamped_fragment_has_colour_gradient_only(oracle):
    from paper_2503_14171_amd import scenes
    pr = dict(mean2d=np.array([[3.0, 3.0]]), conic=np.array([[0.5, 0.0, 0.5]]),
              opacity=np.array([0.999]), rgb=np.array([[0.2, 0.4, 0.6]]), valid=np.ones(1, bool))
    cfg = scenes.render_config(0)
    G = np.ones((1, 12))
    grad = oracle.composite_adjoint(pr, np.zeros(1, np.int64), cfg, [3.0], [3.0], G)
    # alpha = 0.999 > alpha_max at the centre: constant alpha, no geometric gradient
    np.testing.assert_array_equal(grad[0, :6], 0.0)
    # colour weight T alpha = alpha_max; derivative weights vanish
    np.testing.assert_allclose(grad[0, 6:], np.float32(0.99), rtol=1e-7)


def test_loss_grad_matches_finite_differences_of_the_whole_chain(oracle):
    """64 Gaussians, 32x32 rendered, upscaled x2 (and one fractional view):
    the chained adjoint against FP64 central differences of the forward."""
    from paper_2503_14171_amd import scenes
    sc = scenes.make_scene("uniform", 64, 5, 1)
    sc = {k: (np.asarray(v, np.float64) if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
    sc["means"] = sc["means"] * 0.6
    sc["log_scales"] = sc["log_scales"] + 1.6   # footprints of a few pixels
    cams = [scenes.orbit_camera(32, 32, 15.0, 10.0), scenes.orbit_camera(24, 20, -30.0, -5.0)]
    hi = [(64, 64), (37, 31)]
    cfg = scenes.render_config(1)
    rng = np.random.default_rng(9)
    g_up = [rng.standard_normal((H, W, 3)) for (W, H) in hi]
    grads = oracle.loss_grad(sc, cams, hi, cfg, g_up)

    def loss(s):
        tot = 0.0
        for cam, (W, H), g in zip(cams, hi, g_up):
            img = oracle.render(s, cam, cfg)["img"]
            tot += float((oracle.upscale(img, W, H) * g).sum())
        return tot

    checked = 0
    for key in oracle.PARAMS:
        arr = sc[key]
        flat_idx = rng.choice(arr.size, size=min(10, arr.size), replace=False)
        for fi in flat_idx:
            idx = np.unravel_index(fi, arr.shape)
            g = grads[key][idx]
            h = 1e-6 * max(1.0, abs(arr[idx]))
            up = dict(sc)
            dn = dict(sc)
            up[key] = arr.copy()
            dn[key] = arr.copy()
            up[key][idx] += h
            dn[key][idx] -= h
            fd = (loss(up) - loss(dn)) / (2 * h)
            scale = max(1e-3, np.abs(grads[key]).max())
            assert abs(fd - g) <= 2e-5 * scale, (key, idx, fd, g)
            checked += 1
    assert checked >= 40
    assert np.abs(grads["means"]).max() > 0 and np.abs(grads["sh"]).max() > 0
