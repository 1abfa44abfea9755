"""Pins of the oracle's bicubic Hermite patch (Sec. "Image Gradient Based
Upscaling"; Supplement "Spline Image Interpolation").

Checked against: the matrix C printed in the paper (golden fixture), the
interpolation conditions at the nodes, exact reproduction of bicubic
polynomials, continuity across cell edges, the textbook reduction to
Catmull-Rom (Keys a = -1/2) cubic convolution when finite-difference slopes
are fed in, and SciPy's 1D cubic Hermite spline.
"""
import os

import numpy as np
import pytest
from scipy.interpolate import CubicHermiteSpline

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hermite_C.txt")


def _golden_C():
    return np.loadtxt(GOLDEN, comments="#")


def test_C_matches_paper(oracle):
    C, Ci = oracle.hermite_matrices()
    Cg = _golden_C()
    np.testing.assert_array_equal(C, Cg)
    np.testing.assert_allclose(Ci, np.linalg.inv(Cg), atol=1e-15)
    np.testing.assert_allclose(C @ Ci, np.eye(4), atol=1e-15)


def test_patch_equals_matrix_form(oracle):
    """p = [1 x x^2 x^3] C^-1 F C^-T [1 y y^2 y^3]^T with F laid out as printed."""
    rng = np.random.default_rng(0)
    img = rng.standard_normal((2, 2, 12))
    Ci = np.linalg.inv(_golden_C())
    u = rng.uniform(0, 1, 50)
    v = rng.uniform(0, 1, 50)
    out = oracle.patch_eval(img, u, v)
    for ch in range(3):
        f = lambda ox, oy, q: img[oy, ox, 3 * q + ch]
        F = np.array([[f(0, 0, 0), f(0, 1, 0), f(0, 0, 2), f(0, 1, 2)],
                      [f(1, 0, 0), f(1, 1, 0), f(1, 0, 2), f(1, 1, 2)],
                      [f(0, 0, 1), f(0, 1, 1), f(0, 0, 3), f(0, 1, 3)],
                      [f(1, 0, 1), f(1, 1, 1), f(1, 0, 3), f(1, 1, 3)]])
        A = Ci @ F @ Ci.T
        X = np.stack([np.ones_like(u), u, u ** 2, u ** 3], 1)
        Y = np.stack([np.ones_like(v), v, v ** 2, v ** 3], 1)
        np.testing.assert_allclose(out[:, ch], np.einsum("ni,ij,nj->n", X, A, Y), atol=1e-13)


def test_node_reproduction(oracle):
    """Value and x, y, xy derivatives of the spline equal the data at every node."""
    rng = np.random.default_rng(1)
    h, w = 5, 7
    img = rng.standard_normal((h, w, 12))
    jj, ii = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    out = oracle.patch_eval(img, ii.reshape(-1).astype(float), jj.reshape(-1).astype(float))
    np.testing.assert_allclose(out, img.reshape(-1, 12), atol=1e-12)


def _poly_img(a, h, w):
    """Values and exact derivatives of q(x,y) = sum a_ij x^i y^j at the nodes."""
    jj, ii = np.meshgrid(np.arange(h, dtype=float), np.arange(w, dtype=float), indexing="ij")
    img = np.zeros((h, w, 12))
    for ch in range(3):
        for i in range(4):
            for j in range(4):
                c = a[ch, i, j]
                img[..., ch] += c * ii ** i * jj ** j
                if i:
                    img[..., 3 + ch] += c * i * ii ** (i - 1) * jj ** j
                if j:
                    img[..., 6 + ch] += c * j * ii ** i * jj ** (j - 1)
                if i and j:
                    img[..., 9 + ch] += c * i * j * ii ** (i - 1) * jj ** (j - 1)
    return img


def test_bicubic_reproduction_with_border_extrapolation(oracle):
    rng = np.random.default_rng(2)
    h, w = 4, 6
    a = rng.standard_normal((3, 4, 4)) * 0.3
    img = _poly_img(a, h, w)
    u = rng.uniform(-0.5, w - 0.5, 400)
    v = rng.uniform(-0.5, h - 0.5, 400)
    out = oracle.patch_eval(img, u, v)
    for ch in range(3):
        ref = sum(a[ch, i, j] * u ** i * v ** j for i in range(4) for j in range(4))
        np.testing.assert_allclose(out[:, ch], ref, rtol=1e-11, atol=1e-11)


def test_continuity_across_cell_edges(oracle):
    """C^1 across cell edges: value and first derivatives agree on both sides."""
    rng = np.random.default_rng(3)
    img = rng.standard_normal((5, 6, 12))
    eps = 1e-7
    v = rng.uniform(0.0, 4.0, 100)
    for i in range(1, 5):
        lo = oracle.patch_eval(img, np.full(100, i - eps), v)
        hi = oracle.patch_eval(img, np.full(100, i + eps), v)
        np.testing.assert_allclose(lo[:, :9], hi[:, :9], atol=1e-5)
    u = rng.uniform(0.0, 5.0, 100)
    for j in range(1, 4):
        lo = oracle.patch_eval(img, u, np.full(100, j - eps))
        hi = oracle.patch_eval(img, u, np.full(100, j + eps))
        np.testing.assert_allclose(lo[:, :9], hi[:, :9], atol=1e-5)


def test_scale_one_is_identity(oracle):
    rng = np.random.default_rng(4)
    img = rng.standard_normal((6, 9, 12))
    up = oracle.upscale(img, 9, 6)
    np.testing.assert_allclose(up, img[..., :3], atol=1e-13)


def _keys(s, a=-0.5):
    s = np.abs(s)
    return np.where(s <= 1, (a + 2) * s ** 3 - (a + 3) * s ** 2 + 1,
                    np.where(s < 2, a * s ** 3 - 5 * a * s ** 2 + 8 * a * s - 4 * a, 0.0))


def test_fd_slopes_reduce_to_catmull_rom(oracle):
    """Classical bicubic: central-difference slopes turn the patch into Keys'
    cubic convolution with a = -1/2 on interior cells."""
    rng = np.random.default_rng(5)
    h, w = 9, 11
    f = rng.standard_normal((h, w, 3))
    img = np.zeros((h, w, 12))
    img[..., 0:3] = f
    img[1:-1, 1:-1, 3:6] = (f[1:-1, 2:] - f[1:-1, :-2]) / 2
    img[1:-1, 1:-1, 6:9] = (f[2:, 1:-1] - f[:-2, 1:-1]) / 2
    img[1:-1, 1:-1, 9:12] = (f[2:, 2:] - f[2:, :-2] - f[:-2, 2:] + f[:-2, :-2]) / 4
    # interior cells whose 4x4 stencil has FD slopes everywhere: i in [1, w-3]
    u = rng.uniform(1, w - 2, 300)
    v = rng.uniform(1, h - 2, 300)
    u = np.minimum(u, w - 2 - 1e-9)
    v = np.minimum(v, h - 2 - 1e-9)
    out = oracle.patch_eval(img, u, v)
    i0 = np.floor(u).astype(int)
    j0 = np.floor(v).astype(int)
    ref = np.zeros((300, 3))
    for m in range(-1, 3):
        for n in range(-1, 3):
            wgt = _keys(u - (i0 + m)) * _keys(v - (j0 + n))
            ref += wgt[:, None] * f[j0 + n, i0 + m]
    np.testing.assert_allclose(out[:, :3], ref, atol=1e-12)


def test_x_only_field_is_scipy_cubic_hermite(oracle):
    rng = np.random.default_rng(6)
    h, w = 4, 10
    g = rng.standard_normal((w, 3))
    gp = rng.standard_normal((w, 3))
    img = np.zeros((h, w, 12))
    img[..., 0:3] = g[None]
    img[..., 3:6] = gp[None]
    u = rng.uniform(0, w - 1, 200)
    v = rng.uniform(0, h - 1, 200)
    out = oracle.patch_eval(img, u, v)
    for ch in range(3):
        ref = CubicHermiteSpline(np.arange(w, dtype=float), g[:, ch], gp[:, ch])(u)
        np.testing.assert_allclose(out[:, ch], ref, atol=1e-12)
    np.testing.assert_allclose(out[:, 6:12], 0.0, atol=1e-14)


def test_upscale_pixel_mapping(oracle):
    """High-res pixel X samples u = (X + 1/2) w / W - 1/2 (pixel centres on
    integers): for an upscale factor 3 every third pixel lands on a node."""
    rng = np.random.default_rng(7)
    img = rng.standard_normal((5, 4, 12))
    up = oracle.upscale(img, 12, 15)
    np.testing.assert_allclose(up[1::3, 1::3], img[..., :3], atol=1e-13)
    # a fractional factor: compare with the explicit patch evaluation
    W, H = 10, 7
    up = oracle.upscale(img, W, H)
    Yg, Xg = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    u = (Xg + 0.5) * 4 / W - 0.5
    v = (Yg + 0.5) * 5 / H - 0.5
    ref = oracle.patch_eval(img, u.reshape(-1), v.reshape(-1))[:, :3].reshape(H, W, 3)
    np.testing.assert_allclose(up, ref, atol=1e-14)


def test_error_bound_weights(oracle):
    """max over t in [0,1] of |h10| + |h11| is 1/4 (derivative weights of the
    1D Hermite basis); the basis is read from the oracle's C^-1."""
    _, Ci = oracle.hermite_matrices()
    t = np.linspace(0, 1, 100001)
    T = np.stack([np.ones_like(t), t, t * t, t ** 3], 1)
    Hb = T @ Ci  # columns: weights of f(0), f(1), f'(0), f'(1)
    assert abs((np.abs(Hb[:, 2]) + np.abs(Hb[:, 3])).max() - 0.25) < 1e-9
    np.testing.assert_allclose(Hb[:, 0] + Hb[:, 1], 1.0, atol=1e-14)
