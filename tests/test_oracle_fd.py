"""Pins of the oracle's finite-difference slope estimate, the input of the
classical bicubic comparator (Sec. "Image Gradient Based Upscaling",
Spline Interpolation paragraph; Sec. "Motivational Example").

Checked against: NumPy's gradient (central differences inside, first-order
one-sided differences on the border), exactness on quadratic images, and the
textbook identity that Hermite patches with central-difference slopes are
Keys' cubic convolution with a = -1/2 (Catmull-Rom) away from the border.
"""
import numpy as np


def _keys(s, a=-0.5):
    s = np.abs(s)
    return np.where(s <= 1, (a + 2) * s ** 3 - (a + 3) * s ** 2 + 1,
                    np.where(s < 2, a * s ** 3 - 5 * a * s ** 2 + 8 * a * s - 4 * a, 0.0))


def test_fd_slopes_are_numpy_gradient(oracle):
    rng = np.random.default_rng(11)
    for (h, w) in [(2, 2), (2, 5), (7, 3), (13, 17)]:
        f = rng.standard_normal((h, w, 3))
        out = oracle.fd_slopes(f)
        assert out.shape == (h, w, 12)
        gx = np.gradient(f, axis=1)
        gy = np.gradient(f, axis=0)
        np.testing.assert_array_equal(out[..., 0:3], f)
        np.testing.assert_allclose(out[..., 3:6], gx, atol=1e-15)
        np.testing.assert_allclose(out[..., 6:9], gy, atol=1e-15)
        np.testing.assert_allclose(out[..., 9:12], np.gradient(gx, axis=0), atol=1e-15)


def test_fd_slopes_exact_on_quadratics(oracle):
    """Central differences are exact for quadratics; f_xy of a*x*y is a."""
    h, w = 6, 9
    y, x = np.meshgrid(np.arange(h, dtype=float), np.arange(w, dtype=float), indexing="ij")
    f = np.stack([0.3 * x * x - 0.2 * y + 1.0, 0.7 * x * y, -0.4 * y * y + 0.1 * x * y], axis=2)
    out = oracle.fd_slopes(f)
    inner = (slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(out[inner][..., 3], (0.6 * x)[inner], atol=1e-13)
    np.testing.assert_allclose(out[inner][..., 6], np.full((h - 2, w - 2), -0.2), atol=1e-13)
    np.testing.assert_allclose(out[inner][..., 4], (0.7 * y)[inner], atol=1e-13)
    np.testing.assert_allclose(out[inner][..., 7], (0.7 * x)[inner], atol=1e-13)
    np.testing.assert_allclose(out[inner][..., 10], np.full((h - 2, w - 2), 0.7), atol=1e-13)
    np.testing.assert_allclose(out[inner][..., 11], np.full((h - 2, w - 2), 0.1), atol=1e-13)
    np.testing.assert_allclose(out[inner][..., 8], (-0.8 * y + 0.1 * x)[inner], atol=1e-13)
    # border: a one-sided difference of a function linear along that axis is exact
    np.testing.assert_allclose(out[:, 0, 4], 0.7 * np.arange(h), atol=1e-13)
    np.testing.assert_allclose(out[:, -1, 4], 0.7 * np.arange(h), atol=1e-13)
    np.testing.assert_allclose(out[0, :, 6], np.full(w, -0.2), atol=1e-13)
    np.testing.assert_allclose(out[-1, :, 10], np.full(w, 0.7), atol=1e-13)


def test_fd_upscale_is_catmull_rom(oracle):
    """oracle.upscale fed oracle.fd_slopes equals separable Keys a = -1/2
    cubic convolution at every output pixel whose 4x4 stencil is interior."""
    rng = np.random.default_rng(12)
    h, w, s = 10, 12, 3
    H, W = h * s, w * s
    f = rng.standard_normal((h, w, 3))
    up = oracle.upscale(oracle.fd_slopes(f), W, H)
    X = np.arange(W)
    Y = np.arange(H)
    u = (X + 0.5) / s - 0.5
    v = (Y + 0.5) / s - 0.5
    i0 = np.floor(u).astype(int)
    j0 = np.floor(v).astype(int)
    ok_x = (i0 >= 1) & (i0 <= w - 3)
    ok_y = (j0 >= 1) & (j0 <= h - 3)
    checked = 0
    for yy in np.nonzero(ok_y)[0]:
        for xx in np.nonzero(ok_x)[0]:
            ref = np.zeros(3)
            for m in range(-1, 3):
                for n in range(-1, 3):
                    wgt = _keys(u[xx] - (i0[xx] + m)) * _keys(v[yy] - (j0[yy] + n))
                    ref += wgt * f[j0[yy] + n, i0[xx] + m]
            np.testing.assert_allclose(up[yy, xx], ref, atol=1e-12)
            checked += 1
    assert checked > 0.5 * H * W
