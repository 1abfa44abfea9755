"""Seeded synthetic scenes, cameras and render settings.

This module only draws inputs: it holds none of the method's arithmetic and
is shared by the HIP path's tests and benchmark and by the CPU oracle's tests.
All arrays are FP32 (the precision of a trained 3D Gaussian Splatting model);
camera numbers are FP32 values too, so both sides see identical inputs.

Workloads (arXiv 2503.14171 measures on trained MipNeRF360, Tanks&Temples and
Deep Blending models, which are not available here; these synthetic scenes
stand in for them with the same Gaussian counts and image sizes):

* ``tiny``      10k Gaussians, means U[-1,1]^3, log-scales N(-4, 0.5), SH degree 0
                with RGB uniform in [0,1]; 128x128 rendered, upscaled x2.
* ``clusters``  500k Gaussians from a mixture of 32 anisotropic clusters,
                log-scales N(-5, 0.7), SH degree 3 coefficients N(0, 0.2);
                960x540 rendered, upscaled x2 to 1920x1080.
* ``scene``     3M Gaussians: 2.4M from the cluster process plus 0.6M on a
                shell of radius 10 (20 %); same scales, SH and opacity;
                960x540 rendered, upscaled x2, x3, x4 (up to 3840x2160).
* ``batch``     1M Gaussians of the ``scene`` process, seen by 8 stereo pairs
                (16 views, :func:`stereo_rig`): pairs 0-3 at 720x800 upscaled
                x2 to 1440x1600, pairs 4-7 at 480x540 upscaled x3 to 1440x1620.

Draw order from ``numpy.random.default_rng(seed)``: means, log-scales,
quaternions, opacity logits, SH coefficients.  Opacity is sigmoid(N(0, 1)).
"""
from __future__ import annotations

import math

import numpy as np

WORKLOADS = {
    "tiny": dict(n=10_000, kind="uniform", sh_degree=0, size=(128, 128), scales=(2,), seed=1),
    "clusters": dict(n=500_000, kind="clusters", sh_degree=3, size=(960, 540), scales=(2,), seed=2),
    "scene": dict(n=3_000_000, kind="scene", sh_degree=3, size=(960, 540), scales=(2, 3, 4), seed=3),
    "batch": dict(n=1_000_000, kind="scene", sh_degree=3, size=None, scales=None, seed=4),
}


def render_config(sh_degree: int, tile_size: int = 16, **over) -> dict:
    """Render settings: tile size, SH degree, dilation (px^2 added to the 2D
    covariance diagonal), alpha_min (skip), alpha_max (clamp), t_min (stop),
    background colour, and the rasterizer's LDS batch (0 = one splat per
    thread; a speed setting only)."""
    cfg = dict(tile_size=tile_size, sh_degree=sh_degree, dilation=0.3, alpha_min=1.0 / 255.0,
               alpha_max=0.99, t_min=1e-4, bg=(0.0, 0.0, 0.0), batch=0)
    cfg.update(over)
    return cfg


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4), dtype=np.float32).astype(np.float64)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def _random_rotations(rng, k):
    """k random rotation matrices: QR of Gaussian matrices with the sign fixed."""
    g = rng.standard_normal((k, 3, 3))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diagonal(r, axis1=1, axis2=2))[:, None, :]
    det = np.linalg.det(q)
    q[:, :, 0] *= det[:, None]
    return q


def _cluster_means(rng, n, n_clusters=32):
    centres = rng.uniform(-1.0, 1.0, (n_clusters, 3))
    stds = rng.uniform(0.05, 0.25, (n_clusters, 3))
    rots = _random_rotations(rng, n_clusters)
    which = rng.integers(0, n_clusters, n)
    local = rng.standard_normal((n, 3)) * stds[which]
    return centres[which] + np.einsum("nij,nj->ni", rots[which], local)


def make_scene(kind: str, n: int, seed: int, sh_degree: int) -> dict:
    """Synthetic Gaussians: means [n,3], log_scales [n,3], quats [n,4] (w,x,y,z),
    opacity [n] (after the sigmoid), sh [n,(d+1)^2,3]."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        means = rng.uniform(-1.0, 1.0, (n, 3))
        ls_mu, ls_sd = -4.0, 0.5
    elif kind == "clusters":
        means = _cluster_means(rng, n)
        ls_mu, ls_sd = -5.0, 0.7
    elif kind == "scene":
        n_shell = n // 5
        m_cl = _cluster_means(rng, n - n_shell)
        d = rng.standard_normal((n_shell, 3))
        m_sh = 10.0 * d / np.linalg.norm(d, axis=1, keepdims=True)
        means = np.concatenate([m_cl, m_sh], 0)
        ls_mu, ls_sd = -5.0, 0.7
    else:
        raise ValueError(f"unknown scene kind {kind!r}")
    log_scales = rng.normal(ls_mu, ls_sd, (n, 3))
    quats = _unit_quats(rng, n)
    logits = rng.standard_normal(n)
    opacity = 1.0 / (1.0 + np.exp(-logits))
    nb = (sh_degree + 1) ** 2
    if kind == "uniform":
        # degree-0 coefficient such that the evaluated colour Y_00 k + 1/2 is
        # the drawn RGB (Y_00 = 1 / (2 sqrt(pi)))
        rgb = rng.uniform(0.0, 1.0, (n, 3))
        sh = np.zeros((n, nb, 3), np.float32)
        sh[:, 0, :] = (rgb - 0.5) * (2.0 * math.sqrt(math.pi))
    else:
        sh = rng.standard_normal((n, nb, 3), dtype=np.float32) * np.float32(0.2)
    return dict(means=np.ascontiguousarray(means, np.float32),
                log_scales=np.ascontiguousarray(log_scales, np.float32),
                quats=np.ascontiguousarray(quats, np.float32),
                opacity=np.ascontiguousarray(opacity, np.float32),
                sh=np.ascontiguousarray(sh, np.float32), sh_degree=sh_degree)


def workload_scene(name: str, n: int | None = None, seed: int | None = None) -> dict:
    w = WORKLOADS[name]
    return make_scene(w["kind"], w["n"] if n is None else n, w["seed"] if seed is None else seed,
                      w["sh_degree"])


def make_camera(width: int, height: int, eye=(0.0, 0.0, -3.0), target=(0.0, 0.0, 0.0),
                down=(0.0, 1.0, 0.0), fov_x_deg: float = 60.0, near_plane: float = 0.2,
                far_plane: float = 100.0) -> dict:
    """Pinhole camera with OpenCV axes (+x right, +y down, +z forward), looking
    from ``eye`` at ``target``; horizontal field of view ``fov_x_deg``;
    principal point at the image centre, pixel centres at integer coordinates;
    Gaussians closer than ``near_plane`` or farther than ``far_plane`` (0: no
    far plane) are culled.  The default far plane, 100, lies beyond every
    Gaussian of the workloads seen from their cameras (scene extent 10,
    cameras at distance 3), so it culls nothing there."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    x = np.cross(np.asarray(down, np.float64), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z], 0)
    t = -R @ eye
    view = np.concatenate([R, t[:, None]], 1).astype(np.float32)
    f = width / (2.0 * math.tan(math.radians(fov_x_deg) / 2.0))
    return dict(width=int(width), height=int(height), fx=float(np.float32(f)), fy=float(np.float32(f)),
                cx=float(np.float32((width - 1) / 2.0)), cy=float(np.float32((height - 1) / 2.0)),
                view=view, cam_pos=eye.astype(np.float32), near_plane=float(np.float32(near_plane)),
                far_plane=float(np.float32(far_plane)))


def scale_camera(cam: dict, width: int, height: int) -> dict:
    """The same camera with a width x height raster: focal lengths scale with the
    raster and c' = (c + 1/2) s - 1/2, so that pixel X of the new raster sees
    the image-plane point that u = (X + 1/2) w / W - 1/2 denotes on the old one."""
    sx = width / cam["width"]
    sy = height / cam["height"]
    out = dict(cam)
    out.update(width=int(width), height=int(height),
               fx=float(np.float32(cam["fx"] * sx)), fy=float(np.float32(cam["fy"] * sy)),
               cx=float(np.float32((cam["cx"] + 0.5) * sx - 0.5)),
               cy=float(np.float32((cam["cy"] + 0.5) * sy - 0.5)))
    return out


def depth_bound(scene: dict, cam: dict) -> float:
    """A far plane that culls none of the scene's Gaussians seen from `cam`:
    the camera's distance from the origin plus the largest distance of a mean
    from it (a bound on every mean's camera-space depth), rounded up."""
    m = np.asarray(scene["means"], np.float64)
    r = np.sqrt((m[np.isfinite(m).all(1)] ** 2).sum(1)).max(initial=0.0)
    d = float(np.linalg.norm(np.asarray(cam["cam_pos"], np.float64)))
    return float(math.ceil(1.001 * (d + r) + 1e-3))


def orbit_camera(width: int, height: int, azimuth_deg: float, elevation_deg: float,
                 radius: float = 3.0, **kw) -> dict:
    a, e = math.radians(azimuth_deg), math.radians(elevation_deg)
    eye = (radius * math.cos(e) * math.sin(a), -radius * math.sin(e), -radius * math.cos(e) * math.cos(a))
    return make_camera(width, height, eye=eye, **kw)


def workload_camera(name: str) -> dict:
    W, H = WORKLOADS[name]["size"]
    return make_camera(W, H)


def stereo_rig(n_pairs: int = 8, seed: int = 4, baseline: float = 0.064, radius: float = 3.0):
    """Stereo pairs on a random orbit around the origin: azimuth ~ U[0, 360),
    elevation ~ U[-20, 20] degrees, distance ``radius``; the two eyes sit at
    -/+ baseline/2 along the pair's camera x axis with parallel optical axes.
    The first half of the pairs renders 720x800 (upscaled x2 to 1440x1600),
    the second half 480x540 (x3 to 1440x1620).  Returns (low-res cameras,
    high-res sizes), two entries per pair (left eye first)."""
    rng = np.random.default_rng(seed)
    cams, hi = [], []
    for k in range(n_pairs):
        a = math.radians(rng.uniform(0.0, 360.0))
        e = math.radians(rng.uniform(-20.0, 20.0))
        centre = np.array([radius * math.cos(e) * math.sin(a), -radius * math.sin(e),
                           -radius * math.cos(e) * math.cos(a)])
        fwd = -centre / np.linalg.norm(centre)
        right = np.cross(np.array([0.0, 1.0, 0.0]), fwd)
        right /= np.linalg.norm(right)
        (w, h), s = ((720, 800), 2) if k < n_pairs // 2 else ((480, 540), 3)
        for side in (-0.5, 0.5):
            eye = centre + side * baseline * right
            cams.append(make_camera(w, h, eye=tuple(eye), target=tuple(eye + fwd)))
            hi.append((w * s, h * s))
    return cams, hi
