"""Python access to the FP64 CPU oracle (``gsoracle.c``).

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` use this module.  It shares no code with the HIP
implementation and imports nothing from it; scenes and cameras arrive as plain
NumPy arrays and dicts.

Functions (each cites the passage of arXiv 2503.14171 it follows; the C file
holds the arithmetic):

* ``project``       -- EWA projection and SH colour (Sec. "Differentiable 3D
                       Gaussian Splatting", projection equation Sigma' = J W Sigma W^T J^T).
* ``depth_order``   -- front-to-back order of the surviving Gaussians (same section:
                       Gaussians are sorted by the depth of their mean).
* ``composite``     -- alpha blending with dI/dx, dI/dy, d2I/dxdy (Suppl. "3DGS
                       Gradient Computation - Forward pass").
* ``patch_eval`` / ``upscale`` -- bicubic patch F = C A C^T (Sec. "Image Gradient
                       Based Upscaling"; Suppl. "Spline Image Interpolation").
* ``tile_rects`` / ``tile_lists`` -- the tiling that an accelerated renderer may
                       use; it must not change the composited result.
* ``upscale_adjoint`` / ``composite_adjoint`` / ``project_vjp`` / ``loss_grad``
                    -- gradients of a loss on the upscaled image with respect
                       to the low-res buffers, the 2D splat parameters and the
                       3D Gaussian parameters (Suppl. "3DGS Gradient Computation -
                       Backward pass"; the projection's Jacobian by FP64 central
                       differences of ``project``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsoracle.c")
_LIB = os.path.join(_HERE, "libgsoracle.so")
# GS_ORACLE_SANITIZE=1 builds and loads a copy instrumented with AddressSanitizer
# and UndefinedBehaviorSanitizer (the process must preload their runtimes)
_SANITIZE = os.environ.get("GS_ORACLE_SANITIZE") == "1"
if _SANITIZE:
    _LIB = os.path.join(_HERE, "libgsoracle_san.so")

# Relative margins inside which a threshold decision counts as a near tie
# (several outcomes are then correct, see ``composite``).
TIE_ALPHA = 2e-5
TIE_T = 1e-4


def build(force: bool = False) -> str:
    """Compile ``gsoracle.c`` with gcc (plain x86-64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        if _SANITIZE:
            cmd[1:1] = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("view", ctypes.c_double * 12), ("cam_pos", ctypes.c_double * 3),
                ("near_plane", ctypes.c_double), ("far_plane", ctypes.c_double)]


class _Config(ctypes.Structure):
    _fields_ = [("sh_degree", ctypes.c_int32), ("dilation", ctypes.c_double),
                ("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("t_min", ctypes.c_double), ("bg", ctypes.c_double * 3),
                ("tie_alpha", ctypes.c_double), ("tie_t", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        lib.or_sh_basis.argtypes = [i32, i64, P, P]
        lib.or_project.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P]
        lib.or_composite.argtypes = [i64, P, P, P, P, P, P, i64, P, P, P, P, P, P, P]
        lib.or_hermite_matrices.argtypes = [P, P]
        lib.or_patch_eval.argtypes = [P, i32, i32, i64, P, P, P]
        lib.or_upscale.argtypes = [P, i32, i32, i32, i32, i64, P, P, P]
        lib.or_upscale_adjoint.argtypes = [P, i32, i32, i32, i32, P]
        lib.or_composite_adjoint.argtypes = [i64, P, P, P, P, P, P, i64, P, P, P, P]
        lib.or_max_variants.restype = i32
        lib.or_num_threads.restype = i32
        for f in ("or_sh_basis", "or_project", "or_composite", "or_hermite_matrices",
                  "or_patch_eval", "or_upscale", "or_upscale_adjoint", "or_composite_adjoint"):
            getattr(lib, f).restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _camera(cam: dict) -> _Camera:
    c = _Camera()
    c.width, c.height = int(cam["width"]), int(cam["height"])
    # camera values are FP32 numbers; promote exactly
    c.fx, c.fy = float(np.float32(cam["fx"])), float(np.float32(cam["fy"]))
    c.cx, c.cy = float(np.float32(cam["cx"])), float(np.float32(cam["cy"]))
    view = np.asarray(cam["view"], np.float32).reshape(12).astype(np.float64)
    c.view[:] = list(view)
    c.cam_pos[:] = list(np.asarray(cam["cam_pos"], np.float32).astype(np.float64))
    c.near_plane = float(np.float32(cam["near_plane"]))
    c.far_plane = float(np.float32(cam.get("far_plane", 0.0)))
    return c


def _config(cfg: dict, tie_alpha=TIE_ALPHA, tie_t=TIE_T) -> _Config:
    c = _Config()
    c.sh_degree = int(cfg["sh_degree"])
    c.dilation = float(np.float32(cfg["dilation"]))
    c.alpha_min = float(np.float32(cfg["alpha_min"]))
    c.alpha_max = float(np.float32(cfg["alpha_max"]))
    c.t_min = float(np.float32(cfg["t_min"]))
    c.bg[:] = [float(np.float32(v)) for v in cfg["bg"]]
    c.tie_alpha = tie_alpha
    c.tie_t = tie_t
    return c


def sh_basis(deg: int, dirs: np.ndarray) -> np.ndarray:
    """Real orthonormal SH basis values [n, (deg+1)^2] at directions [n, 3]."""
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    out = np.empty((dirs.shape[0], (deg + 1) ** 2), np.float64)
    _load().or_sh_basis(deg, dirs.shape[0], _ptr(dirs), _ptr(out))
    return out


def project(scene: dict, cam: dict, cfg: dict) -> dict:
    """FP64 projection of every Gaussian of ``scene`` (FP32 or FP64 arrays) into ``cam``."""
    n = scene["means"].shape[0]
    # FP32 scene values promote exactly; FP64 values (finite differences) pass as they are
    f64 = lambda k: np.ascontiguousarray(scene[k], np.float64)
    means, ls, quats, opa, sh = f64("means"), f64("log_scales"), f64("quats"), f64("opacity"), f64("sh")
    assert sh.shape[1] == (cfg["sh_degree"] + 1) ** 2
    out = dict(valid=np.empty(n, np.int32), mean2d=np.empty((n, 2)), cov2d=np.empty((n, 3)),
               conic=np.empty((n, 3)), opacity=np.empty(n), rgb=np.empty((n, 3)),
               depth=np.empty(n), bbox=np.empty((n, 4)))
    c, k = _camera(cam), _config(cfg)
    _load().or_project(n, _ptr(means), _ptr(ls), _ptr(quats), _ptr(opa), _ptr(sh),
                       ctypes.byref(c), ctypes.byref(k), _ptr(out["valid"]), _ptr(out["mean2d"]),
                       _ptr(out["cov2d"]), _ptr(out["conic"]), _ptr(out["opacity"]),
                       _ptr(out["rgb"]), _ptr(out["depth"]), _ptr(out["bbox"]))
    out["valid"] = out["valid"].astype(bool)
    return out


def depth_order(proj: dict) -> np.ndarray:
    """Indices of the valid Gaussians, front to back.

    The order decision is taken on camera z rounded to FP32 (the precision in
    which a renderer keys its sort), ties broken by Gaussian index."""
    idx = np.nonzero(proj["valid"])[0]
    z32 = proj["depth"][idx].astype(np.float32)
    return idx[np.lexsort((idx, z32))].astype(np.int64)


def composite(proj: dict, order: np.ndarray, cfg: dict, px, py, variants: bool = False,
              tie_alpha=TIE_ALPHA, tie_t=TIE_T) -> dict:
    """Blend the Gaussians ``order`` (front to back) at image points (px, py).

    Returns ``out`` [n, 12] (I rgb, I_x rgb, I_y rgb, I_xy rgb), ``n_blend``
    and ``n_amb`` (near-tie decisions met).  With ``variants`` also
    ``variants`` [n, 8, 12] and ``n_var``: every result obtained by inverting
    any subset of (at most three) near-tie decisions -- all of them are correct
    results of the method; ``n_var == 0`` marks a point with more near ties."""
    px = np.ascontiguousarray(px, np.float64).reshape(-1)
    py = np.ascontiguousarray(py, np.float64).reshape(-1)
    n = px.shape[0]
    order = np.ascontiguousarray(order, np.int64)
    res = dict(out=np.empty((n, 12)), n_blend=np.empty(n, np.int64), n_amb=np.empty(n, np.int32))
    vptr = nptr = None
    if variants:
        nv = _load().or_max_variants()
        res["variants"] = np.zeros((n, nv, 12))
        res["n_var"] = np.empty(n, np.int32)
        vptr, nptr = _ptr(res["variants"]), _ptr(res["n_var"])
    mean2d = np.ascontiguousarray(proj["mean2d"], np.float64)
    conic = np.ascontiguousarray(proj["conic"], np.float64)
    opa = np.ascontiguousarray(proj["opacity"], np.float64)
    rgb = np.ascontiguousarray(proj["rgb"], np.float64)
    k = _config(cfg, tie_alpha, tie_t)
    _load().or_composite(order.shape[0], _ptr(order), _ptr(mean2d), _ptr(conic), _ptr(opa),
                         _ptr(rgb), ctypes.byref(k), n, _ptr(px), _ptr(py), _ptr(res["out"]),
                         _ptr(res["n_blend"]), _ptr(res["n_amb"]), vptr, nptr)
    return res


def render(scene: dict, cam: dict, cfg: dict, variants: bool = False) -> dict:
    """Whole low-res image: ``img`` [H, W, 12] plus per-pixel statistics."""
    proj = project(scene, cam, cfg)
    order = depth_order(proj)
    H, W = int(cam["height"]), int(cam["width"])
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    r = composite(proj, order, cfg, xx.reshape(-1), yy.reshape(-1), variants=variants)
    out = dict(img=r["out"].reshape(H, W, 12), n_blend=r["n_blend"].reshape(H, W),
               n_amb=r["n_amb"].reshape(H, W), proj=proj, order=order)
    if variants:
        out["variants"] = r["variants"].reshape(H, W, -1, 12)
        out["n_var"] = r["n_var"].reshape(H, W)
    return out


def num_threads() -> int:
    """Host threads the oracle's parallel loops use."""
    return int(_load().or_num_threads())


def hermite_matrices():
    """(C, C^-1) as the oracle uses them."""
    C = np.empty((4, 4))
    Ci = np.empty((4, 4))
    _load().or_hermite_matrices(_ptr(C), _ptr(Ci))
    return C, Ci


def patch_eval(img: np.ndarray, u, v) -> np.ndarray:
    """Patch value and derivatives [n, 12] (p rgb, p_x, p_y, p_xy) at low-res coords (u, v)."""
    img = np.ascontiguousarray(img, np.float64)
    h, w = img.shape[:2]
    assert img.shape[2] == 12 and w >= 2 and h >= 2
    u = np.ascontiguousarray(u, np.float64).reshape(-1)
    v = np.ascontiguousarray(v, np.float64).reshape(-1)
    out = np.empty((u.shape[0], 12))
    _load().or_patch_eval(_ptr(img), w, h, u.shape[0], _ptr(u), _ptr(v), _ptr(out))
    return out


def upscale(img: np.ndarray, W: int, H: int, X=None, Y=None) -> np.ndarray:
    """Upscaled rgb at high-res pixels (X, Y) ([n, 3]), or the whole [H, W, 3] image."""
    img = np.ascontiguousarray(img, np.float64)
    h, w = img.shape[:2]
    whole = X is None
    if whole:
        Yg, Xg = np.meshgrid(np.arange(H, dtype=np.int32), np.arange(W, dtype=np.int32), indexing="ij")
        X, Y = Xg.reshape(-1), Yg.reshape(-1)
    X = np.ascontiguousarray(X, np.int32).reshape(-1)
    Y = np.ascontiguousarray(Y, np.int32).reshape(-1)
    out = np.empty((X.shape[0], 3))
    _load().or_upscale(_ptr(img), w, h, W, H, X.shape[0], _ptr(X), _ptr(Y), _ptr(out))
    return out.reshape(H, W, 3) if whole else out


def upscale_cell(X, Y, w: int, h: int, W: int, H: int):
    """Low-res cell (i, j) whose patch serves high-res pixel (X, Y)."""
    u = (np.asarray(X, np.float64) + 0.5) * w / W - 0.5
    v = (np.asarray(Y, np.float64) + 0.5) * h / H - 0.5
    i = np.clip(np.floor(u).astype(np.int64), 0, w - 2)
    j = np.clip(np.floor(v).astype(np.int64), 0, h - 2)
    return i, j


# ---------------------------------------------------------------------------
# Tiling.  A tiled renderer may only visit, for each pixel, the Gaussians
# whose tile rectangle covers the pixel's tile.  The rectangle is the exact
# alpha_min support box widened by RECT_MARGIN pixels, clipped to the image.
# ---------------------------------------------------------------------------
RECT_MARGIN = 0.25


def tile_rects(proj: dict, W: int, H: int, tile: int) -> np.ndarray:
    """[n, 4] int tile rectangles [tx0, ty0, tx1, ty1) (all zero when empty)."""
    n = proj["valid"].shape[0]
    rect = np.zeros((n, 4), np.int32)
    v = proj["valid"]
    b = proj["bbox"]
    x0 = np.ceil(b[:, 0] - RECT_MARGIN)
    x1 = np.floor(b[:, 1] + RECT_MARGIN)
    y0 = np.ceil(b[:, 2] - RECT_MARGIN)
    y1 = np.floor(b[:, 3] + RECT_MARGIN)
    x0 = np.maximum(x0, 0)
    y0 = np.maximum(y0, 0)
    x1 = np.minimum(x1, W - 1)
    y1 = np.minimum(y1, H - 1)
    ok = v & (x0 <= x1) & (y0 <= y1)
    rect[ok, 0] = (x0[ok] // tile).astype(np.int32)
    rect[ok, 1] = (y0[ok] // tile).astype(np.int32)
    rect[ok, 2] = (x1[ok] // tile).astype(np.int32) + 1
    rect[ok, 3] = (y1[ok] // tile).astype(np.int32) + 1
    return rect


def tile_lists(depth32: np.ndarray, rect: np.ndarray, tiles_x: int, tiles_y: int):
    """Per-tile Gaussian lists in (FP32 depth, index) order.

    Returns (ids, ranges): ids is the concatenation of all tile lists in tile
    order (tile = ty * tiles_x + tx), ranges [T, 2] the [start, end) of each
    ([0, 0) for an empty tile)."""
    n = rect.shape[0]
    cnt = np.maximum(rect[:, 2] - rect[:, 0], 0) * np.maximum(rect[:, 3] - rect[:, 1], 0)
    gid = np.repeat(np.arange(n, dtype=np.int64), cnt)
    tiles = []
    for g in np.nonzero(cnt)[0]:
        tx = np.arange(rect[g, 0], rect[g, 2])
        ty = np.arange(rect[g, 1], rect[g, 3])
        tiles.append((ty[:, None] * tiles_x + tx[None, :]).reshape(-1))
    tile = np.concatenate(tiles) if tiles else np.zeros(0, np.int64)
    z = np.asarray(depth32, np.float32)[gid]
    o = np.lexsort((gid, z, tile))
    T = tiles_x * tiles_y
    counts = np.bincount(tile, minlength=T)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    ranges = np.stack([starts, starts + counts], 1)
    ranges[counts == 0] = 0  # an empty tile's range is [0, 0)
    return gid[o].astype(np.int32), ranges.astype(np.int32)


def fd_slopes(img: np.ndarray) -> np.ndarray:
    """Classical bicubic input: [h, w, 3] -> [h, w, 12] with central-difference
    slopes (one-sided on the border), f_xy the y-difference of f_x (Sec. "Image
    Gradient Based Upscaling": classical bicubic estimates gradients with
    finite differences)."""
    f = np.asarray(img, np.float64)

    def d(a, axis):
        n = a.shape[axis]
        idx = np.arange(n)
        lo, hi = np.maximum(idx - 1, 0), np.minimum(idx + 1, n - 1)
        sc = np.where(hi - lo == 2, 0.5, 1.0)
        shape = [1] * a.ndim
        shape[axis] = n
        return (np.take(a, hi, axis) - np.take(a, lo, axis)) * sc.reshape(shape)

    fx = d(f, 1)
    return np.concatenate([f, fx, d(f, 0), d(fx, 0)], axis=2)


# ---------------------------------------------------------------------------
# Gradients.  A loss L on the upscaled image reaches the Gaussians through the
# upscaler (linear: its adjoint is the transpose), the compositing (adjoint of
# the blend with the index set of every pixel held fixed) and the projection.
# ---------------------------------------------------------------------------
SPLAT_GRAD = ("mean_x", "mean_y", "conic_a", "conic_b", "conic_c", "opacity", "r", "g", "b")


def upscale_adjoint(g: np.ndarray, w: int, h: int) -> np.ndarray:
    """dL/d(low-res [h, w, 12]) for dL/d(upscaled [H, W, 3]) = g."""
    g = np.ascontiguousarray(g, np.float64)
    H, W = g.shape[:2]
    out = np.empty((h, w, 12))
    _load().or_upscale_adjoint(_ptr(g), w, h, W, H, _ptr(out))
    return out


def composite_adjoint(proj: dict, order: np.ndarray, cfg: dict, px, py, G) -> np.ndarray:
    """dL/d(2D parameters) [n, 9] (columns ``SPLAT_GRAD``) for
    L = sum_p G[p] . composite(px[p], py[p]) (G [npts, 12])."""
    px = np.ascontiguousarray(px, np.float64).reshape(-1)
    py = np.ascontiguousarray(py, np.float64).reshape(-1)
    G = np.ascontiguousarray(G, np.float64).reshape(-1, 12)
    assert G.shape[0] == px.shape[0]
    n = proj["mean2d"].shape[0]
    grad = np.zeros((n, 9))
    order = np.ascontiguousarray(order, np.int64)
    args = [np.ascontiguousarray(proj[k], np.float64) for k in ("mean2d", "conic", "opacity", "rgb")]
    k = _config(cfg)
    _load().or_composite_adjoint(order.shape[0], _ptr(order), *[_ptr(a) for a in args], ctypes.byref(k),
                                 px.shape[0], _ptr(px), _ptr(py), _ptr(G), _ptr(grad))
    return grad


PARAMS = ("means", "log_scales", "quats", "opacity", "sh")


def project_vjp(scene: dict, cam: dict, cfg: dict, d2d: np.ndarray, h: float = 1e-6) -> dict:
    """dL/d(3D parameters) for dL/d(2D parameters) = d2d [n, 9] in one view:
    the projection's Jacobian by FP64 central differences (every Gaussian's
    projection depends on its own parameters only, so one pair of projections
    per parameter slot serves all Gaussians)."""
    base = {k: np.asarray(scene[k], np.float64) for k in PARAMS}
    d2d = np.asarray(d2d, np.float64)

    def outputs(sc):
        pr = project(dict(sc, sh_degree=scene.get("sh_degree")), cam, cfg)
        return np.concatenate([pr["mean2d"], pr["conic"], pr["opacity"][:, None], pr["rgb"]], 1)

    grads = {}
    for k in PARAMS:
        arr = base[k]
        g = np.zeros_like(arr)
        flat = arr.reshape(arr.shape[0], -1)
        gflat = g.reshape(arr.shape[0], -1)
        for j in range(flat.shape[1]):
            step = h * np.maximum(1.0, np.abs(flat[:, j]))
            up = flat.copy()
            dn = flat.copy()
            up[:, j] += step
            dn[:, j] -= step
            o_up = outputs(dict(base, **{k: up.reshape(arr.shape)}))
            o_dn = outputs(dict(base, **{k: dn.reshape(arr.shape)}))
            gflat[:, j] = ((o_up - o_dn) * d2d).sum(1) / (2 * step)
        grads[k] = g
    return grads


def loss_grad(scene: dict, cams, hi_sizes, cfg: dict, g_up) -> dict:
    """dL/d(3D parameters) of L = sum_v g_up[v] . upscaled_v, summed over the
    views (cams[v] renders, hi_sizes[v] = (W, H) is its upscaled size)."""
    total = {k: np.zeros(np.shape(scene[k])) for k in PARAMS}
    for cam, (W, H), g in zip(cams, hi_sizes, g_up):
        w, h = int(cam["width"]), int(cam["height"])
        proj = project(scene, cam, cfg)
        order = depth_order(proj)
        G = upscale_adjoint(np.asarray(g).reshape(H, W, 3), w, h)
        yy, xx = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64), indexing="ij")
        d2d = composite_adjoint(proj, order, cfg, xx.reshape(-1), yy.reshape(-1), G.reshape(-1, 12))
        for k, v in project_vjp(scene, cam, cfg, d2d).items():
            total[k] += v
    return total
