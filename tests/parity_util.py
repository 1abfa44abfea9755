"""Helpers shared by the GPU parity tests: moving oracle results into the
splat record layout, comparing against the oracle's set of valid results,
and reporting max / mean errors per buffer."""
from __future__ import annotations

import json
import os

import numpy as np

TOL = 1e-4  # absolute, per channel, FP32 path vs FP64 oracle
BUFFERS = ("I", "I_x", "I_y", "I_xy")


def splat_records(proj: dict, cfg: dict) -> np.ndarray:
    """[n, 12] float32 gs_splat records holding the oracle's projection
    (mean FP64, the rest rounded to FP32), plus the rounded values the
    oracle should composite with."""
    n = proj["valid"].shape[0]
    rec = np.zeros((n, 12), np.float32)
    rec.view(np.float64)[:, 0:2] = proj["mean2d"]
    rec[:, 4:7] = proj["conic"].astype(np.float32)
    rec[:, 7] = proj["opacity"].astype(np.float32)
    rec[:, 8:11] = proj["rgb"].astype(np.float32)
    amin = float(np.float32(cfg["alpha_min"]))
    with np.errstate(divide="ignore", invalid="ignore"):
        sup = 2.0 * np.log(proj["opacity"] / amin)
    rec[:, 11] = np.where(proj["valid"], sup, 0.0).astype(np.float32)
    rec[~proj["valid"]] = 0
    return rec


def rounded_proj(proj: dict) -> dict:
    """The oracle projection with every field the splat record stores in FP32
    rounded to FP32 (so both sides composite identical parameters)."""
    out = dict(proj)
    for k in ("conic", "opacity", "rgb"):
        out[k] = proj[k].astype(np.float32).astype(np.float64)
    return out


def best_variant_error(gpu: np.ndarray, ref: dict):
    """Absolute error [N, C] against the closest of the oracle's valid results
    (the reference walk and its near-tie variants) and the mask of points the
    oracle could not resolve (more near ties than it enumerates)."""
    C = gpu.shape[1]
    base = np.abs(gpu - ref["out"][:, :C])
    if "variants" not in ref:
        return base, np.zeros(gpu.shape[0], bool)
    nv = ref["n_var"]
    masked = nv == 0
    err = base.copy()
    multi = np.nonzero(nv > 1)[0]
    for p in multi:
        cand = np.abs(ref["variants"][p, : nv[p], :C] - gpu[p][None])
        err[p] = cand[np.argmin(cand.max(1))]
    return err, masked


def summarize(err: np.ndarray, masked: np.ndarray, ref_vals: np.ndarray | None = None) -> dict:
    ok = ~masked
    s = {"points": int(err.shape[0]), "masked": int(masked.sum())}
    groups = BUFFERS if err.shape[1] == 12 else ("I",)
    for g, name in enumerate(groups):
        e = err[ok, 3 * g: 3 * g + 3]
        s[name] = {"max": float(e.max()) if e.size else 0.0, "mean": float(e.mean()) if e.size else 0.0}
        if ref_vals is not None:
            v = ref_vals[ok, 3 * g: 3 * g + 3]
            s[name]["rms"] = float(np.sqrt((v ** 2).mean())) if v.size else 0.0
    return s


def report(name: str, summary: dict):
    """Print the error summary and append it to $GS_PARITY_REPORT if set."""
    line = json.dumps({"case": name, **summary})
    print(line, flush=True)
    path = os.environ.get("GS_PARITY_REPORT")
    if path:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        with open(path, "a") as f:
            f.write(line + "\n")


def assert_within(err: np.ndarray, masked: np.ndarray, tol: float = TOL, max_masked_frac: float = 1e-3):
    ok = ~masked
    assert masked.mean() <= max_masked_frac, f"{masked.sum()} unresolved points"
    worst = err[ok].max() if ok.any() else 0.0
    if worst > tol:
        idx = np.unravel_index(np.argmax(np.where(ok[:, None], err, 0)), err.shape)
        raise AssertionError(f"max error {worst:.3e} > {tol:.1e} at point {idx[0]} channel {idx[1]}")


def upscaled_candidates(oracle, corner_variants, u, v, max_combos=256):
    """Every upscaled rgb the oracle accepts at one output pixel.

    corner_variants: four arrays [k_c, 12] of valid results at the cell's
    corners (0,0), (1,0), (0,1), (1,1); (u, v) the local patch coordinates.
    Returns [n_combos, 3], or None when there are too many combinations."""
    import itertools
    sizes = [c.shape[0] for c in corner_variants]
    if min(sizes) == 0 or int(np.prod(sizes)) > max_combos:
        return None
    out = []
    for a, b, c, d in itertools.product(*[range(s) for s in sizes]):
        img = np.stack([np.stack([corner_variants[0][a], corner_variants[1][b]]),
                        np.stack([corner_variants[2][c], corner_variants[3][d]])])
        out.append(oracle.patch_eval(img, [u], [v])[0, :3])
    return np.array(out)


def node_variants(ref: dict, p: int) -> np.ndarray:
    """Valid results [k, 12] of oracle point p (k = 0 when unresolved)."""
    if "variants" not in ref:
        return ref["out"][p][None]
    return ref["variants"][p, : ref["n_var"][p]]
