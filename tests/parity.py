"""Shared helpers for the GPU parity tests (HIP path vs FP64 oracle)."""
from __future__ import annotations

import numpy as np

import oracle

RGBA_TOL = 2e-4          # max-abs per channel on non-fragile pixels (FP32 accumulation)
FRAGILE_MAX = 0.05       # fraction of pixels the oracle may flag before a test is considered degenerate


def compare(gpu_rgba: np.ndarray, ref: oracle.OracleImage, gpu_nominal=None, gpu_composited=None,
            tol: float = RGBA_TOL, label: str = "") -> dict:
    """Element-wise comparison on the pixels whose decisions are not within floating-point
    reach of a threshold (the oracle's fragility mask).  Returns statistics; raises on failure."""
    g = np.asarray(gpu_rgba, np.float64).reshape(ref.rgba.shape)
    frag = ref.fragile.reshape(ref.rgba.shape[:-1])
    ok_rgba = (frag & oracle.FRAGILE_RGBA) == 0
    ok_cnt = frag == 0
    err = np.abs(g - ref.rgba).max(axis=-1)
    worst = float(err[ok_rgba].max()) if ok_rgba.any() else 0.0
    stats = {"label": label, "pixels": int(frag.size), "fragile_rgba": float(1 - ok_rgba.mean()),
             "fragile_any": float(1 - ok_cnt.mean()), "max_abs_err": worst,
             "max_abs_err_all": float(err.max()), "mean_abs_err": float(err[ok_rgba].mean()) if ok_rgba.any() else 0.0}
    print(f"[parity] {stats}", flush=True)
    assert np.isfinite(g).all(), f"{label}: non-finite GPU output"
    assert worst <= tol, f"{label}: max abs RGBA error {worst:.3e} > {tol:.1e} on non-fragile pixels"
    if gpu_nominal is not None:
        gn = np.asarray(gpu_nominal).reshape(frag.shape).astype(np.int64)
        bad = (gn != ref.nominal.reshape(frag.shape).astype(np.int64)) & ok_cnt
        stats["nominal_mismatch"] = int(bad.sum())
        assert not bad.any(), f"{label}: nominal counts differ on {int(bad.sum())} non-fragile pixels"
    if gpu_composited is not None:
        gc = np.asarray(gpu_composited).reshape(frag.shape).astype(np.int64)
        bad = (gc != ref.composited.reshape(frag.shape).astype(np.int64)) & ok_cnt
        assert not bad.any(), f"{label}: composited counts differ on {int(bad.sum())} non-fragile pixels"
    return stats


def sample_pixels(width: int, height: int, k: int, seed: int = 0) -> np.ndarray:
    """Seeded subset of linear pixel indices, sorted, always including the four corners."""
    rng = np.random.default_rng(seed)
    pix = rng.choice(width * height, size=min(k, width * height), replace=False)
    corners = np.array([0, width - 1, (height - 1) * width, height * width - 1])
    return np.unique(np.concatenate([pix, corners]))


def depth_tolerance(alpha, r_outer=1.0):
    """|depth error| bound on a non-fragile pixel.  Writing the depth as t0 + sum w (t - t0) / A with
    t - t0 in [0, 2 r_outer], the numerator is a colour channel scaled by 2 r_outer, so it carries
    at most RGBA_TOL * 2 r_outer of error; the opacity A carries at most RGBA_TOL; together
    |delta depth| <= 2 RGBA_TOL (2 r_outer) / A."""
    return 2 * RGBA_TOL * 2 * r_outer / np.maximum(alpha, 1e-30)


def check_depth(gpu_depth, ref: oracle.OracleImage, label: str = "", min_frac: float = 0.05) -> None:
    """GPU opacity-weighted depth against the oracle's: defined (finite) on the same non-fragile
    pixels, and within depth_tolerance of the oracle's opacity there."""
    g = np.asarray(gpu_depth, np.float64).reshape(ref.depth.shape)
    frag = ref.fragile.reshape(ref.depth.shape)
    ok = (frag & oracle.FRAGILE_RGBA) == 0
    inf_ref = np.isinf(ref.depth)
    assert np.array_equal(np.isinf(g)[ok], inf_ref[ok]), f"{label}: depth defined on different pixels"
    fin = ok & ~inf_ref
    alpha = ref.rgba.reshape(*ref.depth.shape, 4)[..., 3]
    err = np.abs(g[fin] - ref.depth[fin])
    tol = depth_tolerance(alpha[fin])
    print(f"[depth] {label}: {int(fin.sum())} px with depth, max err {err.max() if err.size else 0:.3e}, "
          f"max err / bound {np.max(err / tol) if err.size else 0:.3e}", flush=True)
    assert np.all(err <= tol), f"{label}: depth error above the bound"
    assert fin.sum() > min_frac * fin.size
