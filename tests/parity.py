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
