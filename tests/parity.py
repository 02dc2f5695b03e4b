"""Shared helpers for the GPU parity tests (HIP path vs FP64 oracle).

Every pixel is checked.  A pixel whose decisions all lie beyond floating-point reach of their
thresholds has one legitimate result, the oracle's.  A pixel with brush or termination decisions
within that reach (fragile bits 0 and 1) has several: the oracle enumerates them (every set of
those decisions taken the other way, OracleImage.outcomes) and the GPU's result must equal one of
them.  Only pixels with a ray grazing a sphere or a table lookup at a zero / non-zero opacity
boundary (bits 2 and 4), or with too many flippable decisions to enumerate, stay unchecked, and
their share is bounded by FRAGILE_MAX.
"""
from __future__ import annotations

import numpy as np

import oracle

RGBA_TOL = 2e-4          # max-abs per channel (FP32 accumulation)
FRAGILE_MAX = 0.005      # largest share of pixels that no check covers
UNCHECKED = oracle.FRAGILE_GRAZE | oracle.FRAGILE_TFZERO


def compare(gpu_rgba: np.ndarray, ref: oracle.OracleImage, gpu_nominal=None, gpu_composited=None,
            tol: float = RGBA_TOL, label: str = "", unchecked_max: float = FRAGILE_MAX) -> dict:
    """Element-wise comparison of a GPU image (and its per-pixel counts) with the oracle's.
    Returns statistics, and under "matched" the legitimate result each pixel matched (NaN where
    unchecked); raises on failure."""
    g = np.asarray(gpu_rgba, np.float64).reshape(ref.rgba.shape)
    frag = ref.fragile.reshape(ref.rgba.shape[:-1])
    assert np.isfinite(g).all(), f"{label}: non-finite GPU output"
    gf = g.reshape(-1, 4)
    rf = ref.rgba.reshape(-1, 4)
    ff = frag.reshape(-1)
    npix = ff.size
    gn = None if gpu_nominal is None else np.asarray(gpu_nominal).reshape(-1).astype(np.int64)
    gc = None if gpu_composited is None else np.asarray(gpu_composited).reshape(-1).astype(np.int64)

    single = (ff & oracle.FRAGILE_RGBA) == 0            # one legitimate result
    multi = ((ff & oracle.FRAGILE_FLIPPABLE) != 0) & ((ff & UNCHECKED) == 0)
    unchecked = (ff & UNCHECKED) != 0
    err = np.abs(gf - rf).max(axis=-1)
    worst = float(err[single].max()) if single.any() else 0.0
    stats = {"label": label, "pixels": int(npix), "multi_outcome": float(multi.mean()),
             "max_abs_err": worst, "max_abs_err_all": float(err.max()),
             "mean_abs_err": float(err[single].mean()) if single.any() else 0.0}
    assert worst <= tol, f"{label}: max abs RGBA error {worst:.3e} > {tol:.1e} on single-outcome pixels"
    cnt_ok = ff == 0                                      # counts are defined up to bit 3 as well
    if gn is not None:
        bad = (gn != ref.nominal.reshape(-1).astype(np.int64)) & single & cnt_ok
        stats["nominal_mismatch"] = int(bad.sum())
        assert not bad.any(), f"{label}: nominal counts differ on {int(bad.sum())} single-outcome pixels"
    if gc is not None:
        bad = (gc != ref.composited.reshape(-1).astype(np.int64)) & single & cnt_ok
        assert not bad.any(), f"{label}: composited counts differ on {int(bad.sum())} single-outcome pixels"

    # pixels with several legitimate results: the GPU's must be one of them
    matched = rf.copy()               # the legitimate result each pixel's GPU result matched
    matched[unchecked] = np.nan
    idx = np.nonzero(multi)[0]
    alt_taken = 0
    if idx.size:
        out = ref.outcomes(idx)
        unresolved = out.count < 0
        unchecked[idx[unresolved]] = True
        matched[idx[unresolved]] = np.nan
        for k in np.nonzero(~unresolved)[0]:
            p = idx[k]
            m = int(out.count[k])
            e = np.abs(out.rgba[k, :m] - gf[p]).max(axis=-1)
            ok = e <= tol
            if ff[p] & oracle.FRAGILE_COUNT == 0:
                if gn is not None:
                    ok &= out.nominal[k, :m].astype(np.int64) == gn[p]
                if gc is not None:
                    ok &= out.composited[k, :m].astype(np.int64) == gc[p]
            assert ok.any(), (f"{label}: pixel {p} matches none of its {m} legitimate outcomes "
                              f"(least RGBA error {e.min():.3e})")
            alt_taken += int(not ok[0])
            matched[p] = out.rgba[k, int(np.argmax(ok))]
    stats["alternative_taken"] = alt_taken / npix
    stats["unchecked"] = float(unchecked.mean())
    print(f"[parity] {stats}", flush=True)
    assert stats["unchecked"] <= unchecked_max, f"{label}: {stats['unchecked']:.4f} of the pixels unchecked"
    stats["matched"] = matched.reshape(ref.rgba.shape)
    return stats


def sample_pixels(width: int, height: int, k: int, seed: int = 0) -> np.ndarray:
    """Seeded subset of linear pixel indices, sorted, always including the four corners."""
    rng = np.random.default_rng(seed)
    pix = rng.choice(width * height, size=min(k, width * height), replace=False)
    corners = np.array([0, width - 1, (height - 1) * width, height * width - 1])
    return np.unique(np.concatenate([pix, corners]))


def depth_tolerance(alpha, r_outer=1.0):
    """|depth error| bound on a pixel whose result matches.  Writing the depth as t0 + sum w (t - t0)
    / A with t - t0 in [0, 2 r_outer], the numerator is a colour channel scaled by 2 r_outer, so it
    carries at most RGBA_TOL * 2 r_outer of error; the opacity A carries at most RGBA_TOL; together
    |delta depth| <= 2 RGBA_TOL (2 r_outer) / A."""
    return 2 * RGBA_TOL * 2 * r_outer / np.maximum(alpha, 1e-30)


def check_depth(gpu_depth, ref: oracle.OracleImage, label: str = "", min_frac: float = 0.05,
                gpu_rgba=None) -> None:
    """GPU opacity-weighted depth against the oracle's: defined (finite) on the same pixels, and
    within depth_tolerance of the oracle's opacity there.  Single-outcome pixels use the oracle's
    result; with `gpu_rgba`, pixels with several legitimate results use the outcome whose RGBA the
    GPU's matches."""
    g = np.asarray(gpu_depth, np.float64).reshape(-1)
    frag = ref.fragile.reshape(-1)
    ok = (frag & oracle.FRAGILE_RGBA) == 0
    ref_depth = ref.depth.reshape(-1).copy()
    ref_alpha = ref.rgba.reshape(-1, 4)[:, 3].copy()
    if gpu_rgba is not None:
        gr = np.asarray(gpu_rgba, np.float64).reshape(-1, 4)
        idx = np.nonzero(((frag & oracle.FRAGILE_FLIPPABLE) != 0) & ((frag & UNCHECKED) == 0))[0]
        if idx.size:
            out = ref.outcomes(idx)
            for k in np.nonzero(out.count > 0)[0]:
                m = int(out.count[k])
                e = np.abs(out.rgba[k, :m] - gr[idx[k]]).max(axis=-1)
                o = int(np.argmin(e))
                if e[o] <= RGBA_TOL:
                    ok[idx[k]] = True
                    ref_depth[idx[k]] = out.depth[k, o]
                    ref_alpha[idx[k]] = out.rgba[k, o, 3]
    inf_ref = np.isinf(ref_depth)
    assert np.array_equal(np.isinf(g)[ok], inf_ref[ok]), f"{label}: depth defined on different pixels"
    fin = ok & ~inf_ref
    err = np.abs(g[fin] - ref_depth[fin])
    tol = depth_tolerance(ref_alpha[fin])
    print(f"[depth] {label}: {int(fin.sum())} px with depth ({ok.mean():.4f} checked), max err "
          f"{err.max() if err.size else 0:.3e}, max err / bound {np.max(err / tol) if err.size else 0:.3e}", flush=True)
    assert np.all(err <= tol), f"{label}: depth error above the bound"
    assert fin.sum() > min_frac * fin.size
