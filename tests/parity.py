"""Shared helpers for the GPU parity tests (HIP path vs FP64 oracle).

Every pixel is checked.  A pixel whose decisions all lie beyond floating-point reach of their
thresholds has one legitimate result, the oracle's.  A pixel with decisions within that reach has
several, the oracle's among them: the GPU's result either equals the oracle's, or, for brush and
termination decisions (fragile bits 0 and 1), one of the others, which the oracle enumerates
(every set of those decisions taken the other way, OracleImage.outcomes).  Only a pixel that
differs from the oracle's result and whose other results cannot be enumerated (a ray grazing a
sphere or a table lookup at a zero / non-zero opacity boundary, bits 2 and 4, or too many
decisions) stays unchecked, and their share is bounded by FRAGILE_MAX.
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
    err = np.abs(gf - rf).max(axis=-1)
    worst = float(err[single].max()) if single.any() else 0.0
    stats = {"label": label, "pixels": int(npix), "multi_outcome": float((~single).mean()),
             "max_abs_err": worst, "max_abs_err_all": float(err.max()),
             "mean_abs_err": float(err[single].mean()) if single.any() else 0.0}
    assert worst <= tol, f"{label}: max abs RGBA error {worst:.3e} > {tol:.1e} on single-outcome pixels"
    # the oracle's own (double-precision) result, counts included where they are defined (bit 3
    # clear) and given
    same = err <= tol
    cnt_defined = (ff & oracle.FRAGILE_COUNT) == 0
    if gn is not None:
        same &= (gn == ref.nominal.reshape(-1).astype(np.int64)) | ~cnt_defined
    if gc is not None:
        same &= (gc == ref.composited.reshape(-1).astype(np.int64)) | ~cnt_defined
    bad = single & ~same
    stats["count_mismatch"] = int(bad.sum())
    assert not bad.any(), f"{label}: counts differ on {int(bad.sum())} single-outcome pixels"

    # pixels with several legitimate results whose GPU result is not the oracle's own: it must be
    # one of the others (enumerated where the decisions are brush or termination tests)
    matched = rf.copy()               # the legitimate result each pixel's GPU result matched
    others = ~single & ~same
    flippable = others & ((ff & oracle.FRAGILE_FLIPPABLE) != 0) & ((ff & UNCHECKED) == 0)
    unchecked = others & ~flippable
    idx = np.nonzero(flippable)[0]
    alt_taken = 0
    if idx.size:
        out = ref.outcomes(idx)
        for k in range(idx.size):
            p = idx[k]
            m = int(out.count[k])
            if m < 0:
                unchecked[p] = True
                continue
            e = np.abs(out.rgba[k, :m] - gf[p]).max(axis=-1)
            ok = e <= tol
            if cnt_defined[p]:
                if gn is not None:
                    ok &= out.nominal[k, :m].astype(np.int64) == gn[p]
                if gc is not None:
                    ok &= out.composited[k, :m].astype(np.int64) == gc[p]
            assert ok.any(), (f"{label}: pixel {p} matches none of its {m} legitimate outcomes "
                              f"(least RGBA error {e.min():.3e})")
            alt_taken += 1
            matched[p] = out.rgba[k, int(np.argmax(ok))]
    matched[unchecked] = np.nan
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
    result; with `gpu_rgba`, pixels with several legitimate results use the one whose RGBA the GPU's
    matches (the oracle's own, else an enumerated outcome)."""
    g = np.asarray(gpu_depth, np.float64).reshape(-1)
    frag = ref.fragile.reshape(-1)
    ok = (frag & oracle.FRAGILE_RGBA) == 0
    ref_depth = ref.depth.reshape(-1).copy()
    ref_alpha = ref.rgba.reshape(-1, 4)[:, 3].copy()
    if gpu_rgba is not None:
        gr = np.asarray(gpu_rgba, np.float64).reshape(-1, 4)
        same = np.abs(gr - ref.rgba.reshape(-1, 4)).max(axis=-1) <= RGBA_TOL
        ok |= same
        idx = np.nonzero(~ok & ((frag & oracle.FRAGILE_FLIPPABLE) != 0) & ((frag & UNCHECKED) == 0))[0]
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
