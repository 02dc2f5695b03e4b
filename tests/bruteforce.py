"""Independent vectorised FP64 ray caster for tiny inputs (<= 16^3, <= 16x16 px).

Used only to pin the C oracle: it is written a different way (numpy arrays of
all sample positions per ray, scipy's `map_coordinates` with order 1 and
edge replication for the trilinear fetch, cumulative products for the
transmittance and a post-hoc cut at early termination) so that a dropped
term, a wrong sign or a swapped index in either implementation shows up as a
disagreement.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.ndimage import map_coordinates


def camera_rays(cam, width, height):
    cam = np.asarray(np.asarray(cam, np.float32), np.float64)
    eye, target, up, fov = cam[0:3], cam[3:6], cam[6:9], cam[9]
    fwd = target - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    upv = np.cross(right, fwd)
    th = math.tan(math.radians(fov) / 2)
    px, py = np.meshgrid(np.arange(width) + 0.5, np.arange(height) + 0.5)
    sx = (2 * px / width - 1) * th * (width / height)
    sy = (1 - 2 * py / height) * th
    d = fwd[None, None, :] + sx[..., None] * right + sy[..., None] * upv
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return eye, d


def _ball(o, d, rho):
    """Hit interval of the ray with the ball |x| <= rho (None when it misses or touches)."""
    b = o @ d
    c = o @ o - rho * rho
    disc = b * b - c
    if disc <= 0:
        return None
    s = math.sqrt(disc)
    return (-b - s, -b + s)


def segments(o, d, r_inner, r_outer):
    outer = _ball(o, d, r_outer)
    if outer is None:
        return []
    inner = _ball(o, d, r_inner) if r_inner > 0 else None
    pieces = [outer] if inner is None else [(outer[0], min(outer[1], inner[0])), (max(outer[0], inner[1]), outer[1])]
    out = []
    for a, b in pieces:
        a = max(a, 0.0)
        if b > a:
            out.append((a, b))
    return out


def render(level_fields, cam, width, height, step, *, active, lo, hi, tf_field, vmin, vmax,
           tf_rgba, ref_step=2 / 256, ert=0.99, r_inner=0.55, r_outer=1.0, coord=None, with_depth=False):
    f64 = lambda x: float(np.float32(x))
    lf = np.asarray(level_fields, np.float32).astype(np.float64)
    nf, n = lf.shape[0], lf.shape[1]
    lo = np.asarray(np.asarray(lo, np.float32), np.float64)
    hi = np.asarray(np.asarray(hi, np.float32), np.float64)
    tab = np.asarray(np.asarray(tf_rgba, np.float32), np.float64).reshape(256, 4)
    vmin, vmax, ref_step, ert, step = f64(vmin), f64(vmax), f64(ref_step), f64(ert), f64(step)
    r_inner, r_outer = f64(r_inner), f64(r_outer)
    eye, dirs = camera_rays(cam, width, height)
    h = 2.0 / n
    ds = step * h
    rgba = np.zeros((height, width, 4))
    nominal = np.zeros((height, width), np.int64)
    composited = np.zeros((height, width), np.int64)
    depth = np.full((height, width), np.inf)
    for py in range(height):
        for px in range(width):
            d = dirs[py, px]
            mids, lens = [], []
            for a, b in segments(eye, d, r_inner, r_outer):
                k = int(math.ceil((b - a) / ds))
                t0 = a + ds * np.arange(k)
                t1 = np.minimum(a + ds * np.arange(1, k + 1), b)
                mids.append(0.5 * (t0 + t1))
                lens.append(t1 - t0)
            if not mids:
                continue
            tm = np.concatenate(mids)
            ln = np.concatenate(lens)
            pos = eye[None, :] + tm[:, None] * d[None, :]
            u = (pos + 1.0) / h - 0.5                      # x, y, z continuous indices
            coords = u[:, ::-1].T                           # array axes are z, y, x
            vals = np.stack([map_coordinates(lf[f], coords, order=1, mode="nearest", prefilter=False)
                             for f in range(nf)])
            keep = np.ones(tm.size, bool)
            for f in range(nf):
                if active[f]:
                    keep &= (vals[f] >= lo[f]) & (vals[f] <= hi[f])
            if coord is not None:
                cvals = [pos[:, 0], pos[:, 1], pos[:, 2], np.linalg.norm(pos, axis=1)]
                for ax in range(4):
                    if coord[0][ax]:
                        keep &= (cvals[ax] >= f64(coord[1][ax])) & (cvals[ax] <= f64(coord[2][ax]))
            x = np.clip((vals[tf_field] - vmin) / (vmax - vmin), 0.0, 1.0) * 255.0
            i = np.minimum(np.floor(x).astype(np.int64), 254)
            w = (x - i)[:, None]
            s = (1 - w) * tab[i] + w * tab[i + 1]
            alpha = np.where(s[:, 3] >= 1.0, 1.0, 1.0 - np.power(1.0 - np.minimum(s[:, 3], 1.0), ln / ref_step))
            alpha = np.where(keep, alpha, 0.0)
            trans_after = np.cumprod(1.0 - alpha)
            trans_before = np.concatenate([[1.0], trans_after[:-1]])
            acc_after = 1.0 - trans_after
            stop = tm.size
            if ert < 1.0:
                hit = np.flatnonzero(keep & (alpha > 0) & (acc_after >= ert))
                if hit.size:
                    stop = int(hit[0]) + 1
            wgt = (trans_before * alpha)[:stop]
            rgba[py, px, :3] = (wgt[:, None] * s[:stop, :3]).sum(axis=0)
            rgba[py, px, 3] = 1.0 - trans_after[stop - 1]
            nominal[py, px] = stop
            composited[py, px] = int(np.count_nonzero(keep[:stop] & (s[:stop, 3] > 0)))
            if rgba[py, px, 3] > 0:
                depth[py, px] = float(wgt @ tm[:stop]) / rgba[py, px, 3]
    if with_depth:
        return rgba, nominal, composited, depth
    return rgba, nominal, composited
