"""Image warping of a rendered frame to another camera pose (reference definition).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's CPU-baseline
leg, never by the product library, with which it shares no code.

The paper (Section 2, and Section 2.2 "Rendering") decouples the display from the ray caster and
fills the frames the caster has not delivered yet by warping the last image it did deliver; it names
no warping method.  The reading taken here is a forward reprojection of every pixel of the last
image with its opacity-weighted depth:

  * each source pixel's ray (through its centre, row 0 at the top, as in the render) is followed to
    its depth d, giving a world point; a pixel whose depth is not finite (nothing was composited) is
    a point at infinity in its ray's direction;
  * the point is projected through the destination camera; a point on or behind the destination's
    image plane (view depth z <= 0) or outside its image is dropped;
  * it lands on the destination pixel that contains its projection (floor of the continuous pixel
    coordinate); where several land on one pixel, the nearest wins (a z-buffer on the distance from
    the destination eye, +inf for points at infinity), and among equal distances the lowest source
    index;
  * a destination pixel that nothing landed on takes the winner of its eight neighbours with the
    greatest key (the farthest: cracks from forward warping open where a nearer surface uncovers a
    farther one); with no landed neighbour it stays empty (RGBA 0, depth +inf, source -1);
  * the result is the winning source pixel's RGBA unchanged, with the winner's distance from the
    destination eye as the new depth (so a warped frame can be warped again).

Which destination pixel a point lands on is a floating-point decision deciding an integer, so it is
taken here in float32, one correctly rounded operation at a time in the order written below (no
fused multiply-adds), from the camera frame rounded to float32 after computing it in double.  A
warp that reaches the same decisions must follow the same sequence.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

F32 = np.float32
EMPTY = np.int64(-1)


@dataclass
class Frame32:
    """A camera's frame in float32: eye, unit forward / right / up, and the image-plane scales."""
    eye: np.ndarray
    fwd: np.ndarray
    right: np.ndarray
    up: np.ndarray
    sx_scale: np.float32   # tan(fov_y / 2) * width / height
    sy_scale: np.float32   # tan(fov_y / 2)
    inv_w2: np.float32     # 2 / width
    inv_h2: np.float32     # 2 / height


def camera_frame(camera, width: int, height: int) -> Frame32:
    """Pinhole frame of camera = [eye(3), target(3), up(3), fov_y_deg]: forward = normalised
    (target - eye), right = normalised (forward x up), up' = right x forward, computed in double from
    the float32 camera and rounded to float32."""
    c = [float(F32(x)) for x in np.asarray(camera).reshape(10)]
    eye, target, up, fov = c[0:3], c[3:6], c[6:9], c[9]
    f = [target[k] - eye[k] for k in range(3)]
    fl = math.sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2])
    f = [x / fl for x in f]
    r = [f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]]
    rl = math.sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2])
    r = [x / rl for x in r]
    t = [r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]]
    th = math.tan(0.5 * fov * math.pi / 180.0)
    return Frame32(np.array(eye, F32), np.array(f, F32), np.array(r, F32), np.array(t, F32),
                   F32(th * width / height), F32(th), F32(2.0 / width), F32(2.0 / height))


def _dot(v, a):
    """(v0 a0 + v1 a1) + v2 a2 in float32, each product and sum rounded."""
    return (v[0] * a[0] + v[1] * a[1]) + v[2] * a[2]


def landing(depth, src: Frame32, src_w: int, src_h: int, dst: Frame32, dst_w: int, dst_h: int):
    """For every source pixel (row-major): destination pixel index (-1 when dropped) and the key
    depth (distance from the destination eye, +inf for points at infinity), both float32-decided."""
    with np.errstate(all="ignore"):
        d = np.asarray(depth, F32).reshape(-1)
        py, px = np.divmod(np.arange(src_w * src_h, dtype=np.int64), src_w)
        a = px.astype(F32) + F32(0.5)
        b = py.astype(F32) + F32(0.5)
        sx = (a * src.inv_w2 - F32(1.0)) * src.sx_scale
        sy = (F32(1.0) - b * src.inv_h2) * src.sy_scale
        e = [(src.fwd[k] + sx * src.right[k]) + sy * src.up[k] for k in range(3)]
        ln = np.sqrt(_dot(e, e))
        n = [e[k] / ln for k in range(3)]
        finite = d < F32(np.inf)     # NaN and +inf: a point at infinity along the ray
        v = [np.where(finite, (src.eye[k] + d * n[k]) - dst.eye[k], n[k]) for k in range(3)]
        z = _dot(v, dst.fwd)
        xr = _dot(v, dst.right)
        yu = _dot(v, dst.up)
        xn = xr / (z * dst.sx_scale)
        yn = yu / (z * dst.sy_scale)
        fx = (xn + F32(1.0)) * F32(0.5 * dst_w)
        fy = (F32(1.0) - yn) * F32(0.5 * dst_h)
        ok = (z > F32(0.0)) & (fx >= F32(0.0)) & (fx < F32(dst_w)) & (fy >= F32(0.0)) & (fy < F32(dst_h))
        ix = np.where(ok, np.floor(np.where(ok, fx, 0)), 0).astype(np.int64)
        iy = np.where(ok, np.floor(np.where(ok, fy, 0)), 0).astype(np.int64)
        target = np.where(ok, iy * dst_w + ix, -1)
        q = np.where(finite, np.sqrt(_dot(v, v)), F32(np.inf)).astype(F32)
    return target, q


def splat(target, q, dst_w: int, dst_h: int) -> np.ndarray:
    """z-buffer of the landed points: per destination pixel the least key (distance bits << 32 |
    source index), -1 where nothing landed.  Distances are >= 0, so their float32 bit patterns order
    as the distances do."""
    keys = np.full(dst_w * dst_h, np.iinfo(np.int64).max, np.int64)
    src = np.flatnonzero(target >= 0)
    k = (q[src].view(np.uint32).astype(np.int64) << 32) | src
    np.minimum.at(keys, target[src], k)
    keys[keys == np.iinfo(np.int64).max] = EMPTY
    return keys


def fill(keys: np.ndarray, dst_w: int, dst_h: int) -> np.ndarray:
    """Empty pixels take the greatest key among their eight neighbours' landed keys (read from the
    splat, not from other filled pixels); still -1 when none landed."""
    k2 = keys.reshape(dst_h, dst_w)
    pad = np.full((dst_h + 2, dst_w + 2), EMPTY, np.int64)
    pad[1:-1, 1:-1] = k2
    best = np.full((dst_h, dst_w), EMPTY, np.int64)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx or dy:
                best = np.maximum(best, pad[1 + dy:1 + dy + dst_h, 1 + dx:1 + dx + dst_w])
    return np.where(k2 == EMPTY, best, k2).reshape(-1)


def warp(rgba, depth, src_camera, src_w: int, src_h: int, dst_camera, dst_w: int, dst_h: int):
    """Warp a frame (rgba float32 [src_h, src_w, 4], depth float32 [src_h, src_w]) to dst_camera.
    Returns (rgba float32 [dst_h, dst_w, 4], depth float32 [dst_h, dst_w], source int64 [dst_h,
    dst_w]) with source -1, RGBA 0 and depth +inf where the destination pixel stays empty."""
    src = camera_frame(src_camera, src_w, src_h)
    dst = camera_frame(dst_camera, dst_w, dst_h)
    target, q = landing(depth, src, src_w, src_h, dst, dst_w, dst_h)
    keys = fill(splat(target, q, dst_w, dst_h), dst_w, dst_h)
    has = keys != EMPTY
    source = np.where(has, keys & 0xFFFFFFFF, -1)
    out_depth = np.where(has, (keys >> 32).astype(np.uint32).view(F32), F32(np.inf)).astype(F32)
    col = np.asarray(rgba, F32).reshape(-1, 4)
    out = np.where(has[:, None], col[np.where(has, source, 0)], F32(0.0)).astype(F32)
    return out.reshape(dst_h, dst_w, 4), out_depth.reshape(dst_h, dst_w), source.reshape(dst_h, dst_w)
