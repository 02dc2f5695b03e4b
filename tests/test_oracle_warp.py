"""Pins for the image-warping oracle and the opacity-weighted depth it reprojects with (CPU only).

The warp is tied to the geometry of a pinhole camera (a fronto-parallel plane under a camera
translation moves by a whole number of pixels that follows from the focal length; a reversed camera
sees nothing), to a float64 brute force written with plain loops on tiny images, and to its own
invariants (identity, z-buffer order, hole filling).  The depth is tied to the brute-force ray caster
and to the closed form of a homogeneous medium.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import warp as WP
from paper_2207_12011_amd import workloads as W

from . import bruteforce as bf

F32 = np.float32


def cam(eye, target=(0, 0, 0), up=(0, 1, 0), fov=90.0):
    return np.array([*eye, *target, *up, fov], np.float32)


def rays64(c, w, h):
    """Unit ray directions (float64) through the pixel centres of camera c."""
    eye, d = bf.camera_rays(c, w, h)
    return eye, d


def plane_depth(c, w, h, z_plane=0.0):
    """Distance along each ray of camera c to the plane z = z_plane (float64)."""
    eye, d = rays64(c, w, h)
    return (z_plane - eye[2]) / d[..., 2]


def frame64(c, w, h):
    c = np.asarray(np.asarray(c, np.float32), np.float64)
    eye, target, up, fov = c[0:3], c[3:6], c[6:9], c[9]
    f = (target - eye) / np.linalg.norm(target - eye)
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = math.tan(math.radians(fov) / 2)
    return eye, f, r, u, th * w / h, th


def brute_warp(depth, c_src, sw, sh, c_dst, dw, dh, margin=1e-4):
    """Float64 forward warp with explicit loops: (source index per destination pixel or -1, mask of
    destination pixels whose outcome no float32 rounding can change)."""
    eye_s, dirs = rays64(c_src, sw, sh)
    eye_d, f, r, u, sxs, sys_ = frame64(c_dst, dw, dh)
    best = {}
    unsure = np.zeros((dh, dw), bool)
    for py in range(sh):
        for px in range(sw):
            d = float(depth[py, px])
            if np.isfinite(d):
                v = eye_s + d * dirs[py, px] - eye_d
                dist = float(np.linalg.norm(v))
            else:
                v = dirs[py, px]
                dist = math.inf
            z = float(v @ f)
            if z <= 1e-9:
                continue
            fx = (float(v @ r) / (z * sxs) + 1) * 0.5 * dw
            fy = (1 - float(v @ u) / (z * sys_)) * 0.5 * dh
            ix, iy = math.floor(fx), math.floor(fy)
            near_edge = min(abs(fx - round(fx)), abs(fy - round(fy))) < margin
            for jx, jy in {(ix, iy), (math.floor(fx - margin), math.floor(fy - margin)),
                           (math.floor(fx + margin), math.floor(fy + margin))}:
                if 0 <= jx < dw and 0 <= jy < dh and near_edge:
                    unsure[jy, jx] = True
            if not (0 <= ix < dw and 0 <= iy < dh):
                continue
            key = (dist, py * sw + px)
            cur = best.get((iy, ix))
            if cur is not None and cur[0] != math.inf and dist != math.inf and abs(cur[0] - dist) < 2e-6 * dist:
                unsure[iy, ix] = True
            if cur is None or key < cur:
                best[(iy, ix)] = key
    src = np.full((dh, dw), -1, np.int64)
    for (iy, ix), (_, s) in best.items():
        src[iy, ix] = s
    return src, ~unsure


def smooth_depth(rng, w, h, lo=2.0, hi=3.5, hole_frac=0.2):
    """Seeded smooth depth map in [lo, hi] with about hole_frac of the pixels at +inf."""
    yy, xx = np.mgrid[0:h, 0:w] / max(w, h)
    d = np.zeros((h, w))
    for _ in range(4):
        a, b, ph = rng.uniform(1, 6, 2).tolist() + [rng.uniform(0, 6.28)]
        d += np.sin(a * xx * 6.28 + b * yy * 6.28 + ph)
    d = lo + (hi - lo) * (d - d.min()) / max(d.max() - d.min(), 1e-9)
    d[rng.random((h, w)) < hole_frac] = np.inf
    return d.astype(np.float32)


# ----------------------------------------------------------------------------- warp geometry
def test_identity_warp():
    rng = np.random.default_rng(1)
    c = cam((0.3, -0.2, 3.0), (0.1, 0, 0), (0, 1, 0.2), 50)
    for w, h in ((37, 23), (16, 16), (1, 1), (64, 1)):
        depth = smooth_depth(rng, w, h)
        rgba = rng.random((h, w, 4)).astype(F32)
        out, od, src = WP.warp(rgba, depth, c, w, h, c, w, h)
        assert np.array_equal(src.reshape(-1), np.arange(w * h))
        assert np.array_equal(out, rgba)
        fin = np.isfinite(depth)
        assert np.all(np.isinf(od[~fin]))
        assert np.all(np.abs(od[fin] / depth[fin] - 1) <= 1e-6)


@pytest.mark.parametrize("axis,delta,shift", [(0, 0.375, -4), (1, 0.1875, 2), (0, -0.75, 8)])
def test_plane_translation_closed_form(axis, delta, shift):
    """A plane 3 units in front of a 90-degree camera, 64 x 64: moving the camera by delta along its
    right (up) axis moves the image by delta * 32 / 3 pixels to the left (downwards)."""
    w = h = 64
    src_c = cam((0, 0, 3))
    e = [0.0, 0.0, 3.0]
    e[axis] += delta
    t = [0.0, 0.0, 0.0]
    t[axis] += delta
    dst_c = cam(e, t)
    depth = plane_depth(src_c, w, h).astype(F32)
    rgba = np.random.default_rng(2).random((h, w, 4)).astype(F32)
    out, od, src = WP.warp(rgba, depth, src_c, w, h, dst_c, w, h)
    sy, sx = np.divmod(src, w)
    ty, tx = np.mgrid[0:h, 0:w]
    moved = (sx - tx) if axis == 0 else (sy - ty)
    # the destination pixels whose source is inside the image received it, shifted by `shift`
    if axis == 0:
        inner = (tx + (-shift) >= 0) & (tx + (-shift) < w)
        assert np.all(moved[inner] == -shift) and np.all(sy[inner] == ty[inner])
    else:
        inner = (ty - shift >= 0) & (ty - shift < h)
        assert np.all(moved[inner] == -shift) and np.all(sx[inner] == tx[inner])
    assert np.array_equal(out[inner], rgba.reshape(-1, 4)[src[inner]])
    # the first uncovered row or column is filled from its neighbours, the rest stay empty
    n_uncovered = abs(shift)
    strip = ~inner
    if axis == 0:
        cols = np.arange(w - n_uncovered, w) if shift < 0 else np.arange(0, n_uncovered)
        first = cols[0] if shift < 0 else cols[-1]
        filled = np.zeros_like(strip)
        filled[:, first] = True
    else:
        rows = np.arange(0, n_uncovered) if shift > 0 else np.arange(h - n_uncovered, h)
        first = rows[-1] if shift > 0 else rows[0]
        filled = np.zeros_like(strip)
        filled[first, :] = True
    assert np.all(src[filled] >= 0)
    assert np.all(src[strip & ~filled] == -1) and np.all(out[strip & ~filled] == 0)
    assert np.all(np.isinf(od[strip & ~filled]))
    # new depth: distance from the moved eye to the plane point
    eye_s, dirs = rays64(src_c, w, h)
    pts = eye_s + plane_depth(src_c, w, h)[..., None] * dirs
    want = np.linalg.norm(pts.reshape(-1, 3)[src[inner]] - np.asarray(e), axis=-1)
    assert np.abs(od[inner] / want - 1).max() <= 2e-6


def test_reversed_camera_sees_nothing():
    w, h = 24, 16
    src_c = cam((0, 0, 3))
    depth = plane_depth(src_c, w, h).astype(F32)
    depth[::3] = np.inf
    rgba = np.ones((h, w, 4), F32)
    out, od, src = WP.warp(rgba, depth, src_c, w, h, cam((0, 0, 3), (0, 0, 6)), w, h)
    assert np.all(src == -1) and np.all(out == 0) and np.all(np.isinf(od))


@pytest.mark.parametrize("case", range(6))
def test_warp_matches_bruteforce(case):
    """Seeded depth maps (with empty pixels) under translation, rotation, zoom, a size change and
    a large move; the float64 loop brute force must pick the same winners wherever no float32
    rounding can change the outcome, and the filled pixels must follow the neighbour rule."""
    rng = np.random.default_rng(10 + case)
    sw, sh = [(20, 14), (16, 16), (24, 10), (13, 17), (20, 14), (9, 9)][case]
    dw, dh = [(20, 14), (16, 16), (24, 10), (26, 11), (20, 14), (13, 7)][case]
    src_c = cam((0.2, 0.1, 3.0), (0, 0, 0), (0, 1, 0), 60)
    dst_c = [cam((0.35, 0.1, 2.9), (0.1, 0, 0), (0, 1, 0), 60),           # translate
             cam((0.2, 0.1, 3.0), (0.4, -0.2, 0), (0.1, 1, 0), 60),        # rotate about the eye
             cam((0.2, 0.1, 2.2), (0, 0, 0), (0, 1, 0), 60),                # move closer (magnify)
             cam((0.1, 0.1, 3.1), (0, 0.05, 0), (0, 1, 0), 45),             # zoom and resize
             cam((2.0, 0.5, 2.0), (0, 0, 0), (0, 1, 0), 60),                # large move: occlusions
             cam((0.2, 0.1, 3.0), (0, 0, 0), (0, 1, 0), 90)][case]          # wider field of view
    depth = smooth_depth(rng, sw, sh, 2.0, 3.5, 0.15)
    depth[rng.random((sh, sw)) < 0.1] = np.float32(1.2)  # near specks that occlude
    rgba = rng.random((sh, sw, 4)).astype(F32)
    out, od, src = WP.warp(rgba, depth, src_c, sw, sh, dst_c, dw, dh)
    want, sure = brute_warp(depth, src_c, sw, sh, dst_c, dw, dh)
    target, q = WP.landing(depth, WP.camera_frame(src_c, sw, sh), sw, sh, WP.camera_frame(dst_c, dw, dh), dw, dh)
    landed = np.zeros(dw * dh, bool)
    landed[target[target >= 0]] = True
    landed = landed.reshape(dh, dw)
    assert sure[landed].mean() > 0.8
    assert np.array_equal(src[landed & sure], want[landed & sure])
    assert np.array_equal(landed & sure, (want >= 0) & sure & landed)
    assert np.all(want[~landed & sure] == -1)
    # filled pixels: the farthest of the landed neighbours' winners
    keys = WP.splat(target, q, dw, dh).reshape(dh, dw)
    for iy, ix in zip(*np.nonzero(~landed)):
        nb = [keys[y, x] for y in range(iy - 1, iy + 2) for x in range(ix - 1, ix + 2)
              if (y, x) != (iy, ix) and 0 <= y < dh and 0 <= x < dw and keys[y, x] >= 0]
        assert src[iy, ix] == (max(nb) & 0xFFFFFFFF if nb else -1)
    assert np.array_equal(out.reshape(-1, 4)[src.reshape(-1) >= 0], rgba.reshape(-1, 4)[src[src >= 0]])
    assert (src >= 0).sum() > dw * dh // 3


def test_magnification_fills_cracks():
    """Moving towards a plane by 20 % spreads the image; after the fill no interior pixel is empty."""
    w = h = 48
    src_c = cam((0, 0, 3))
    depth = plane_depth(src_c, w, h).astype(F32)
    rgba = np.random.default_rng(3).random((h, w, 4)).astype(F32)
    target, q = WP.landing(depth, WP.camera_frame(src_c, w, h), w, h, WP.camera_frame(cam((0, 0, 2.4)), w, h), w, h)
    landed = np.zeros(w * h, bool)
    landed[target[target >= 0]] = True
    assert (~landed).sum() > 100                       # forward warping alone leaves cracks
    _, _, src = WP.warp(rgba, depth, src_c, w, h, cam((0, 0, 2.4)), w, h)
    assert np.all(src >= 0)


# ----------------------------------------------------------------------------- depth
@pytest.fixture(scope="module")
def tiny():
    return W.make_workload(0, n=16, width=16, height=16)


@pytest.mark.parametrize("brushed", [True, False])
@pytest.mark.parametrize("ert", [0.99, 0.6])
def test_depth_matches_bruteforce(tiny, brushed, ert):
    wl = tiny
    act = wl.brush.active if brushed else np.zeros(2, np.uint8)
    kw = dict(active=act, lo=wl.brush.lo, hi=wl.brush.hi, tf_field=0, vmin=wl.tf.vmin, vmax=wl.tf.vmax,
              tf_rgba=wl.tf.rgba, ert=ert)
    c = wl.camera.as_array()
    o = oracle.render(wl.fields, c, 16, 16, 0.5, **kw)
    _, _, _, dep = bf.render(wl.fields, c, 16, 16, 0.5, with_depth=True, **kw)
    ok = (o.fragile & oracle.FRAGILE_ERT) == 0
    assert np.array_equal(np.isinf(o.depth), np.isinf(dep))
    fin = ok & np.isfinite(dep)
    assert fin.sum() > 20
    assert np.abs(o.depth[fin] - dep[fin]).max() <= 1e-12
    assert np.all(np.isinf(o.depth[o.rgba[..., 3] == 0]))


@pytest.mark.parametrize("a0", [0.05, 0.4])
@pytest.mark.parametrize("step", [0.5, 1.0])
def test_depth_homogeneous_closed_form(a0, step):
    """Constant field and table, no termination, rays that miss the inner sphere: the samples of the
    one segment [a, b] carry weights q^j alpha (q = 1 - alpha), the last partial one q^(k-1)
    alpha_last, so the depth is a geometric series in closed form."""
    n = 16
    vol = np.full((1, n, n, n), 0.5, np.float32)
    c = np.array([3, 0, 0, 0, 0, 0, 0, 0, 1, 60], np.float32)
    w = h = 15
    o = oracle.render(vol, c, w, h, step, active=[0], lo=[0], hi=[1], tf_field=0, vmin=0, vmax=1,
                      tf_rgba=np.tile(np.float32([0.3, 0.3, 0.3, a0]), (256, 1)), ert=1.0)
    eye, dirs = bf.camera_rays(c, w, h)
    ref = float(np.float32(2 / 256))
    r_in, r_out = float(np.float32(0.55)), 1.0
    ds = step * 2 / n
    A0 = float(np.float32(a0))
    checked = 0
    for py in range(h):
        for px in range(w):
            d = dirs[py, px]
            b = eye @ d
            p2 = eye @ eye - b * b
            if not (r_in ** 2 + 1e-3 < p2 < r_out ** 2 - 1e-3):
                continue
            s = math.sqrt(r_out ** 2 - p2)
            a, e = -b - s, -b + s
            k = math.ceil((e - a) / ds)
            m = k - 1                                          # full samples
            alpha = 1 - (1 - A0) ** (ds / ref)
            q = 1 - alpha
            last_len = e - (a + m * ds)
            alpha_l = 1 - (1 - A0) ** (last_len / ref)
            s0 = (1 - q ** m) / (1 - q)
            s1 = q * (1 - m * q ** (m - 1) + (m - 1) * q ** m) / (1 - q) ** 2
            num = alpha * (a * s0 + ds * (s1 + 0.5 * s0)) + q ** m * alpha_l * (a + m * ds + 0.5 * last_len)
            den = 1 - q ** m * (1 - alpha_l)
            assert abs(o.depth[py, px] - num / den) <= 1e-9 * num / den
            checked += 1
    assert checked >= 20


def test_depth_of_a_thin_slab():
    """Field = world x; a brush keeping only x in [0.70, 0.72] along the axis ray x = 3 - t leaves
    samples with midpoints in that slab: the depth is their weighted mean, between 2.28 and 2.30."""
    n = 64
    x = ((np.arange(n) + 0.5) * 2 / n - 1).astype(np.float32)
    vol = np.broadcast_to(x[None, None, None, :], (1, n, n, n)).copy()
    c = np.array([3, 0, 0, 0, 0, 0, 0, 0, 1, 60], np.float32)
    o = oracle.render(vol, c, 3, 3, 0.25, active=[1], lo=[0.70], hi=[0.72], tf_field=0, vmin=-1, vmax=1,
                      tf_rgba=np.tile(np.float32([1, 1, 1, 0.2]), (256, 1)), ert=1.0, r_inner=0.0)
    assert o.rgba[1, 1, 3] > 0
    assert 2.28 - 1e-3 <= o.depth[1, 1] <= 2.30 + 1e-3
