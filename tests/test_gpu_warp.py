"""GPU parity of the opacity-weighted depth and of image warping.

The depth render is compared with the FP64 oracle (RGBA <= 2e-4 on non-fragile pixels, the image
bit-identical to the plain render, depth within the bound derived from the RGBA tolerance); the
warp is compared bit for bit (source index, RGBA and depth) with the float32 warp oracle on the same
seeded inputs, which never come from the HIP path: synthetic depth maps, or the oracle's own render
rounded to float32.
"""
import zlib

import numpy as np
import pytest
import torch

import oracle
from oracle import preprocess as pp
from oracle import warp as WP
from paper_2207_12011_amd import workloads as W

from .parity import check_depth, compare

pytestmark = pytest.mark.gpu

F32 = np.float32


@pytest.fixture(scope="module")
def rp():
    from paper_2207_12011_amd import raypc
    return raypc


@pytest.fixture(scope="module")
def ctx(rp):
    c = rp.create(0)
    yield c
    rp.destroy(c)


def cpu(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def cam(eye, target=(0, 0, 0), up=(0, 1, 0), fov=60.0):
    return np.array([*eye, *target, *up, fov], np.float32)


@pytest.mark.parametrize("storage", ["f32", "f16", "u8"])
def test_render_depth_matches_oracle(rp, ctx, storage):
    wl = W.make_workload(1, n=64, width=200, height=136)
    vid = rp.load_fields(ctx, torch.from_numpy(wl.fields).cuda(), storage, 3, wl.r_inner, wl.r_outer)
    rp.set_brush(ctx, vid, wl.brush.active, wl.brush.lo, wl.brush.hi)
    rp.set_transfer_function(ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, wl.tf.ref_step)
    rp.set_options(ctx, wl.ert)
    levels = pp.stored_levels(wl.fields, 3, storage)
    c = wl.camera.as_array()
    for lod, step, brushed in ((0, wl.step, True), (0, wl.step, False), (1, 0.7, True), (2, 1.3, True)):
        act = wl.brush.active if brushed else np.zeros(wl.n_fields, np.uint8)
        rp.set_brush(ctx, vid, act, wl.brush.lo, wl.brush.hi)
        label = f"{storage} lod {lod} step {step} brushed {brushed}"
        print(f"[case] depth {label}", flush=True)
        rgba, dep = rp.render_depth(ctx, vid, c, wl.width, wl.height, lod, step)
        plain = rp.render(ctx, vid, c, wl.width, wl.height, lod, step)
        assert np.array_equal(cpu(rgba), cpu(plain)), label
        ref = oracle.render_workload(wl, levels[lod], active=act, step=step)
        compare(cpu(rgba), ref, label=label)
        check_depth(cpu(dep), ref, label, gpu_rgba=cpu(rgba))
    with pytest.raises(rp.RaypcError):
        rp._check(rp._render_depth(ctx, vid, rp.ctypes.byref(rp.Camera.make(c)), 8, 8, 0, 0.5,
                                   rgba.data_ptr(), None, None))
    rp.unload(ctx, vid)


def test_render_depth_with_termination_and_background(rp, ctx):
    """An opaque table (early termination on most rays) and a background: the depth stops at the
    termination sample and ignores the background."""
    wl = W.make_workload(1, n=64, width=96, height=80)
    vid = rp.load_fields(ctx, torch.from_numpy(wl.fields).cuda(), "f16", 1, wl.r_inner, wl.r_outer)
    tab = wl.tf.rgba.copy()
    tab[:, 3] = np.linspace(0.3, 0.9, 256, dtype=np.float32)
    rp.set_brush(ctx, vid, np.zeros(wl.n_fields, np.uint8), wl.brush.lo, wl.brush.hi)
    rp.set_transfer_function(ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, tab, wl.tf.ref_step)
    bg = np.array([0.1, 0.2, 0.3, 1.0], np.float32)
    rp.set_options(ctx, 0.95, bg)
    try:
        rgba, dep = rp.render_depth(ctx, vid, wl.camera.as_array(), wl.width, wl.height, 0, wl.step)
        level = pp.stored_levels(wl.fields, 1, "f16")[0]
        kw = dict(active=np.zeros(wl.n_fields, np.uint8), tf_rgba=tab, ert=0.95)
        ref = oracle.render_workload(wl, level, bg=bg, **kw)
        compare(cpu(rgba), ref, label="opaque + background")
        # the background has no depth: the same depth as without it, bounded with the volume's opacity
        ref_vol = oracle.render_workload(wl, level, **kw)
        assert np.array_equal(ref.depth, ref_vol.depth)
        assert (ref_vol.rgba[..., 3] >= 0.95).sum() > 500
        check_depth(cpu(dep), ref_vol, "opaque + background")
    finally:
        rp.set_options(ctx, 0.99, None)
        rp.unload(ctx, vid)


# ----------------------------------------------------------------------------- warp
def smooth_depth(rng, w, h, lo=2.0, hi=3.5, hole_frac=0.2, speck_frac=0.05):
    yy, xx = np.mgrid[0:h, 0:w] / max(w, h)
    d = np.zeros((h, w))
    for _ in range(4):
        a, b, ph = rng.uniform(1, 6), rng.uniform(1, 6), rng.uniform(0, 6.28)
        d += np.sin(a * xx * 6.28 + b * yy * 6.28 + ph)
    d = lo + (hi - lo) * (d - d.min()) / max(d.max() - d.min(), 1e-9)
    d[rng.random((h, w)) < speck_frac] = 1.2
    d[rng.random((h, w)) < hole_frac] = np.inf
    return d.astype(F32)


def run_warp(rp, ctx, rgba, depth, src_c, dst_c, dw, dh, label):
    sh, sw = depth.shape
    print(f"[case] warp {label}: {sw}x{sh} -> {dw}x{dh}", flush=True)
    out, od, src = rp.warp(ctx, torch.from_numpy(rgba).cuda(), torch.from_numpy(depth).cuda(), src_c, dst_c, dw, dh)
    want_rgba, want_depth, want_src = WP.warp(rgba, depth, src_c, sw, sh, dst_c, dw, dh)
    g_src = cpu(src).astype(np.int64)
    bad = g_src != want_src
    assert not bad.any(), f"{label}: source differs on {int(bad.sum())} of {bad.size} pixels"
    assert np.array_equal(cpu(out).view(np.uint32), want_rgba.view(np.uint32)), label
    assert np.array_equal(cpu(od).view(np.uint32), want_depth.view(np.uint32)), label
    filled = (g_src >= 0).mean()
    print(f"[warp] {label}: {filled:.3f} of the pixels covered", flush=True)
    return g_src


MOVES = {
    "identity": lambda: cam((0.2, 0.1, 3.0)),
    "translate": lambda: cam((0.35, 0.1, 2.9), (0.1, 0, 0)),
    "rotate": lambda: cam((0.2, 0.1, 3.0), (0.4, -0.2, 0), (0.1, 1, 0)),
    "closer": lambda: cam((0.2, 0.1, 2.2)),
    "zoom": lambda: cam((0.1, 0.1, 3.1), (0, 0.05, 0), (0, 1, 0), 45),
    "large": lambda: cam((2.0, 0.5, 2.0)),
    "reversed": lambda: cam((0.2, 0.1, 3.0), (0.4, 0.2, 6.0)),
}


@pytest.mark.parametrize("move", list(MOVES))
@pytest.mark.parametrize("sizes", [((64, 48), (64, 48)), ((200, 136), (131, 77)), ((37, 23), (50, 41))])
def test_warp_bitexact(rp, ctx, move, sizes):
    (sw, sh), (dw, dh) = sizes
    rng = np.random.default_rng(zlib.crc32(f"{move} {sizes}".encode()))
    depth = smooth_depth(rng, sw, sh)
    rgba = rng.random((sh, sw, 4)).astype(F32)
    src = run_warp(rp, ctx, rgba, depth, cam((0.2, 0.1, 3.0)), MOVES[move](), dw, dh, f"{move} {sizes}")
    if move == "identity" and (sw, sh) == (dw, dh):
        assert np.array_equal(src.reshape(-1), np.arange(sw * sh))
    if move == "reversed":
        assert np.all(src == -1)


def test_warps_in_a_row_of_changing_sizes(rp, ctx):
    """Warps use two z-buffers in turn, each emptied by the previous warp's resolve up to that warp's
    size: a sequence that grows, shrinks and grows again (fill passes needed and not needed) must
    give the oracle's result every time."""
    rng = np.random.default_rng(11)
    sizes = [((64, 48), (64, 48)), ((64, 48), (64, 48)), ((90, 40), (100, 30)), ((20, 20), (20, 20)),
             ((64, 48), (100, 30)), ((40, 40), (64, 48)), ((64, 48), (64, 48)), ((300, 200), (320, 240)),
             ((64, 48), (64, 48))]
    for (sw, sh), (dw, dh) in sizes:
        depth = smooth_depth(rng, sw, sh)
        rgba = rng.random((sh, sw, 4)).astype(F32)
        run_warp(rp, ctx, rgba, depth, cam((0.2, 0.1, 3.0)), MOVES["translate"](), dw, dh, f"sequence {sw}x{sh}->{dw}x{dh}")


def test_warp_degenerate_shapes(rp, ctx):
    rng = np.random.default_rng(7)
    for (sw, sh), (dw, dh) in (((1, 1), (1, 1)), ((1, 1), (5, 3)), ((4096, 1), (1, 4096)), ((1, 777), (300, 2)),
                               ((17, 3), (1, 1))):
        depth = smooth_depth(rng, sw, sh, hole_frac=0.1)
        rgba = rng.random((sh, sw, 4)).astype(F32)
        run_warp(rp, ctx, rgba, depth, cam((0.2, 0.1, 3.0)), MOVES["translate"](), dw, dh, f"{sw}x{sh}->{dw}x{dh}")
    depth = np.full((9, 11), np.inf, F32)
    depth[::2] = np.nan
    rgba = rng.random((9, 11, 4)).astype(F32)
    run_warp(rp, ctx, rgba, depth, cam((0.2, 0.1, 3.0)), MOVES["rotate"](), 11, 9, "points at infinity")


def test_warp_full_hd_bitexact(rp, ctx):
    """1920x1080 -> 1920x1080 under a small head motion and under a larger one (every pixel)."""
    rng = np.random.default_rng(2207)
    depth = smooth_depth(rng, 1920, 1080, hole_frac=0.3, speck_frac=0.02)
    rgba = rng.random((1080, 1920, 4)).astype(F32)
    src_c = cam((0.0, 0.0, 3.0), fov=60)
    run_warp(rp, ctx, rgba, depth, src_c, cam((0.02, 0.01, 2.99), (0.01, 0, 0), fov=60), 1920, 1080, "1080p small")
    run_warp(rp, ctx, rgba, depth, src_c, cam((0.6, 0.3, 2.6), (0.05, 0, 0), fov=60), 1920, 1080, "1080p large")


def test_warp_of_oracle_render_bitexact(rp, ctx):
    """The oracle's own render and depth of the small workload, rounded to float32, warped by both."""
    wl = W.make_workload(1, n=64, width=120, height=90)
    level = pp.stored_levels(wl.fields, 1, "f16")[0]
    ref = oracle.render_workload(wl, level)
    rgba = ref.rgba.astype(F32)
    depth = ref.depth.astype(F32)
    c = wl.camera.as_array()
    eye = c[:3]
    for k, delta in enumerate(([0.05, 0.0, 0.0], [0.0, -0.08, 0.03], [0.2, 0.1, -0.1])):
        d = c.copy()
        d[:3] = eye + np.array(delta, F32)
        src = run_warp(rp, ctx, rgba, depth, c, d, wl.width, wl.height, f"oracle frame move {k}")
        # a pure sideways shift keeps every pixel covered; the larger moves turn part of the view
        # beyond the source frame, which stays empty
        assert (src >= 0).mean() == 1.0 if k == 0 else (src >= 0).mean() > 0.9


def test_warp_reduces_the_error_of_a_stale_frame(rp, ctx):
    """Showing the frame of an older pose is worse than warping it to the new pose (both measured
    against the frame rendered at the new pose) once the view moves by a pixel or more; below a
    pixel the stale frame is already close and the nearest-pixel splat cannot improve on it."""
    wl = W.make_workload(1, n=64, width=256, height=192)
    vid = rp.load_fields(ctx, torch.from_numpy(wl.fields).cuda(), "f16", 1, wl.r_inner, wl.r_outer)
    rp.set_brush(ctx, vid, wl.brush.active, wl.brush.lo, wl.brush.hi)
    rp.set_transfer_function(ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, wl.tf.ref_step)
    rp.set_options(ctx, wl.ert)
    c0 = wl.camera.as_array()
    rgba0, dep0 = rp.render_depth(ctx, vid, c0, wl.width, wl.height, 0, wl.step)
    for delta in ([0.2, 0.0, 0.0], [0.1, 0.0, 0.0]):
        c1 = c0.copy()
        c1[:3] += np.array(delta, F32)
        truth = cpu(rp.render(ctx, vid, c1, wl.width, wl.height, 0, wl.step))
        warped, _, _ = rp.warp(ctx, rgba0, dep0, c0, c1)
        e_stale = np.abs(cpu(rgba0) - truth).mean()
        e_warp = np.abs(cpu(warped) - truth).mean()
        print(f"[warp] move {delta}: mean-abs error stale {e_stale:.4e}, warped {e_warp:.4e}", flush=True)
        assert e_warp < 0.8 * e_stale
    rp.unload(ctx, vid)


def test_warp_arguments(rp, ctx):
    c = cam((0.2, 0.1, 3.0))
    rgba = torch.zeros((8, 8, 4), dtype=torch.float32, device="cuda")
    depth = torch.zeros((8, 8), dtype=torch.float32, device="cuda")
    # every output pointer below has room for what a call that got through would write
    big = torch.zeros((16385 * 4,), dtype=torch.float32, device="cuda")
    P = rp.ctypes.byref
    C = rp.Camera.make
    # output overlapping an input, outputs overlapping each other, NULL input, bad sizes, bad camera
    for args in ((8, 8, rgba.data_ptr(), depth.data_ptr(), 8, 8, rgba.data_ptr(), None, None),
                 (8, 8, rgba.data_ptr(), depth.data_ptr(), 8, 8, big.data_ptr(), None, big.data_ptr()),
                 (8, 8, rgba.data_ptr(), depth.data_ptr(), 8, 8, big.data_ptr(), depth.data_ptr(), None),
                 (8, 8, None, depth.data_ptr(), 8, 8, big.data_ptr(), None, None),
                 (0, 8, rgba.data_ptr(), depth.data_ptr(), 8, 8, big.data_ptr(), None, None),
                 (8, 8, rgba.data_ptr(), depth.data_ptr(), 16385, 1, big.data_ptr(), None, None)):
        sw, sh, a, d, dw, dh, o, od, os_ = args
        with pytest.raises(rp.RaypcError):
            rp._check(rp._warp(ctx, P(C(c)), sw, sh, a, d, P(C(c)), dw, dh, o, od, os_, None))
    bad = c.copy()
    bad[3:6] = bad[0:3]
    with pytest.raises(rp.RaypcError):
        rp.warp(ctx, rgba, depth, c, bad)
    torch.cuda.synchronize()
