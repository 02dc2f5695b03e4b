"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Bit-exact: level data, min/max tables, skip lists, voxel masks, skip on/off and
inclusive-brush invariants.  Within 2e-4 max-abs per RGBA channel, with exact
nominal/composited sample counts, on every pixel the oracle does not flag as
fragile (a brush, termination or shell-grazing decision within floating-point
reach of its threshold).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import preprocess as pp
from paper_2207_12011_amd import workloads as W

from .parity import check_depth, compare, sample_pixels

pytestmark = pytest.mark.gpu

STORAGES = ["f32", "f16", "u8"]


@pytest.fixture(scope="module")
def rp():
    from paper_2207_12011_amd import raypc
    return raypc


@pytest.fixture(scope="module")
def ctx(rp):
    c = rp.create(0)
    yield c
    rp.destroy(c)


@pytest.fixture(scope="module")
def c0():
    return W.make_workload(0)


@pytest.fixture(scope="module")
def small5():
    """The five-field recipe at 64^3 with a ragged image size."""
    return W.make_workload(1, n=64, width=200, height=136)


def load(rp, ctx, wl, storage="f32", n_lods=3):
    vid = rp.load_fields(ctx, torch.from_numpy(wl.fields).cuda(), storage, n_lods, wl.r_inner, wl.r_outer)
    rp.set_brush(ctx, vid, wl.brush.active, wl.brush.lo, wl.brush.hi)
    rp.set_transfer_function(ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, wl.tf.ref_step)
    rp.set_options(ctx, wl.ert)
    return vid


def cpu(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def gpu_render(rp, ctx, vid, wl, lod=0, step=None, camera=None, width=None, height=None, skip=True):
    rgba, nom, comp = rp.render_debug(ctx, vid, camera if camera is not None else wl.camera.as_array(),
                                      width or wl.width, height or wl.height, lod, step or wl.step, skip=skip)
    return cpu(rgba), cpu(nom), cpu(comp)


# ----------------------------------------------------------------------------- preprocessing
@pytest.mark.parametrize("storage", STORAGES)
def test_levels_and_minmax_bitexact(rp, ctx, c0, small5, storage):
    for wl in (c0, small5):
        print(f"[case] levels/minmax {wl.name} {storage}", flush=True)
        vid = load(rp, ctx, wl, storage)
        levels = pp.stored_levels(wl.fields, 3, storage)
        for lod in range(3):
            for f in range(wl.n_fields):
                got = cpu(rp.export_level(ctx, vid, lod, f))
                assert np.array_equal(got.view(np.uint32), levels[lod][f].view(np.uint32)), (lod, f)
                mm = cpu(rp.export_minmax(ctx, vid, lod, f))
                mn, mx = pp.brick_minmax(levels[lod][f])
                assert np.array_equal(mm[..., 0], mn) and np.array_equal(mm[..., 1], mx), (lod, f)
                sub = cpu(rp.export_minmax_sub(ctx, vid, lod, f))     # [bz, by, bx, sx + 2 sy + 4 sz, 2]
                smn, smx = pp.brick_minmax(levels[lod][f], pp.SUB)   # [sz, sy, sx] over the 2 nb grid
                for i in range(8):
                    sx, sy, sz = i & 1, (i >> 1) & 1, i >> 2
                    assert np.array_equal(sub[..., i, 0], smn[sz::2, sy::2, sx::2]), (lod, f, i)
                    assert np.array_equal(sub[..., i, 1], smx[sz::2, sy::2, sx::2]), (lod, f, i)
        rp.unload(ctx, vid)


@pytest.mark.parametrize("storage", STORAGES)
def test_skiplist_and_mask_bitexact(rp, ctx, small5, storage):
    wl = small5
    print(f"[case] skiplist {storage}", flush=True)
    vid = load(rp, ctx, wl, storage)
    levels = pp.stored_levels(wl.fields, 3, storage)
    tab = wl.tf.rgba.copy()
    tab[:40, 3] = 0.0
    tab[200:, 3] = 0.0
    rp.set_transfer_function(ctx, 1, wl.tf.field, wl.tf.vmin, wl.tf.vmax, tab, wl.tf.ref_step)
    nf = wl.n_fields
    brushes = [(wl.brush.active, wl.brush.lo, wl.brush.hi),
               (np.zeros(nf, np.uint8), wl.brush.lo, wl.brush.hi),
               (np.ones(nf, np.uint8), np.full(nf, 1.0, np.float32), np.full(nf, 0.0, np.float32)),
               (np.array([1, 0, 1, 0, 0], np.uint8), np.array([0.6, 0, 4.0, 0, 0], np.float32),
                np.array([1.2, 0, 5.0, 0, 0], np.float32))]
    for bi, (act, lo, hi) in enumerate(brushes):
        rp.set_brush(ctx, vid, act, lo, hi)
        for lod in range(3):
            mins, maxs = zip(*[pp.brick_minmax(levels[lod][f]) for f in range(nf)])
            for slot, t in ((0, wl.tf.rgba), (1, tab)):
                brick_skip = pp.skip_bits(mins, maxs, act, lo, hi, wl.tf.field, wl.tf.vmin, wl.tf.vmax, t)
                want = pp.pack_bits(brick_skip)
                got = cpu(rp.export_skiplist(ctx, vid, lod, slot)).view(np.uint32)
                assert np.array_equal(got, want), (bi, lod, slot)
                want_sub = pp.sub_skip(levels[lod], act, lo, hi, wl.tf.field, wl.tf.vmin, wl.tf.vmax, t)
                got_sub = cpu(rp.export_subskip(ctx, vid, lod, slot))
                assert np.array_equal(got_sub, want_sub), (bi, lod, slot)
                nb = (wl.n >> lod) // 8
                got_words = cpu(rp.export_skip_words(ctx, vid, lod, slot)).view(np.uint16)
                assert np.array_equal(got_words, pp.skip_words(want_sub, nb, brick_skip)), (bi, lod, slot)
            m = cpu(rp.export_voxel_mask(ctx, vid, lod))
            assert np.array_equal(m, pp.voxel_mask(levels[lod], act, lo, hi)), (bi, lod)
    rp.unload(ctx, vid)


def test_brush_change_leaves_volume_untouched(rp, ctx, small5):
    wl = small5
    vid = load(rp, ctx, wl, "f16")
    before = [cpu(rp.export_level(ctx, vid, 0, f)).copy() for f in range(wl.n_fields)]
    mm_before = cpu(rp.export_minmax(ctx, vid, 1, 2)).copy()
    rp.set_brush(ctx, vid, np.ones(5, np.uint8), np.zeros(5, np.float32), np.ones(5, np.float32))
    rp.render(ctx, vid, wl.camera.as_array(), 64, 64, 0, 0.5)
    for f in range(wl.n_fields):
        assert np.array_equal(cpu(rp.export_level(ctx, vid, 0, f)), before[f])
    assert np.array_equal(cpu(rp.export_minmax(ctx, vid, 1, 2)), mm_before)
    rp.unload(ctx, vid)


# ----------------------------------------------------------------------------- rendering
@pytest.mark.parametrize("storage", STORAGES)
@pytest.mark.parametrize("lod", [0, 1, 2])
def test_render_tiny_full_frame(rp, ctx, c0, storage, lod):
    wl = c0
    print(f"[case] tiny full frame {storage} lod {lod}", flush=True)
    vid = load(rp, ctx, wl, storage)
    level = pp.stored_levels(wl.fields, 3, storage)[lod]
    rgba, nom, comp = gpu_render(rp, ctx, vid, wl, lod)
    ref = oracle.render_workload(wl, level)
    compare(rgba, ref, nom, comp, label=f"tiny {storage} lod{lod}")
    assert ref.nominal.sum() > 0 and (ref.rgba[..., 3] > 0).mean() > 0.1
    rp.unload(ctx, vid)


@pytest.mark.parametrize("storage", STORAGES)
@pytest.mark.parametrize("step", [0.5, 0.37, 2.0])
def test_render_ragged_five_fields(rp, ctx, small5, storage, step):
    wl = small5
    print(f"[case] ragged 200x136 {storage} step {step}", flush=True)
    vid = load(rp, ctx, wl, storage)
    level = pp.stored_levels(wl.fields, 1, storage)[0]
    rgba, nom, comp = gpu_render(rp, ctx, vid, wl, 0, step)
    ref = oracle.render_workload(wl, level, step=step)
    compare(rgba, ref, nom, comp, label=f"ragged {storage} step {step}")
    rp.unload(ctx, vid)


@pytest.mark.parametrize("case", ["inside_shell", "inside_core", "grazing", "opaque_ert", "no_inner"])
def test_render_special_views(rp, ctx, small5, case):
    wl = small5
    print(f"[case] special view {case}", flush=True)
    r_inner = 0.0 if case == "no_inner" else wl.r_inner
    vid = rp.load_fields(ctx, torch.from_numpy(wl.fields).cuda(), "f32", 1, r_inner, wl.r_outer)
    rp.set_brush(ctx, vid, wl.brush.active, wl.brush.lo, wl.brush.hi)
    tab = wl.tf.rgba.copy()
    ert = wl.ert
    cam = wl.camera.as_array()
    if case == "inside_shell":
        cam = np.array([0.8, 0.1, 0.1, 0, 0, 0, 0, 0, 1, 90], np.float32)
    elif case == "inside_core":
        cam = np.array([0.1, 0.2, 0.05, 1, 0, 0, 0, 0, 1, 100], np.float32)
    elif case == "grazing":
        cam = np.array([3, 0, 0, 0, 0.55, 0, 0, 0, 1, 20], np.float32)
    elif case == "opaque_ert":
        tab[:, 3] = np.linspace(0.2, 0.95, 256, dtype=np.float32)
        rp.set_brush(ctx, vid, np.zeros(5, np.uint8), wl.brush.lo, wl.brush.hi)
        ert = 0.95
    rp.set_transfer_function(ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, tab, wl.tf.ref_step)
    rp.set_options(ctx, ert)
    rgba, nom, comp = gpu_render(rp, ctx, vid, wl, 0, 0.5, camera=cam, width=96, height=80)
    active = np.zeros(5, np.uint8) if case == "opaque_ert" else wl.brush.active
    ref = oracle.render(wl.fields, cam, 96, 80, 0.5, active=active, lo=wl.brush.lo, hi=wl.brush.hi,
                        tf_field=wl.tf.field, vmin=wl.tf.vmin, vmax=wl.tf.vmax, tf_rgba=tab, ert=ert,
                        r_inner=r_inner, r_outer=wl.r_outer)
    compare(rgba, ref, nom, comp, label=case)
    rp.unload(ctx, vid)


def test_skip_on_off_bitexact(rp, ctx, small5):
    wl = small5
    for storage in STORAGES:
        vid = load(rp, ctx, wl, storage)
        for lod in range(3):
            a = gpu_render(rp, ctx, vid, wl, lod, skip=True)
            b = gpu_render(rp, ctx, vid, wl, lod, skip=False)
            for x, y in zip(a, b):
                assert np.array_equal(x, y), (storage, lod)
        plain = cpu(rp.render(ctx, vid, wl.camera.as_array(), wl.width, wl.height, 0, wl.step))
        assert np.array_equal(plain, gpu_render(rp, ctx, vid, wl, 0)[0])
        rp.unload(ctx, vid)


@pytest.mark.parametrize("base", ["f16", "f32", "u8"])
def test_records_equal_compact_layout(rp, ctx, small5, c0, base):
    """Both layouts hold the same stored values (8-bit records hold the decoded values); every render
    is bit-identical."""
    for wl in (small5, c0):
        rec = load(rp, ctx, wl, base)
        cmp_ = load(rp, ctx, wl, base + "c")
        assert rp.volume_info(ctx, rec)["bytes"] > 2 * rp.volume_info(ctx, cmp_)["bytes"]
        views = [(wl.camera.as_array(), 0, 0.5), (wl.camera.as_array(), 1, 0.37),
                 (np.array([0.8, 0.1, 0.1, 0, 0, 0, 0, 0, 1, 90], np.float32), 0, 1.0),
                 (np.array([3, 0, 0, 0, 0.55, 0, 0, 0, 1, 20], np.float32), 2, 0.5)]
        for cam, lod, step in views:
            a = gpu_render(rp, ctx, rec, wl, lod, step, camera=cam, width=120, height=72)
            b = gpu_render(rp, ctx, cmp_, wl, lod, step, camera=cam, width=120, height=72)
            for x, y in zip(a, b):
                assert np.array_equal(x, y), (base, lod, step)
        rp.unload(ctx, rec)
        rp.unload(ctx, cmp_)


@pytest.mark.parametrize("base", ["u8", "f16"])
def test_blocks_at_the_grid_faces(rp, ctx, small5, base):
    """The 8-bit and binary16 blocks at the grid's faces: with the shell touching the cube (r_outer =
    1), samples next to each face centre have base voxels on the last (or first) voxel plane, where
    the upper corner clamps onto the base voxel and the block reads its copied values.  The compact
    layout equals the records (gathered from the stored values themselves) bit for bit there, on
    every level, with all five fields fetched (an all-inclusive brush)."""
    wl = small5
    nf = wl.n_fields
    vids = {}
    for st in (base, base + "c"):
        print(f"[case] blocks at the faces {st}", flush=True)
        vid = rp.load_fields(ctx, torch.from_numpy(wl.fields).cuda(), st, 3, 0.0, 1.0)
        rp.set_brush(ctx, vid, np.ones(nf, np.uint8), np.full(nf, -np.inf, np.float32),
                     np.full(nf, np.inf, np.float32))
        vids[st] = vid
    rp.set_transfer_function(ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, wl.tf.ref_step)
    rp.set_options(ctx, wl.ert)
    ups = {0: (0, 0, 1), 1: (0, 0, 1), 2: (0, 1, 0)}
    for axis in range(3):
        for sign in (1.0, -1.0):
            eye = [0.0, 0.0, 0.0]
            eye[axis] = 3.0 * sign
            cam = np.array(eye + [0, 0, 0] + list(ups[axis]) + [12], np.float32)
            for lod in range(3):
                a = gpu_render(rp, ctx, vids[base], wl, lod, 0.5, camera=cam, width=48, height=40)
                b = gpu_render(rp, ctx, vids[base + "c"], wl, lod, 0.5, camera=cam, width=48, height=40)
                assert a[0][..., 3].max() > 0.0, (axis, sign, lod)
                for x, y in zip(a, b):
                    assert np.array_equal(x, y), (axis, sign, lod)
    for vid in vids.values():
        rp.unload(ctx, vid)


def test_inclusive_brush_equals_none_and_empty_is_background(rp, ctx, small5):
    wl = small5
    vid = load(rp, ctx, wl, "f16")
    nf = wl.n_fields
    rp.set_brush(ctx, vid, np.zeros(nf, np.uint8), wl.brush.lo, wl.brush.hi)
    none = gpu_render(rp, ctx, vid, wl, 0)
    rp.set_brush(ctx, vid, np.ones(nf, np.uint8), np.full(nf, -np.inf, np.float32), np.full(nf, np.inf, np.float32))
    inf = gpu_render(rp, ctx, vid, wl, 0)
    mn, mx = wl.fields.min(axis=(1, 2, 3)), wl.fields.max(axis=(1, 2, 3))
    rp.set_brush(ctx, vid, np.ones(nf, np.uint8), mn - 1.0, mx + 1.0)
    wide = gpu_render(rp, ctx, vid, wl, 0)
    for other in (inf, wide):
        for x, y in zip(none, other):
            assert np.array_equal(x, y)
    rp.set_brush(ctx, vid, np.ones(nf, np.uint8), np.full(nf, 1.0, np.float32), np.full(nf, 0.0, np.float32))
    empty = gpu_render(rp, ctx, vid, wl, 0)
    assert np.all(empty[0] == 0.0) and np.all(empty[2] == 0)
    skip = cpu(rp.export_skiplist(ctx, vid, 0, 0)).view(np.uint32)
    assert np.all(skip == 0xFFFFFFFF)
    assert np.all(cpu(rp.export_subskip(ctx, vid, 0, 0)) == 0xFF)
    rp.set_options(ctx, 0.99, [0.1, 0.2, 0.3, 1.0])
    bg = gpu_render(rp, ctx, vid, wl, 0)[0]
    assert np.all(bg == np.array([0.1, 0.2, 0.3, 1.0], np.float32))
    rp.set_options(ctx, 0.99)
    rp.unload(ctx, vid)


def test_constant_density_closed_form(rp, ctx):
    n = 64
    vol = np.full((1, n, n, n), 0.25, np.float32)
    vid = rp.load_fields(ctx, torch.from_numpy(vol).cuda(), "f32", 3, 0.55, 1.0)
    rp.set_brush(ctx, vid, [0], [0], [0])
    tab = np.zeros((256, 4), np.float32)
    tab[:, :3] = (0.2, 0.5, 0.9)
    tab[:, 3] = 0.3
    rp.set_transfer_function(ctx, 0, 0, 0.0, 1.0, tab)
    rp.set_options(ctx, 1.0)
    cam = np.array([3, 0, 0, 0, 0, 0, 0, 0, 1, 60], np.float32)
    from .bruteforce import camera_rays
    eye, dirs = camera_rays(cam, 33, 33)
    p = np.linalg.norm(np.cross(eye[None, None, :], dirs), axis=-1)
    r_in = float(np.float32(0.55))
    L = np.where(p < 1, 2 * np.sqrt(np.maximum(1 - p ** 2, 0)), 0) - np.where(p < r_in, 2 * np.sqrt(np.maximum(r_in ** 2 - p ** 2, 0)), 0)
    want = 1 - (1 - float(np.float32(0.3))) ** (L / float(np.float32(2 / 256)))
    for lod in range(3):
        for step in (0.25, 0.5, 1.0):
            got = cpu(rp.render(ctx, vid, cam, 33, 33, lod, step))
            graze = np.abs(p - r_in) < 1e-3
            assert np.abs(got[..., 3] - want)[~graze].max() <= 2e-5, (lod, step)
    rp.set_options(ctx, 0.99)
    rp.unload(ctx, vid)


def test_progressive_passes_equal_single_renders(rp, ctx, small5):
    wl = small5
    vid = load(rp, ctx, wl, "f16")
    cam = wl.camera.as_array()
    outs = rp.render_progressive(ctx, vid, cam, 120, 90, 0, 0.25, 3)
    for k, o in enumerate(outs):
        single = rp.render(ctx, vid, cam, 120, 90, 0, 0.25 * 2 ** (2 - k))
        assert np.array_equal(cpu(o), cpu(single)), k
    # each pass matches the oracle at its own step, and the passes converge
    level = pp.stored_levels(wl.fields, 1, "f16")[0]
    errs = []
    for k, o in enumerate(outs):
        ref = oracle.render_workload(wl, level, step=0.25 * 2 ** (2 - k), width=120, height=90)
        compare(cpu(o), ref, label=f"progressive pass {k}")
        errs.append(np.abs(cpu(o) - cpu(outs[-1])).mean())
    assert errs[0] >= errs[1] >= errs[2] == 0.0
    rp.unload(ctx, vid)


@pytest.mark.parametrize("n0", [256, 512])
def test_select_lod_matches_rule(rp, ctx, n0):
    vol = np.zeros((1, n0, n0, n0), np.float32)
    vid = rp.load_fields(ctx, torch.from_numpy(vol).cuda(), "f16", 3, 0.55, 1.0)
    rng = np.random.default_rng(9)
    for _ in range(40):
        d = rng.uniform(0.5, 8.0)
        cam = W.orbit_camera(rng.uniform(0, 2 * math.pi), rng.uniform(-1, 1), d, rng.uniform(20, 90))
        for size in (64, 256, 512, 1024, 1080, 2048):
            want = pp.select_lod(n0, 3, cam.eye, cam.fov_y_deg, size)
            assert rp.select_lod(ctx, vid, cam, size, size) == want
    rp.unload(ctx, vid)


def test_invalid_arguments_leave_state(rp, ctx, small5):
    wl = small5
    vid = load(rp, ctx, wl, "f32", 1)
    cam = wl.camera.as_array()
    ref = cpu(rp.render(ctx, vid, cam, 48, 40, 0, 0.5))
    bad_calls = [
        lambda: rp.render(ctx, vid, cam, 0, 40, 0, 0.5),
        lambda: rp.render(ctx, vid, cam, 48, 40, 1, 0.5),          # only one level
        lambda: rp.render(ctx, vid, cam, 48, 40, 0, 1e-3),
        lambda: rp.render(ctx, vid, np.array([3, 0, 0, 0, 0, 0, 1, 0, 0, 60], np.float32), 48, 40, 0, 0.5),
        lambda: rp.render(ctx, vid, np.array([3, 0, 0, 0, 0, 0, 0, 0, 1, 180], np.float32), 48, 40, 0, 0.5),
        lambda: rp.render(ctx, 12345, cam, 48, 40, 0, 0.5),
        lambda: rp.set_brush(ctx, vid, [1] * 4, [0] * 4, [1] * 4),
        lambda: rp.set_brush(ctx, vid, [1] * 5, [np.nan] * 5, [1] * 5),
        lambda: rp.set_transfer_function(ctx, 0, 0, 1.0, 1.0, wl.tf.rgba),
        lambda: rp.set_transfer_function(ctx, 0, 0, 0.0, 1.0, wl.tf.rgba * 2),
        lambda: rp.set_transfer_function(ctx, 9, 0, 0.0, 1.0, wl.tf.rgba),
        lambda: rp.set_options(ctx, float("nan")),
        lambda: rp.load_fields(ctx, torch.zeros((1, 40, 40, 40), device="cuda"), "f32", 1),
        lambda: rp.load_fields(ctx, torch.zeros((9, 32, 32, 32), device="cuda"), "f32", 1),
        lambda: rp.load_fields(ctx, torch.full((1, 32, 32, 32), float("inf"), device="cuda"), "f32", 1),
    ]
    for i, call in enumerate(bad_calls):
        with pytest.raises(rp.RaypcError) as ei:
            call()
        assert ei.value.code == rp.ERR_INVALID, (i, str(ei.value))
        assert rp.last_error(), i
    assert np.array_equal(cpu(rp.render(ctx, vid, cam, 48, 40, 0, 0.5)), ref)
    rp.unload(ctx, vid)
    with pytest.raises(rp.RaypcError):
        rp.unload(ctx, vid)


def test_extreme_image_shapes(rp, ctx, c0):
    wl = c0
    vid = load(rp, ctx, wl, "f32", 1)
    for w, h in ((1, 1), (16384, 1), (1, 4096), (17, 3)):
        rgba, nom, comp = gpu_render(rp, ctx, vid, wl, 0, width=w, height=h)
        pix = sample_pixels(w, h, 3000)
        ref = oracle.render_workload(wl, wl.fields, width=w, height=h, pixels=pix)
        compare(rgba.reshape(-1, 4)[pix], ref, nom.reshape(-1)[pix], comp.reshape(-1)[pix], label=f"{w}x{h}")
    rp.unload(ctx, vid)


# ----------------------------------------------------------------------------- full-size sampled
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_single_request_256_full_size_sampled(rp, ctx, storage):
    wl = W.make_workload(1)
    print(f"[case] 256^3 x 5, 1024^2, {storage}", flush=True)
    vid = load(rp, ctx, wl, storage)
    rgba, nom, comp = gpu_render(rp, ctx, vid, wl, 0)
    level = pp.stored_levels(wl.fields, 1, storage)[0]
    pix = sample_pixels(wl.width, wl.height, 6000, seed=1)
    ref = oracle.render_workload(wl, level, pixels=pix)
    compare(rgba.reshape(-1, 4)[pix], ref, nom.reshape(-1)[pix], comp.reshape(-1)[pix], label=f"c1 {storage}")
    rp.unload(ctx, vid)


@pytest.mark.parametrize("storage", STORAGES)
def test_field_order_does_not_change_the_image(rp, ctx, small5, storage):
    """The renderer tests brushed fields in an order it picks per brush (to fetch fewer fields per
    sample).  Loading the same fields in other orders (brush and transfer function permuted with
    them) changes that order but never the image or the counts, which match the oracle."""
    wl = small5
    cam = wl.camera.as_array()
    first = None
    for perm in ([0, 1, 2, 3, 4], [4, 3, 2, 1, 0], [2, 0, 4, 1, 3]):
        print(f"[case] field order {perm} {storage}", flush=True)
        vid = rp.load_fields(ctx, torch.from_numpy(np.ascontiguousarray(wl.fields[perm])).cuda(), storage, 1,
                             wl.r_inner, wl.r_outer)
        rp.set_brush(ctx, vid, wl.brush.active[perm], wl.brush.lo[perm], wl.brush.hi[perm])
        rp.set_transfer_function(ctx, 0, perm.index(wl.tf.field), wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, wl.tf.ref_step)
        rp.set_options(ctx, wl.ert)
        for act in (wl.brush.active[perm], np.array([1, 0, 1, 0, 1], np.uint8)[perm]):
            rp.set_brush(ctx, vid, act, wl.brush.lo[perm], wl.brush.hi[perm])
            got = gpu_render(rp, ctx, vid, wl, 0)
            if first is None:
                first = {}
            key = tuple(act[np.argsort(perm)].tolist())
            if key in first:
                assert all(np.array_equal(a, b) for a, b in zip(got, first[key])), (perm, key)
            else:
                first[key] = got
                level = pp.stored_levels(wl.fields[perm], 1, storage)[0]
                ref = oracle.render_workload(wl, level, active=act, lo=wl.brush.lo[perm], hi=wl.brush.hi[perm],
                                             tf_field=perm.index(wl.tf.field))
                compare(got[0], ref, got[1], got[2], label=f"field order {perm} {storage}")
        rp.unload(ctx, vid)


@pytest.mark.parametrize("storage", ["f32", "f16", "u8c"])
def test_work_counts(rp, ctx, small5, storage):
    """The renderer's work counts (the roofline's numerator): with an all-inclusive brush and a table
    positive everywhere nothing is skipped, every sample is evaluated and fetches each needed field
    once (5 with every field brushed, 1 with none); with the real brush, evaluated samples lie
    between the passing and the nominal ones and fetch between 1 and 5 fields each.  The image is
    raypc_render's."""
    wl = small5
    vid = load(rp, ctx, wl, storage, 1)
    cam = wl.camera.as_array()
    nf = wl.n_fields
    try:
        for act, lo, hi, per in ((np.ones(nf, np.uint8), np.full(nf, -np.inf, np.float32), np.full(nf, np.inf, np.float32), 5),
                                 (np.zeros(nf, np.uint8), wl.brush.lo, wl.brush.hi, 1),
                                 (wl.brush.active, wl.brush.lo, wl.brush.hi, None)):
            rp.set_brush(ctx, vid, act, lo, hi)
            rgba, ev, fe = (cpu(t).astype(np.int64) if i else cpu(t) for i, t in
                            enumerate(rp.render_work(ctx, vid, cam, wl.width, wl.height, 0, wl.step)))
            plain = cpu(rp.render(ctx, vid, cam, wl.width, wl.height, 0, wl.step))
            assert np.array_equal(rgba.view(np.uint32), plain.view(np.uint32))
            _, nom, comp = (cpu(t).astype(np.int64) for t in rp.render_debug(ctx, vid, cam, wl.width, wl.height, 0,
                                                                              wl.step))
            print(f"[work] {storage} per-sample fields {per}: nominal {nom.sum()}, evaluated {ev.sum()}, "
                  f"fetched {fe.sum()}, passed {comp.sum()}", flush=True)
            if per is not None:
                assert np.array_equal(ev, nom)
                assert np.array_equal(fe, per * nom)
            else:
                assert np.all(comp <= ev) and np.all(ev <= nom) and np.all(ev <= fe) and np.all(fe <= 5 * ev)
                assert ev.sum() < nom.sum() and fe.sum() < 5 * ev.sum() and comp.sum() > 0
    finally:
        rp.unload(ctx, vid)


def test_narrow_storage_equals_float32_on_representable_data(rp, ctx, small5):
    """Fields of integers in [0, 255] with a 0 and a 255 in every 8^3 brick: binary16 holds them
    exactly and the 8-bit scale of every brick is exactly 1, so all storages and layouts store the
    same values and must render the same image and counts, bit for bit (level 0)."""
    wl = small5
    f = wl.fields
    lo_f, hi_f = f.reshape(5, -1).min(axis=1), f.reshape(5, -1).max(axis=1)
    q = np.rint((f - lo_f[:, None, None, None]) / (hi_f - lo_f)[:, None, None, None] * 255).astype(np.float32)
    q[:, ::8, ::8, ::8] = 0.0
    q[:, ::8, ::8, 1::8] = 255.0
    fields = np.ascontiguousarray(q)
    m = W.shell_mask(W.radius(64))
    # bounds half-way between integers, so that few samples sit on a bound
    brush_lo = np.array([np.quantile(fields[k][m], 0.3) + 0.5 for k in range(5)], np.float32)
    brush_hi = np.array([np.quantile(fields[k][m], 0.95) - 0.5 for k in range(5)], np.float32)
    act = np.array([1, 1, 0, 1, 1], np.uint8)
    cam = wl.camera.as_array()
    want = None
    for storage in ("f32", "f16", "u8", "f32c", "f16c", "u8c"):
        print(f"[case] representable data, {storage}", flush=True)
        vid = rp.load_fields(ctx, torch.from_numpy(fields).cuda(), storage, 1, wl.r_inner, wl.r_outer)
        rp.set_brush(ctx, vid, act, brush_lo, brush_hi)
        rp.set_transfer_function(ctx, 0, 1, 0.0, 255.0, wl.tf.rgba, wl.tf.ref_step)
        rp.set_options(ctx, wl.ert)
        level = cpu(rp.export_level(ctx, vid, 0, 2))
        assert np.array_equal(level, fields[2]), storage
        got = gpu_render(rp, ctx, vid, wl, 0)
        rp.unload(ctx, vid)
        if want is None:
            want = got
            ref = oracle.render_workload(wl, fields, active=act, lo=brush_lo, hi=brush_hi, tf_field=1, vmin=0.0,
                                         vmax=255.0)
            compare(got[0], ref, got[1], got[2], label="representable data f32")
        else:
            assert all(np.array_equal(a, b) for a, b in zip(got, want)), storage


@pytest.fixture(scope="module")
def c2():
    return W.make_workload(2)


def test_precision_512_full_size_sampled(rp, ctx, c2):
    wl = c2
    print("[case] 512^3 x 5, 1920x1080, all storages", flush=True)
    fields_dev = torch.from_numpy(wl.fields).cuda()
    pix = sample_pixels(wl.width, wl.height, 3000, seed=2)
    for storage in STORAGES:
        vid = rp.load_fields(ctx, fields_dev, storage, 3, wl.r_inner, wl.r_outer)
        rp.set_brush(ctx, vid, wl.brush.active, wl.brush.lo, wl.brush.hi)
        rp.set_transfer_function(ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, wl.tf.ref_step)
        rp.set_options(ctx, wl.ert)
        rgba, nom, comp = gpu_render(rp, ctx, vid, wl, 0)
        # the kernel that is timed and served (one-wave blocks, 32-bit record offsets, no counts) gives
        # the counting variant's image bit for bit, at the level the selection rule picks too
        for lod in (0, -1):
            plain = cpu(rp.render(ctx, vid, wl.camera.as_array(), wl.width, wl.height, lod, wl.step))
            assert np.array_equal(plain.view(np.uint32), rgba.view(np.uint32)), (storage, lod)
        level = np.stack([rp_level for rp_level in
                          (cpu(rp.export_level(ctx, vid, 0, f)) for f in range(wl.n_fields))])
        want_level = np.stack([pp.stored_values(wl.fields[f], storage) for f in range(wl.n_fields)])
        assert np.array_equal(level.view(np.uint32), want_level.view(np.uint32))
        ref = oracle.render_workload(wl, want_level, pixels=pix)
        compare(rgba.reshape(-1, 4)[pix], ref, nom.reshape(-1)[pix], comp.reshape(-1)[pix], label=f"c2 {storage}")
        # the depth that image warping reprojects with, from the same frame
        rgba_d, dep = rp.render_depth(ctx, vid, wl.camera.as_array(), wl.width, wl.height, 0, wl.step)
        assert np.array_equal(cpu(rgba_d), rgba)
        check_depth(cpu(dep).reshape(-1)[pix], ref, label=f"c2 {storage} depth", min_frac=0.02,
                    gpu_rgba=rgba.reshape(-1, 4)[pix])
        rp.unload(ctx, vid)
        # the compact layout's timed kernel (8-bit: the code blocks) gives the records' image bit for bit
        print(f"[case] 512^3 x 5, 1920x1080, {storage} compact", flush=True)
        vid = rp.load_fields(ctx, fields_dev, storage + "c", 3, wl.r_inner, wl.r_outer)
        rp.set_brush(ctx, vid, wl.brush.active, wl.brush.lo, wl.brush.hi)
        plain = cpu(rp.render(ctx, vid, wl.camera.as_array(), wl.width, wl.height, 0, wl.step))
        assert np.array_equal(plain.view(np.uint32), rgba.view(np.uint32)), storage + "c"
        rp.unload(ctx, vid)


def test_served_requests_match_oracle(rp, ctx, c2):
    """Serving at full size: requests of the serving trace (the 256^3 and 512^3 x 5 binary16 volumes
    resident, images up to 2048^2, orbit cameras, 1-5-axis quantile brushes, level by the selection
    rule) submitted together, so that they share batched launches, each checked against the oracle
    on sampled pixels of the level the rule picks, and equal to its single render bit for bit."""
    wl512 = c2
    wl256 = W.make_workload(1)
    rng = np.random.default_rng(3)
    tables = [W.quantile_table(wl256.fields, W.shell_mask(W.radius(256)), rng),
              W.quantile_table(wl512.fields, W.shell_mask(W.radius(512)), rng)]
    trace = W.serving_trace(tables, n=40)
    # twelve requests covering both volumes and every image size
    chosen, seen = [], set()
    for i, q in enumerate(trace):
        key = (q.volume, (q.width, q.height))
        if key not in seen or len(chosen) < 6:
            seen.add(key)
            chosen.append(i)
        if len(chosen) == 12:
            break
    wls = [wl256, wl512]
    tf = wl512.tf
    rp.set_transfer_function(ctx, 0, tf.field, tf.vmin, tf.vmax, tf.rgba, tf.ref_step)
    rp.set_options(ctx, wl512.ert)
    vols = [rp.load_fields(ctx, torch.from_numpy(w.fields).cuda(), "f16", 3) for w in wls]
    levels = [pp.stored_levels(w.fields, 3, "f16") for w in wls]
    outs = [torch.full((trace[i].height, trace[i].width, 4), -1.0, dtype=torch.float32, device="cuda") for i in chosen]
    rp.server_start(ctx, 8 << 30, 64, 32768, 2)
    try:
        tickets = [rp.submit(ctx, rp.make_request(vols[trace[i].volume], trace[i].camera, trace[i].width,
                                                  trace[i].height, o, -1, 0.5, trace[i].active, trace[i].lo,
                                                  trace[i].hi, 0))
                   for i, o in zip(chosen, outs)]
        for t in tickets:
            rp.wait(ctx, t, 120000)
            rp.release(ctx, t)
    finally:
        rp.server_stop(ctx)
    try:
        for i, o in zip(chosen, outs):
            q = trace[i]
            w = wls[q.volume]
            cam = q.camera.as_array()
            lod = pp.select_lod(w.n, 3, cam[:3], float(cam[9]), q.height)
            assert rp.select_lod(ctx, vols[q.volume], cam, q.width, q.height) == lod
            label = f"served #{i} {w.n}^3 {q.width}x{q.height} lod {lod} k={int(q.active.sum())}"
            print(f"[case] {label}", flush=True)
            served = cpu(o)
            rp.set_brush(ctx, vols[q.volume], q.active, q.lo, q.hi)
            single = cpu(rp.render(ctx, vols[q.volume], cam, q.width, q.height, -1, 0.5))
            assert np.array_equal(served.view(np.uint32), single.view(np.uint32)), label
            pix = sample_pixels(q.width, q.height, 400, seed=i)
            ref = oracle.render(levels[q.volume][lod], cam, q.width, q.height, 0.5, active=q.active, lo=q.lo,
                                hi=q.hi, tf_field=tf.field, vmin=tf.vmin, vmax=tf.vmax, tf_rgba=tf.rgba,
                                ref_step=tf.ref_step, ert=wl512.ert, pixels=pix)
            compare(served.reshape(-1, 4)[pix], ref, label=label)
    finally:
        for v in vols:
            rp.unload(ctx, v)


@pytest.mark.timeout(1200)
def test_large_progressive_1024_4k_sampled(rp, ctx, capsys):
    """The large progressive configuration at its size: 1024^3 x 5 fields stored binary16 (level 0's
    record fields above 4 GiB, read at 64-bit offsets), a 3840x2160 view, progressive passes at step
    1.0 / 0.5 / 0.25 voxel for the final (~10 %) brush and for a brush half-way along the narrowing
    sequence; the first and final passes checked against the oracle on 1 000 sampled pixels, with
    exact counts where the counting variant is asked; the final pass served, and rendered from the
    compact binary16 blocks, equal to it bit for bit."""
    import time
    t0 = time.perf_counter()

    def say(msg):
        with capsys.disabled():
            print(f"[c4] {msg} ({time.perf_counter() - t0:.0f}s)", flush=True)

    wl = W.make_workload(4, progress=lambda m: say(f"generated {m}"))
    mask = W.shell_mask(W.radius(wl.n))
    brushes = W.narrowing_brushes(wl.fields, mask, np.random.default_rng(W.SEED_BASE + 4), wl.brush)
    del mask
    rp.set_transfer_function(ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, wl.tf.ref_step)
    rp.set_options(ctx, wl.ert)
    vid = rp.load_fields(ctx, torch.from_numpy(wl.fields).cuda(), "f16", 3, wl.r_inner, wl.r_outer)
    torch.cuda.synchronize()
    say("loaded f16 with records")
    level = np.stack([pp.stored_values(wl.fields[f], "f16") for f in range(wl.n_fields)])
    say("oracle level 0 stored values")
    cam = wl.camera.as_array()
    assert rp.select_lod(ctx, vid, cam, wl.width, wl.height) == 0
    pix = sample_pixels(wl.width, wl.height, 1000, seed=44)
    try:
        for b in (brushes[5], brushes[-1]):
            rp.set_brush(ctx, vid, b.active, b.lo, b.hi)
            passes = rp.render_progressive(ctx, vid, cam, wl.width, wl.height, -1, wl.step, 3)
            passes = [cpu(p) for p in passes]
            for k, st in ((0, wl.step * 4), (2, wl.step)):
                label = f"c4 f16 pass {k} step {st} brush lo {b.lo[0]:.3g}"
                ref = oracle.render_workload(wl, level, pixels=pix, step=st, active=b.active, lo=b.lo, hi=b.hi)
                say(f"oracle {label}")
                if k == 2 and b is brushes[-1]:
                    rgba, nom, comp = gpu_render(rp, ctx, vid, wl, 0, step=st)
                    assert np.array_equal(rgba.view(np.uint32), passes[k].view(np.uint32)), label
                    compare(rgba.reshape(-1, 4)[pix], ref, nom.reshape(-1)[pix], comp.reshape(-1)[pix], label=label)
                else:
                    compare(passes[k].reshape(-1, 4)[pix], ref, label=label)
        # the same final pass served (the batched kernel at 64-bit record offsets, two samples per
        # lane) equals the single render bit for bit
        b = brushes[-1]
        out = torch.empty((wl.height, wl.width, 4), dtype=torch.float32, device="cuda")
        rp.server_start(ctx, 8 << 30, 8, 32768, 2)
        try:
            req = rp.make_request(vid, cam, wl.width, wl.height, out, -1, wl.step, b.active, b.lo, b.hi, 0)
            rp.wait(ctx, rp.submit(ctx, req), 120000)
        finally:
            rp.server_stop(ctx)
        say("served the final pass")
        assert np.array_equal(cpu(out).view(np.uint32), passes[2].view(np.uint32))
        # the compact binary16 blocks (2.4 GB per field at level 0, byte offsets beyond 2^31) give
        # the final pass of the records bit for bit
        cvid = rp.load_fields(ctx, torch.from_numpy(wl.fields).cuda(), "f16c", 3, wl.r_inner, wl.r_outer)
        try:
            rp.set_brush(ctx, cvid, b.active, b.lo, b.hi)
            plain = cpu(rp.render(ctx, cvid, cam, wl.width, wl.height, 0, wl.step))
            say("compact binary16 final pass")
            assert np.array_equal(plain.view(np.uint32), passes[2].view(np.uint32))
        finally:
            rp.unload(ctx, cvid)
    finally:
        rp.unload(ctx, vid)



def test_jitter_and_coordinates_512_full_size_sampled(rp, ctx, c2):
    """The widened rows at the full 512^3 x 5 / 1920x1080 size (f16, sampled pixels): one jittered
    pass against the oracle given the same per-pixel offsets, and a coordinate cut (an x slab with a
    radius floor) against the oracle, with exact counts on non-fragile pixels."""
    from oracle import jitter as J
    wl = c2
    print("[case] 512^3 x 5, 1920x1080, jittered pass and coordinate cut (f16)", flush=True)
    vid = rp.load_fields(ctx, torch.from_numpy(wl.fields).cuda(), "f16", 1, wl.r_inner, wl.r_outer)
    rp.set_brush(ctx, vid, wl.brush.active, wl.brush.lo, wl.brush.hi)
    rp.set_transfer_function(ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, wl.tf.ref_step)
    rp.set_options(ctx, wl.ert)
    level = np.stack([pp.stored_values(wl.fields[f], "f16") for f in range(wl.n_fields)])
    pix = sample_pixels(wl.width, wl.height, 2000, seed=5)
    cam = wl.camera.as_array()
    try:
        rgba, nom, comp = rp.render_jittered(ctx, vid, cam, wl.width, wl.height, 0, wl.step, 3, 8, 0x2207, counts=True)
        s = J.offsets(wl.width, pix, 3, 8, 0x2207)
        ref = oracle.render_workload(wl, level, pixels=pix, jitter=s)
        compare(cpu(rgba).reshape(-1, 4)[pix], ref, cpu(nom).reshape(-1)[pix], cpu(comp).reshape(-1)[pix],
                label="c2 f16 jittered pass 3 of 8")
        # the plain jittered kernel (two samples per lane) gives the counting kernel's image
        plain = rp.render_jittered(ctx, vid, cam, wl.width, wl.height, 0, wl.step, 3, 8, 0x2207)[0]
        assert np.array_equal(cpu(plain), cpu(rgba))
        coord = ([1, 0, 0, 1], [-0.3, 0, 0, 0.7], [0.4, 0, 0, 2.0])
        rp.set_coordinate_brush(ctx, vid, *coord)
        rgba, nom, comp = gpu_render(rp, ctx, vid, wl, 0)
        ref = oracle.render_workload(wl, level, pixels=pix, coord=coord)
        compare(rgba.reshape(-1, 4)[pix], ref, nom.reshape(-1)[pix], comp.reshape(-1)[pix], label="c2 f16 coordinate cut")
        assert np.array_equal(cpu(rp.render(ctx, vid, cam, wl.width, wl.height, 0, wl.step)), rgba)
    finally:
        rp.unload(ctx, vid)


# Bounds on the storage-precision error of whole images (every pixel, fragile ones included) against
# the FP64 oracle on the original float32 fields.  float32 storage differs from the reference only by
# FP32 arithmetic and the threshold decisions it flips; binary16 and 8-bit codes move sample values by
# up to half a unit in the last place / half a quantisation step, which flips brush decisions near the
# bounds and shifts colours.  The bounds are about 3x the values measured on this seeded workload
# (f32 0.015 / 2.2e-6 / 0.005 %, f16 0.043 / 9.1e-5 / 0.32 %, u8 0.039 / 1.4e-4 / 0.44 %): a report
# with a guard against regressions, not a parity tolerance.
PRECISION_BOUNDS = {"f32": (0.05, 1e-5, 2e-4), "f16": (0.15, 3e-4, 0.01), "u8": (0.15, 5e-4, 0.015)}
#                    storage: (max-abs, mean-abs, fraction of pixels with error > 1e-2)


def test_storage_precision_report(rp, ctx, c2):
    """Precision study (512^3 x 5 fields, 1920x1080): per storage, max-abs / mean-abs RGBA error and the fraction of pixels
    with error > 1e-2 against the FP64 oracle on the ORIGINAL float32 fields (every 4th row and
    column of the 1920x1080 frame)."""
    wl = c2
    fields_dev = torch.from_numpy(wl.fields).cuda()
    ys, xs = np.meshgrid(np.arange(0, wl.height, 4), np.arange(0, wl.width, 4), indexing="ij")
    pix = (ys * wl.width + xs).reshape(-1)
    print(f"[case] precision report, {pix.size} pixels, oracle on the original float32 fields", flush=True)
    ref = oracle.render_workload(wl, wl.fields, pixels=pix)
    for storage in STORAGES:
        vid = rp.load_fields(ctx, fields_dev, storage, 3, wl.r_inner, wl.r_outer)
        rp.set_brush(ctx, vid, wl.brush.active, wl.brush.lo, wl.brush.hi)
        rp.set_transfer_function(ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, wl.tf.ref_step)
        rp.set_options(ctx, wl.ert)
        rgba = gpu_render(rp, ctx, vid, wl, 0)[0].reshape(-1, 4)[pix].astype(np.float64)
        rp.unload(ctx, vid)
        err = np.abs(rgba - ref.rgba).max(axis=-1)
        stats = {"storage": storage, "pixels": int(pix.size), "max_abs": float(err.max()),
                 "mean_abs": float(err.mean()), "p99_abs": float(np.percentile(err, 99)),
                 "frac_gt_1e-2": float((err > 1e-2).mean()), "frac_gt_1e-3": float((err > 1e-3).mean())}
        print(f"[precision] {stats}", flush=True)
        assert np.isfinite(rgba).all()
        mx, mean, frac = PRECISION_BOUNDS[storage]
        assert stats["max_abs"] <= mx and stats["mean_abs"] <= mean and stats["frac_gt_1e-2"] <= frac, stats
        if storage == "f32":
            continue
        # attribution (oracle only): the error of the image whose fields are the original float32 ones
        # except field f, stored as `storage`
        per_field = {}
        for f in range(wl.n_fields):
            lv = wl.fields.copy()
            lv[f] = pp.stored_values(wl.fields[f], storage)
            e_f = np.abs(oracle.render_workload(wl, lv, pixels=pix).rgba - ref.rgba).max(axis=-1)
            per_field[wl.field_names[f]] = {"max_abs": float(e_f.max()), "mean_abs": float(e_f.mean()),
                                            "frac_gt_1e-2": float((e_f > 1e-2).mean())}
        print(f"[precision] {storage} per field: {per_field}", flush=True)
        assert sum(v["mean_abs"] for v in per_field.values()) <= 2 * stats["mean_abs"] + 1e-6


@pytest.mark.timeout(600)
def test_max_size_1024_sampled(rp, ctx):
    """The largest grid (1024^3): 64-bit record addressing, a 4 GiB float32 field and a 2 GiB
    binary16 field in the compact layout (buffer ranges at their limits), all levels; sampled pixels
    of a 1920x1080 frame against the oracle on the stored values."""
    wl = W.analytic_workload(1024)
    print(f"[case] {wl.name}", flush=True)
    fields_dev = torch.from_numpy(wl.fields).cuda()
    pix = sample_pixels(wl.width, wl.height, 1500, seed=4)
    for storage in ("f16", "u8", "f32c", "f16c"):
        print(f"[case] 1024^3 {storage}", flush=True)
        vid = rp.load_fields(ctx, fields_dev, storage, 3, wl.r_inner, wl.r_outer)
        rp.set_brush(ctx, vid, wl.brush.active, wl.brush.lo, wl.brush.hi)
        rp.set_transfer_function(ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, wl.tf.ref_step)
        rp.set_options(ctx, wl.ert)
        rgba, nom, comp = gpu_render(rp, ctx, vid, wl, 0)
        base = storage.rstrip("c")
        want_level = np.stack([pp.stored_values(wl.fields[f], base) for f in range(wl.n_fields)])
        ref = oracle.render_workload(wl, want_level, pixels=pix)
        del want_level
        compare(rgba.reshape(-1, 4)[pix], ref, nom.reshape(-1)[pix], comp.reshape(-1)[pix], label=f"1024 {storage}")
        lod2 = gpu_render(rp, ctx, vid, wl, 2, width=480, height=270)[0]
        assert np.isfinite(lod2).all() and lod2[..., 3].max() > 0
        if storage in ("f16", "u8"):
            # served requests at this size: level 0's record fields reach 4 GiB, so the batched kernel
            # reads them at 64-bit offsets (level 1 at 32-bit ones); either way the image is the
            # single render's bit for bit
            print(f"[case] 1024^3 {storage} served", flush=True)
            cam = wl.camera.as_array()
            rp.server_start(ctx, 0, 4, 0, 0)
            try:
                for lod, (w, h) in ((0, (320, 180)), (1, (256, 144))):
                    single = cpu(rp.render(ctx, vid, cam, w, h, lod, wl.step))
                    out = torch.empty((h, w, 4), dtype=torch.float32, device="cuda")
                    t = rp.submit(ctx, rp.make_request(vid, cam, w, h, out, lod, wl.step, wl.brush.active,
                                                       wl.brush.lo, wl.brush.hi))
                    rp.wait(ctx, t, 60000)
                    assert np.array_equal(cpu(out), single), (storage, lod)
                    assert single[..., 3].max() > 0
                    rp.release(ctx, t)
            finally:
                rp.server_stop(ctx)
        rp.unload(ctx, vid)
