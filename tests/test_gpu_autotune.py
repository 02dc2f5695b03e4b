"""GPU tests of the launch-shape autotuner: every wave tile shape and super-tile size gives the image
of the default shape bit for bit (with its counts), the tuner times all shapes and keeps the
fastest, the server sweep picks one of its candidates, and invalid arguments are rejected."""
import numpy as np
import pytest
import torch

from paper_2207_12011_amd import autotune as AT
from paper_2207_12011_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def load(rp, ctx, wl, storage="f16"):
    vid = rp.load_fields(ctx, torch.from_numpy(wl.fields).cuda(), storage, 3, wl.r_inner, wl.r_outer)
    rp.set_brush(ctx, vid, wl.brush.active, wl.brush.lo, wl.brush.hi)
    rp.set_transfer_function(ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, wl.tf.ref_step)
    rp.set_options(ctx, wl.ert)
    return vid


SHAPES = [(0, 2), (1, 2), (3, 2), (2, 0), (2, 1), (2, 3), (2, 4), (0, 4), (3, 0), (1, 3)]


@pytest.mark.parametrize("storage", ["f32", "f16", "u8"])
def test_every_launch_shape_gives_the_same_image(rp, ctx, storage):
    wl = W.make_workload(1, n=64, width=200, height=136)
    vid = load(rp, ctx, wl, storage)
    cam = wl.camera.as_array()
    try:
        for w, h, lod in ((200, 136, 0), (1, 1, 0), (517, 3, 1), (64, 300, 2), (1920, 1080, 0)):
            rp.set_launch_shape(ctx, 2, 2)
            want = [cpu(x) for x in rp.render_debug(ctx, vid, cam, w, h, lod, 0.5)]
            want_jit = cpu(rp.render_jittered(ctx, vid, cam, w, h, lod, 0.5, 1, 4, 7)[0])
            want_depth = cpu(rp.render_depth(ctx, vid, cam, w, h, lod, 0.5)[1])
            for s, t in SHAPES:
                print(f"[case] launch shape s={s} t={t} {storage} {w}x{h} lod {lod}", flush=True)
                rp.set_launch_shape(ctx, s, t)
                assert rp.get_launch_shape(ctx) == (s, t)
                got = [cpu(x) for x in rp.render_debug(ctx, vid, cam, w, h, lod, 0.5)]
                assert all(np.array_equal(a, b) for a, b in zip(got, want)), (s, t, w, h)
                # the plain render (one-wave blocks, 32-bit record offsets) and the counting variant
                # (four-wave blocks, 64-bit offsets for the record kinds) march the same samples
                assert np.array_equal(cpu(rp.render(ctx, vid, cam, w, h, lod, 0.5)), want[0]), (s, t, w, h)
                jit = cpu(rp.render_jittered(ctx, vid, cam, w, h, lod, 0.5, 1, 4, 7)[0])
                assert np.array_equal(jit, want_jit), (s, t, w, h)
                rgba_d, dep = rp.render_depth(ctx, vid, cam, w, h, lod, 0.5)
                assert np.array_equal(cpu(rgba_d), want[0]) and np.array_equal(cpu(dep), want_depth), (s, t, w, h)
    finally:
        rp.set_launch_shape(ctx, 2, 2)
        rp.unload(ctx, vid)


def test_autotune_render_keeps_the_fastest(rp, ctx):
    wl = W.make_workload(1, n=64, width=640, height=360)
    vid = load(rp, ctx, wl)
    cam = wl.camera.as_array()
    try:
        (bs, bt), times = rp.autotune_render(ctx, vid, cam, wl.width, wl.height, 0, 0.5, repeats=5)
        print(f"[autotune] ms per render [tile_log2w][super_log2]: {times}, best s={bs} t={bt}", flush=True)
        flat = [ms for row in times for ms in row]
        assert 0 <= bs <= 3 and 0 <= bt <= 4 and len(flat) == 20 and all(x > 0 for x in flat)
        if (bs, bt) != (2, 2):
            assert times[bt][bs] == min(flat) and times[bt][bs] < 0.99 * times[2][2]
        else:
            assert min(flat) >= 0.99 * times[2][2]
        assert rp.get_launch_shape(ctx) == (bs, bt)
        cache = {}
        key = AT.render_key(AT.device_name(), 64, "f16", wl.width, wl.height, 0, 0.5)
        r = AT.tune_render(rp, ctx, vid, cam, wl.width, wl.height, 0, 0.5, repeats=3, cache=cache, key=key)
        assert not r["cached"] and key in cache
        rp.set_launch_shape(ctx, 0, 0)
        r = AT.tune_render(rp, ctx, vid, cam, wl.width, wl.height, 0, 0.5, cache=cache, key=key)
        assert r["cached"] and rp.get_launch_shape(ctx) == (cache[key]["super_log2"], cache[key]["tile_log2w"])
        for bad in (0, 1001):
            with pytest.raises(rp.RaypcError):
                rp.autotune_render(ctx, vid, cam, wl.width, wl.height, 0, 0.5, repeats=bad)
        with pytest.raises(rp.RaypcError):
            rp.autotune_render(ctx, vid, cam, 0, wl.height, 0, 0.5)
        for bad in ((-1, 2), (4, 2), (2, -1), (2, 5)):
            with pytest.raises(rp.RaypcError):
                rp.set_launch_shape(ctx, *bad)
        assert rp.get_launch_shape(ctx) == (cache[key]["super_log2"], cache[key]["tile_log2w"])
    finally:
        rp.set_launch_shape(ctx, 2, 2)
        rp.unload(ctx, vid)


def test_tune_server_picks_a_candidate(rp, ctx):
    wl = W.make_workload(1, n=64, width=200, height=136)
    vid = load(rp, ctx, wl)
    cam = wl.camera.as_array()
    outs = [torch.empty((h, w, 4), dtype=torch.float32, device="cuda") for w, h in ((200, 136), (64, 64), (333, 97))
            for _ in range(4)]
    reqs = [rp.make_request(vid, cam, o.shape[1], o.shape[0], o, 0, 0.5, wl.brush.active, wl.brush.lo, wl.brush.hi)
            for o in outs]
    try:
        r = AT.tune_server(rp, ctx, reqs, candidates=((2048, 1), (8192, 2)), rounds=1)
        print(f"[autotune] server: {r}", flush=True)
        assert (r["tiles_per_step"], r["steps_in_flight"]) in ((2048, 1), (8192, 2))
        single = cpu(rp.render(ctx, vid, cam, 333, 97, 0, 0.5))
        assert np.array_equal(cpu(outs[-1]), single)
    finally:
        rp.unload(ctx, vid)
