"""GPU tests of transfer-function changes: a render already enqueued keeps its table, a render
enqueued after the change uses the new one, and the stream-ordered form does not wait."""
import numpy as np
import pytest
import torch

from paper_2207_12011_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rp():
    from paper_2207_12011_amd import raypc
    return raypc


def setup(rp, ctx, wl):
    vid = rp.load_fields(ctx, torch.from_numpy(wl.fields).cuda(), "f16", 1, wl.r_inner, wl.r_outer)
    rp.set_brush(ctx, vid, wl.brush.active, wl.brush.lo, wl.brush.hi)
    rp.set_options(ctx, wl.ert)
    return vid


def coloured(tab, v):
    t = tab.copy()
    t[:, :3] = v
    return t


def test_change_is_ordered(rp):
    """A render enqueued before a definition (behind queued work on its stream) keeps the old table;
    one enqueued after it uses the new one."""
    ctx = rp.create(0)
    try:
        wl = W.make_workload(1, n=64, width=96, height=64)
        tf = wl.tf
        vid = setup(rp, ctx, wl)
        cam = wl.camera.as_array()
        tab_a, tab_b = coloured(tf.rgba, 0.25), coloured(tf.rgba, 0.75)
        rp.set_transfer_function(ctx, 0, tf.field, tf.vmin, tf.vmax, tab_a, tf.ref_step)
        want_a = rp.render(ctx, vid, cam, wl.width, wl.height, 0, wl.step)
        rp.set_transfer_function(ctx, 0, tf.field, tf.vmin, tf.vmax, tab_b, tf.ref_step)
        want_b = rp.render(ctx, vid, cam, wl.width, wl.height, 0, wl.step)
        torch.cuda.synchronize()
        rp.set_transfer_function(ctx, 0, tf.field, tf.vmin, tf.vmax, tab_a, tf.ref_step)
        s = torch.cuda.Stream()
        x = torch.randn(4096, 4096, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            for _ in range(40):          # about 5 TFLOP queued ahead of the renders
                torch.mm(x, x, out=y)
            got_a = rp.render(ctx, vid, cam, wl.width, wl.height, 0, wl.step, stream=s)
            rp.set_transfer_function(ctx, 0, tf.field, tf.vmin, tf.vmax, tab_b, tf.ref_step)
            got_b = rp.render(ctx, vid, cam, wl.width, wl.height, 0, wl.step, stream=s)
        s.synchronize()
        assert torch.equal(got_a, want_a) and torch.equal(got_b, want_b)
        assert not torch.equal(want_a, want_b)
        rp.unload(ctx, vid)
    finally:
        rp.destroy(ctx)


def test_change_on_a_stream_does_not_wait(rp):
    """The stream-ordered definition returns while the stream's queued work still runs; the render
    enqueued before it on that stream keeps the old table, the one after it uses the new one."""
    ctx = rp.create(0)
    try:
        wl = W.make_workload(1, n=64, width=96, height=64)
        tf = wl.tf
        vid = setup(rp, ctx, wl)
        cam = wl.camera.as_array()
        tab_a, tab_b = coloured(tf.rgba, 0.25), coloured(tf.rgba, 0.75)
        rp.set_transfer_function(ctx, 0, tf.field, tf.vmin, tf.vmax, tab_b, tf.ref_step)
        want_b = rp.render(ctx, vid, cam, wl.width, wl.height, 0, wl.step)
        rp.set_transfer_function(ctx, 0, tf.field, tf.vmin, tf.vmax, tab_a, tf.ref_step)
        want_a = rp.render(ctx, vid, cam, wl.width, wl.height, 0, wl.step)
        s = torch.cuda.Stream()
        x = torch.randn(4096, 4096, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            for _ in range(40):
                torch.mm(x, x, out=y)
            got_a = rp.render(ctx, vid, cam, wl.width, wl.height, 0, wl.step, stream=s)
            t = tab_b.copy()
            rp.set_transfer_function(ctx, 0, tf.field, tf.vmin, tf.vmax, t, tf.ref_step, stream=s,
                                     ordered_on_stream=True)
            busy = not s.query()         # the upload is queued behind the work: nothing waited for it
            t[:] = 0.0                   # the caller's array may change at once (it was staged)
            got_b = rp.render(ctx, vid, cam, wl.width, wl.height, 0, wl.step, stream=s)
        s.synchronize()
        assert busy, "the stream-ordered definition waited for the stream"
        assert torch.equal(got_a, want_a) and torch.equal(got_b, want_b)
        rp.unload(ctx, vid)
    finally:
        rp.destroy(ctx)


@pytest.mark.parametrize("ordered_on_stream", [False, True])
def test_many_changes_wrap_the_versions(rp, ordered_on_stream):
    """More definitions of a slot than it keeps versions (256): every render, enqueued between two
    definitions without waiting, used the table defined just before it (with the stream-ordered
    form, the staging copies are reused too)."""
    ctx = rp.create(0)
    try:
        wl = W.make_workload(1, n=64, width=32, height=32)
        tf = wl.tf
        vid = setup(rp, ctx, wl)
        cam = wl.camera.as_array()
        outs = []
        n = 600
        s = torch.cuda.current_stream()
        for i in range(n):
            rp.set_transfer_function(ctx, 0, tf.field, tf.vmin, tf.vmax, coloured(tf.rgba, (i + 1) / (n + 1)),
                                     tf.ref_step, stream=s, ordered_on_stream=ordered_on_stream)
            outs.append(rp.render(ctx, vid, cam, wl.width, wl.height, 0, wl.step, stream=s))
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            a = o.cpu().numpy()
            m = a[..., 3] > 0.05
            assert m.sum() > 20
            ratio = a[..., 0][m] / a[..., 3][m]   # a constant colour c gives premultiplied c * opacity
            assert np.abs(ratio - (i + 1) / (n + 1)).max() < 1e-5, i
        rp.unload(ctx, vid)
    finally:
        rp.destroy(ctx)
