"""GPU test of frames in flight: renders of one volume with different brushes, enqueued on two
streams without waiting (one stream held back behind queued work), each give the image the same
brush gives alone; every brush change computes its skip flags into a new version, so a frame never
reads the flags of a later brush."""
import numpy as np
import pytest
import torch

from paper_2207_12011_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rp():
    from paper_2207_12011_amd import raypc
    return raypc


def test_frames_in_flight_keep_their_skip_flags(rp):
    ctx = rp.create(0)
    try:
        wl = W.make_workload(1, n=64, width=200, height=136)
        tf = wl.tf
        vid = rp.load_fields(ctx, torch.from_numpy(wl.fields).cuda(), "f16", 1, wl.r_inner, wl.r_outer)
        rp.set_transfer_function(ctx, 0, tf.field, tf.vmin, tf.vmax, tf.rgba, tf.ref_step)
        rp.set_options(ctx, wl.ert)
        cam = wl.camera.as_array()
        rng = np.random.default_rng(5)
        brushes = [(wl.brush.active, wl.brush.lo, wl.brush.hi)]
        for _ in range(4):
            lo = (wl.brush.lo - np.abs(wl.brush.lo) * rng.uniform(0.0, 0.3, wl.n_fields)).astype(np.float32)
            act = (rng.random(wl.n_fields) < 0.7).astype(np.uint8)
            brushes.append((act, lo, wl.brush.hi))
        want = []
        for act, lo, hi in brushes:
            rp.set_brush(ctx, vid, act, lo, hi)
            want.append(rp.render(ctx, vid, cam, wl.width, wl.height, 0, wl.step))
            torch.cuda.synchronize()
        assert len({w.cpu().numpy().tobytes() for w in want}) == len(brushes)
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        x = torch.randn(2048, 2048, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        with torch.cuda.stream(streams[0]):
            for _ in range(20):
                torch.mm(x, x, out=y)          # holds stream 0 back
        got = []
        for i in range(23):
            k = i % len(brushes)
            rp.set_brush(ctx, vid, *brushes[k])
            got.append((k, rp.render(ctx, vid, cam, wl.width, wl.height, 0, wl.step, stream=streams[i % 2])))
        torch.cuda.synchronize()
        for i, (k, img) in enumerate(got):
            assert torch.equal(img, want[k]), (i, k)
        rp.unload(ctx, vid)
    finally:
        rp.destroy(ctx)
