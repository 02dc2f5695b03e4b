"""GPU test of raypc_warp_noalloc, the warp for callers that cannot allocate device memory.

It must give raypc_warp's outputs bit for bit (RGBA, depth and source index of every destination
pixel), on two calls in a row whose second is smaller (the fixed z-buffer keeps the first call's
keys, which the second must not see), allocate no device memory, and reject a destination larger
than its fixed z-buffer before launching anything.  Inputs are seeded synthetic frames.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

F32 = np.float32


@pytest.fixture(scope="module")
def rp():
    from paper_2207_12011_amd import raypc
    return raypc


def cam(eye, target=(0, 0, 0), up=(0, 1, 0), fov=60.0):
    return np.array([*eye, *target, *up, fov], np.float32)


def frame(rng, w, h):
    """A smooth depth map with holes (points at infinity) and near specks, and random RGBA."""
    yy, xx = np.mgrid[0:h, 0:w] / max(w, h)
    d = np.zeros((h, w))
    for _ in range(4):
        a, b, ph = rng.uniform(1, 6), rng.uniform(1, 6), rng.uniform(0, 6.28)
        d += np.sin(a * xx * 6.28 + b * yy * 6.28 + ph)
    d = 2.0 + 1.5 * (d - d.min()) / max(d.max() - d.min(), 1e-9)
    d[rng.random((h, w)) < 0.03] = 1.2
    d[rng.random((h, w)) < 0.25] = np.inf
    rgba = rng.random((h, w, 4)).astype(F32)
    return torch.from_numpy(rgba).cuda(), torch.from_numpy(d.astype(F32)).cuda()


def outputs(w, h):
    return (torch.full((h, w, 4), -7.0, dtype=torch.float32, device="cuda"),
            torch.full((h, w), -7.0, dtype=torch.float32, device="cuda"),
            torch.full((h, w), -7, dtype=torch.int32, device="cuda"))


def test_noalloc_warp_equals_warp_on_two_calls(rp):
    ctx = rp.create(0)
    try:
        rng = np.random.default_rng(2212)
        src_c = cam((0.0, 0.0, 3.0))
        cases = [((1920, 1080), (1920, 1080), cam((0.05, 0.02, 2.98), (0.01, 0, 0))),
                 ((640, 360), (500, 300), cam((0.4, 0.2, 2.7), (0.05, 0, 0), fov=55.0))]
        for k, ((sw, sh), (dw, dh), dst_c) in enumerate(cases):
            print(f"[case] warp_noalloc call {k}: {sw}x{sh} -> {dw}x{dh}", flush=True)
            rgba, depth = frame(rng, sw, sh)
            o_n, d_n, s_n = outputs(dw, dh)
            torch.cuda.synchronize()
            free_before = torch.cuda.mem_get_info()[0]
            rp.warp(ctx, rgba, depth, src_c, dst_c, dw, dh, out=o_n, out_depth=d_n, out_source=s_n, noalloc=True)
            torch.cuda.synchronize()
            free_after = torch.cuda.mem_get_info()[0]
            # a z-buffer allocation would take dw * dh * 8 bytes (16.6 MB at 1080p)
            assert free_before - free_after < dw * dh * 8 // 2, (free_before, free_after)
            o_w, d_w, s_w = rp.warp(ctx, rgba, depth, src_c, dst_c, dw, dh)
            torch.cuda.synchronize()
            src_n = s_n.cpu().numpy()
            assert np.array_equal(src_n, s_w.cpu().numpy()), f"call {k}: source indices differ"
            assert np.array_equal(o_n.cpu().numpy().view(np.uint32), o_w.cpu().numpy().view(np.uint32)), k
            assert np.array_equal(d_n.cpu().numpy().view(np.uint32), d_w.cpu().numpy().view(np.uint32)), k
            covered = (src_n >= 0).mean()
            print(f"[warp_noalloc] call {k}: {covered:.3f} of the pixels covered", flush=True)
            assert 0.3 < covered < 1.0
    finally:
        rp.destroy(ctx)


def test_noalloc_warp_rejects_oversized_destination(rp):
    ctx = rp.create(0)
    try:
        c = cam((0.2, 0.1, 3.0))
        rgba = torch.zeros((8, 8, 4), dtype=torch.float32, device="cuda")
        depth = torch.zeros((8, 8), dtype=torch.float32, device="cuda")
        out = torch.zeros((4, 4, 4), dtype=torch.float32, device="cuda")
        P = rp.ctypes.byref
        C = rp.Camera.make
        # 2049 x 2048 pixels: one row over the fixed z-buffer; refused before any launch, so the
        # small output buffer is never written
        with pytest.raises(rp.RaypcError, match="fixed z-buffer"):
            rp._check(rp._warp_noalloc(ctx, P(C(c)), 8, 8, rgba.data_ptr(), depth.data_ptr(), P(C(c)), 2048, 2049,
                                       out.data_ptr(), None, None, None))
        torch.cuda.synchronize()
        assert float(out.abs().sum()) == 0.0
        assert rp.WARP_NOALLOC_MAX_PIXELS == 2048 * 2048
    finally:
        rp.destroy(ctx)
