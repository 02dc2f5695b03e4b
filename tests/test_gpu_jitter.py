"""GPU parity of jittered progressive passes: each pass against the oracle given the same per-pixel
sample-grid offsets (the oracle's own SplitMix64 implementation), the running mean, and the
convergence of the mean towards the fine-step render."""
import numpy as np
import pytest
import torch

import oracle
from oracle import jitter as J
from oracle import preprocess as pp
from paper_2207_12011_amd import workloads as W

from .parity import compare

pytestmark = pytest.mark.gpu

SEED = 0x5EED2207


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
def small5():
    return W.make_workload(1, n=64, width=200, height=136)


def cpu(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def load(rp, ctx, wl, storage):
    vid = rp.load_fields(ctx, torch.from_numpy(wl.fields).cuda(), storage, 3, wl.r_inner, wl.r_outer)
    rp.set_brush(ctx, vid, wl.brush.active, wl.brush.lo, wl.brush.hi)
    rp.set_transfer_function(ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, wl.tf.ref_step)
    rp.set_options(ctx, wl.ert)
    return vid


@pytest.mark.parametrize("storage", ["f32", "f16", "u8"])
def test_jittered_passes_match_oracle(rp, ctx, small5, storage):
    wl = small5
    vid = load(rp, ctx, wl, storage)
    level = pp.stored_levels(wl.fields, 1, storage)[0]
    npx = wl.width * wl.height
    mean = torch.empty((wl.height, wl.width, 4), dtype=torch.float32, device="cuda")
    K = 4
    ref_sum = np.zeros((npx, 4))
    gpu_passes = []
    for k in range(K):
        print(f"[case] jittered {storage} pass {k}/{K}", flush=True)
        rgba, nom, comp = rp.render_jittered(ctx, vid, wl.camera.as_array(), wl.width, wl.height, 0, wl.step, k, K,
                                             SEED, mean=mean, counts=True)
        s = J.offsets(wl.width, np.arange(npx), k, K, SEED)
        ref = oracle.render_workload(wl, level, pixels=np.arange(npx), jitter=s)
        st = compare(cpu(rgba).reshape(-1, 4), ref, cpu(nom).reshape(-1), cpu(comp).reshape(-1),
                     label=f"{storage} pass {k}")
        # the plain jittered kernel (two samples per lane for binary16 records) marches the same samples
        # as the counting one (one per lane)
        plain = rp.render_jittered(ctx, vid, wl.camera.as_array(), wl.width, wl.height, 0, wl.step, k, K, SEED)[0]
        assert np.array_equal(cpu(plain), cpu(rgba)), (storage, k)
        gpu_passes.append(cpu(rgba).reshape(-1, 4).astype(np.float64))
        ref_sum += st["matched"]
    m = cpu(mean).reshape(-1, 4).astype(np.float64)
    assert np.abs(m - np.mean(gpu_passes, axis=0)).max() <= 1e-6
    # the running mean against the mean of the legitimate results the passes matched
    ok = np.isfinite(ref_sum).all(axis=-1)
    assert ok.mean() >= 0.99
    assert np.abs(m - ref_sum / K)[ok].max() <= 2e-4
    rp.unload(ctx, vid)


def test_jittered_mean_converges(rp, ctx, small5):
    """The running mean of K passes approaches the render at a 16x finer step as K grows."""
    wl = small5
    vid = load(rp, ctx, wl, "f16")
    fine = cpu(rp.render(ctx, vid, wl.camera.as_array(), wl.width, wl.height, 0, wl.step / 16)).astype(np.float64)
    errs = []
    for K in (1, 4, 16):
        mean = torch.empty((wl.height, wl.width, 4), dtype=torch.float32, device="cuda")
        for k in range(K):
            rp.render_jittered(ctx, vid, wl.camera.as_array(), wl.width, wl.height, 0, wl.step, k, K, SEED, mean=mean)
        errs.append(float(np.abs(cpu(mean) - fine).mean()))
    print(f"[jitter] mean-abs error of the pass mean against step/16, K = 1, 4, 16: {errs}", flush=True)
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.35 * errs[0], errs
    rp.unload(ctx, vid)


def test_jittered_arguments(rp, ctx, small5):
    wl = small5
    vid = load(rp, ctx, wl, "f16")
    cam = wl.camera.as_array()
    for k, K in ((4, 4), (-1, 4), (0, 0), (0, 257)):
        with pytest.raises(rp.RaypcError):
            rp.render_jittered(ctx, vid, cam, 32, 32, 0, 0.5, k, K, SEED)
    a = cpu(rp.render_jittered(ctx, vid, cam, 32, 32, 0, 0.5, 255, 256, SEED)[0])
    b = cpu(rp.render_jittered(ctx, vid, cam, 32, 32, 0, 0.5, 255, 256, SEED)[0])
    assert np.isfinite(a).all() and np.array_equal(a, b)
    rp.unload(ctx, vid)
