"""GPU tests of the continuous-batching server: every served image equals the
single-request render of the same view, brush and table (bit for bit), alone
and in a mix of requests of different sizes, brushes, levels, steps, tables and
storage types; admission is FIFO under a memory budget; oversized requests,
deadlines, cancellation and busy volumes are reported as documented."""
import math

import time

import numpy as np
import pytest
import torch

from paper_2207_12011_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rp():
    from paper_2207_12011_amd import raypc
    return raypc


@pytest.fixture(scope="module")
def setup(rp):
    ctx = rp.create(0)
    five = W.make_workload(1, n=64)
    tiny = W.make_workload(0, n=64)
    v5 = rp.load_fields(ctx, torch.from_numpy(five.fields).cuda(), "f16", 3)
    v2 = rp.load_fields(ctx, torch.from_numpy(tiny.fields).cuda(), "f32", 2)
    v5u = rp.load_fields(ctx, torch.from_numpy(five.fields).cuda(), "u8", 2)
    rp.set_transfer_function(ctx, 0, five.tf.field, five.tf.vmin, five.tf.vmax, five.tf.rgba)
    tab = tiny.tf.rgba.copy()
    tab[:30, 3] = 0.0
    rp.set_transfer_function(ctx, 1, 0, tiny.tf.vmin, tiny.tf.vmax, tab)
    rp.set_options(ctx, 0.99)
    yield ctx, {v5: five, v2: tiny, v5u: five}, {0: (five.tf, five.tf.rgba), 1: (tiny.tf, tab)}
    rp.destroy(ctx)


def random_requests(rng, vols, k):
    sizes = [(32, 32), (64, 48), (96, 96), (200, 136), (128, 64), (17, 9)]
    reqs = []
    for i in range(k):
        vid = list(vols)[i % len(vols)]
        wl = vols[vid]
        nf = wl.n_fields
        cam = W.orbit_camera(rng.uniform(0, 2 * math.pi), rng.uniform(-1.0, 1.0), rng.uniform(2.2, 4.0),
                             rng.uniform(35, 70))
        w, h = sizes[rng.integers(len(sizes))]
        act = np.zeros(nf, np.uint8)
        act[rng.choice(nf, size=rng.integers(1, nf + 1), replace=False)] = 1
        q = W.shell_quantiles(wl.fields, W.shell_mask(W.radius(wl.n)), [0.1, 0.35, 0.6, 0.95])
        lo = np.array([q[f, rng.integers(0, 2)] for f in range(nf)], np.float32)
        hi = np.array([q[f, rng.integers(2, 4)] for f in range(nf)], np.float32)
        slot = 1 if (nf == 2 and rng.random() < 0.5) else 0
        lod = int(rng.integers(-1, 2))
        step = float(rng.choice([0.5, 1.0, 0.37]))
        reqs.append(dict(vid=vid, cam=cam, w=w, h=h, act=act, lo=lo, hi=hi, slot=slot, lod=lod, step=step))
    return reqs


def single_render(rp, ctx, tfs, q):
    """The same view through raypc_render (volume brush + slot 0 set to the request's table)."""
    tf, tab = tfs[q["slot"]]
    rp.set_transfer_function(ctx, 0, tf.field if q["slot"] == 0 else 0, tf.vmin, tf.vmax, tab)
    rp.set_brush(ctx, q["vid"], q["act"], q["lo"], q["hi"])
    img = rp.render(ctx, q["vid"], q["cam"], q["w"], q["h"], q["lod"], q["step"])
    torch.cuda.synchronize()
    out = img.cpu().numpy()
    t0, tab0 = tfs[0]
    rp.set_transfer_function(ctx, 0, t0.field, t0.vmin, t0.vmax, tab0)
    return out


def submit_all(rp, ctx, reqs, deadline_ms=0.0):
    outs, tickets = [], []
    for q in reqs:
        out = torch.full((q["h"], q["w"], 4), float("nan"), device="cuda")
        r = rp.make_request(q["vid"], q["cam"], q["w"], q["h"], out, q["lod"], q["step"], q["act"], q["lo"], q["hi"],
                            q["slot"], deadline_ms)
        tickets.append(rp.submit(ctx, r))
        outs.append(out)
    return tickets, outs


@pytest.mark.parametrize("tiles_per_step,max_inflight", [(64, 6), (8192, 64), (7, 2)])
def test_served_images_equal_single_renders(rp, setup, tiles_per_step, max_inflight):
    ctx, vols, tfs = setup
    rng = np.random.default_rng(tiles_per_step)
    reqs = random_requests(rng, vols, 18)
    print(f"[case] serving mix tiles_per_step={tiles_per_step} max_inflight={max_inflight}", flush=True)
    rp.server_start(ctx, 0, max_inflight, tiles_per_step, 2)
    try:
        tickets, outs = submit_all(rp, ctx, reqs)
        for t in tickets:
            rp.wait(ctx, t, 60000)
            assert rp.poll(ctx, t) == rp.REQ_DONE
        stats = rp.server_get_stats(ctx)
        assert stats["completed"] == len(reqs) and stats["bytes_in_use"] == 0
        times = [rp.request_times(ctx, t) for t in tickets]
    finally:
        rp.server_stop(ctx)
    for q, o, tm in zip(reqs, outs, times):
        got = o.cpu().numpy()
        want = single_render(rp, ctx, tfs, q)
        assert np.array_equal(got, want), (q["w"], q["h"], q["lod"], q["step"])
        assert tm[0] <= tm[1] <= tm[2] <= tm[3]
    # admission follows submission order
    admits = [tm[1] for tm in times]
    assert admits == sorted(admits)
    if max_inflight > 2:
        # the work of several requests overlapped on the device
        overlap = sum(1 for i in range(1, len(times)) if times[i][1] < times[i - 1][3])
        assert overlap > 0


def test_budget_queues_requests_fifo(rp, setup):
    ctx, vols, tfs = setup
    rng = np.random.default_rng(5)
    reqs = random_requests(rng, vols, 8)
    for q in reqs:
        q["w"], q["h"] = 96, 96
    per_req = 96 * 96 * 16 + 8 * 8 * 8 * 2    # image + the two-byte skip flag word per brick
    rp.server_start(ctx, per_req + 100, 8, 16, 2)       # room for exactly one request at a time
    try:
        tickets, outs = submit_all(rp, ctx, reqs)
        for t in tickets:
            rp.wait(ctx, t, 60000)
        times = [rp.request_times(ctx, t) for t in tickets]
        stats = rp.server_get_stats(ctx)
    finally:
        rp.server_stop(ctx)
    assert stats["peak_bytes_in_use"] <= per_req + 100
    for i in range(1, len(times)):
        assert times[i][1] >= times[i - 1][3] - 1e-6       # admitted only once the previous one finished
    for q, o in zip(reqs, outs):
        assert np.array_equal(o.cpu().numpy(), single_render(rp, ctx, tfs, q))


def test_oversized_request_is_rejected(rp, setup):
    ctx, vols, _ = setup
    vid = list(vols)[0]
    rp.server_start(ctx, 1000, 4, 0, 0)
    try:
        out = torch.empty((64, 64, 4), device="cuda")
        r = rp.make_request(vid, W.default_camera(), 64, 64, out, active=[0] * 5, lo=[0] * 5, hi=[0] * 5)
        with pytest.raises(rp.RaypcError) as ei:
            rp.submit(ctx, r)
        assert ei.value.code == rp.ERR_NOMEM
        bad = rp.make_request(vid, W.default_camera(), 0 + 8, 8, out, step=100.0)
        with pytest.raises(rp.RaypcError) as ei:
            rp.submit(ctx, bad)
        assert ei.value.code == rp.ERR_INVALID
    finally:
        rp.server_stop(ctx)


def test_deadline_cancel_and_busy_volume(rp, setup):
    ctx, vols, _ = setup
    vid = list(vols)[0]
    cam = W.default_camera()
    rp.server_start(ctx, 0, 1, 1, 1)   # one slot, one tile per step: a big request occupies it for a while
    try:
        big = torch.empty((512, 512, 4), device="cuda")
        t_big = rp.submit(ctx, rp.make_request(vid, cam, 512, 512, big, active=[0] * 5, lo=[0] * 5, hi=[0] * 5))
        # the scheduler thread admits it asynchronously: wait until it holds the slot
        t0 = time.monotonic()
        while rp.poll(ctx, t_big) == rp.REQ_QUEUED and time.monotonic() - t0 < 10.0:
            time.sleep(0.0005)
        assert rp.poll(ctx, t_big) == rp.REQ_RUNNING
        small = [torch.empty((16, 16, 4), device="cuda") for _ in range(3)]
        t_dead = rp.submit(ctx, rp.make_request(vid, cam, 16, 16, small[0], deadline_ms=0.01))
        t_cancel = rp.submit(ctx, rp.make_request(vid, cam, 16, 16, small[1]))
        t_ok = rp.submit(ctx, rp.make_request(vid, cam, 16, 16, small[2]))
        rp.cancel(ctx, t_cancel)
        with pytest.raises(rp.RaypcError) as ei:
            rp.unload(ctx, vid)
        assert ei.value.code == rp.ERR_BUSY
        with pytest.raises(rp.RaypcError) as ei:
            rp.cancel(ctx, t_big)          # already admitted
        assert ei.value.code == rp.ERR_BUSY
        rp.wait(ctx, t_big, 120000)
        with pytest.raises(rp.RaypcError) as ei:
            rp.wait(ctx, t_dead, 10000)
        assert ei.value.code == rp.ERR_TIMEOUT
        assert rp.poll(ctx, t_dead) == -rp.ERR_TIMEOUT
        assert rp.poll(ctx, t_cancel) == -rp.ERR_CANCELLED
        rp.wait(ctx, t_ok, 10000)
        stats = rp.server_get_stats(ctx)
        assert stats["timed_out"] == 1 and stats["cancelled"] == 1 and stats["completed"] == 2
        for t in (t_big, t_dead, t_cancel, t_ok):
            rp.release(ctx, t)
        with pytest.raises(rp.RaypcError):
            rp.poll(ctx, t_ok)
    finally:
        rp.server_stop(ctx)


def test_many_tiny_requests(rp, setup):
    ctx, vols, tfs = setup
    rng = np.random.default_rng(11)
    reqs = random_requests(rng, vols, 300)
    for q in reqs:
        q["w"], q["h"] = 8, 8
    rp.server_start(ctx, 0, 32, 100, 3)
    try:
        tickets, outs = submit_all(rp, ctx, reqs)
        for t in tickets:
            rp.wait(ctx, t, 60000)
        stats = rp.server_get_stats(ctx)
    finally:
        rp.server_stop(ctx)
    assert stats["completed"] == 300 and stats["failed"] == 0
    for i in range(0, 300, 37):
        assert np.array_equal(outs[i].cpu().numpy(), single_render(rp, ctx, tfs, reqs[i]))


def test_server_state_errors(rp, setup):
    ctx, vols, _ = setup
    with pytest.raises(rp.RaypcError) as ei:
        rp.server_stop(ctx)
    assert ei.value.code == rp.ERR_STATE
    rp.server_start(ctx, 0, 4)
    try:
        with pytest.raises(rp.RaypcError) as ei:
            rp.server_start(ctx, 0, 4)
        assert ei.value.code == rp.ERR_STATE
    finally:
        rp.server_stop(ctx)
    with pytest.raises(rp.RaypcError):
        rp.server_start(ctx, 0, 0)
