"""GPU parity of the coordinate axes of the brush (sample x, y, z and radius): renders against the
oracle, skip on/off, voxel masks and parallel-coordinates lines bit-exact, served requests equal to
single renders."""
import numpy as np
import pytest
import torch

import oracle
from oracle import preprocess as pp
from paper_2207_12011_amd import workloads as W

from .parity import compare

pytestmark = pytest.mark.gpu

CUTS = [([1, 0, 0, 0], [0.0, 0, 0, 0], [1.0, 0, 0, 0]),                 # half space x >= 0
        ([0, 1, 1, 0], [0, -0.4, -1.0, 0], [0, 0.3, 0.2, 0]),           # slab in y, z
        ([0, 0, 0, 1], [0, 0, 0, 0.7], [0, 0, 0, 0.85]),               # radius band (an altitude range)
        ([1, 0, 0, 1], [-0.2, 0, 0, 0.6], [0.5, 0, 0, 2.0])]           # x slab with a radius floor


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
def test_coordinate_cuts_match_oracle(rp, ctx, small5, storage):
    wl = small5
    vid = load(rp, ctx, wl, storage)
    level = pp.stored_levels(wl.fields, 1, storage)[0]
    cam = wl.camera.as_array()
    nf = wl.n_fields
    for ci, coord in enumerate(CUTS):
        for brushed in (True, False):
            act = wl.brush.active if brushed else np.zeros(nf, np.uint8)
            rp.set_brush(ctx, vid, act, wl.brush.lo, wl.brush.hi)
            rp.set_coordinate_brush(ctx, vid, *coord)
            print(f"[case] coordinate cut {ci} brushed={brushed} {storage}", flush=True)
            rgba, nom, comp = rp.render_debug(ctx, vid, cam, wl.width, wl.height, 0, wl.step)
            ref = oracle.render_workload(wl, level, active=act, coord=coord)
            compare(cpu(rgba), ref, cpu(nom), cpu(comp), label=f"{storage} cut {ci} brushed {brushed}")
            a = rp.render_debug(ctx, vid, cam, wl.width, wl.height, 0, wl.step, skip=False)
            assert all(np.array_equal(cpu(x), cpu(y)) for x, y in zip((rgba, nom, comp), a))
            # the plain render (run-time field count; two samples per lane for binary16 records)
            assert np.array_equal(cpu(rp.render(ctx, vid, cam, wl.width, wl.height, 0, wl.step)), cpu(rgba))
    rp.set_coordinate_brush(ctx, vid, [0, 0, 0, 0], [0] * 4, [0] * 4)
    rp.unload(ctx, vid)


@pytest.mark.parametrize("storage", ["f32", "f16", "u8"])
def test_coordinate_cuts_on_cells_bitexact(rp, ctx, small5, storage):
    wl = small5
    nf = wl.n_fields
    vid = load(rp, ctx, wl, storage)
    levels = pp.stored_levels(wl.fields, 3, storage)
    axis_lo = wl.fields.reshape(nf, -1).min(axis=1)
    axis_hi = wl.fields.reshape(nf, -1).max(axis=1)
    for coord in CUTS + [([0, 0, 0, 1], [0, 0, 0, 0.0], [0, 0, 0, -0.5])]:
        rp.set_coordinate_brush(ctx, vid, *coord)
        for lod in range(3):
            n = 64 >> lod
            want = pp.voxel_mask(levels[lod], wl.brush.active, wl.brush.lo, wl.brush.hi, coord=coord)
            assert np.array_equal(cpu(rp.export_voxel_mask(ctx, vid, lod)), want), (coord, lod)
            mins, maxs = zip(*[pp.brick_minmax(levels[lod][f]) for f in range(nf)])
            brick_skip = pp.skip_bits(mins, maxs, wl.brush.active, wl.brush.lo, wl.brush.hi, wl.tf.field,
                                      wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, coord, n)
            bits = pp.pack_bits(brick_skip)
            assert np.array_equal(cpu(rp.export_skiplist(ctx, vid, lod, 0)).view(np.uint32), bits), (coord, lod)
            sub = pp.sub_skip(levels[lod], wl.brush.active, wl.brush.lo, wl.brush.hi, wl.tf.field, wl.tf.vmin,
                              wl.tf.vmax, wl.tf.rgba, coord=coord)
            assert np.array_equal(cpu(rp.export_subskip(ctx, vid, lod, 0)), sub), (coord, lod)
            assert np.array_equal(cpu(rp.export_skip_words(ctx, vid, lod, 0)).view(np.uint16),
                                  pp.skip_words(sub, n // 8, brick_skip)), (coord, lod)
            cells = W.pc_line_cells(n, 2000 >> lod, seed=lod)
            _, passes, hist = rp.pc_lines(ctx, vid, lod, torch.from_numpy(cells.astype(np.int32)).cuda(),
                                          axis_lo, axis_hi, 32)
            _, want_p, want_h = pp.pc_lines(levels[lod], cells, wl.brush.active, wl.brush.lo, wl.brush.hi,
                                            axis_lo, axis_hi, 32, coord=coord)
            assert np.array_equal(cpu(passes), want_p) and np.array_equal(cpu(hist).astype(np.uint32), want_h)
    with pytest.raises(rp.RaypcError):
        rp.set_coordinate_brush(ctx, vid, [1, 0, 0, 0], [float("nan"), 0, 0, 0], [1, 0, 0, 0])
    rp.set_coordinate_brush(ctx, vid, [0, 0, 0, 0], [0] * 4, [0] * 4)
    rp.unload(ctx, vid)


def test_served_coordinate_cut_equals_single_render(rp, ctx, small5):
    wl = small5
    vid = load(rp, ctx, wl, "f16")
    cam = wl.camera.as_array()
    coord = CUTS[3]
    rp.set_coordinate_brush(ctx, vid, *coord)
    single = cpu(rp.render(ctx, vid, cam, wl.width, wl.height, 0, wl.step))
    rp.set_coordinate_brush(ctx, vid, [0, 0, 0, 0], [0] * 4, [0] * 4)
    plain = cpu(rp.render(ctx, vid, cam, wl.width, wl.height, 0, wl.step))
    assert not np.array_equal(single, plain)
    out = torch.empty((wl.height, wl.width, 4), dtype=torch.float32, device="cuda")
    rp.server_start(ctx, 0, 8, 64, 2)
    try:
        req = rp.make_request(vid, cam, wl.width, wl.height, out, 0, wl.step, wl.brush.active, wl.brush.lo,
                              wl.brush.hi, 0, coord=coord)
        t = rp.submit(ctx, req)
        rp.wait(ctx, t, 20000)
    finally:
        rp.server_stop(ctx)
    assert np.array_equal(cpu(out), single)
    rp.unload(ctx, vid)
