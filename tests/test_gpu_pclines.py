"""GPU parity of the parallel-coordinates lines (the plot's lines, their brush flags and per-axis
histograms) against the oracle: bit-exact values, flags and bin counts."""
import numpy as np
import pytest
import torch

from oracle import preprocess as pp
from paper_2207_12011_amd import workloads as W

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
def small5():
    return W.make_workload(1, n=64, width=64, height=64)


def cpu(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def check(rp, ctx, vid, wl, lod, cells, axis_lo, axis_hi, n_bins, level, brush, label):
    act, lo, hi = brush
    rp.set_brush(ctx, vid, act, lo, hi)
    dev = torch.from_numpy(cells.astype(np.int32)).cuda()
    vals, passes, hist = rp.pc_lines(ctx, vid, lod, dev, axis_lo, axis_hi, n_bins)
    want_v, want_p, want_h = pp.pc_lines(level, cells, act, lo, hi, axis_lo, axis_hi, n_bins)
    got_v = cpu(vals)
    assert np.array_equal(got_v.view(np.uint32), want_v.view(np.uint32)), label
    assert np.array_equal(cpu(passes), want_p), label
    assert np.array_equal(cpu(hist).astype(np.uint32), want_h), label
    print(f"[pclines] {label}: {cells.size} lines, {int(want_p.sum())} pass", flush=True)


@pytest.mark.parametrize("storage", STORAGES)
def test_pc_lines_bitexact(rp, ctx, small5, storage):
    wl = small5
    nf = wl.n_fields
    vid = rp.load_fields(ctx, torch.from_numpy(wl.fields).cuda(), storage, 3, wl.r_inner, wl.r_outer)
    levels = pp.stored_levels(wl.fields, 3, storage)
    brushes = [(wl.brush.active, wl.brush.lo, wl.brush.hi),
               (np.zeros(nf, np.uint8), wl.brush.lo, wl.brush.hi),
               (np.ones(nf, np.uint8), np.full(nf, 1.0, np.float32), np.full(nf, 0.0, np.float32)),
               (np.array([0, 1, 0, 0, 1], np.uint8), np.array([0, -0.1, 0, 0, 0.5], np.float32),
                np.array([0, 0.2, 0, 0, 1.5], np.float32))]
    full_lo = wl.fields.reshape(nf, -1).min(axis=1)
    full_hi = wl.fields.reshape(nf, -1).max(axis=1)
    narrow_lo = full_lo + 0.25 * (full_hi - full_lo)
    narrow_hi = full_lo + 0.5 * (full_hi - full_lo)       # many values clamp into the end bins
    for lod in range(3):
        n = 64 >> lod
        cells = W.pc_line_cells(n, 3000 >> lod, seed=lod)
        for bi, br in enumerate(brushes):
            for axes, nb in (((full_lo, full_hi), 64), ((narrow_lo, narrow_hi), 1), ((narrow_lo, narrow_hi), 512)):
                check(rp, ctx, vid, wl, lod, cells, axes[0], axes[1], nb, levels[lod], br,
                      f"{storage} lod {lod} brush {bi} bins {nb}")
    rp.unload(ctx, vid)


def test_pc_lines_edges(rp, ctx, small5):
    """No lines; cells outside the grid (ignored: NaN values, flag 0, not counted); lines not
    written when the outputs are omitted; invalid arguments rejected."""
    wl = small5
    nf = wl.n_fields
    vid = rp.load_fields(ctx, torch.from_numpy(wl.fields).cuda(), "f16", 1, wl.r_inner, wl.r_outer)
    lo_ax, hi_ax = np.zeros(nf, np.float32), np.ones(nf, np.float32)
    vals, passes, hist = rp.pc_lines(ctx, vid, 0, torch.zeros(0, dtype=torch.int32, device="cuda"), lo_ax, hi_ax, 8)
    assert vals.shape == (0, nf) and np.all(cpu(hist) == 0)
    cells = np.array([5, 64 ** 3, 7, 2 ** 31 - 1], np.int64).astype(np.int32)
    vals, passes, hist = rp.pc_lines(ctx, vid, 0, torch.from_numpy(cells).cuda(), lo_ax, hi_ax, 8)
    v, p, h = cpu(vals), cpu(passes), cpu(hist)
    assert np.isnan(v[1]).all() and np.isnan(v[3]).all() and p[1] == 0 and p[3] == 0
    assert np.all(h[:, :, 0].sum(axis=1) == 2)
    level = pp.stored_levels(wl.fields, 1, "f16")[0]
    want_v, _, want_h = pp.pc_lines(level, cells[[0, 2]], wl.brush.active, wl.brush.lo, wl.brush.hi,
                                    lo_ax, hi_ax, 8)
    rp.set_brush(ctx, vid, wl.brush.active, wl.brush.lo, wl.brush.hi)
    vals, passes, hist = rp.pc_lines(ctx, vid, 0, torch.from_numpy(cells).cuda(), lo_ax, hi_ax, 8)
    assert np.array_equal(cpu(vals)[[0, 2]], want_v) and np.array_equal(cpu(hist).astype(np.uint32), want_h)
    for bad in ((lo_ax, lo_ax, 8), (lo_ax, hi_ax, 0), (lo_ax, hi_ax, 513)):
        with pytest.raises(rp.RaypcError):
            rp.pc_lines(ctx, vid, 0, torch.from_numpy(cells).cuda(), *bad)
    with pytest.raises(rp.RaypcError):
        rp.pc_lines(ctx, vid, 3, torch.from_numpy(cells).cuda(), lo_ax, hi_ax, 8)
    rp.unload(ctx, vid)
