"""Exactness pins of the oracle's empty-space skip rule (brick bits and 4^3 sub-brick flags).

The conservativeness tests elsewhere only catch a rule that skips too much.  These catch a rule
that skips too little: every box's decision is rebuilt here from first principles and compared
with the oracle's for equality.

* The voxels a box can make a sample read are enumerated from the sampling definition (a sample
  whose clamped floor index c lies in the box reads c and min(c + 1, N - 1) per axis), not taken
  from the oracle's window formula.
* A field blocks skipping unless the interval of those voxels' values meets [lo, hi].
* The transfer function blocks skipping unless its piecewise-linear opacity, evaluated in float64,
  is positive somewhere on the index interval [x(min), x(max)] of the table field's values.  A
  piecewise-linear function is positive somewhere on an interval iff it is positive at an end
  or at a knot inside, so only those points are evaluated.  x(v) is the float32 index map
  (paper, Section 2.2: the brush and the table decide which samples count; the float32 map is
  the reading that makes the GPU's skip lists reproducible).
* Coordinate axes may skip a box only if no position within half a voxel of the positions that
  map into it passes them.

Adversarial brushes put bounds exactly on a box's extreme value and one float32 step beyond it,
and adversarial tables put zero bands exactly around a box's index interval.  Both the oracle's
bits and this enumeration must agree everywhere (paper, Section 2.2: a brush change rebuilds
nothing, so the per-brush skip decision is all the renderer has).
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import preprocess as pp
from paper_2207_12011_amd import workloads as W

F32 = np.float32


def readable_axis(b: int, box: int, n: int) -> list:
    """Voxel indices on one axis that samples with clamped floor index in [box b, box b + box) read."""
    s = set()
    for c in range(box * b, box * b + box):
        s.add(min(max(c, 0), n - 1))
        s.add(min(max(c + 1, 0), n - 1))
    return sorted(s)


def box_ranges(field: np.ndarray, box: int):
    """Per box: (min, max) over the enumerated readable voxels, float32 [nb]^3 each."""
    n = field.shape[0]
    nb = n // box
    axes = [readable_axis(b, box, n) for b in range(nb)]
    mn = np.empty((nb, nb, nb), F32)
    mx = np.empty((nb, nb, nb), F32)
    for bz in range(nb):
        for by in range(nb):
            for bx in range(nb):
                win = field[np.ix_(axes[bz], axes[by], axes[bx])]
                mn[bz, by, bx] = win.min()
                mx[bz, by, bx] = win.max()
    return mn, mx


def x_index(v, vmin, vmax) -> np.ndarray:
    """Float32 table index of value v: fl32(clamp(fl32(fl32(v - vmin) inv), 0, 1) 255), inv = fl32(1 / (vmax - vmin))."""
    inv = F32(F32(1.0) / (F32(vmax) - F32(vmin)))
    t = F32(F32(F32(v) - F32(vmin)) * inv)
    t = min(max(t, F32(0.0)), F32(1.0))
    return float(F32(t * F32(255.0)))


def opacity_at(x: float, alpha: np.ndarray) -> float:
    """Piecewise-linear table opacity at index x in [0, 255] (float64)."""
    i = min(int(np.floor(x)), 254)
    w = x - i
    return (1.0 - w) * float(alpha[i]) + w * float(alpha[i + 1])


def tf_positive(x0: float, x1: float, alpha: np.ndarray) -> bool:
    pts = [x0, x1] + [float(k) for k in range(int(np.floor(x0)) + 1, int(np.ceil(x1))) if x0 < k < x1]
    return any(opacity_at(x, alpha) > 0.0 for x in pts)


def coord_may_pass(i0: int, i1: int, n: int, coord) -> bool:
    """Some position within half a voxel of the positions that map into voxel boxes [i0, i1]^3
    (per axis: [(i0 + 1/2) h - 1, (i1 + 3/2) h - 1), open at the grid faces) passes the axes; a
    little float32 slack (1e-6) is allowed beyond the half voxel."""
    act, lo, hi = coord
    h = 2.0 / n
    rng = []
    for a in range(3):
        lo_p = -np.inf if i0[a] == 0 else i0[a] * h - 1.0 - 1e-6
        hi_p = np.inf if i1[a] == n - 1 else (i1[a] + 2) * h - 1.0 + 1e-6
        rng.append((lo_p, hi_p))
        if act[a] and (hi_p < lo[a] or lo_p > hi[a]):
            return False
    if act[3]:
        dmin = sum(max(0.0, r[0], -r[1]) ** 2 for r in rng)
        dmax = sum(max(r[0] ** 2, r[1] ** 2) for r in rng)
        if np.sqrt(dmin) > hi[3] + 1e-6 or np.sqrt(dmax) < lo[3] - 1e-6:
            return False
    return True


def enumerated_skip(fields, box, active, lo, hi, tf_field, vmin, vmax, table, coord=None) -> np.ndarray:
    n = fields[0].shape[0]
    nb = n // box
    ranges = [box_ranges(np.asarray(f, F32), box) for f in fields]
    alpha = np.asarray(table, F32).reshape(256, 4)[:, 3].astype(np.float64)
    skip = np.zeros((nb, nb, nb), bool)
    for bz in range(nb):
        for by in range(nb):
            for bx in range(nb):
                passable = True
                for f in range(len(fields)):
                    if active[f]:
                        mn, mx = ranges[f][0][bz, by, bx], ranges[f][1][bz, by, bx]
                        if max(mn, F32(lo[f])) > min(mx, F32(hi[f])):
                            passable = False
                tmn, tmx = ranges[tf_field][0][bz, by, bx], ranges[tf_field][1][bz, by, bx]
                if not tf_positive(x_index(tmn, vmin, vmax), x_index(tmx, vmin, vmax), alpha):
                    passable = False
                if coord is not None and any(coord[0]):
                    i0 = (bx * box, by * box, bz * box)
                    i1 = tuple(i + box - 1 for i in i0)
                    if not coord_may_pass(i0, i1, n, coord):
                        passable = False
                skip[bz, by, bx] = not passable
    return skip


def oracle_brick_skip(fields, active, lo, hi, tf_field, vmin, vmax, table, coord=None):
    mins, maxs = zip(*[pp.brick_minmax(f) for f in fields])
    return pp.skip_bits(mins, maxs, active, lo, hi, tf_field, vmin, vmax, table, coord, fields[0].shape[0])


def oracle_sub_skip(fields, active, lo, hi, tf_field, vmin, vmax, table, coord=None):
    """Sub-brick flags unpacked to bool [2 nb]^3 (the inverse of the byte packing is written out)."""
    by = pp.sub_skip(fields, active, lo, hi, tf_field, vmin, vmax, table, coord)
    n = fields[0].shape[0]
    nb = n // pp.BRICK
    cube = by.reshape(nb, nb, nb)
    out = np.zeros((2 * nb,) * 3, bool)
    for sz in range(2):
        for sy in range(2):
            for sx in range(2):
                out[sz::2, sy::2, sx::2] = (cube >> (sx + 2 * sy + 4 * sz)) & 1
    return out


@pytest.fixture(scope="module")
def small5():
    """The five-field recipe at 32^3 (4^3 bricks, 8^3 sub-bricks) with its table field."""
    wl = W.make_workload(1, n=32, width=16, height=16)
    return wl


def _cases(wl, box):
    """Brushes and tables: the workload's own, and adversarial ones built on box extremes."""
    fields = wl.fields
    nf = fields.shape[0]
    table = wl.tf.rgba.copy()
    base = (wl.brush.active.copy(), wl.brush.lo.copy(), wl.brush.hi.copy(), table)
    out = [base]
    rng = np.random.default_rng(1000 + box)
    ranges = [box_ranges(fields[f], box) for f in range(nf)]
    nb = fields.shape[1] // box
    for _ in range(6):
        f = int(rng.integers(nf))
        b = tuple(int(i) for i in rng.integers(nb, size=3))
        mn, mx = ranges[f][0][b], ranges[f][1][b]
        act = np.zeros(nf, np.uint8)
        act[f] = 1
        lo = np.full(nf, -np.inf, F32)
        hi = np.full(nf, np.inf, F32)
        # lo exactly on the box's maximum (kept), one float32 step above (skipped)
        for lo_f in (mx, np.nextafter(mx, F32(np.inf))):
            l2 = lo.copy()
            l2[f] = lo_f
            out.append((act, l2, hi, table))
        for hi_f in (mn, np.nextafter(mn, F32(-np.inf))):
            h2 = hi.copy()
            h2[f] = hi_f
            out.append((act, lo, h2, table))
    # tables with zero bands around a box's index interval of the table field
    tf = wl.tf.field
    for _ in range(4):
        b = tuple(int(i) for i in rng.integers(nb, size=3))
        x0 = x_index(ranges[tf][0][b], wl.tf.vmin, wl.tf.vmax)
        x1 = x_index(ranges[tf][1][b], wl.tf.vmin, wl.tf.vmax)
        i0, i1 = int(np.floor(x0)), min(int(np.ceil(x1)), 255)
        t_zero = table.copy()
        t_zero[max(i0 - 1, 0):i1 + 1, 3] = 0.0          # every reachable entry zero: skipped
        out.append((np.zeros(nf, np.uint8), np.full(nf, -np.inf, F32), np.full(nf, np.inf, F32), t_zero))
        t_edge = t_zero.copy()
        t_edge[i1, 3] = 0.05                            # only the top reachable entry positive: kept
        out.append((np.zeros(nf, np.uint8), np.full(nf, -np.inf, F32), np.full(nf, np.inf, F32), t_edge))
        t_above = t_zero.copy()
        t_above[:, 3] = 0.0
        t_above[min(i1 + 1, 255):min(i1 + 4, 256), 3] = 0.05  # positive just above the interval
        out.append((np.zeros(nf, np.uint8), np.full(nf, -np.inf, F32), np.full(nf, np.inf, F32), t_above))
    # banded table: zero over two bands
    t_band = table.copy()
    t_band[60:121, 3] = 0.0
    t_band[200:231, 3] = 0.0
    out.append((wl.brush.active.copy(), wl.brush.lo.copy(), wl.brush.hi.copy(), t_band))
    return out


@pytest.mark.parametrize("box", [pp.BRICK, pp.SUB])
def test_skip_rule_equals_enumeration(small5, box):
    wl = small5
    fields = [wl.fields[f] for f in range(wl.n_fields)]
    kept_and_skipped = [0, 0]
    for act, lo, hi, table in _cases(wl, box):
        want = enumerated_skip(fields, box, act, lo, hi, wl.tf.field, wl.tf.vmin, wl.tf.vmax, table)
        if box == pp.BRICK:
            got = oracle_brick_skip(fields, act, lo, hi, wl.tf.field, wl.tf.vmin, wl.tf.vmax, table)
        else:
            got = oracle_sub_skip(fields, act, lo, hi, wl.tf.field, wl.tf.vmin, wl.tf.vmax, table)
        assert np.array_equal(got, want), (box, int((got != want).sum()))
        kept_and_skipped[0] += int((~want).sum())
        kept_and_skipped[1] += int(want.sum())
    assert min(kept_and_skipped) > 0


def test_skip_rule_adversarial_cases_decide_both_ways(small5):
    """The bounds on a box's extremes keep that box, one float32 step beyond skips it: the pin
    distinguishes <= from <, and a rule widened by any amount fails it."""
    wl = small5
    fields = [wl.fields[f] for f in range(wl.n_fields)]
    ranges = box_ranges(fields[2], pp.BRICK)
    b = (1, 2, 1)
    nf = wl.n_fields
    act = np.zeros(nf, np.uint8)
    act[2] = 1
    hi = np.full(nf, np.inf, F32)
    for lo_f, skipped in ((ranges[1][b], False), (np.nextafter(ranges[1][b], F32(np.inf)), True)):
        lo = np.full(nf, -np.inf, F32)
        lo[2] = lo_f
        got = oracle_brick_skip(fields, act, lo, hi, wl.tf.field, wl.tf.vmin, wl.tf.vmax, wl.tf.rgba)
        assert bool(got[b]) == skipped


def test_skip_rule_with_coordinate_axes_equals_enumeration():
    """Coordinate axes: a box is skipped exactly when no position within half a voxel of the
    positions mapping into it passes (the margin of the rule), for slab, band and shell cuts."""
    wl = W.make_workload(0, n=32)
    fields = [wl.fields[f] for f in range(2)]
    none = (np.zeros(2, np.uint8), np.full(2, -np.inf, F32), np.full(2, np.inf, F32))
    cuts = [
        ([1, 0, 0, 0], [0.0, 0, 0, 0], [1.0, 0, 0, 0]),
        ([0, 1, 1, 0], [-1.0, -0.3, 0, 0], [1.0, 0.27, 0.5, 0]),
        ([0, 0, 0, 1], [0, 0, 0, 0.7], [0, 0, 0, 0.85]),
        ([1, 0, 0, 1], [-0.13, 0, 0, 0.0], [0.41, 0, 0, 0.62]),
    ]
    table = wl.tf.rgba
    for box in (pp.BRICK, pp.SUB):
        for act, lo, hi in cuts:
            coord = (np.array(act, np.uint8), np.array(lo, F32), np.array(hi, F32))
            want = enumerated_skip(fields, box, none[0], none[1], none[2], 0, wl.tf.vmin, wl.tf.vmax, table, coord)
            if box == pp.BRICK:
                got = oracle_brick_skip(fields, none[0], none[1], none[2], 0, wl.tf.vmin, wl.tf.vmax, table, coord)
            else:
                got = oracle_sub_skip(fields, none[0], none[1], none[2], 0, wl.tf.vmin, wl.tf.vmax, table, coord)
            # the rule works in float32 with the stated margin; the enumeration allows 1e-6 of
            # slack, so the rule may keep (never skip) boxes within that slack of a bound
            assert not np.any(got & ~want), (box, act)
            assert np.array_equal(got, want), (box, act, int((got != want).sum()))
