"""Reference definitions of the preprocessing steps (numpy).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  Shares no code with
the HIP library.

Paper, Section 2.1: an octree level-of-detail structure with two coarser
levels, each holding one eighth of the cells of the previous one.  Section 2.2:
changing the brush modifies no volume data and rebuilds no acceleration
structure -- so everything brush-dependent here (voxel mask, brick skip bits)
is derived from brush-independent tables at render time.

Every definition below is written in float32 with an explicit operation order
(numpy float32 arithmetic rounds after each operation), because the GPU
library must reproduce these arrays bit for bit:

* level build: parent = fl32(fl32(fl32((a+b)+(c+d)) + fl32((e+f)+(g+h))) * 0.125)
  with the eight children in (z, y, x) lexicographic order;
* FP16 storage: the field times a power of two 2^k, rounded to nearest even
  binary16 (subnormals kept), then times 2^-k; k = max(0, 14 - e) for the
  field's largest |value| f 2^e at level 0 (f in [0.5, 1)), the same k for
  every level, so a field of small values keeps binary16's normal-range
  precision (both scalings are exact in float32);
* 8-bit storage: per 8^3 brick of its own 512 voxels, offset = min,
  scale = fl32((max - min)/255), q = clamp(rint(fl32(fl32(v - offset)/scale)), 0, 255)
  (scale 0 and q 0 for a constant brick); value = fl32(fl32(scale*q) + offset);
* brick min/max: over the dequantised values of voxel indices
  [8b, min(8b+8, N-1)] per axis (the brick plus a one-voxel apron), which is
  every voxel a sample whose clamped floor index lies in the brick can read;
* skip bit: some active field's brick range misses its [lo, hi] (or lo > hi, an
  empty interval), or the table
  opacity is zero over every entry the transfer-function field's brick range
  can address; the index map is x(v) = fl32(min(max(fl32(fl32(v - vmin)*inv), 0), 1)*255)
  with inv = fl32(1/(vmax - vmin));
* sub-brick skip flags: the same rule over the eight 4^3 sub-bricks of every
  brick, each with its own apron window [4s, min(4s+4, N-1)] per axis, packed
  one byte per brick with sub-brick (sx, sy, sz) in bit sx + 2 sy + 4 sz.  A
  sub-brick window lies inside its brick's window, so a skipped brick has all
  eight sub-bricks skipped; the finer flags let a ray skip part of a brick.
"""
from __future__ import annotations

import math

import numpy as np

BRICK = 8
SUB = 4
F32 = np.float32


def build_level(v: np.ndarray) -> np.ndarray:
    """2x2x2 box mean of a float32 [N,N,N] array, fixed order, float32 [N/2]^3."""
    v = np.ascontiguousarray(v, dtype=F32)
    a = v[0::2, 0::2, 0::2]
    b = v[0::2, 0::2, 1::2]
    c = v[0::2, 1::2, 0::2]
    d = v[0::2, 1::2, 1::2]
    e = v[1::2, 0::2, 0::2]
    f = v[1::2, 0::2, 1::2]
    g = v[1::2, 1::2, 0::2]
    h = v[1::2, 1::2, 1::2]
    s0 = (a + b) + (c + d)
    s1 = (e + f) + (g + h)
    return ((s0 + s1) * F32(0.125)).astype(F32)


def build_levels(v: np.ndarray, n_lods: int):
    """[L0, L1, ...] float32 levels, each built from the float32 level above it."""
    out = [np.ascontiguousarray(v, dtype=F32)]
    for _ in range(1, n_lods):
        out.append(build_level(out[-1]))
    return out


# ----------------------------------------------------------------------------- storage
def encode_f16(v: np.ndarray) -> np.ndarray:
    """float32 -> IEEE binary16 bit patterns (round to nearest even, subnormals kept)."""
    return np.asarray(v, F32).astype(np.float16).view(np.uint16)


def decode_f16(bits: np.ndarray) -> np.ndarray:
    return np.asarray(bits, np.uint16).view(np.float16).astype(F32)


def _bricks_view(v: np.ndarray) -> np.ndarray:
    n = v.shape[0]
    nb = n // BRICK
    return v.reshape(nb, BRICK, nb, BRICK, nb, BRICK).transpose(0, 2, 4, 1, 3, 5).reshape(nb, nb, nb, BRICK ** 3)


def _unbricks(b: np.ndarray, n: int) -> np.ndarray:
    nb = n // BRICK
    return b.reshape(nb, nb, nb, BRICK, BRICK, BRICK).transpose(0, 3, 1, 4, 2, 5).reshape(n, n, n)


def encode_u8(v: np.ndarray):
    """Per-8^3-brick 8-bit codes.  Returns (q uint8 [N,N,N], scale f32 [nb]^3, offset f32 [nb]^3)."""
    v = np.asarray(v, F32)
    n = v.shape[0]
    bv = _bricks_view(v)
    mn = bv.min(axis=-1)
    mx = bv.max(axis=-1)
    scale = ((mx - mn) / F32(255.0)).astype(F32)
    d = (bv - mn[..., None]).astype(F32)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = (d / scale[..., None]).astype(F32)
    r = np.where(scale[..., None] > 0, r, F32(0.0))
    q = np.clip(np.rint(r), 0, 255).astype(np.uint8)
    return _unbricks(q, n), scale, mn.astype(F32)


def decode_u8(q: np.ndarray, scale: np.ndarray, offset: np.ndarray) -> np.ndarray:
    n = q.shape[0]
    bq = _bricks_view(q).astype(F32)
    val = ((scale[..., None] * bq).astype(F32) + offset[..., None]).astype(F32)
    return _unbricks(val, n)


def f16_exponent(v: np.ndarray) -> int:
    """k of binary16 storage: max(0, 14 - e) with the largest |value| m = f 2^e, f in [0.5, 1)
    (0 for an all-zero field), so that m 2^k < 2^14."""
    m = float(np.max(np.abs(np.asarray(v, F32)))) if np.size(v) else 0.0
    if m == 0.0:
        return 0
    return max(0, 14 - math.frexp(m)[1])


def stored_values(v: np.ndarray, storage: str, f16_exp: int = None) -> np.ndarray:
    """What a renderer reads after storing float32 level data as `storage`.  binary16 uses the
    exponent `f16_exp` (default: the one of `v` itself, right for level 0)."""
    if storage == "f32":
        return np.asarray(v, F32)
    if storage == "f16":
        k = f16_exponent(v) if f16_exp is None else f16_exp
        up, down = F32(2.0 ** k), F32(2.0 ** -k)
        return (decode_f16(encode_f16((np.asarray(v, F32) * up).astype(F32))) * down).astype(F32)
    if storage == "u8":
        return decode_u8(*encode_u8(v))
    raise ValueError(storage)


def stored_levels(fields: np.ndarray, n_lods: int, storage: str):
    """levels[l] = float32 [F, N_l, N_l, N_l] stored (dequantised) values of level l."""
    per_field = [build_levels(fields[f], n_lods) for f in range(fields.shape[0])]
    exps = [f16_exponent(fields[f]) for f in range(fields.shape[0])]
    return [np.stack([stored_values(per_field[f][l], storage, exps[f]) for f in range(fields.shape[0])])
            for l in range(n_lods)]


# ----------------------------------------------------------------------------- tables
def brick_minmax(v: np.ndarray, brick: int = BRICK):
    """(min, max) float32 [N/brick]^3 over the apron window [brick*b, min(brick*b+brick, N-1)] per axis."""
    v = np.asarray(v, F32)
    n = v.shape[0]
    nb = n // brick
    # pad one voxel at the far end by edge replication: the window then is [B b, B b + B]
    p = np.pad(v, ((0, 1), (0, 1), (0, 1)), mode="edge")
    mn = np.empty((nb, nb, nb), F32)
    mx = np.empty((nb, nb, nb), F32)
    for bz in range(nb):
        slab = p[brick * bz:brick * bz + brick + 1]
        for by in range(nb):
            row = slab[:, brick * by:brick * by + brick + 1]
            win = np.lib.stride_tricks.sliding_window_view(row, brick + 1, axis=2)[:, :, ::brick][:, :, :nb]
            mn[bz, by] = win.min(axis=(0, 1, 3))
            mx[bz, by] = win.max(axis=(0, 1, 3))
    return mn, mx


def tf_index(v, vmin: float, vmax: float) -> np.ndarray:
    """x(v) in float32 with the host-precomputed reciprocal."""
    vmin32 = F32(vmin)
    inv = F32(F32(1.0) / (F32(vmax) - vmin32))
    t = ((np.asarray(v, F32) - vmin32).astype(F32) * inv).astype(F32)
    t = np.minimum(np.maximum(t, F32(0.0)), F32(1.0))
    return (t * F32(255.0)).astype(F32)


def coord_skip(n: int, box: int, coord) -> np.ndarray:
    """bool [n/box]^3: boxes of box^3 voxels (voxel indices [i0, i1] per axis) in which no sample
    position can pass the coordinate axes of ``coord``.  The positions whose clamped floor index
    lies in the box are inside [fl32(fl32(i0 h) - 1), fl32(fl32((i1 + 2) h) - 1)] per axis (half a
    voxel of margin on each side; open at the grid faces), h = fl32(2 / n).  An axis skips the box
    when that range misses its bounds; the radius axis when the box's squared radius range
    (float32, summed x, y, z) misses the bounds' squares (see coord_pass)."""
    act, lo, hi = coord
    nbx = n // box
    h = F32(F32(2.0) / F32(n))
    i0 = np.arange(nbx, dtype=np.int64) * box
    i1 = i0 + box - 1
    with np.errstate(over="ignore", invalid="ignore"):
        bmin = ((i0.astype(F32) * h).astype(F32) - F32(1.0)).astype(F32)
        bmax = (((i1 + 2).astype(F32) * h).astype(F32) - F32(1.0)).astype(F32)
        bmin[i0 == 0] = -np.inf
        bmax[i1 == n - 1] = np.inf
        shapes = ((1, 1, nbx), (1, nbx, 1), (nbx, 1, 1))          # x, y, z along the array axes
        skip = np.zeros((nbx, nbx, nbx), bool)
        for ax in range(3):
            if act[ax]:
                miss = (bmax < F32(lo[ax])) | (bmin > F32(hi[ax]))
                skip |= miss.reshape(shapes[ax])
        if act[3]:
            d = np.maximum(np.maximum(F32(0.0), bmin), -bmax).astype(F32)
            d2 = (d * d).astype(F32)
            m2 = np.maximum((bmin * bmin).astype(F32), (bmax * bmax).astype(F32)).astype(F32)
            rmin2 = ((d2.reshape(shapes[0]) + d2.reshape(shapes[1])).astype(F32) + d2.reshape(shapes[2])).astype(F32)
            rmax2 = ((m2.reshape(shapes[0]) + m2.reshape(shapes[1])).astype(F32) + m2.reshape(shapes[2])).astype(F32)
            l3, h3 = F32(lo[3]), F32(hi[3])
            clo = F32(l3 * l3) if l3 > 0 else F32(-np.inf)
            chi = F32(h3 * h3) if h3 >= 0 else F32(-1.0)
            skip |= (rmin2 > chi) | (rmax2 < clo)
    return skip


def skip_bits(mins, maxs, active, lo, hi, tf_field: int, vmin: float, vmax: float, tf_rgba, coord=None,
              n: int = 0, box: int = BRICK) -> np.ndarray:
    """bool [nb]^3 brick skip flags from per-field tables (lists of [nb]^3 arrays); with ``coord``
    (coordinate axes) and the level size ``n``, boxes of ``box`` voxels that no sample position
    passing the axes can reach are skipped too (coord_skip)."""
    nb = mins[0].shape[0]
    skip = np.zeros((nb, nb, nb), bool)
    if coord is not None and any(coord[0]):
        skip |= coord_skip(n, box, coord)
    for f in range(len(mins)):
        if active[f]:
            skip |= (maxs[f] < F32(lo[f])) | (mins[f] > F32(hi[f])) | (F32(lo[f]) > F32(hi[f]))
    alpha = np.asarray(tf_rgba, F32).reshape(256, 4)[:, 3]
    x0 = tf_index(mins[tf_field], vmin, vmax)
    x1 = tf_index(maxs[tf_field], vmin, vmax)
    i0 = np.floor(x0).astype(np.int64)
    i1 = np.minimum(np.ceil(x1).astype(np.int64), 255)
    # zero over [i0, i1]  <=>  no positive entry in that range
    csum = np.concatenate([[0], np.cumsum(alpha > 0)])
    nz = csum[i1 + 1] - csum[i0]
    skip |= nz == 0
    return skip


def sub_skip_bytes(sub_flags: np.ndarray) -> np.ndarray:
    """bool [2 nb]^3 sub-brick skip flags -> uint8 [nb^3] (linear brick order), one byte per brick
    with sub-brick (sx, sy, sz) in bit sx + 2 sy + 4 sz."""
    f = np.asarray(sub_flags, bool)
    nb = f.shape[0] // 2
    out = np.zeros((nb, nb, nb), np.uint8)
    for sz in range(2):
        for sy in range(2):
            for sx in range(2):
                out |= (f[sz::2, sy::2, sx::2].astype(np.uint8) << (sx + 2 * sy + 4 * sz)).astype(np.uint8)
    return out.reshape(-1)


def sub_skip(fields_level, active, lo, hi, tf_field: int, vmin: float, vmax: float, tf_rgba,
             coord=None) -> np.ndarray:
    """Sub-brick skip bytes of one level's stored fields: the skip rule over 4^3 windows, packed."""
    mins, maxs = zip(*[brick_minmax(f, SUB) for f in fields_level])
    n = np.asarray(fields_level[0]).shape[0]
    return sub_skip_bytes(skip_bits(mins, maxs, active, lo, hi, tf_field, vmin, vmax, tf_rgba, coord, n, SUB))


def skip_words(sub_bytes: np.ndarray, nb: int, brick_skip=None) -> np.ndarray:
    """Per-brick flag words of the renderer (an empty-space structure of this implementation; the
    paper has only bricks): uint16 [nb^3], bits 0-7 the sub-brick skip byte, bit 8 set when every
    brick of the brick's aligned 2x2x2-brick group has all eight sub-bricks skipped, bit 9 the same
    for its aligned 4x4x4-brick group (a group cut by the grid's upper faces counts only the bricks
    inside the grid), bit 10 the brick's own skip bit (`brick_skip`, bool per brick in linear
    order; bit 10 clear when it is None)."""
    sub = np.asarray(sub_bytes, np.uint8).reshape(nb, nb, nb)
    full = sub == 0xFF
    words = sub.astype(np.uint16)
    for g, bit in ((2, 0x100), (4, 0x200)):
        ng = -(-nb // g)
        padded = np.ones((ng * g,) * 3, bool)
        padded[:nb, :nb, :nb] = full
        empty = padded.reshape(ng, g, ng, g, ng, g).all(axis=(1, 3, 5))
        spread = np.repeat(np.repeat(np.repeat(empty, g, 0), g, 1), g, 2)[:nb, :nb, :nb]
        words |= np.where(spread, bit, 0).astype(np.uint16)
    words = words.reshape(-1)
    if brick_skip is not None:
        words |= np.where(np.asarray(brick_skip, bool).reshape(-1), 0x400, 0).astype(np.uint16)
    return words


def pack_bits(flags: np.ndarray) -> np.ndarray:
    """bool array (linear brick order) -> uint32 words, brick k in word k//32 bit k%32."""
    flat = np.asarray(flags, bool).ravel()
    nw = (flat.size + 31) // 32
    padded = np.zeros(nw * 32, bool)
    padded[:flat.size] = flat
    w = padded.reshape(nw, 32).astype(np.uint64) << np.arange(32, dtype=np.uint64)
    return w.sum(axis=1).astype(np.uint32)


def pc_bin(v, axis_lo: float, axis_hi: float, n_bins: int) -> np.ndarray:
    """Histogram bin of values on one parallel-coordinates axis, decided in float32:
    inv = fl32(1 / fl32(hi - lo)), x = fl32(fl32(fl32(v - lo) * inv) * n_bins),
    bin = clamp(floor(x), 0, n_bins - 1)."""
    lo32, hi32 = F32(axis_lo), F32(axis_hi)
    inv = F32(F32(1.0) / F32(hi32 - lo32))
    t = ((np.asarray(v, F32) - lo32).astype(F32) * inv).astype(F32)
    x = (t * F32(n_bins)).astype(F32)
    return np.clip(np.floor(x), 0, n_bins - 1).astype(np.int64)


def cell_coord(i, n: int) -> np.ndarray:
    """World coordinate of cell index i on an N-cell axis, in float32: fl32(fl32(2 i + 1) / N) - 1."""
    return ((np.asarray(2 * np.asarray(i, np.int64) + 1).astype(F32) / F32(n)).astype(F32) - F32(1.0)).astype(F32)


def coord_pass(x, y, z, coord) -> np.ndarray:
    """The coordinate axes of the brush at positions (float32 arrays): axes 0..2 need
    lo <= x, y, z <= hi; axis 3 (radius) needs lo <= r <= hi, decided on squares in float32:
    r2 = fl32(fl32(fl32(x x) + fl32(y y)) + fl32(z z)) >= fl32(lo lo) (when lo > 0) and
    r2 <= fl32(hi hi) (when hi >= 0; nothing passes when hi < 0)."""
    act, lo, hi = coord
    keep = np.ones(np.broadcast_shapes(np.shape(x), np.shape(y), np.shape(z)), bool)
    for ax, v in enumerate((x, y, z)):
        if act[ax]:
            keep &= (v >= F32(lo[ax])) & (v <= F32(hi[ax]))
    if act[3]:
        x, y, z = (np.asarray(a, F32) for a in (x, y, z))
        r2 = ((x * x).astype(F32) + (y * y).astype(F32)).astype(F32)
        r2 = (r2 + (z * z).astype(F32)).astype(F32)
        l3, h3 = F32(lo[3]), F32(hi[3])
        if l3 > 0:
            keep &= r2 >= F32(l3 * l3)
        keep &= (r2 <= F32(h3 * h3)) if h3 >= 0 else np.zeros(keep.shape, bool)
    return keep


def pc_lines(level_fields: np.ndarray, cells, active, lo, hi, axis_lo, axis_hi, n_bins: int, coord=None):
    """Parallel-coordinates lines (paper, Section 2.1: up to 100 000 randomly chosen cells give the
    lines of the plot; Section 2: the brush selects the subset that is shown).  For cell indices
    z N^2 + y N + x of one level: the stored value of every field (the line's coordinates), whether
    the line passes the brush (every active field inside its inclusive [lo, hi], and the cell centre
    inside the coordinate axes of ``coord`` = (active[4], lo[4], hi[4]), see coord_pass), and per field a
    histogram over ``n_bins`` bins of [axis_lo, axis_hi] (pc_bin) of all lines and of passing lines.
    Returns (values float32 [L, F], passes uint8 [L], hist uint32 [F, n_bins, 2])."""
    lf = np.asarray(level_fields, F32)
    nf, n = lf.shape[0], lf.shape[1]
    c = np.asarray(cells, np.int64)
    z, y, x = c // (n * n), (c // n) % n, c % n
    values = np.stack([lf[f, z, y, x] for f in range(nf)], axis=1).astype(F32)
    keep = np.ones(c.size, bool)
    for f in range(nf):
        if active[f]:
            keep &= (values[:, f] >= F32(lo[f])) & (values[:, f] <= F32(hi[f]))
    if coord is not None:
        keep &= coord_pass(cell_coord(x, n), cell_coord(y, n), cell_coord(z, n), coord)
    hist = np.zeros((nf, n_bins, 2), np.uint32)
    for f in range(nf):
        b = pc_bin(values[:, f], axis_lo[f], axis_hi[f], n_bins)
        hist[f, :, 0] = np.bincount(b, minlength=n_bins)
        hist[f, :, 1] = np.bincount(b[keep], minlength=n_bins)
    return values, keep.astype(np.uint8), hist


def voxel_mask(level_fields: np.ndarray, active, lo, hi, coord=None) -> np.ndarray:
    """uint8 [N]^3: 1 where every active field lies in its inclusive [lo, hi] and the cell centre
    passes the coordinate axes of ``coord`` (see coord_pass)."""
    m = np.ones(level_fields.shape[1:], bool)
    for f in range(level_fields.shape[0]):
        if active[f]:
            m &= (level_fields[f] >= F32(lo[f])) & (level_fields[f] <= F32(hi[f]))
    if coord is not None and any(coord[0]):
        n = level_fields.shape[1]
        c = cell_coord(np.arange(n), n)
        m &= coord_pass(c[None, None, :], c[None, :, None], c[:, None, None], coord)
    return m.astype(np.uint8)


# ----------------------------------------------------------------------------- LOD choice
def select_lod(n0: int, n_lods: int, eye, fov_y_deg: float, height: int, r_outer: float = 1.0) -> int:
    """Keep about one finest-level voxel per pixel: with P the projected diameter of the
    outer sphere in pixels, lod = clamp(ceil(log2(N0/P)), 0, n_lods-1) when N0 > P, else 0;
    an eye inside the outer sphere gets level 0."""
    dist = math.sqrt(sum(float(e) ** 2 for e in eye))
    if dist <= r_outer:
        return 0
    p = height * math.tan(math.asin(r_outer / dist)) / math.tan(math.radians(fov_y_deg) / 2)
    if n0 <= p:
        return 0
    return int(min(max(math.ceil(math.log2(n0 / p)), 0), n_lods - 1))
