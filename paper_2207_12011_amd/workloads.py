"""Seeded synthetic workloads: volumes, brushes, transfer functions, cameras.

This module only *makes inputs*.  It holds none of the renderer's arithmetic
(no sampling, interpolation, classification or compositing) and is the one
module that both the HIP path and the FP64 oracle are fed from.

The paper's simulation snapshots (Section 3, the contest's mantle-convection
data) are not available, so these generators stand in for them.  Their
variables mirror the ones the paper names: temperature, temperature anomaly,
thermal conductivity, expansivity (Section 1) and the derived radial velocity
(Section 2.1); velocity enters through its magnitude.

Geometry: a cubic N^3 grid, cell-centred over [-1,1]^3, C order [z][y][x];
the planetary shell is r_inner <= r <= r_outer with r_inner = 0.55,
r_outer = 1 and every field is zero outside it.

Random streams: ``np.random.SeedSequence(220712011 + config_id)`` spawns, in
this fixed order, the children
``plumes, noise1, noise2, noise3, vel_x, vel_y, vel_z, workload``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

SEED_BASE = 220712011
CHILDREN = ("plumes", "noise1", "noise2", "noise3", "vel_x", "vel_y", "vel_z", "workload")
R_INNER = 0.55
R_OUTER = 1.0
COARSE = 128          # resolution the smooth random fields are drawn at
REF_STEP = 2.0 / 256  # opacity reference length in world units

FIELD_NAMES_5 = ("temperature", "temperature_anomaly", "conductivity",
                 "expansivity", "velocity_magnitude")
FIELD_NAMES_2 = ("temperature", "radial_velocity")


# --------------------------------------------------------------------------
# small value types handed to both the GPU library and the oracle
# --------------------------------------------------------------------------
@dataclass
class Camera:
    eye: Sequence[float]
    target: Sequence[float] = (0.0, 0.0, 0.0)
    up: Sequence[float] = (0.0, 0.0, 1.0)
    fov_y_deg: float = 60.0

    def as_array(self) -> np.ndarray:
        """[eye(3), target(3), up(3), fov_y_deg] as float32 (boundary precision)."""
        return np.array(list(self.eye) + list(self.target) + list(self.up) + [self.fov_y_deg],
                        dtype=np.float32)


@dataclass
class Brush:
    active: np.ndarray   # uint8[F]
    lo: np.ndarray       # float32[F]
    hi: np.ndarray       # float32[F]

    @staticmethod
    def none(n_fields: int) -> "Brush":
        return Brush(np.zeros(n_fields, np.uint8), np.full(n_fields, -np.inf, np.float32),
                     np.full(n_fields, np.inf, np.float32))

    def n_active(self) -> int:
        return int(np.count_nonzero(self.active))


@dataclass
class TransferFunction:
    field: int
    vmin: float
    vmax: float
    rgba: np.ndarray          # float32[256,4], straight (non-premultiplied) colour
    ref_step: float = REF_STEP


@dataclass
class Workload:
    config_id: int
    name: str
    fields: np.ndarray        # float32[F,N,N,N]
    field_names: tuple
    brush: Brush
    tf: TransferFunction
    camera: Camera
    width: int
    height: int
    step: float               # in voxels of the rendered level
    ert: float = 0.99
    r_inner: float = R_INNER
    r_outer: float = R_OUTER
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.fields.shape[1])

    @property
    def n_fields(self) -> int:
        return int(self.fields.shape[0])


# --------------------------------------------------------------------------
# grid helpers
# --------------------------------------------------------------------------
def cell_centres(n: int) -> np.ndarray:
    """x_i = -1 + (i + 1/2) * 2/n, float64."""
    return -1.0 + (np.arange(n, dtype=np.float64) + 0.5) * (2.0 / n)


def radius(n: int) -> np.ndarray:
    """|x| at every cell centre, float32[N,N,N] (computed in float64 per z-slice)."""
    c = cell_centres(n)
    yx = c[None, :] ** 2 + c[:, None] ** 2
    out = np.empty((n, n, n), np.float32)
    for k in range(n):
        out[k] = np.sqrt(yx + c[k] ** 2)
    return out


def shell_mask(r: np.ndarray, r_inner: float = R_INNER, r_outer: float = R_OUTER) -> np.ndarray:
    return (r >= np.float32(r_inner)) & (r <= np.float32(r_outer))


def _resample_matrix(n: int, m: int = COARSE) -> np.ndarray:
    """(n, m) linear-interpolation weights from an m-cell to an n-cell grid over [-1,1]
    (both cell centred, clamp to edge)."""
    u = (cell_centres(n) + 1.0) / (2.0 / m) - 0.5
    u = np.clip(u, 0.0, m - 1.0)
    i0 = np.floor(u).astype(np.int64)
    i0 = np.minimum(i0, m - 2)
    w = u - i0
    mat = np.zeros((n, m))
    mat[np.arange(n), i0] += 1.0 - w
    mat[np.arange(n), i0 + 1] += w
    return mat


def smooth_field(rng: np.random.Generator, n: int, mask: np.ndarray) -> np.ndarray:
    """White noise on a 128^3 grid, Gaussian-filtered (sigma = 2 coarse cells, periodic),
    resampled to n^3 cell centres and normalised to zero mean / unit std over ``mask``."""
    from scipy.ndimage import gaussian_filter
    coarse = gaussian_filter(rng.standard_normal((COARSE,) * 3), 2.0, mode="wrap")
    mat = _resample_matrix(n)
    a = np.tensordot(mat, coarse, axes=([1], [0]))                 # (n, m, m)
    a = np.tensordot(a, mat, axes=([2], [1]))                       # (n, m, n)
    out = np.empty((n, n, n), np.float32)
    for k in range(n):
        out[k] = (mat @ a[k]).astype(np.float32)                    # (n, n)
    sel = out[mask].astype(np.float64)
    mu, sd = sel.mean(), sel.std()
    out -= np.float32(mu)
    out /= np.float32(sd)
    out[~mask] = 0.0
    return out


def _plume_centres(rng: np.random.Generator, k: int = 8):
    cs = []
    while len(cs) < k:
        c = rng.uniform(-1.0, 1.0, 3)
        if R_INNER <= np.linalg.norm(c) <= R_OUTER:
            cs.append(c)
    amps = rng.uniform(0.3, 1.0, k)
    return np.array(cs), amps


def temperature(rng: np.random.Generator, n: int, r: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """clamp(sum of 8 Gaussian plumes (sigma 0.08, amplitude U(0.3,1)), 0, 1) + (1 - r)/0.45."""
    centres, amps = _plume_centres(rng)
    c = cell_centres(n)
    s2 = 2.0 * 0.08 ** 2
    acc = np.zeros((n, n, n), np.float32)
    for (cx, cy, cz), a in zip(centres, amps):
        ex = np.exp(-(c - cx) ** 2 / s2).astype(np.float32)
        ey = np.exp(-(c - cy) ** 2 / s2).astype(np.float32)
        ez = (a * np.exp(-(c - cz) ** 2 / s2)).astype(np.float32)
        eyx = ey[:, None] * ex[None, :]
        for k in range(n):
            if ez[k] > 1e-30:
                acc[k] += ez[k] * eyx
    np.clip(acc, 0.0, 1.0, out=acc)
    acc += (np.float32(1.0) - r) / np.float32(0.45)
    acc[~mask] = 0.0
    return acc


def temperature_anomaly(t: np.ndarray, r: np.ndarray, mask: np.ndarray, n: int) -> np.ndarray:
    """T minus its mean over radial bins of width h = 2/n (shell voxels only)."""
    h = 2.0 / n
    b = np.floor(r[mask].astype(np.float64) / h).astype(np.int64)
    tv = t[mask].astype(np.float64)
    sums = np.bincount(b, weights=tv)
    cnts = np.bincount(b)
    mean = np.where(cnts > 0, sums / np.maximum(cnts, 1), 0.0)
    out = np.zeros_like(t)
    out[mask] = (tv - mean[b]).astype(np.float32)
    return out


# --------------------------------------------------------------------------
# transfer function, brushes, cameras
# --------------------------------------------------------------------------
def default_tf_table() -> np.ndarray:
    """Blue -> grey (middle) -> red, alpha 0.02 + 0.10 (2i/255 - 1)^2; float32[256,4]."""
    blue = np.array([0.23, 0.30, 0.75])
    grey = np.array([0.87, 0.87, 0.87])
    red = np.array([0.71, 0.02, 0.15])
    tab = np.zeros((256, 4))
    for i in range(256):
        s = i / 255.0
        if s <= 0.5:
            rgb = blue + (grey - blue) * (2 * s)
        else:
            rgb = grey + (red - grey) * (2 * s - 1)
        tab[i, :3] = rgb
        tab[i, 3] = 0.02 + 0.10 * (2 * i / 255.0 - 1) ** 2
    return tab.astype(np.float32)


def default_tf(fields: np.ndarray, mask: np.ndarray, tf_field: int) -> TransferFunction:
    v = fields[tf_field][mask]
    return TransferFunction(tf_field, float(v.min()), float(v.max()), default_tf_table())


def shell_quantiles(fields: np.ndarray, mask: np.ndarray, qs) -> np.ndarray:
    """float32[F, len(qs)] quantiles of every field over shell voxels."""
    out = np.zeros((fields.shape[0], len(qs)), np.float32)
    for f in range(fields.shape[0]):
        out[f] = np.quantile(fields[f][mask], qs).astype(np.float32)
    return out


def _subsample_shell(fields: np.ndarray, mask: np.ndarray, rng, k: int = 1 << 21) -> np.ndarray:
    idx = np.flatnonzero(mask.ravel())
    if idx.size > k:
        idx = np.sort(rng.choice(idx, size=k, replace=False))
    return np.stack([fields[f].ravel()[idx] for f in range(fields.shape[0])])


def joint_fraction(sample: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> float:
    keep = np.ones(sample.shape[1], bool)
    for f in range(sample.shape[0]):
        keep &= (sample[f] >= lo[f]) & (sample[f] <= hi[f])
    return float(keep.mean())


def upper_tail_brush(fields: np.ndarray, mask: np.ndarray, rng, target=0.10, tol=0.005) -> Brush:
    """Every field keeps its upper tail [Q_f(1 - w), max_f]; w is bisected until the joint
    fraction of shell voxels is within target +- tol (evaluated on a seeded subsample of
    up to 2^21 shell voxels)."""
    nf = fields.shape[0]
    sample = _subsample_shell(fields, mask, rng)
    srt = np.sort(sample, axis=1)
    hi = srt[:, -1].copy()
    lo_w, hi_w = 0.0, 1.0
    lo = None
    for _ in range(60):
        w = 0.5 * (lo_w + hi_w)
        q = np.clip(int(math.floor((1.0 - w) * (srt.shape[1] - 1))), 0, srt.shape[1] - 1)
        lo = srt[:, q].copy()
        frac = joint_fraction(sample, lo, hi)
        if abs(frac - target) <= tol * 0.5:
            break
        if frac < target:
            lo_w = w
        else:
            hi_w = w
    hi = np.array([fields[f][mask].max() for f in range(nf)], np.float32)
    return Brush(np.ones(nf, np.uint8), lo.astype(np.float32), hi)


def narrowing_brushes(fields: np.ndarray, mask: np.ndarray, rng, final: Brush, count: int = 10) -> list:
    """``count`` brushes narrowing linearly in quantile space from all-inclusive to ``final`` (an
    upper-tail brush): brush k keeps [Q_f(u_f k / (count - 1)), hi_f] on every field, where u_f is
    the shell quantile of final.lo[f] (on a seeded subsample); brush 0 has lo = -inf, the last one
    is ``final``."""
    sample = _subsample_shell(fields, mask, rng)
    srt = np.sort(sample, axis=1)
    nf = fields.shape[0]
    out = []
    for k in range(count):
        if k == 0:
            lo = np.full(nf, -np.inf, np.float32)
        elif k == count - 1:
            lo = final.lo.copy()
        else:
            lo = np.empty(nf, np.float32)
            for f in range(nf):
                u = np.searchsorted(srt[f], final.lo[f]) / (srt.shape[1] - 1)
                q = int(round(u * k / (count - 1) * (srt.shape[1] - 1)))
                lo[f] = srt[f, min(q, srt.shape[1] - 1)]
        out.append(Brush(final.active.copy(), lo, final.hi.copy()))
    return out


def orbit_camera(az: float, el: float, dist: float = 3.0, fov: float = 60.0) -> Camera:
    eye = (dist * math.cos(el) * math.cos(az), dist * math.cos(el) * math.sin(az), dist * math.sin(el))
    return Camera(eye, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), fov)


def default_camera() -> Camera:
    return orbit_camera(math.radians(30.0), math.radians(20.0))


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------
def _children(config_id: int):
    ss = np.random.SeedSequence(SEED_BASE + config_id)
    kids = ss.spawn(len(CHILDREN))
    return {name: np.random.default_rng(k) for name, k in zip(CHILDREN, kids)}


def make_fields_5(n: int, rngs, progress=None) -> np.ndarray:
    """The five-field volume (temperature, anomaly, conductivity, expansivity, |v|).  ``progress``,
    if given, is called with a short message as each field is finished."""
    done = progress or (lambda msg: None)
    r = radius(n)
    m = shell_mask(r)
    t = temperature(rngs["plumes"], n, r, m)
    done("temperature")
    dt = temperature_anomaly(t, r, m, n)
    done("anomaly")
    cond = np.float32(3.0) + np.float32(2.0) * t + np.float32(0.05) * rngs["noise2"].standard_normal(
        (n, n, n), dtype=np.float32)
    cond[~m] = 0.0
    done("conductivity")
    expn = np.float32(3e-5) * (np.float32(1.0) - np.float32(0.5) * r) + np.float32(1e-6) * \
        rngs["noise3"].standard_normal((n, n, n), dtype=np.float32)
    expn[~m] = 0.0
    done("expansivity")
    vx = smooth_field(rngs["vel_x"], n, m)
    vy = smooth_field(rngs["vel_y"], n, m)
    vz = smooth_field(rngs["vel_z"], n, m)
    vmag = np.sqrt(vx * vx + vy * vy + vz * vz)
    del vx, vy, vz
    vmag[~m] = 0.0
    done("velocity magnitude")
    return np.stack([t, dt, cond, expn, vmag]), m


def make_workload(config_id: int, n: Optional[int] = None, width: Optional[int] = None,
                  height: Optional[int] = None, progress=None) -> Workload:
    """Configurations: 0 tiny (64^3, 2 fields, 128^2), 1 single request (256^3, 5 fields,
    1024^2), 2 precision study (512^3, 5 fields, 1920x1080), 4 large progressive (1024^3,
    5 fields, 3840x2160, final step 0.25 voxel).  ``n``/``width``/``height`` override the sizes
    (used for small cases of the same recipe)."""
    rngs = _children(config_id)
    cam = default_camera()
    if config_id == 0:
        n = n or 64
        r = radius(n)
        m = shell_mask(r)
        t = temperature(rngs["plumes"], n, r, m)
        vr = smooth_field(rngs["noise1"], n, m)
        fields = np.stack([t, vr])
        q = shell_quantiles(fields, m, [0.25, 0.5, 0.75])
        mx = np.array([fields[f][m].max() for f in range(2)], np.float32)
        brush = Brush(np.ones(2, np.uint8), np.array([q[0, 1], q[1, 0]], np.float32),
                      np.array([mx[0], q[1, 2]], np.float32))
        tf = default_tf(fields, m, 0)
        return Workload(0, "tiny 64^3 x 2 fields fp32, 128x128", fields, FIELD_NAMES_2, brush, tf, cam,
                        width or 128, height or 128, 0.5)
    if config_id in (1, 2, 4):
        n = n or {1: 256, 2: 512, 4: 1024}[config_id]
        fields, m = make_fields_5(n, rngs, progress)
        brush = upper_tail_brush(fields, m, rngs["workload"])
        tf = default_tf(fields, m, 1)
        step = 0.5
        if config_id == 1:
            w, h, name = width or 1024, height or 1024, f"single request {n}^3 x 5 fields, {width or 1024}x{height or 1024}"
        elif config_id == 2:
            w, h, name = width or 1920, height or 1080, f"precision {n}^3 x 5 fields, {width or 1920}x{height or 1080}"
        else:
            w, h, step = width or 3840, height or 2160, 0.25
            name = f"large progressive {n}^3 x 5 fields, {w}x{h}"
        return Workload(config_id, name, fields, FIELD_NAMES_5, brush, tf, cam, w, h, step)
    raise ValueError(f"unknown config {config_id}")


def analytic_workload(n: int = 1024, width: int = 1920, height: int = 1080) -> Workload:
    """Two closed-form fields over the shell (zero outside), cheap at the largest grid size:
    f0 = 0.5 + 0.25 sin(5x) sin(4y) sin(3z) + 0.25 (1 - r) / 0.45 and f1 = r, built one z-slab
    at a time.  Brush f0 in [0.55, 1], f1 in [0.6, 0.95]; table on f0 over [0, 1]; default camera,
    step 0.5 voxel."""
    c = cell_centres(n)
    sx = np.sin(5.0 * c).astype(np.float32)
    sy = np.sin(4.0 * c).astype(np.float32)
    sz = np.sin(3.0 * c).astype(np.float32)
    yx = (c[None, :] ** 2 + c[:, None] ** 2).astype(np.float32)
    sxy = sy[:, None] * sx[None, :]
    fields = np.empty((2, n, n, n), np.float32)
    for k in range(n):
        r = np.sqrt(yx + np.float32(c[k] ** 2))
        m = (r >= np.float32(R_INNER)) & (r <= np.float32(R_OUTER))
        f0 = np.float32(0.5) + np.float32(0.25) * sxy * sz[k] + np.float32(0.25) * (np.float32(1.0) - r) / np.float32(0.45)
        fields[0, k] = np.where(m, f0, np.float32(0.0))
        fields[1, k] = np.where(m, r, np.float32(0.0))
    brush = Brush(np.ones(2, np.uint8), np.array([0.55, 0.6], np.float32), np.array([1.0, 0.95], np.float32))
    tf = TransferFunction(0, 0.0, 1.0, default_tf_table())
    return Workload(5, f"analytic {n}^3 x 2 fields, {width}x{height}", fields, FIELD_NAMES_2, brush, tf,
                    default_camera(), width, height, 0.5)


def pc_line_cells(n: int, count: int = 100_000, seed: int = SEED_BASE + 6) -> np.ndarray:
    """Seeded choice (without replacement) of up to ``count`` shell cells of an N^3 grid, as
    uint32 linear indices z N^2 + y N + x: the cells whose values are the lines of the
    parallel-coordinates plot."""
    idx = np.flatnonzero(shell_mask(radius(n)).ravel())
    rng = np.random.default_rng(seed)
    return rng.choice(idx, size=min(count, idx.size), replace=False).astype(np.uint32)


# --------------------------------------------------------------------------
# serving trace
# --------------------------------------------------------------------------
SERVING_SIZES = ((256, 256), (512, 512), (1024, 1024), (1920, 1080), (2048, 2048))


def quantile_table(fields: np.ndarray, mask: np.ndarray, rng, levels: int = 1001,
                   sample: int = 1 << 21) -> np.ndarray:
    """float32 [F, levels]: shell-voxel quantiles of every field at linspace(0, 1, levels),
    estimated on a seeded subsample of up to `sample` shell voxels."""
    s = _subsample_shell(fields, mask, rng, sample)
    return np.quantile(s, np.linspace(0.0, 1.0, levels), axis=1).T.astype(np.float32)


@dataclass
class ServingRequest:
    volume: int            # index into the list of resident volumes
    camera: Camera
    width: int
    height: int
    active: np.ndarray     # uint8[5]
    lo: np.ndarray         # float32[5]
    hi: np.ndarray         # float32[5]
    gap: float             # unit-rate exponential inter-arrival gap (divide by QPS)


def serving_trace(qtables, n: int = 512, seed: int = SEED_BASE + 3):
    """Requests of the serving configuration: volume uniform over the resident ones, image size
    uniform over SERVING_SIZES, orbit camera (azimuth U[0, 2 pi), elevation U[-60, 60] deg,
    distance 3, up +z, 60 deg FOV), brush on k ~ U{1..5} distinct fields, each [Q(u), Q(u + w)]
    with w ~ U(0.3, 0.9), u ~ U(0, 1 - w) in shell quantiles; Poisson arrivals (unit-rate gaps)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        vi = int(rng.integers(len(qtables)))
        qt = qtables[vi]
        nf, levels = qt.shape
        w_, h_ = SERVING_SIZES[int(rng.integers(len(SERVING_SIZES)))]
        cam = orbit_camera(rng.uniform(0.0, 2 * math.pi), math.radians(rng.uniform(-60.0, 60.0)))
        k = int(rng.integers(1, nf + 1))
        act = np.zeros(nf, np.uint8)
        lo = np.zeros(nf, np.float32)
        hi = np.zeros(nf, np.float32)
        for f in rng.choice(nf, size=k, replace=False):
            w = rng.uniform(0.3, 0.9)
            u = rng.uniform(0.0, 1.0 - w)
            act[f] = 1
            lo[f] = np.interp(u, np.linspace(0, 1, levels), qt[f])
            hi[f] = np.interp(u + w, np.linspace(0, 1, levels), qt[f])
        out.append(ServingRequest(vi, cam, w_, h_, act, lo, hi, float(rng.exponential(1.0))))
    return out
