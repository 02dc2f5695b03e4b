"""FP64 CPU oracle for brushed spherical-shell volume ray casting.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the product library never does, and
the two share no code.  The ray caster itself is plain C (raypc_oracle.c,
double precision, one pixel at a time); the preprocessing definitions are
numpy float32 with explicit operation order (preprocess.py).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import preprocess  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libraypc_oracle.so")
_lib = None

FRAGILE_BRUSH = 1
FRAGILE_ERT = 2
FRAGILE_GRAZE = 4
FRAGILE_COUNT = 8
FRAGILE_TFZERO = 16
# bits whose decision can move RGBA by more than rounding; bit 3 only moves counts
FRAGILE_RGBA = FRAGILE_BRUSH | FRAGILE_ERT | FRAGILE_GRAZE | FRAGILE_TFZERO
# decisions whose two outcomes OracleImage.outcomes enumerates
FRAGILE_FLIPPABLE = FRAGILE_BRUSH | FRAGILE_ERT


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(
                os.path.join(_HERE, "raypc_oracle.c")):
            from .build import build
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.oracle_render.restype = ctypes.c_int
        L.oracle_render.argtypes = [
            ctypes.c_int, ctypes.c_int, P, ctypes.c_double, ctypes.c_double,
            P, P, P, P, P, P, ctypes.c_int, ctypes.c_double, ctypes.c_double, P, ctypes.c_double,
            ctypes.c_double, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_long,
            P, P, P, P, P, P, P, P, ctypes.c_int]
        L.oracle_outcomes.restype = ctypes.c_int
        L.oracle_outcomes.argtypes = [
            ctypes.c_int, ctypes.c_int, P, ctypes.c_double, ctypes.c_double,
            P, P, P, P, P, P, ctypes.c_int, ctypes.c_double, ctypes.c_double, P, ctypes.c_double,
            ctypes.c_double, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_long,
            P, P, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, ctypes.c_int]
        L.oracle_trilinear.restype = None
        L.oracle_trilinear.argtypes = [P, ctypes.c_int, P, ctypes.c_int, P]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Outcomes:
    """Legitimate results of some pixels whose flippable decisions (fragile bits 0 and 1) may go
    either way: for pixel k, count[k] outcomes (-1: more than the limit), outcome 0 being the
    double-precision result; rgba [k, o, 4], nominal / composited / depth / flips [k, o]."""
    count: np.ndarray
    rgba: np.ndarray
    nominal: np.ndarray
    composited: np.ndarray
    depth: np.ndarray
    flips: np.ndarray


@dataclass
class OracleImage:
    rgba: np.ndarray        # float64 [npix, 4] (or [H, W, 4] for full frames)
    nominal: np.ndarray     # uint32
    composited: np.ndarray  # uint32
    fragile: np.ndarray     # uint8 bit mask
    pathlen: np.ndarray     # float64
    depth: np.ndarray       # float64 opacity-weighted mean sample distance (+inf: nothing composited)
    _call: Optional[tuple] = None  # the render's prepared arguments (for outcomes)

    def outcomes(self, index: np.ndarray, max_flips: int = 8, max_out: int = 256,
                 threads: Optional[int] = None) -> Outcomes:
        """Every outcome of the pixels at positions `index` of this image's (flattened) pixel list
        with at most `max_flips` flippable decisions taken the other way."""
        args, pix, jit, width = self._call
        index = np.asarray(index, np.int64).reshape(-1)
        lin = np.ascontiguousarray(index if pix is None else pix[index])
        j = None if jit is None else np.ascontiguousarray(jit[index])
        k = lin.size
        count = np.zeros(k, np.int32)
        rgba = np.zeros((k, max_out, 4))
        nom = np.zeros((k, max_out), np.uint32)
        comp = np.zeros((k, max_out), np.uint32)
        dep = np.zeros((k, max_out))
        fl = np.zeros((k, max_out), np.uint8)
        if k:
            rc = lib().oracle_outcomes(*args, int(k), _ptr(lin), _ptr(j), int(max_flips), int(max_out), _ptr(count),
                                       _ptr(rgba), _ptr(nom), _ptr(comp), _ptr(dep), _ptr(fl),
                                       int(threads or os.cpu_count() or 1))
            if rc != 0:
                raise ValueError("oracle_outcomes: invalid arguments")
        return Outcomes(count, rgba, nom, comp, dep, fl)


def render(level_fields: np.ndarray, camera, width: int, height: int, step: float, *,
           active, lo, hi, tf_field: int, vmin: float, vmax: float, tf_rgba,
           ref_step: float = 2.0 / 256, ert: float = 0.99, bg=None,
           r_inner: float = 0.55, r_outer: float = 1.0,
           pixels: Optional[np.ndarray] = None, threads: Optional[int] = None,
           jitter: Optional[np.ndarray] = None, coord=None) -> OracleImage:
    """Render `pixels` (linear indices py*W+px; None = full frame) of one level.  `jitter` gives
    each rendered pixel's sample-grid offset in [0, 1) steps (None: the regular partition).
    `coord` = (active[4], lo[4], hi[4]) restricts the sample position (world x, y, z, radius).

    `level_fields` holds the level's stored values as float32 [F, N, N, N];
    scalars and tables are taken at float32 boundary precision and widened
    exactly to float64.  `camera` is a 10-vector [eye, target, up, fov_y_deg].
    """
    lf = np.ascontiguousarray(level_fields, dtype=np.float32)
    nf, n = lf.shape[0], lf.shape[1]
    ptrs = (ctypes.c_void_p * nf)(*[lf[f].ctypes.data for f in range(nf)])
    act = np.ascontiguousarray(np.asarray(active, np.uint8))
    lo64 = np.asarray(np.asarray(lo, np.float32), np.float64)
    hi64 = np.asarray(np.asarray(hi, np.float32), np.float64)
    tf64 = np.ascontiguousarray(np.asarray(np.asarray(tf_rgba, np.float32), np.float64).reshape(256, 4))
    cam = np.asarray(np.asarray(camera, np.float32), np.float64)
    bg64 = None if bg is None else np.asarray(np.asarray(bg, np.float32), np.float64)
    full = pixels is None
    pix = None if full else np.ascontiguousarray(np.asarray(pixels, np.int64))
    npix = width * height if full else pix.size
    jit = None if jitter is None else np.ascontiguousarray(np.asarray(jitter, np.float64).reshape(npix))
    cact = clo = chi = None
    if coord is not None:
        cact = np.ascontiguousarray(np.asarray(coord[0], np.uint8).reshape(4))
        clo = np.asarray(np.asarray(coord[1], np.float32).reshape(4), np.float64)
        chi = np.asarray(np.asarray(coord[2], np.float32).reshape(4), np.float64)
    rgba = np.zeros((npix, 4))
    nom = np.zeros(npix, np.uint32)
    comp = np.zeros(npix, np.uint32)
    frag = np.zeros(npix, np.uint8)
    plen = np.zeros(npix)
    dep = np.zeros(npix)
    threads = threads or os.cpu_count() or 1
    args = (nf, n, ctypes.cast(ptrs, ctypes.c_void_p), float(np.float32(r_inner)), float(np.float32(r_outer)),
            _ptr(act), _ptr(lo64), _ptr(hi64), _ptr(cact), _ptr(clo), _ptr(chi), int(tf_field),
            float(np.float32(vmin)), float(np.float32(vmax)), _ptr(tf64), float(np.float32(ref_step)),
            float(np.float32(ert)), _ptr(bg64), _ptr(cam), int(width), int(height), float(np.float32(step)))
    rc = lib().oracle_render(*args, int(npix), _ptr(pix), _ptr(jit),
                             _ptr(rgba), _ptr(nom), _ptr(comp), _ptr(frag), _ptr(plen), _ptr(dep), int(threads))
    if rc != 0:
        raise ValueError("oracle_render: invalid arguments")
    # keep the arrays the pointers in `args` refer to alive with the image
    call = (args, pix, jit, width)
    call_refs = (lf, ptrs, act, lo64, hi64, tf64, cam, bg64, cact, clo, chi)
    if full:
        img = OracleImage(rgba.reshape(height, width, 4), nom.reshape(height, width),
                          comp.reshape(height, width), frag.reshape(height, width),
                          plen.reshape(height, width), dep.reshape(height, width), call)
    else:
        img = OracleImage(rgba, nom, comp, frag, plen, dep, call)
    img._refs = call_refs
    return img


def trilinear(field: np.ndarray, u_xyz: np.ndarray) -> np.ndarray:
    """Values of one float32 [N,N,N] field at continuous voxel indices u (k x 3, x-y-z order)."""
    f = np.ascontiguousarray(field, np.float32)
    u = np.ascontiguousarray(np.asarray(u_xyz, np.float64).reshape(-1, 3))
    out = np.zeros(u.shape[0])
    lib().oracle_trilinear(_ptr(f), f.shape[0], _ptr(u), u.shape[0], _ptr(out))
    return out


def render_workload(wl, level_fields: np.ndarray, **kw) -> OracleImage:
    """Convenience: render a workloads.Workload's view from given level data."""
    args = dict(active=wl.brush.active, lo=wl.brush.lo, hi=wl.brush.hi, tf_field=wl.tf.field,
                vmin=wl.tf.vmin, vmax=wl.tf.vmax, tf_rgba=wl.tf.rgba, ref_step=wl.tf.ref_step,
                ert=wl.ert, r_inner=wl.r_inner, r_outer=wl.r_outer)
    args.update(kw)
    step = args.pop("step", wl.step)
    width = args.pop("width", wl.width)
    height = args.pop("height", wl.height)
    camera = args.pop("camera", wl.camera.as_array())
    return render(level_fields, camera, width, height, step, **args)
