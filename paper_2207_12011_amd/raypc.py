"""Python binding of libraypc.so -- argument marshalling only.

Each function wraps the C entry point of the same name in include/raypc.h
(``render`` wraps ``raypc_render`` and so on).  Device buffers are torch CUDA
tensors (passed by ``data_ptr()``) and streams are torch streams (passed by
their HIP handle); torch provides memory and streams, every step of the
rendering runs in the library's HIP kernels.  There is no fallback: if the
library is not built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch  # must load before libraypc.so so that one HIP runtime serves both

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libraypc.so")

OK, ERR_INVALID, ERR_NOMEM, ERR_DEVICE, ERR_BUSY, ERR_TIMEOUT, ERR_CANCELLED, ERR_STATE = range(8)
STORAGE_COMPACT = 0x100
# "f32" / "f16" / "u8" keep 8-byte neighbourhood records besides the compact layout; the "c" forms keep only
# the compact layout
STORAGE = {"f32": 0, "f16": 1, "u8": 2, "f32c": 0 | STORAGE_COMPACT, "f16c": 1 | STORAGE_COMPACT,
           "u8c": 2 | STORAGE_COMPACT}
MAX_FIELDS = 8
TF_ENTRIES = 256

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                      "or `python paper_2207_12011_amd/build.py`")
_lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.c_void_p
_I = ctypes.c_int
_F = ctypes.c_float


class Camera(ctypes.Structure):
    _fields_ = [("eye", _F * 3), ("target", _F * 3), ("up", _F * 3), ("fov_y_deg", _F)]

    @staticmethod
    def make(cam) -> "Camera":
        """From a 10-vector [eye, target, up, fov_y_deg] or an object with those attributes."""
        if hasattr(cam, "eye"):
            v = list(cam.eye) + list(cam.target) + list(cam.up) + [cam.fov_y_deg]
        else:
            v = [float(x) for x in cam]
        c = Camera()
        c.eye[:] = v[0:3]
        c.target[:] = v[3:6]
        c.up[:] = v[6:9]
        c.fov_y_deg = v[9]
        return c


def _sig(name, restype, *argtypes):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(argtypes)
    return f


_create = _sig("raypc_create", _I, _I, ctypes.POINTER(_P))
_destroy = _sig("raypc_destroy", None, _P)
_last_error = _sig("raypc_last_error", ctypes.c_char_p)
_version = _sig("raypc_version", _I)
_load_fields = _sig("raypc_load_fields", _I, _P, _I, _I, _P, _I, _I, _I, _F, _F, _P, ctypes.POINTER(_I))
_unload = _sig("raypc_unload", _I, _P, _I)
_volume_info = _sig("raypc_volume_info", _I, _P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I),
                    ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_uint64))
_set_brush = _sig("raypc_set_brush", _I, _P, _I, _I, _P, _P, _P)
_set_coord = _sig("raypc_set_coordinate_brush", _I, _P, _I, _P, _P, _P)
_set_tf = _sig("raypc_set_transfer_function", _I, _P, _I, _I, _F, _F, _P, _I, _F)
_set_tf_async = _sig("raypc_set_transfer_function_async", _I, _P, _I, _I, _F, _F, _P, _I, _F, _P)
_set_options = _sig("raypc_set_options", _I, _P, _F, _P)
_select_lod = _sig("raypc_select_lod", _I, _P, _I, ctypes.POINTER(Camera), _I, _I, ctypes.POINTER(_I))
_render = _sig("raypc_render", _I, _P, _I, ctypes.POINTER(Camera), _I, _I, _I, _F, _P, _P)
_render_prog = _sig("raypc_render_progressive", _I, _P, _I, ctypes.POINTER(Camera), _I, _I, _I, _F, _I, _P, _P)
_export_level = _sig("raypc_export_level", _I, _P, _I, _I, _I, _P, _P)
_export_minmax = _sig("raypc_export_minmax", _I, _P, _I, _I, _I, _P, _P)
_export_minmax_sub = _sig("raypc_export_minmax_sub", _I, _P, _I, _I, _I, _P, _P)
_pc_lines = _sig("raypc_pc_lines", _I, _P, _I, _I, _I, _P, _P, _P, _I, _P, _P, _P, _P)
_render_jittered = _sig("raypc_render_jittered", _I, _P, _I, _P, _I, _I, _I, ctypes.c_float, _I, _I,
                        ctypes.c_uint64, _P, _P, _P, _P, _P)
_export_skip = _sig("raypc_export_skiplist", _I, _P, _I, _I, _I, _P, _P)
_export_subskip = _sig("raypc_export_subskip", _I, _P, _I, _I, _I, _P, _P)
_export_skip_words = _sig("raypc_export_skip_words", _I, _P, _I, _I, _I, _P, _P)
_export_mask = _sig("raypc_export_voxel_mask", _I, _P, _I, _I, _P, _P)
_render_debug = _sig("raypc_render_debug", _I, _P, _I, ctypes.POINTER(Camera), _I, _I, _I, _F, _P, _P, _P, _P, _I,
                     _P)
_measure_peaks = _sig("raypc_measure_peaks", _I, _P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                      _P)
_render_work = _sig("raypc_render_work", _I, _P, _I, ctypes.POINTER(Camera), _I, _I, _I, _F, _P, _P, _P, _P)
_render_depth = _sig("raypc_render_depth", _I, _P, _I, ctypes.POINTER(Camera), _I, _I, _I, _F, _P, _P, _P)
_set_launch_shape = _sig("raypc_set_launch_shape", _I, _P, _I, _I)
_get_launch_shape = _sig("raypc_get_launch_shape", _I, _P, ctypes.POINTER(_I), ctypes.POINTER(_I))
_autotune_render = _sig("raypc_autotune_render", _I, _P, _I, ctypes.POINTER(Camera), _I, _I, _I, _F, _I, _P,
                        ctypes.POINTER(_I), ctypes.POINTER(_I))
_warp = _sig("raypc_warp", _I, _P, ctypes.POINTER(Camera), _I, _I, _P, _P, ctypes.POINTER(Camera), _I, _I, _P, _P, _P,
             _P)
_warp_noalloc = _sig("raypc_warp_noalloc", _I, _P, ctypes.POINTER(Camera), _I, _I, _P, _P, ctypes.POINTER(Camera), _I,
                     _I, _P, _P, _P, _P)
WARP_NOALLOC_MAX_PIXELS = 2048 * 2048

class ServerCfg(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_uint64), ("max_inflight", _I), ("tiles_per_step", _I),
                ("steps_in_flight", _I)]


class Request(ctypes.Structure):
    _fields_ = [("volume_id", _I), ("camera", Camera), ("width", _I), ("height", _I), ("lod", _I), ("step", _F),
                ("active", ctypes.c_uint8 * MAX_FIELDS), ("lo", _F * MAX_FIELDS), ("hi", _F * MAX_FIELDS),
                ("coord_active", ctypes.c_uint8 * 4), ("coord_lo", _F * 4), ("coord_hi", _F * 4),
                ("tf_slot", _I), ("out", _P), ("deadline_ms", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "timed_out", "cancelled", "failed", "steps",
                                                "tiles", "bytes_in_use", "peak_bytes_in_use")] + \
               [("inflight", _I), ("queued", _I)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE = 0, 1, 2

_server_start = _sig("raypc_server_start", _I, _P, ctypes.POINTER(ServerCfg))
_server_stop = _sig("raypc_server_stop", _I, _P)
_submit = _sig("raypc_submit", _I, _P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64))
_poll = _sig("raypc_poll", _I, _P, ctypes.c_uint64, ctypes.POINTER(_I))
_wait = _sig("raypc_wait", _I, _P, ctypes.c_uint64, _I)
_cancel = _sig("raypc_cancel", _I, _P, ctypes.c_uint64)
_request_times = _sig("raypc_request_times", _I, _P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double * 4))
_release = _sig("raypc_release", _I, _P, ctypes.c_uint64)
_server_get_stats = _sig("raypc_server_get_stats", _I, _P, ctypes.POINTER(ServerStats))

EXPORTED = ["raypc_server_start", "raypc_server_stop", "raypc_submit", "raypc_poll", "raypc_wait", "raypc_cancel",
            "raypc_request_times", "raypc_release", "raypc_server_get_stats",
            "raypc_create", "raypc_destroy", "raypc_last_error", "raypc_version", "raypc_load_fields",
            "raypc_unload", "raypc_volume_info", "raypc_set_brush", "raypc_set_transfer_function", "raypc_set_transfer_function_async",
            "raypc_set_options", "raypc_select_lod", "raypc_render", "raypc_render_progressive",
            "raypc_export_level", "raypc_export_minmax", "raypc_export_minmax_sub", "raypc_export_skiplist",
            "raypc_export_subskip", "raypc_export_skip_words", "raypc_export_voxel_mask", "raypc_render_debug",
            "raypc_render_work", "raypc_measure_peaks", "raypc_pc_lines",
            "raypc_render_jittered", "raypc_set_coordinate_brush", "raypc_render_depth", "raypc_warp", "raypc_warp_noalloc",
            "raypc_set_launch_shape", "raypc_get_launch_shape", "raypc_autotune_render"]


class RaypcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"raypc error {code}: {msg}")
        self.code = code


def last_error() -> str:
    return (_last_error() or b"").decode()


def _check(rc: int):
    if rc != OK:
        raise RaypcError(rc, last_error())


def _stream(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


def _dptr(t: torch.Tensor, dtype, numel: int, what: str) -> int:
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"{what} must be a contiguous CUDA tensor of {dtype}")
    if t.numel() < numel:
        raise ValueError(f"{what} holds {t.numel()} elements, needs {numel}")
    return t.data_ptr()


def version() -> int:
    return _version()


# ----------------------------------------------------------------------------- context
def create(device: int = 0):
    h = _P()
    _check(_create(int(device), ctypes.byref(h)))
    return h


def destroy(ctx) -> None:
    _destroy(ctx)


def load_fields(ctx, fields, storage: str = "f32", n_lods: int = 3, r_inner: float = 0.55,
                r_outer: float = 1.0, stream=None) -> int:
    """`fields`: float32 [F, N, N, N] as a numpy array (host copy) or a CUDA tensor, or a list of
    per-field arrays/tensors."""
    seq = list(fields) if not isinstance(fields, (np.ndarray, torch.Tensor)) else [fields[i] for i in range(fields.shape[0])]
    if not seq:
        raise ValueError("no fields")
    on_device = isinstance(seq[0], torch.Tensor) and seq[0].is_cuda
    n = int(seq[0].shape[0])
    for f in seq:
        if tuple(f.shape) != (n, n, n):
            raise ValueError(f"every field must have shape ({n}, {n}, {n}), got {tuple(f.shape)}")
    keep = []
    ptrs = []
    for f in seq:
        if on_device:
            if not (isinstance(f, torch.Tensor) and f.is_cuda and f.dtype == torch.float32 and f.is_contiguous()):
                raise TypeError("device fields must be contiguous float32 CUDA tensors")
            ptrs.append(f.data_ptr())
        else:
            a = np.ascontiguousarray(np.asarray(f), dtype=np.float32)
            keep.append(a)
            ptrs.append(a.ctypes.data)
    arr = (_P * len(ptrs))(*ptrs)
    vid = _I()
    _check(_load_fields(ctx, len(ptrs), n, ctypes.cast(arr, _P), 1 if on_device else 0, STORAGE[storage],
                        int(n_lods), float(r_inner), float(r_outer), _stream(stream), ctypes.byref(vid)))
    return vid.value


def unload(ctx, volume_id: int) -> None:
    _check(_unload(ctx, int(volume_id)))


def volume_info(ctx, volume_id: int) -> dict:
    nf, n, nl, st = _I(), _I(), _I(), _I()
    by = ctypes.c_uint64()
    _check(_volume_info(ctx, int(volume_id), ctypes.byref(nf), ctypes.byref(n), ctypes.byref(nl), ctypes.byref(st),
                        ctypes.byref(by)))
    return {"n_fields": nf.value, "n": n.value, "n_lods": nl.value, "storage": st.value, "bytes": by.value}


def set_brush(ctx, volume_id: int, active, lo, hi) -> None:
    a = np.ascontiguousarray(np.asarray(active, np.uint8))
    l = np.ascontiguousarray(np.asarray(lo, np.float32))
    h = np.ascontiguousarray(np.asarray(hi, np.float32))
    _check(_set_brush(ctx, int(volume_id), int(a.size), a.ctypes.data, l.ctypes.data, h.ctypes.data))


def set_coordinate_brush(ctx, volume_id: int, active, lo, hi) -> None:
    """Coordinate axes (x, y, z of the sample position, its radius): 4 flags and bounds."""
    a = np.ascontiguousarray(np.asarray(active, np.uint8).reshape(4))
    l = np.ascontiguousarray(np.asarray(lo, np.float32).reshape(4))
    h = np.ascontiguousarray(np.asarray(hi, np.float32).reshape(4))
    _check(_set_coord(ctx, int(volume_id), a.ctypes.data, l.ctypes.data, h.ctypes.data))


def set_transfer_function(ctx, slot: int, field: int, vmin: float, vmax: float, rgba,
                          ref_step: float = 2.0 / 256, stream=None, ordered_on_stream: bool = False) -> None:
    """ordered_on_stream: raypc_set_transfer_function_async on `stream` (the current one when None)."""
    t = np.ascontiguousarray(np.asarray(rgba, np.float32).reshape(-1))
    if ordered_on_stream:
        _check(_set_tf_async(ctx, int(slot), int(field), float(vmin), float(vmax), t.ctypes.data, int(t.size // 4),
                             float(ref_step), _stream(stream)))
    else:
        _check(_set_tf(ctx, int(slot), int(field), float(vmin), float(vmax), t.ctypes.data, int(t.size // 4),
                       float(ref_step)))


def set_options(ctx, ert: float = 0.99, bg=None) -> None:
    b = None if bg is None else np.ascontiguousarray(np.asarray(bg, np.float32))
    _check(_set_options(ctx, float(ert), None if b is None else b.ctypes.data))


def select_lod(ctx, volume_id: int, camera, width: int, height: int) -> int:
    out = _I()
    _check(_select_lod(ctx, int(volume_id), ctypes.byref(Camera.make(camera)), int(width), int(height),
                       ctypes.byref(out)))
    return out.value


# ----------------------------------------------------------------------------- rendering
def _image(out, width, height, device):
    if out is None:
        out = torch.empty((height, width, 4), dtype=torch.float32, device=device)
    _dptr(out, torch.float32, width * height * 4, "out")
    return out


def render(ctx, volume_id: int, camera, width: int, height: int, lod: int = -1, step: float = 0.5,
           out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Async render into `out` (allocated as [H, W, 4] float32 when None)."""
    out = _image(out, width, height, "cuda")
    _check(_render(ctx, int(volume_id), ctypes.byref(Camera.make(camera)), int(width), int(height), int(lod),
                   float(step), out.data_ptr(), _stream(stream)))
    return out


def render_progressive(ctx, volume_id: int, camera, width: int, height: int, lod: int = -1, step: float = 0.5,
                       n_passes: int = 3, outs: Optional[Sequence[torch.Tensor]] = None, stream=None):
    if outs is None:
        outs = [torch.empty((height, width, 4), dtype=torch.float32, device="cuda") for _ in range(n_passes)]
    ptrs = (_P * n_passes)(*[_dptr(o, torch.float32, width * height * 4, "outs[k]") for o in outs])
    _check(_render_prog(ctx, int(volume_id), ctypes.byref(Camera.make(camera)), int(width), int(height), int(lod),
                        float(step), int(n_passes), ctypes.cast(ptrs, _P), _stream(stream)))
    return list(outs)


def render_debug(ctx, volume_id: int, camera, width: int, height: int, lod: int = -1, step: float = 0.5,
                 skip: bool = True, touched: Optional[torch.Tensor] = None, stream=None):
    """(rgba [H,W,4] f32, nominal [H,W] i32, composited [H,W] i32) as CUDA tensors (async).
    `touched`, if given, is a zeroed int32 CUDA tensor of ceil(nb^3/32) words (nb of the
    rendered level) that receives the touched-brick bits."""
    out = torch.empty((height, width, 4), dtype=torch.float32, device="cuda")
    nom = torch.empty((height, width), dtype=torch.int32, device="cuda")
    comp = torch.empty((height, width), dtype=torch.int32, device="cuda")
    tptr = None
    if touched is not None:
        info = volume_info(ctx, volume_id)
        lv = lod if lod >= 0 else select_lod(ctx, volume_id, camera, width, height)
        nb = (info["n"] >> lv) // 8
        tptr = _dptr(touched, torch.int32, (nb ** 3 + 31) // 32, "touched")
    _check(_render_debug(ctx, int(volume_id), ctypes.byref(Camera.make(camera)), int(width), int(height), int(lod),
                         float(step), out.data_ptr(), nom.data_ptr(), comp.data_ptr(), tptr, 0 if skip else 1,
                         _stream(stream)))
    return out, nom, comp


def render_work(ctx, volume_id: int, camera, width: int, height: int, lod: int = -1, step: float = 0.5, stream=None):
    """(rgba [H,W,4] f32, evaluated [H,W] i32, fetched [H,W] i32) as CUDA tensors (async): the samples the
    renderer did not skip and the field values it interpolated for them, per pixel."""
    out = torch.empty((height, width, 4), dtype=torch.float32, device="cuda")
    ev = torch.empty((height, width), dtype=torch.int32, device="cuda")
    fe = torch.empty((height, width), dtype=torch.int32, device="cuda")
    _check(_render_work(ctx, int(volume_id), ctypes.byref(Camera.make(camera)), int(width), int(height), int(lod),
                        float(step), out.data_ptr(), ev.data_ptr(), fe.data_ptr(), _stream(stream)))
    return out, ev, fe


def measure_peaks(ctx, stream=None) -> dict:
    """Measured device ceilings: {"copy_bytes_per_s", "fma_lane_ops_per_s"} (raypc_measure_peaks)."""
    c, f = ctypes.c_double(), ctypes.c_double()
    _check(_measure_peaks(ctx, ctypes.byref(c), ctypes.byref(f), _stream(stream)))
    return {"copy_bytes_per_s": c.value, "fma_lane_ops_per_s": f.value}


def render_jittered(ctx, volume_id: int, camera, width: int, height: int, lod: int, step: float, pass_index: int,
                    n_passes: int, seed: int, mean: Optional[torch.Tensor] = None, counts: bool = False,
                    stream=None):
    """One jittered progressive pass: (rgba [H,W,4] f32, nominal, composited) as CUDA tensors (the
    counts are None unless `counts`).  `mean`, if given, is an [H,W,4] float32 CUDA tensor holding
    the running mean of the passes (overwritten on pass 0)."""
    out = torch.empty((height, width, 4), dtype=torch.float32, device="cuda")
    nom = comp = None
    if counts:
        nom = torch.empty((height, width), dtype=torch.int32, device="cuda")
        comp = torch.empty((height, width), dtype=torch.int32, device="cuda")
    mptr = None if mean is None else _dptr(mean, torch.float32, height * width * 4, "mean")
    _check(_render_jittered(ctx, int(volume_id), ctypes.byref(Camera.make(camera)), int(width), int(height), int(lod),
                            float(step), int(pass_index), int(n_passes), int(seed) & ((1 << 64) - 1),
                            out.data_ptr(), mptr, None if nom is None else nom.data_ptr(),
                            None if comp is None else comp.data_ptr(), _stream(stream)))
    return out, nom, comp


TILE_SHAPES = tuple((1 << t, 16 >> t) for t in range(5))   # wave tile (width, height) per tile_log2w
SUPER_LOG2S = (0, 1, 2, 3)


def set_launch_shape(ctx, super_log2: int, tile_log2w: int = 2) -> None:
    _check(_set_launch_shape(ctx, int(super_log2), int(tile_log2w)))


def get_launch_shape(ctx):
    """(super_log2, tile_log2w) of the context's single-image launches."""
    s, t = _I(), _I()
    _check(_get_launch_shape(ctx, ctypes.byref(s), ctypes.byref(t)))
    return s.value, t.value


def autotune_render(ctx, volume_id: int, camera, width: int, height: int, lod: int = -1, step: float = 0.5,
                    repeats: int = 10):
    """Time the launch shapes on this view and keep the fastest: ((best super_log2, best tile_log2w),
    ms per render [tile_log2w][super_log2])."""
    times = (_F * 20)()
    best_s, best_t = _I(), _I()
    _check(_autotune_render(ctx, int(volume_id), ctypes.byref(Camera.make(camera)), int(width), int(height), int(lod),
                            float(step), int(repeats), ctypes.cast(times, _P), ctypes.byref(best_s),
                            ctypes.byref(best_t)))
    return (best_s.value, best_t.value), [[float(times[4 * t + k]) for k in range(4)] for t in range(5)]


def render_depth(ctx, volume_id: int, camera, width: int, height: int, lod: int = -1, step: float = 0.5,
                 out: Optional[torch.Tensor] = None, depth: Optional[torch.Tensor] = None, stream=None):
    """Async render plus opacity-weighted depth: (rgba [H,W,4] f32, depth [H,W] f32) CUDA tensors."""
    out = _image(out, width, height, "cuda")
    if depth is None:
        depth = torch.empty((height, width), dtype=torch.float32, device="cuda")
    _dptr(depth, torch.float32, width * height, "depth")
    _check(_render_depth(ctx, int(volume_id), ctypes.byref(Camera.make(camera)), int(width), int(height), int(lod),
                         float(step), out.data_ptr(), depth.data_ptr(), _stream(stream)))
    return out, depth


def warp(ctx, rgba: torch.Tensor, depth: torch.Tensor, src_camera, dst_camera, dst_width: Optional[int] = None,
         dst_height: Optional[int] = None, out: Optional[torch.Tensor] = None, out_depth: Optional[torch.Tensor] = None,
         out_source: Optional[torch.Tensor] = None, want_depth: bool = True, want_source: bool = True, stream=None,
         noalloc: bool = False):
    """Warp a frame (rgba [H,W,4] f32, depth [H,W] f32 CUDA tensors rendered with src_camera) to
    dst_camera: (rgba [H',W',4] f32, depth [H',W'] f32 or None, source [H',W'] int32 or None), async.
    noalloc: call raypc_warp_noalloc (the library's fixed z-buffer; outputs must be passed in by a
    caller that cannot allocate, else they are allocated here)."""
    sh, sw = int(rgba.shape[0]), int(rgba.shape[1])
    dw = sw if dst_width is None else int(dst_width)
    dh = sh if dst_height is None else int(dst_height)
    _dptr(rgba, torch.float32, sw * sh * 4, "rgba")
    _dptr(depth, torch.float32, sw * sh, "depth")
    out = _image(out, dw, dh, "cuda")
    if want_depth and out_depth is None:
        out_depth = torch.empty((dh, dw), dtype=torch.float32, device="cuda")
    if want_source and out_source is None:
        out_source = torch.empty((dh, dw), dtype=torch.int32, device="cuda")
    dptr = None if out_depth is None else _dptr(out_depth, torch.float32, dw * dh, "out_depth")
    sptr = None if out_source is None else _dptr(out_source, torch.int32, dw * dh, "out_source")
    fn = _warp_noalloc if noalloc else _warp
    _check(fn(ctx, ctypes.byref(Camera.make(src_camera)), sw, sh, rgba.data_ptr(), depth.data_ptr(),
              ctypes.byref(Camera.make(dst_camera)), dw, dh, out.data_ptr(), dptr, sptr, _stream(stream)))
    return out, out_depth, out_source


# ----------------------------------------------------------------------------- exports
def export_level(ctx, volume_id: int, lod: int, field: int, stream=None) -> torch.Tensor:
    info = volume_info(ctx, volume_id)
    n = info["n"] >> lod
    out = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
    _check(_export_level(ctx, int(volume_id), int(lod), int(field), out.data_ptr(), _stream(stream)))
    return out


def export_minmax(ctx, volume_id: int, lod: int, field: int, stream=None) -> torch.Tensor:
    nb = (volume_info(ctx, volume_id)["n"] >> lod) // 8
    out = torch.empty((nb, nb, nb, 2), dtype=torch.float32, device="cuda")
    _check(_export_minmax(ctx, int(volume_id), int(lod), int(field), out.data_ptr(), _stream(stream)))
    return out


def export_minmax_sub(ctx, volume_id: int, lod: int, field: int, stream=None) -> torch.Tensor:
    """[nb, nb, nb, 8 sub-bricks (bit sx + 2 sy + 4 sz), 2] float32."""
    nb = (volume_info(ctx, volume_id)["n"] >> lod) // 8
    out = torch.empty((nb, nb, nb, 8, 2), dtype=torch.float32, device="cuda")
    _check(_export_minmax_sub(ctx, int(volume_id), int(lod), int(field), out.data_ptr(), _stream(stream)))
    return out


def export_subskip(ctx, volume_id: int, lod: int, slot: int = 0, stream=None) -> torch.Tensor:
    nb = (volume_info(ctx, volume_id)["n"] >> lod) // 8
    out = torch.empty((nb ** 3,), dtype=torch.uint8, device="cuda")
    _check(_export_subskip(ctx, int(volume_id), int(lod), int(slot), out.data_ptr(), _stream(stream)))
    return out


def export_skip_words(ctx, volume_id: int, lod: int, slot: int = 0, stream=None) -> torch.Tensor:
    nb = (volume_info(ctx, volume_id)["n"] >> lod) // 8
    out = torch.empty((nb ** 3,), dtype=torch.int16, device="cuda")
    _check(_export_skip_words(ctx, int(volume_id), int(lod), int(slot), out.data_ptr(), _stream(stream)))
    return out


def export_skiplist(ctx, volume_id: int, lod: int, slot: int = 0, stream=None) -> torch.Tensor:
    nb = (volume_info(ctx, volume_id)["n"] >> lod) // 8
    out = torch.empty(((nb ** 3 + 31) // 32,), dtype=torch.int32, device="cuda")
    _check(_export_skip(ctx, int(volume_id), int(lod), int(slot), out.data_ptr(), _stream(stream)))
    return out


def pc_lines(ctx, volume_id: int, lod: int, cells: torch.Tensor, axis_lo=None, axis_hi=None, n_bins: int = 64,
             stream=None):
    """Parallel-coordinates lines of `cells` (a device tensor of uint32 or int32 linear indices):
    (values float32 [L, F], passes uint8 [L], hist int32 [F, n_bins, 2] or None without axis ranges)."""
    info = volume_info(ctx, volume_id)
    nf = info["n_fields"]
    if cells.dtype not in (torch.int32, torch.uint32) or not cells.is_cuda:
        raise ValueError("cells must be a CUDA tensor of 32-bit integers")
    c = cells.contiguous()
    nl = c.numel()
    values = torch.empty((nl, nf), dtype=torch.float32, device="cuda")
    passes = torch.empty((nl,), dtype=torch.uint8, device="cuda")
    hist = None
    lo_p = hi_p = None
    if axis_lo is not None:
        lo_a = np.ascontiguousarray(np.asarray(axis_lo, np.float32).reshape(nf))
        hi_a = np.ascontiguousarray(np.asarray(axis_hi, np.float32).reshape(nf))
        # at least one bin so that the library, not a NULL pointer, rejects a bad n_bins
        hist = torch.empty((nf, max(int(n_bins), 1), 2), dtype=torch.int32, device="cuda")
        lo_p, hi_p = lo_a.ctypes.data, hi_a.ctypes.data
    _check(_pc_lines(ctx, int(volume_id), int(lod), nl, c.data_ptr() if nl else None, lo_p, hi_p, int(n_bins),
                     values.data_ptr() if nl else None, passes.data_ptr() if nl else None,
                     hist.data_ptr() if hist is not None else None, _stream(stream)))
    return values, passes, hist


def export_voxel_mask(ctx, volume_id: int, lod: int, stream=None) -> torch.Tensor:
    n = volume_info(ctx, volume_id)["n"] >> lod
    out = torch.empty((n, n, n), dtype=torch.uint8, device="cuda")
    _check(_export_mask(ctx, int(volume_id), int(lod), out.data_ptr(), _stream(stream)))
    return out


# ----------------------------------------------------------------------------- serving
def server_start(ctx, mem_budget_bytes: int = 0, max_inflight: int = 64, tiles_per_step: int = 0,
                 steps_in_flight: int = 0) -> None:
    cfg = ServerCfg(int(mem_budget_bytes), int(max_inflight), int(tiles_per_step), int(steps_in_flight))
    _check(_server_start(ctx, ctypes.byref(cfg)))


def server_stop(ctx) -> None:
    _check(_server_stop(ctx))


def make_request(volume_id: int, camera, width: int, height: int, out: torch.Tensor, lod: int = -1,
                 step: float = 0.5, active=(), lo=(), hi=(), tf_slot: int = 0, deadline_ms: float = 0.0,
                 coord=None) -> Request:
    """A serving request; `coord` = (active[4], lo[4], hi[4]) coordinate axes (None: none)."""
    r = Request()
    r.volume_id = int(volume_id)
    r.camera = Camera.make(camera)
    r.width, r.height, r.lod, r.step = int(width), int(height), int(lod), float(step)
    a = np.zeros(MAX_FIELDS, np.uint8)
    l = np.zeros(MAX_FIELDS, np.float32)
    h = np.zeros(MAX_FIELDS, np.float32)
    a[:len(active)] = np.asarray(active, np.uint8)
    l[:len(lo)] = np.asarray(lo, np.float32)
    h[:len(hi)] = np.asarray(hi, np.float32)
    r.active[:] = a.tolist()
    r.lo[:] = l.tolist()
    r.hi[:] = h.tolist()
    if coord is not None:
        r.coord_active[:] = np.asarray(coord[0], np.uint8).reshape(4).tolist()
        r.coord_lo[:] = np.asarray(coord[1], np.float32).reshape(4).tolist()
        r.coord_hi[:] = np.asarray(coord[2], np.float32).reshape(4).tolist()
    r.tf_slot = int(tf_slot)
    r.out = _dptr(out, torch.float32, width * height * 4, "out")
    r.deadline_ms = float(deadline_ms)
    return r


def submit(ctx, request: Request) -> int:
    t = ctypes.c_uint64()
    _check(_submit(ctx, ctypes.byref(request), ctypes.byref(t)))
    return t.value


def poll(ctx, ticket: int) -> int:
    st = _I()
    _check(_poll(ctx, int(ticket), ctypes.byref(st)))
    return st.value


def wait(ctx, ticket: int, timeout_ms: int = -1) -> None:
    _check(_wait(ctx, int(ticket), int(timeout_ms)))


def cancel(ctx, ticket: int) -> None:
    _check(_cancel(ctx, int(ticket)))


def request_times(ctx, ticket: int):
    arr = (ctypes.c_double * 4)()
    _check(_request_times(ctx, int(ticket), ctypes.byref(arr)))
    return list(arr)


def release(ctx, ticket: int) -> None:
    _check(_release(ctx, int(ticket)))


def server_get_stats(ctx) -> dict:
    st = ServerStats()
    _check(_server_get_stats(ctx, ctypes.byref(st)))
    return {n: getattr(st, n) for n, _ in ServerStats._fields_}


class Renderer:
    """Owns one context; thin convenience over the functions above."""

    def __init__(self, device: int = 0):
        self.ctx = create(device)

    def close(self):
        if self.ctx is not None:
            destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_workload_volume(self, wl, storage="f32", n_lods=3, device_input=True):
        """Load a workloads.Workload's fields, brush and transfer function (slot 0)."""
        fields = torch.from_numpy(wl.fields).cuda() if device_input else wl.fields
        vid = load_fields(self.ctx, fields, storage, n_lods, wl.r_inner, wl.r_outer)
        set_brush(self.ctx, vid, wl.brush.active, wl.brush.lo, wl.brush.hi)
        set_transfer_function(self.ctx, 0, wl.tf.field, wl.tf.vmin, wl.tf.vmax, wl.tf.rgba, wl.tf.ref_step)
        set_options(self.ctx, wl.ert)
        return vid
