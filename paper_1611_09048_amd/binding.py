"""ctypes binding of libisaac_mi355x.so (argument marshalling only).

Every call maps one-to-one onto a C entry point of include/isaac_mi355x.h;
all work of the ray caster runs in the HIP library.  Importing this module
never touches a GPU; loading the library fails loudly when it is not built.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libisaac_mi355x.so")

ISAAC_OK = 0
ERRORS = {
    -1: "ISAAC_ERR_INVALID_ARGUMENT", -2: "ISAAC_ERR_BAD_FUNCTOR", -3: "ISAAC_ERR_BAD_TRANSFER",
    -4: "ISAAC_ERR_OUT_OF_MEMORY", -5: "ISAAC_ERR_BUSY", -6: "ISAAC_ERR_NOT_FOUND", -7: "ISAAC_ERR_DEVICE",
}
DTYPES = {"f32": 0, "f16": 1, "bf16": 2}
PERSPECTIVE, ORTHOGRAPHIC = 0, 1
NEAREST, TRILINEAR = 0, 1
VOLUME, ISO = 0, 1
ASYNC, TIMING, NO_GRAPH, DIRECT, DERIVE = 1, 2, 4, 8, 16
MAX_SOURCES, MAX_FUNCTORS, MAX_CLIP, MAX_BATCH = 8, 8, 8, 256


class IsaacError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


UPDATE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p)


INIT_NULL_STREAM = 1


class InitDesc(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("mem_budget_bytes", ctypes.c_size_t),
                ("max_inflight", ctypes.c_int), ("max_volumes", ctypes.c_int), ("flags", ctypes.c_uint)]


class SourceDesc(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("f_dim", ctypes.c_int), ("dtype", ctypes.c_int),
                ("comp", ctypes.c_void_p * 4), ("stride", ctypes.c_int64 * 3), ("guard", ctypes.c_int),
                ("persistent", ctypes.c_int), ("functor_chain", ctypes.c_char_p), ("weight", ctypes.c_float),
                ("enabled", ctypes.c_int), ("update", UPDATE_FN), ("user", ctypes.c_void_p)]


class TfPoint(ctypes.Structure):
    _fields_ = [("x", ctypes.c_double), ("rgba", ctypes.c_double * 4)]


class ClipPlane(ctypes.Structure):
    _fields_ = [("n", ctypes.c_double * 3), ("d", ctypes.c_double)]


class RenderDesc(ctypes.Structure):
    _fields_ = [("volume_id", ctypes.c_int), ("width", ctypes.c_int), ("height", ctypes.c_int),
                ("projection", ctypes.c_int), ("eye", ctypes.c_double * 3), ("center", ctypes.c_double * 3),
                ("up", ctypes.c_double * 3), ("fovy_deg", ctypes.c_double), ("ortho_height", ctypes.c_double),
                ("step", ctypes.c_double), ("interpolation", ctypes.c_int), ("n_clip", ctypes.c_int),
                ("clip", ctypes.POINTER(ClipPlane)), ("tf_handles", ctypes.POINTER(ctypes.c_int32)),
                ("weights", ctypes.POINTER(ctypes.c_float)), ("enabled", ctypes.POINTER(ctypes.c_int32)),
                ("ert_threshold", ctypes.c_float), ("out_rgba", ctypes.c_void_p),
                ("out_samples", ctypes.c_void_p), ("update_pointer", ctypes.c_void_p),
                ("brick_origin", ctypes.POINTER(ctypes.c_int32)), ("global_dims", ctypes.POINTER(ctypes.c_int32)),
                ("out_depth", ctypes.c_void_p), ("mode", ctypes.c_int32),
                ("iso_values", ctypes.POINTER(ctypes.c_float))]


EXPORTS = ["isaac_init", "isaac_destroy", "isaac_last_error", "isaac_init_error", "isaac_set_sources",
           "isaac_set_transfer", "isaac_release_transfer", "isaac_render", "isaac_render_noalloc",
           "isaac_composite", "isaac_encode_rgba8",
           "isaac_timing", "isaac_set_tile_shape", "isaac_get_tile_shape", "isaac_submit", "isaac_submit_batch",
           "isaac_poll", "isaac_release", "isaac_read_image", "isaac_read_image_rgba8", "isaac_encode_jpeg", "isaac_read_image_jpeg", "isaac_freeze_volume", "isaac_serving_usage",
           "isaac_check_functor_chain", "isaac_version"]

_lib = None


def load(path: Optional[str] = None):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with `python -m paper_1611_09048_amd.build`")
    lib = ctypes.CDLL(p)
    c_ctx = ctypes.c_void_p
    lib.isaac_init.argtypes = [ctypes.POINTER(InitDesc), ctypes.POINTER(c_ctx)]
    lib.isaac_destroy.argtypes = [c_ctx]
    lib.isaac_destroy.restype = None
    lib.isaac_last_error.argtypes = [c_ctx]
    lib.isaac_last_error.restype = ctypes.c_char_p
    lib.isaac_init_error.argtypes = []
    lib.isaac_init_error.restype = ctypes.c_char_p
    lib.isaac_version.restype = ctypes.c_char_p
    lib.isaac_set_sources.argtypes = [c_ctx, ctypes.c_int, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(SourceDesc),
                                      ctypes.c_int]
    lib.isaac_set_transfer.argtypes = [c_ctx, ctypes.c_int, ctypes.c_int, ctypes.POINTER(TfPoint), ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int32)]
    lib.isaac_release_transfer.argtypes = [c_ctx, ctypes.c_int32]
    lib.isaac_render.argtypes = [c_ctx, ctypes.POINTER(RenderDesc), ctypes.c_int, ctypes.c_uint]
    lib.isaac_render_noalloc.argtypes = [c_ctx, ctypes.POINTER(RenderDesc), ctypes.c_int, ctypes.c_uint]
    lib.isaac_timing.argtypes = [c_ctx, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
    lib.isaac_composite.argtypes = [c_ctx, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint]
    lib.isaac_encode_rgba8.argtypes = [c_ctx, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_uint]
    lib.isaac_read_image_rgba8.argtypes = [c_ctx, ctypes.c_uint64, ctypes.POINTER(ctypes.c_float), ctypes.c_void_p]
    lib.isaac_freeze_volume.argtypes = [c_ctx, ctypes.c_int]
    lib.isaac_encode_jpeg.argtypes = [c_ctx, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    lib.isaac_read_image_jpeg.argtypes = [c_ctx, ctypes.c_uint64, ctypes.POINTER(ctypes.c_float), ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    lib.isaac_set_tile_shape.argtypes = [c_ctx] + [ctypes.c_int] * 7
    lib.isaac_get_tile_shape.argtypes = [c_ctx, ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 6
    lib.isaac_submit.argtypes = [c_ctx, ctypes.POINTER(RenderDesc), ctypes.POINTER(ctypes.c_uint64)]
    lib.isaac_submit_batch.argtypes = [c_ctx, ctypes.POINTER(RenderDesc), ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_uint64)]
    lib.isaac_poll.argtypes = [c_ctx, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_void_p)]
    lib.isaac_release.argtypes = [c_ctx, ctypes.c_uint64]
    lib.isaac_read_image.argtypes = [c_ctx, ctypes.c_uint64, ctypes.c_void_p]
    lib.isaac_serving_usage.argtypes = [c_ctx, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                        ctypes.POINTER(ctypes.c_int)]
    lib.isaac_check_functor_chain.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_int), ctypes.c_char_p, ctypes.c_int]
    for name in EXPORTS:
        f = getattr(lib, name)
        if f.restype is ctypes.c_int and name not in ("isaac_destroy",):
            f.restype = ctypes.c_int32
    if path is None:
        _lib = lib
    return lib


def check_functor_chain(chain: str, f_dim: int):
    """(result dimension, functor count after simplification); raises IsaacError on a bad chain."""
    lib = load()
    d, n = ctypes.c_int(), ctypes.c_int()
    err = ctypes.create_string_buffer(256)
    rc = lib.isaac_check_functor_chain((chain or "").encode(), int(f_dim), ctypes.byref(d), ctypes.byref(n), err, 256)
    if rc != ISAAC_OK:
        raise IsaacError(rc, err.value.decode())
    return d.value, n.value


def _arr(ctype, values):
    if values is None:
        return None
    return (ctype * len(values))(*values)


class Context:
    """One library context on one device (not thread-safe, like the C context).

    stream: where the context enqueues its work.  "current" (the default):
    torch's current stream on `device` when the context is made, so work the
    caller issues there through torch (allocations, fills, copies) and the
    library's work are ordered, and events recorded there bracket a render;
    torch's default stream is HIP's null stream, passed as
    ISAAC_INIT_NULL_STREAM.  A torch stream or a raw hipStream_t handle: that
    stream.  None: a stream of the library's own."""

    def __init__(self, device: int = 0, stream="current", mem_budget: int = 0, max_inflight: int = 0,
                 max_volumes: int = 0):
        self.lib = load()
        if isinstance(stream, str) and stream == "current":
            import torch
            # no visible device: the null stream (isaac_init then reports the missing device)
            stream = torch.cuda.current_stream(device) if torch.cuda.is_available() else 0
        handle, flags = None, 0
        if stream is not None:
            handle = _stream_handle(stream)
            if not handle:
                handle, flags = None, INIT_NULL_STREAM
        d = InitDesc(device=device, stream=handle, mem_budget_bytes=mem_budget,
                     max_inflight=max_inflight, max_volumes=max_volumes, flags=flags)
        h = ctypes.c_void_p()
        rc = self.lib.isaac_init(ctypes.byref(d), ctypes.byref(h))
        if rc != ISAAC_OK:
            raise IsaacError(rc, self.lib.isaac_init_error().decode())
        self.h = h
        self._keep = {}

    # -- error handling -------------------------------------------------------
    def _check(self, rc):
        if rc != ISAAC_OK:
            raise IsaacError(rc, self.lib.isaac_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.isaac_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- volumes and transfer functions --------------------------------------
    def set_sources(self, volume_id: int, dims: Sequence[int], sources: Sequence[SourceDesc]):
        arr = (SourceDesc * max(1, len(sources)))(*sources)
        self._keep[("src", volume_id)] = (arr, list(sources))
        self._check(self.lib.isaac_set_sources(self.h, volume_id, _arr(ctypes.c_int32, list(dims)), arr,
                                               len(sources)))

    def set_transfer(self, volume_id: int, source: int, points) -> int:
        pts = (TfPoint * len(points))(*[TfPoint(x=float(p[0]), rgba=(ctypes.c_double * 4)(*map(float, p[1:5])))
                                        for p in points])
        h = ctypes.c_int32(-1)
        self._check(self.lib.isaac_set_transfer(self.h, volume_id, source, pts, len(points), ctypes.byref(h)))
        return h.value

    def release_transfer(self, handle: int):
        self._check(self.lib.isaac_release_transfer(self.h, int(handle)))

    # -- rendering ------------------------------------------------------------
    def render(self, jobs: Sequence[RenderDesc], flags: int = 0):
        arr = (RenderDesc * len(jobs))(*jobs)
        self._check(self.lib.isaac_render(self.h, arr, len(jobs), flags))

    def render_noalloc(self, jobs: Sequence[RenderDesc], flags: int = 0):
        """isaac_render_noalloc: the same images, no device allocation (static scratch)."""
        arr = (RenderDesc * len(jobs))(*jobs)
        self._check(self.lib.isaac_render_noalloc(self.h, arr, len(jobs), flags))

    def composite(self, rgba_ptrs, depth_ptrs, width: int, height: int, out_ptr: int, flags: int = 0):
        """Sort-last over-compositing of partial images (device pointers) into out_ptr."""
        n = len(rgba_ptrs)
        r = (ctypes.c_void_p * n)(*rgba_ptrs)
        d = (ctypes.c_void_p * n)(*depth_ptrs)
        self._check(self.lib.isaac_composite(self.h, r, d, n, width, height, out_ptr, flags))

    def encode_rgba8(self, rgba_ptr: int, width: int, height: int, out_ptr: int, background=None, flags: int = 0):
        """Quantize a device RGBA32F image to device RGBA8 (optionally over an opaque rgb background)."""
        bg = (ctypes.c_float * 3)(*map(float, background)) if background is not None else None
        self._check(self.lib.isaac_encode_rgba8(self.h, rgba_ptr, width, height, bg, out_ptr, flags))

    def freeze_volume(self, volume_id: int):
        """Evaluate the volume's chains once per voxel; later renders read those values (sources must not change)."""
        self._check(self.lib.isaac_freeze_volume(self.h, volume_id))

    def _jpeg_call(self, call, width: int, height: int) -> bytes:
        # a reused host buffer (first guess at most 16 MiB); on a too small one the
        # library reports the size it needs and the call is repeated once
        size = ctypes.c_size_t(0)
        need = min(width * height * 4 + 4096, 16 << 20)
        for _ in range(2):
            buf = getattr(self, "_jpeg_buf", None)
            if buf is None or len(buf) < need:
                self._jpeg_buf = buf = (ctypes.c_char * need)()
            rc = call(buf, len(buf), size)
            if rc == 0:
                return ctypes.string_at(buf, size.value)
            if rc != -1 or size.value <= len(buf):
                break
            need = size.value
        self._check(rc)
        raise IsaacError(rc, "jpeg encode failed")

    def encode_jpeg(self, rgba8_ptr: int, width: int, height: int, quality: int = 90) -> bytes:
        """JPEG bytes of a device RGBA8 frame (rows top to bottom, alpha ignored)."""
        return self._jpeg_call(lambda buf, cap, size: self.lib.isaac_encode_jpeg(
            self.h, rgba8_ptr, width, height, quality, buf, cap, ctypes.byref(size)), width, height)

    def timing(self):
        ms, n = ctypes.c_double(), ctypes.c_int()
        self._check(self.lib.isaac_timing(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def set_tile_shape(self, size_class: int, wave_w: int, waves_x: int, unroll: int = 1, lanes: int = 1,
                       min_waves: int = 0, pooled: int = 0):
        self._check(self.lib.isaac_set_tile_shape(self.h, size_class, wave_w, waves_x, unroll, lanes, min_waves,
                                                  pooled))

    def get_tile_shape(self, size_class: int):
        v = [ctypes.c_int() for _ in range(6)]
        self._check(self.lib.isaac_get_tile_shape(self.h, size_class, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    # -- serving ----------------------------------------------------------------
    def submit_batch(self, jobs: Sequence[RenderDesc]):
        """Tickets for the jobs, or None if admission was refused (ISAAC_ERR_BUSY)."""
        arr = (RenderDesc * len(jobs))(*jobs)
        t = (ctypes.c_uint64 * len(jobs))()
        rc = self.lib.isaac_submit_batch(self.h, arr, len(jobs), t)
        if rc == -5:
            return None
        self._check(rc)
        return list(t)

    def submit(self, job: RenderDesc):
        t = self.submit_batch([job])
        return None if t is None else t[0]

    def poll(self, ticket: int):
        done, ptr = ctypes.c_int(), ctypes.c_void_p()
        self._check(self.lib.isaac_poll(self.h, ctypes.c_uint64(ticket), ctypes.byref(done), ctypes.byref(ptr)))
        return bool(done.value), ptr.value

    def release(self, ticket: int):
        self._check(self.lib.isaac_release(self.h, ctypes.c_uint64(ticket)))

    def read_image(self, ticket: int, out):
        """Copy a ticket's image into the float32 numpy array `out` (height, width, 4)."""
        self._check(self.lib.isaac_read_image(self.h, ctypes.c_uint64(ticket), out.ctypes.data))
        return out

    def read_image_rgba8(self, ticket: int, out, background=None):
        """Encode a ticket's image to RGBA8 on the device and copy it into the uint8 array `out` (h, w, 4)."""
        bg = (ctypes.c_float * 3)(*map(float, background)) if background is not None else None
        self._check(self.lib.isaac_read_image_rgba8(self.h, ctypes.c_uint64(ticket), bg, out.ctypes.data))
        return out

    def read_image_jpeg(self, ticket: int, width: int, height: int, quality: int = 90, background=None) -> bytes:
        """JPEG bytes of a ticket's image (encoded to RGBA8 over `background`, then compressed, on the device)."""
        bg = (ctypes.c_float * 3)(*map(float, background)) if background is not None else None
        return self._jpeg_call(lambda buf, cap, size: self.lib.isaac_read_image_jpeg(
            self.h, ctypes.c_uint64(ticket), bg, quality, buf, cap, ctypes.byref(size)), width, height)

    def serving_usage(self):
        u, b, n = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int()
        self._check(self.lib.isaac_serving_usage(self.h, ctypes.byref(u), ctypes.byref(b), ctypes.byref(n)))
        return u.value, b.value, n.value


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def source_desc(*, name: str, f_dim: int, dtype: str, comp: Sequence[int], stride: Sequence[int], guard: int,
                chain: str = "", weight: float = 1.0, enabled: bool = True, persistent: bool = True,
                update=None, user: int = 0) -> SourceDesc:
    d = SourceDesc()
    d.name = name.encode()
    d.f_dim = f_dim
    d.dtype = DTYPES[dtype]
    for c in range(4):
        d.comp[c] = int(comp[c]) if c < len(comp) and comp[c] else None
    d.stride[:] = [int(s) for s in stride]
    d.guard = guard
    d.persistent = 1 if persistent else 0
    d.functor_chain = (chain or "").encode()
    d.weight = weight
    d.enabled = 1 if enabled else 0
    d.update = UPDATE_FN(update) if update is not None else UPDATE_FN()
    d.user = user
    return d


def render_desc(*, volume_id: int, width: int, height: int, eye, center, up, fovy_deg: float = 60.0,
                projection: int = PERSPECTIVE, ortho_height: float = 0.0, step: float = 0.5,
                interpolation: int = NEAREST, clip=(), tf_handles=None, weights=None, enabled=None,
                ert_threshold: float = 0.0, out_rgba: int = 0, out_samples: int = 0, brick_origin=None,
                global_dims=None, out_depth: int = 0, mode: int = 0, iso_values=None) -> RenderDesc:
    j = RenderDesc()
    j.volume_id = volume_id
    j.width, j.height = width, height
    j.projection = projection
    j.eye[:] = [float(v) for v in eye]
    j.center[:] = [float(v) for v in center]
    j.up[:] = [float(v) for v in up]
    j.fovy_deg = fovy_deg
    j.ortho_height = ortho_height
    j.step = step
    j.interpolation = interpolation
    clip = list(clip)
    j.n_clip = len(clip)
    keep = []
    if clip:
        arr = (ClipPlane * len(clip))(*[ClipPlane(n=(ctypes.c_double * 3)(*map(float, c[:3])), d=float(c[3]))
                                        for c in clip])
        keep.append(arr)
        j.clip = arr
    if tf_handles is not None:
        a = _arr(ctypes.c_int32, list(tf_handles))
        keep.append(a)
        j.tf_handles = a
    if weights is not None:
        a = _arr(ctypes.c_float, list(weights))
        keep.append(a)
        j.weights = a
    if enabled is not None:
        a = _arr(ctypes.c_int32, [1 if e else 0 for e in enabled])
        keep.append(a)
        j.enabled = a
    j.ert_threshold = ert_threshold
    j.out_rgba = out_rgba or None
    j.out_samples = out_samples or None
    if brick_origin is not None:
        a = _arr(ctypes.c_int32, [int(v) for v in brick_origin])
        b = _arr(ctypes.c_int32, [int(v) for v in global_dims])
        keep.extend([a, b])
        j.brick_origin = a
        j.global_dims = b
    j.out_depth = out_depth or None
    j.mode = mode
    if iso_values is not None:
        a = _arr(ctypes.c_float, [float(v) for v in iso_values])
        keep.append(a)
        j.iso_values = a
    j._keep = keep          # arrays referenced by pointer stay alive with the struct
    return j
