"""ctypes marshalling for the C oracle (test infrastructure only).

The functions here convert a `scenes.Scene` into the oracle's C structures and
return numpy arrays; all arithmetic of the method runs in isaac_oracle.c.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "isaac_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_DT = {"f32": 0, "f16": 1, "bf16": 2}


class _Source(ctypes.Structure):
    _fields_ = [("f_dim", ctypes.c_int), ("dtype", ctypes.c_int),
                ("comp", ctypes.c_void_p * 4), ("stride", ctypes.c_int64 * 3),
                ("guard", ctypes.c_int), ("chain", ctypes.c_char_p), ("weight", ctypes.c_double),
                ("enabled", ctypes.c_int), ("n_tf", ctypes.c_int), ("tf", ctypes.POINTER(ctypes.c_double)),
                ("iso", ctypes.c_double)]


class _Scene(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 3), ("n_src", ctypes.c_int), ("src", ctypes.POINTER(_Source)),
                ("orthographic", ctypes.c_int), ("eye", ctypes.c_double * 3),
                ("center", ctypes.c_double * 3), ("up", ctypes.c_double * 3),
                ("fovy_deg", ctypes.c_double), ("ortho_height", ctypes.c_double),
                ("width", ctypes.c_int), ("height", ctypes.c_int), ("step", ctypes.c_double),
                ("interpolation", ctypes.c_int), ("n_clip", ctypes.c_int),
                ("clip", ctypes.POINTER(ctypes.c_double)), ("ert_threshold", ctypes.c_double),
                ("mode", ctypes.c_int), ("iso_margin", ctypes.c_double),
                ("delta", ctypes.c_double), ("ert_margin", ctypes.c_double)]


PIXEL_DTYPE = np.dtype([("rgba", np.float64, 4), ("samples", np.int64), ("allowance", np.float64),
                        ("flags", np.int32), ("kinds", np.int32), ("count_slack", np.int32), ("pad", np.int32)])
assert PIXEL_DTYPE.itemsize == 64
FLAG_NEAREST, FLAG_CLIP, FLAG_EXIT, FLAG_ERT, FLAG_ISO = 1, 2, 4, 8, 16
NO_TERMINATION = 2.0        # a threshold opacity never reaches

DELTA = 2.0 ** -12          # voxels: decisions closer than this may go either way on the GPU
ERT_MARGIN = 1e-4           # opacity margin around the termination threshold
ISO_MARGIN = 2.0 ** -16     # iso mode: relative FP32 arithmetic error of a value; with the value's change over
                            # +-DELTA per axis it bounds how far the GPU's value can lie from the oracle's

_lib = None
_lock = threading.Lock()


def build(force: bool = True, src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle with gcc (-O2, no contraction, no fast-math)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp"
        subprocess.run(["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-O2", "-ffp-contract=off", "-fno-fast-math",
                        "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, src, "-lm"], check=True)
        os.replace(tmp, out)
    return out


def _declare(lib):
    lib.oracle_render_range.argtypes = [ctypes.POINTER(_Scene), ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int]
    lib.oracle_render_list.argtypes = [ctypes.POINTER(_Scene), ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int]
    lib.oracle_chain_eval.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                                      ctypes.c_char_p, ctypes.c_int]
    lib.oracle_tf_table.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double), ctypes.c_char_p, ctypes.c_int]
    lib.oracle_ray.argtypes = [ctypes.POINTER(_Scene), ctypes.c_int, ctypes.c_int,
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.oracle_encode_rgba8.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_int64,
                                        ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_ubyte)]
    lib.oracle_encode_rgba8.restype = None
    for f in ("oracle_render_range", "oracle_render_list", "oracle_chain_eval", "oracle_tf_table",
              "oracle_ray"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


def load(path: Optional[str] = None):
    """Load liboracle.so (building it if missing); `path` loads another build (e.g. a mutant)."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build(force=True)
            _lib = _declare(ctypes.CDLL(LIB))
    return _lib


class _Marshalled:
    """Keeps every buffer referenced by the C structs alive."""

    def __init__(self, scene, delta: float, ert_margin: float, ert_threshold: Optional[float]):
        self.keep = []
        n = len(scene.sources)
        self.srcs = (_Source * max(n, 1))()
        for k, s in enumerate(scene.sources):
            cs = self.srcs[k]
            cs.f_dim = s.f_dim
            cs.dtype = _DT[s.dtype]
            for c, (bi, off) in enumerate(s.comp):
                buf = s.buffers[bi]
                self.keep.append(buf)
                cs.comp[c] = buf.ctypes.data + int(off)
            cs.stride[:] = [int(v) for v in s.strides]
            cs.guard = int(s.guard)
            chain = (s.chain or "").encode()
            self.keep.append(chain)
            cs.chain = chain
            cs.weight = float(s.weight)
            cs.enabled = 1 if s.enabled else 0
            tf = np.ascontiguousarray(np.array(s.tf, dtype=np.float64).reshape(-1))
            self.keep.append(tf)
            cs.n_tf = len(s.tf)
            cs.tf = tf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            cs.iso = float(s.iso)
        sc = _Scene()
        sc.dims[:] = [int(v) for v in scene.dims]
        sc.n_src = n
        sc.src = self.srcs
        cam = scene.camera
        sc.orthographic = 1 if cam.projection == "orthographic" else 0
        sc.eye[:] = [float(v) for v in cam.eye]
        sc.center[:] = [float(v) for v in cam.center]
        sc.up[:] = [float(v) for v in cam.up]
        sc.fovy_deg = float(cam.fovy_deg)
        sc.ortho_height = float(cam.ortho_height)
        sc.width, sc.height = int(scene.width), int(scene.height)
        sc.step = float(scene.step)
        sc.interpolation = int(scene.interpolation)
        clip = np.ascontiguousarray(np.array(scene.clip, dtype=np.float64).reshape(-1))
        if clip.size == 0:
            clip = np.zeros(4)
        self.keep.append(clip)
        sc.n_clip = len(scene.clip)
        sc.clip = clip.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        sc.ert_threshold = float(scene.ert_threshold if ert_threshold is None else ert_threshold)
        sc.mode = {"volume": 0, "iso": 1}[scene.mode]
        sc.iso_margin = ISO_MARGIN
        sc.delta = float(delta)
        sc.ert_margin = float(ert_margin)
        self.scene = sc


def _check(rc, err):
    if rc != 0:
        raise ValueError(err.value.decode(errors="replace"))


def render(scene, first: int = 0, count: Optional[int] = None, *, delta: float = DELTA,
           ert_margin: float = ERT_MARGIN, ert_threshold: Optional[float] = None, lib=None,
           threads: int = 1) -> np.ndarray:
    """Render pixels [first, first+count) (default: the whole image); returns PIXEL_DTYPE records.

    threads > 1 splits the pixel range over host threads running the same
    single-threaded C function (ctypes releases the GIL).
    """
    lib = lib or load()
    total = scene.width * scene.height
    count = total - first if count is None else count
    m = _Marshalled(scene, delta, ert_margin, ert_threshold)
    out = np.zeros(count, dtype=PIXEL_DTYPE)
    if threads <= 1 or count < 2 * threads:
        err = ctypes.create_string_buffer(256)
        _check(lib.oracle_render_range(ctypes.byref(m.scene), first, count, out.ctypes.data, err, 256), err)
        return out
    bounds = np.linspace(0, count, threads + 1).astype(np.int64)
    errors = []

    def work(a, b):
        err = ctypes.create_string_buffer(256)
        rc = lib.oracle_render_range(ctypes.byref(m.scene), first + int(a), int(b - a),
                                     out.ctypes.data + int(a) * PIXEL_DTYPE.itemsize, err, 256)
        if rc:
            errors.append(err.value.decode(errors="replace"))

    ts = [threading.Thread(target=work, args=(bounds[t], bounds[t + 1])) for t in range(threads)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    if errors:
        raise ValueError(errors[0])
    return out


def render_pixels(scene, px: Sequence, *, delta: float = DELTA, ert_margin: float = ERT_MARGIN,
                  ert_threshold: Optional[float] = None, lib=None) -> np.ndarray:
    """Render the listed (column, row) pixels."""
    lib = lib or load()
    px = np.ascontiguousarray(np.asarray(px, dtype=np.int32).reshape(-1, 2))
    m = _Marshalled(scene, delta, ert_margin, ert_threshold)
    out = np.zeros(px.shape[0], dtype=PIXEL_DTYPE)
    err = ctypes.create_string_buffer(256)
    _check(lib.oracle_render_list(ctypes.byref(m.scene), px.ctypes.data, px.shape[0], out.ctypes.data,
                                  err, 256), err)
    return out


def image(records: np.ndarray, scene) -> np.ndarray:
    return records["rgba"].reshape(scene.height, scene.width, 4)


def chain_eval(chain: str, f_dim: int, value, lib=None):
    """(classification value, result dimension) of a functor chain applied to one date."""
    lib = lib or load()
    v = (ctypes.c_double * 4)(*([float(x) for x in np.asarray(value, dtype=np.float64).reshape(-1)] + [0.0] * 4)[:4])
    out = ctypes.c_double()
    dim = ctypes.c_int()
    err = ctypes.create_string_buffer(256)
    _check(lib.oracle_chain_eval((chain or "").encode(), int(f_dim), v, ctypes.byref(out), ctypes.byref(dim),
                                 err, 256), err)
    return out.value, dim.value


def tf_table(points, lib=None) -> np.ndarray:
    lib = lib or load()
    pts = np.ascontiguousarray(np.array(points, dtype=np.float64).reshape(-1))
    table = np.zeros(256 * 4, dtype=np.float64)
    err = ctypes.create_string_buffer(256)
    _check(lib.oracle_tf_table(len(points), pts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               table.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), err, 256), err)
    return table.reshape(256, 4)


def encode_rgba8(rgba, background=None, lib=None) -> np.ndarray:
    """uint8 (..., 4) frame of a float32 premultiplied RGBA image (..., 4)."""
    lib = lib or load()
    a = np.ascontiguousarray(np.asarray(rgba, dtype=np.float32))
    assert a.shape[-1] == 4
    out = np.zeros(a.shape, dtype=np.uint8)
    bg = None
    if background is not None:
        bg = (ctypes.c_float * 3)(*[float(np.float32(v)) for v in background])
    lib.oracle_encode_rgba8(a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.c_int64(a.size // 4), bg,
                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
    return out


def ray(scene, i: int, j: int, lib=None):
    """(hit, origin, direction, t0, t1) of pixel (i, j)."""
    lib = lib or load()
    m = _Marshalled(scene, DELTA, ERT_MARGIN, None)
    o = (ctypes.c_double * 3)()
    d = (ctypes.c_double * 3)()
    t0 = ctypes.c_double()
    t1 = ctypes.c_double()
    hit = lib.oracle_ray(ctypes.byref(m.scene), int(i), int(j), o, d, ctypes.byref(t0), ctypes.byref(t1))
    if hit < 0:
        raise ValueError("bad scene")
    return bool(hit), np.array(o[:]), np.array(d[:]), t0.value, t1.value
