"""Storage layouts for source fields and the scene containers.

A source field is held as raw bytes exactly as a simulation would hold it in
device memory: a guard layer around the local volume, rows padded to a byte
pitch, the vector components either interleaved (array of structures) or in
separate arrays, with any axis order and direction.  A source is then
described the way the library receives it: one byte address per component of
interior voxel (0,0,0) and a signed byte stride per axis.

Bytes outside the stored field (row padding, and optional extra layers around
the guard) are filled with 0xFF, which is a NaN in every storage type, so an
out-of-range read shows up as a non-finite pixel.
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

DTYPE_SIZE = {"f32": 4, "f16": 2, "bf16": 2}


def f32_to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even); return the 16-bit patterns."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    bias = ((u >> 16) & 1) + 0x7FFF
    out = ((u + bias) >> 16).astype(np.uint16)
    nan = np.isnan(a)
    if nan.any():
        out[nan] = 0x7FC0
    return out


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    """Exact widening of bfloat16 bit patterns to float32."""
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return (b.astype(np.uint32) << 16).view(np.float32)


def quantize(values: np.ndarray, dtype: str) -> Tuple[np.ndarray, np.ndarray]:
    """Return (storage elements, the same values widened exactly to float64)."""
    v32 = np.asarray(values, dtype=np.float32)
    if dtype == "f32":
        return v32, v32.astype(np.float64)
    if dtype == "f16":
        h = v32.astype(np.float16)
        return h, h.astype(np.float64)
    if dtype == "bf16":
        b = f32_to_bf16_bits(v32)
        return b, bf16_bits_to_f32(b).astype(np.float64)
    raise ValueError(f"unknown storage type {dtype!r}")


@dataclasses.dataclass
class SourceSpec:
    """One source: its stored bytes, how to address them, and its render settings."""
    name: str
    f_dim: int
    dtype: str
    buffers: List[np.ndarray]            # raw uint8 storage
    comp: List[Tuple[int, int]]          # per component: (buffer index, byte offset of voxel (0,0,0))
    strides: Tuple[int, int, int]        # signed byte strides along x, y, z
    guard: int                           # guard layers present around the local volume
    values: np.ndarray                   # stored values as float64, [z+g][y+g][x+g][c]
    chain: str = ""
    weight: float = 1.0
    enabled: bool = True
    persistent: bool = True
    tf: List[Tuple[float, float, float, float, float]] = dataclasses.field(default_factory=list)
    iso: float = float("nan")            # iso value in iso-surface mode (NaN: the source draws no surface)

    def nbytes(self) -> int:
        return int(sum(b.nbytes for b in self.buffers))

    def field_bytes(self) -> int:
        """Bytes of field data stored (guards included, padding excluded)."""
        n = self.values.shape[0] * self.values.shape[1] * self.values.shape[2]
        return int(n * self.f_dim * DTYPE_SIZE[self.dtype])


@dataclasses.dataclass
class Camera:
    eye: Tuple[float, float, float]
    center: Tuple[float, float, float]
    up: Tuple[float, float, float]
    fovy_deg: float = 60.0
    projection: str = "perspective"      # or "orthographic"
    ortho_height: float = 0.0


@dataclasses.dataclass
class Scene:
    dims: Tuple[int, int, int]           # local volume size in cells (x, y, z)
    sources: List[SourceSpec]
    camera: Camera
    width: int
    height: int
    step: float = 0.5
    interpolation: int = 0               # 0 nearest, 1 trilinear
    clip: List[Tuple[float, float, float, float]] = dataclasses.field(default_factory=list)
    ert_threshold: float = 0.999
    seed: Optional[int] = None
    label: str = ""
    mode: str = "volume"                 # "volume" (emission-absorption) or "iso" (first iso-surface)

    def with_(self, **kw) -> "Scene":
        return dataclasses.replace(self, **kw)


def _poisoned(nbytes: int) -> np.ndarray:
    return np.full(int(nbytes), 0xFF, dtype=np.uint8)


def store_field(values: np.ndarray, dtype: str = "f32", guard: int = 1, *,
                layout: str = "aos", order: Sequence[int] = (0, 1, 2),
                flip: Sequence[bool] = (False, False, False), pitch_align: int = 256,
                extra_layers: int = 0):
    """Lay out a logical field in raw bytes.

    values: float array [z][y][x][c] (or [z][y][x] for a scalar) covering the
        local volume plus `guard` layers on every side.
    layout: "aos" (components interleaved per voxel) or "soa" (one array per
        component).
    order: logical axes (0=x, 1=y, 2=z) from the fastest-varying to the slowest.
    flip: per logical axis, store it in decreasing address order (negative stride).
    pitch_align: the fastest rows are padded to a multiple of this many bytes.
    extra_layers: NaN-filled layers stored around the guard layers, i.e. memory
        that exists but that the source does not declare.

    Returns (buffers, comp, strides, stored_values_float64).
    """
    v = np.asarray(values)
    if v.ndim == 3:
        v = v[..., None]
    f_dim = v.shape[3]
    if not 1 <= f_dim <= 4:
        raise ValueError("f_dim must be 1..4")
    storage, stored64 = quantize(v, dtype)
    esize = DTYPE_SIZE[dtype]
    e = int(extra_layers)
    if e:
        full = np.empty(tuple(s + 2 * e for s in storage.shape[:3]) + (f_dim,), dtype=storage.dtype)
        full.view(np.uint8)[...] = 0xFF
        full[e:-e, e:-e, e:-e] = storage
        storage = full
    # logical axis extents including guard and extra layers, x,y,z order
    ext = (storage.shape[2], storage.shape[1], storage.shape[0])
    order = tuple(int(a) for a in order)
    assert sorted(order) == [0, 1, 2]
    # permute to physical [slow][mid][fast][c]
    zyx_axis = {0: 2, 1: 1, 2: 0}
    phys = np.transpose(storage, (zyx_axis[order[2]], zyx_axis[order[1]], zyx_axis[order[0]], 3))
    for ax in range(3):
        if flip[ax]:
            phys = np.flip(phys, axis=2 - order.index(ax))
    n_slow, n_mid, n_fast = phys.shape[:3]
    comps_per_buf = f_dim if layout == "aos" else 1
    row_bytes = n_fast * comps_per_buf * esize
    pitch = -(-row_bytes // pitch_align) * pitch_align
    phys_stride = {order[0]: comps_per_buf * esize, order[1]: pitch, order[2]: pitch * n_mid}
    buffers = []
    if layout == "aos":
        buf = _poisoned(pitch * n_mid * n_slow)
        view = buf.reshape(n_slow, n_mid, pitch)
        view[:, :, :row_bytes] = np.ascontiguousarray(phys).view(np.uint8).reshape(n_slow, n_mid, row_bytes)
        buffers.append(buf)
    elif layout == "soa":
        for c in range(f_dim):
            buf = _poisoned(pitch * n_mid * n_slow)
            view = buf.reshape(n_slow, n_mid, pitch)
            view[:, :, :row_bytes] = np.ascontiguousarray(phys[..., c]).view(np.uint8).reshape(
                n_slow, n_mid, row_bytes)
            buffers.append(buf)
    else:
        raise ValueError(f"unknown layout {layout!r}")
    # byte offset of interior voxel (0,0,0): array index g + e along each axis
    g = int(guard)
    strides = []
    origin = 0
    for ax in range(3):
        s = phys_stride[ax]
        a = g + e
        if flip[ax]:
            origin += (ext[ax] - 1 - a) * s
            strides.append(-s)
        else:
            origin += a * s
            strides.append(s)
    comp = []
    for c in range(f_dim):
        if layout == "aos":
            comp.append((0, origin + c * esize))
        else:
            comp.append((c, origin))
    return buffers, comp, tuple(strides), stored64


def make_source(name: str, values: np.ndarray, *, dtype: str = "f32", guard: int = 1,
                chain: str = "", weight: float = 1.0, tf=None, enabled: bool = True,
                persistent: bool = True, iso: float = float("nan"), **layout_kw) -> SourceSpec:
    buffers, comp, strides, stored = store_field(values, dtype, guard, **layout_kw)
    if stored.ndim == 3:
        stored = stored[..., None]
    return SourceSpec(name=name, f_dim=stored.shape[3], dtype=dtype, buffers=buffers, comp=comp,
                      strides=strides, guard=guard, values=stored, chain=chain, weight=weight,
                      enabled=enabled, persistent=persistent, tf=list(tf or []), iso=float(iso))


def logical_values(src: SourceSpec) -> np.ndarray:
    """The stored values, float64, indexed [z+g][y+g][x+g][c]."""
    return src.values


def relayout(src: SourceSpec, dtype: Optional[str] = None, **layout_kw) -> SourceSpec:
    """The same source stored in another layout (values re-quantized only if dtype changes)."""
    dt = dtype or src.dtype
    buffers, comp, strides, stored = store_field(src.values, dt, src.guard, **layout_kw)
    return dataclasses.replace(src, dtype=dt, buffers=buffers, comp=comp, strides=strides,
                               values=stored)
