"""The benchmark workloads and the small scenes used by tests.

Workloads (seeded; sizes can be scaled down for tests):
  plain_scalar   one FP32 Gaussian-blob scalar, 64^3, nearest, 256x256
  pic3           PIConGPU-shaped density + E + B, 256^3 with one guard layer,
                 trilinear, two clipping planes, 1920x1080
  pic3 (f16/bf16 storage) the same scene quantized once, round-to-nearest-even
  batch64        64 uneven sub-volumes with their own cameras and image sizes
  serving        a resident 512x512x256 three-source volume and a Poisson
                 stream of steering edits from four clients

Only inputs are produced here: no ray-casting arithmetic.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

from . import fields
from .layout import Camera, Scene, SourceSpec, make_source

# View direction (from the volume centre towards the eye) of the fixed camera.
D0 = (1.0, 0.8, 0.6)

# Functor chains of the three PIConGPU-shaped sources.
CHAIN_DENSITY = ""
CHAIN_E = "length"
CHAIN_B = "length | mul(2) | pow(0.5)"


def _unit(v) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def orbit_camera(dims, direction, distance_factor: float = 2.0, fovy_deg: float = 60.0) -> Camera:
    """Perspective camera looking at the volume centre from `distance_factor` diagonals away.

    The up vector is +z, or +y when the view direction is along +-z.
    """
    nx, ny, nz = dims
    c = np.array([nx, ny, nz], dtype=np.float64) / 2.0
    diag = math.sqrt(nx * nx + ny * ny + nz * nz)
    d = _unit(direction)
    eye = c + distance_factor * diag * d
    up = (0.0, 1.0, 0.0) if abs(d[0]) < 1e-12 and abs(d[1]) < 1e-12 else (0.0, 0.0, 1.0)
    return Camera(eye=tuple(eye), center=tuple(c), up=up, fovy_deg=fovy_deg)


def views26() -> List[tuple]:
    """The 26 neighbour directions of a cube cell, {-1,0,1}^3 without the origin."""
    out = []
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                if (i, j, k) != (0, 0, 0):
                    out.append((float(i), float(j), float(k)))
    return out


def random_tf(rng: np.random.Generator, n_points: int, alpha_max: float, grid: int = 255):
    """Piecewise-linear RGBA control points on the 1/grid lattice spanning [0, 1]."""
    if n_points < 2:
        raise ValueError("need at least two control points")
    interior = np.sort(rng.choice(np.arange(1, grid), size=n_points - 2, replace=False))
    xs = [0] + [int(i) for i in interior] + [grid]
    pts = []
    for xi in xs:
        r, g, b = rng.uniform(0.0, 1.0, size=3)
        a = rng.uniform(0.0, alpha_max)
        pts.append((xi / grid, float(r), float(g), float(b), float(a)))
    return pts


def random_clip_plane(rng: np.random.Generator, dims):
    """Plane through a point in the middle half of the volume, keeping the volume centre."""
    n = _unit(rng.standard_normal(3))
    lo = np.array(dims, dtype=np.float64) / 4.0
    q = lo + rng.uniform(0.0, 1.0, size=3) * (2.0 * lo)
    d = -float(n @ q)
    c = np.array(dims, dtype=np.float64) / 2.0
    if float(n @ c) + d < 0.0:
        n, d = -n, -d
    return (float(n[0]), float(n[1]), float(n[2]), float(d))


def plain_scalar(seed: int = 1, n: int = 64, width: int = 256, height: int = 256,
                 direction=D0) -> Scene:
    """One FP32 Gaussian-blob scalar, no guard, nearest sampling, step 0.5, one 4-point TF."""
    ss = np.random.SeedSequence(seed).spawn(2)
    dims = (n, n, n)
    field = fields.gaussian_blobs(np.random.default_rng(ss[0]), dims, guard=0, scale=n / 64.0)
    tf = random_tf(np.random.default_rng(ss[1]), 4, 0.03)
    src = make_source("density", field, guard=0, chain="", tf=tf)
    return Scene(dims=dims, sources=[src], camera=orbit_camera(dims, direction), width=width,
                 height=height, step=0.5, interpolation=0, seed=seed,
                 label=f"plain_scalar n={n} {width}x{height}")


def pic3_sources(seed: int, dims, dtype: str = "f32", guard: int = 1,
                 layout_kw: Optional[dict] = None) -> List[SourceSpec]:
    """Density, E and B sources with their chains, 8-point TFs and weights."""
    ss = np.random.SeedSequence(seed).spawn(5)
    rng_d, rng_e, rng_b, rng_tf, rng_w = (np.random.default_rng(s) for s in ss)
    lk = dict(layout_kw or {})
    dens = fields.lognormal_wake(rng_d, dims, guard)
    e = fields.divergence_free_sinusoids(rng_e, dims, guard)
    b = fields.divergence_free_sinusoids(rng_b, dims, guard)
    tfs = [random_tf(rng_tf, 8, 0.03) for _ in range(3)]
    w = rng_w.uniform(0.3, 1.0, size=3)
    out = [
        make_source("density", dens, dtype=dtype, guard=guard, chain=CHAIN_DENSITY, weight=float(w[0]),
                    tf=tfs[0], **lk),
        make_source("E", e, dtype=dtype, guard=guard, chain=CHAIN_E, weight=float(w[1]), tf=tfs[1], **lk),
        make_source("B", b, dtype=dtype, guard=guard, chain=CHAIN_B, weight=float(w[2]), tf=tfs[2], **lk),
    ]
    return out


def pic3(seed: int = 2, n: int = 256, width: int = 1920, height: int = 1080, dtype: str = "f32",
         n_clip: int = 2, direction=D0, dims=None) -> Scene:
    """Three PIConGPU-shaped sources on an n^3 grid with one guard layer, trilinear, clipped."""
    dims = tuple(dims) if dims is not None else (n, n, n)
    srcs = pic3_sources(seed, dims, dtype)
    rng_c = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[5])
    clip = [random_clip_plane(rng_c, dims) for _ in range(n_clip)]
    return Scene(dims=dims, sources=srcs, camera=orbit_camera(dims, direction), width=width,
                 height=height, step=0.5, interpolation=1, clip=clip, seed=seed,
                 label=f"pic3 {dims[0]}x{dims[1]}x{dims[2]} {dtype} {width}x{height}")


def batch64(seed: int = 4, n_jobs: int = 64, edge=(32, 192), sizes=(128, 256, 512, 1024)) -> List[Scene]:
    """Uneven sub-volumes, each a Gaussian-blob scalar with its own camera and image size."""
    out = []
    for j, s in enumerate(np.random.SeedSequence(seed).spawn(n_jobs)):
        rng = np.random.default_rng(s)
        dims = tuple(int(v) for v in rng.integers(edge[0], edge[1] + 1, size=3))
        field = fields.gaussian_blobs(rng, dims, guard=1, scale=float(np.mean(dims)) / 64.0)
        tf = random_tf(rng, 4, 0.03)
        size = int(rng.choice(np.array(sizes)))
        direction = _unit(rng.standard_normal(3))
        src = make_source("density", field, guard=1, chain="", tf=tf)
        out.append(Scene(dims=dims, sources=[src], camera=orbit_camera(dims, direction), width=size,
                         height=size, step=0.5, interpolation=1, seed=seed,
                         label=f"batch64[{j}] {dims} {size}^2"))
    return out


RESOLUTIONS = ((512, 512), (1280, 720), (1920, 1080))


@dataclasses.dataclass
class Request:
    """One steering request: a complete render description after the client's edit."""
    arrival: float                 # seconds from the start of the run
    client: int
    edit: str                      # "camera" | "tf" | "clip"
    width: int
    height: int
    direction: tuple               # camera direction from the volume centre
    tfs: List[list]                # control points per source
    tf_version: List[int]          # per source: bumps on each edit (a new table upload)
    clip: List[tuple]


def serving_requests(seed: int, dims, n_clients: int = 4, rate_per_client: float = 50.0,
                     duration: float = 60.0, base_tfs: Optional[List[list]] = None) -> List[Request]:
    """Merged Poisson request streams; each request applies one random edit to its client's view."""
    reqs = []
    for c, s in enumerate(np.random.SeedSequence(seed).spawn(n_clients)):
        rng = np.random.default_rng(s)
        direction = tuple(_unit(rng.standard_normal(3)))
        tfs = [list(t) for t in (base_tfs or [random_tf(rng, 8, 0.03) for _ in range(3)])]
        ver = [0] * len(tfs)
        clip: List[tuple] = []
        t = 0.0
        while True:
            t += rng.exponential(1.0 / rate_per_client)
            if t >= duration:
                break
            edit = ("camera", "tf", "clip")[int(rng.integers(0, 3))]
            if edit == "camera":
                direction = tuple(_unit(rng.standard_normal(3)))
            elif edit == "tf":
                k = int(rng.integers(0, len(tfs)))
                tfs = list(tfs)
                tfs[k] = random_tf(rng, 8, 0.03)
                ver = list(ver)
                ver[k] += 1
            else:
                clip = [random_clip_plane(rng, dims)]
            w, h = RESOLUTIONS[int(rng.integers(0, len(RESOLUTIONS)))]
            reqs.append(Request(arrival=t, client=c, edit=edit, width=w, height=h, direction=direction,
                                tfs=tfs, tf_version=list(ver), clip=list(clip)))
    reqs.sort(key=lambda r: (r.arrival, r.client))
    return reqs


# ---------------------------------------------------------------------------
# Small scenes for closed-form and brute-force tests
# ---------------------------------------------------------------------------

def axis_camera(dims, axis: int = 0, sign: float = 1.0, width: int = 8, height: int = 8,
                ortho_height: Optional[float] = None, distance: float = 10.0) -> Camera:
    """Orthographic camera whose rays run along +axis (sign=+1) or -axis, centred on the box."""
    c = np.array(dims, dtype=np.float64) / 2.0
    d = np.zeros(3)
    d[axis] = sign
    eye = c - d * (dims[axis] / 2.0 + distance)
    up = np.zeros(3)
    up[2 if axis != 2 else 1] = 1.0
    oh = float(ortho_height if ortho_height is not None else max(dims) * 1.5)
    return Camera(eye=tuple(eye), center=tuple(c), up=tuple(up), fovy_deg=60.0,
                  projection="orthographic", ortho_height=oh)


def constant_tf(rgb, a):
    return [(0.0, rgb[0], rgb[1], rgb[2], a), (1.0, rgb[0], rgb[1], rgb[2], a)]


def linear_alpha_tf(rgb, a_max):
    return [(0.0, rgb[0], rgb[1], rgb[2], 0.0), (1.0, rgb[0], rgb[1], rgb[2], a_max)]


def random_chain(rng: np.random.Generator, f_dim: int, max_ops: int = 4) -> str:
    """A random valid functor chain for an f_dim-component source."""
    ops = []
    dim = f_dim
    for _ in range(int(rng.integers(0, max_ops + 1))):
        kind = ("add", "mul", "pow", "length", "sum")[int(rng.integers(0, 5))]
        if kind in ("length", "sum"):
            ops.append(kind)
            dim = 1
            continue
        nargs = 1 if (dim == 1 or rng.random() < 0.5) else dim
        if kind == "pow":
            args = [float(rng.choice([0.5, 2.0, 1.5, 3.0, 1.0]) ) for _ in range(nargs)]
        elif kind == "mul":
            args = [float(np.round(rng.uniform(-2.0, 2.0), 3)) for _ in range(nargs)]
        else:
            args = [float(np.round(rng.uniform(-0.5, 0.5), 3)) for _ in range(nargs)]
        ops.append(f"{kind}({', '.join(repr(a) for a in args)})")
    return " | ".join(ops)


def random_small_scene(seed: int, max_edge: int = 8, max_px: int = 12) -> Scene:
    """A random tiny scene exercising every feature (for brute-force comparison)."""
    rng = np.random.default_rng(seed)
    dims = tuple(int(v) for v in rng.integers(2, max_edge + 1, size=3))
    n_src = int(rng.integers(1, 4))
    srcs = []
    for s in range(n_src):
        f_dim = int(rng.integers(1, 5))
        guard = int(rng.integers(0, 2))
        dtype = ("f32", "f32", "f16", "bf16")[int(rng.integers(0, 4))]
        vals = fields.uniform_random(rng, dims, guard, f_dim, -1.0, 1.5)
        layout = dict(layout=("aos", "soa")[int(rng.integers(0, 2))],
                      order=tuple(int(a) for a in rng.permutation(3)),
                      flip=tuple(bool(b) for b in rng.integers(0, 2, size=3)),
                      pitch_align=int(rng.choice([4, 64, 256])))
        tf = random_tf(rng, int(rng.integers(2, 7)), float(rng.choice([0.05, 0.3, 1.0])))
        srcs.append(make_source(f"s{s}", vals, dtype=dtype, guard=guard, chain=random_chain(rng, f_dim),
                                weight=float(rng.uniform(0.0, 1.0)), tf=tf,
                                enabled=bool(rng.random() < 0.85), **layout))
    c = np.array(dims, dtype=np.float64) / 2.0
    if rng.random() < 0.15:
        eye = rng.uniform(0.0, 1.0, size=3) * np.array(dims)      # inside the box
    else:
        eye = c + _unit(rng.standard_normal(3)) * rng.uniform(6.0, 20.0)
    center = c + rng.uniform(-1.0, 1.0, size=3)
    fwd = _unit(center - eye)
    up = _unit(rng.standard_normal(3))
    if abs(float(up @ fwd)) > 0.95:
        up = _unit(np.cross(fwd, [1.0, 0.0, 0.0]) + 0.1)
    ortho = rng.random() < 0.3
    cam = Camera(eye=tuple(eye), center=tuple(center), up=tuple(up),
                 fovy_deg=float(rng.uniform(20.0, 90.0)),
                 projection="orthographic" if ortho else "perspective",
                 ortho_height=float(rng.uniform(4.0, 14.0)))
    clip = [random_clip_plane(rng, dims) for _ in range(int(rng.integers(0, 4)))]
    return Scene(dims=dims, sources=srcs, camera=cam, width=int(rng.integers(3, max_px + 1)),
                 height=int(rng.integers(3, max_px + 1)), step=float(rng.choice([0.5, 0.3, 0.7, 1.0])),
                 interpolation=int(rng.integers(0, 2)), clip=clip,
                 ert_threshold=float(rng.choice([0.999, 0.9, 0.5, 1.0])), seed=seed,
                 label=f"random_small[{seed}]")
