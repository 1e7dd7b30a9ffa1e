"""Autotuner for the ray-tile shape and sample schedule of each image-size class.

For every size class present in a workload it times the ray-casting kernel
(HIP events around the launch, ISAAC_TIMING) for each candidate
(wave_w, waves_x, unroll, lanes_per_ray, min_waves) and keeps the fastest.  Results are cached as JSON
keyed by device architecture, size class and a source signature (source
count, storage types, feature dimensions, interpolation), and applied with
isaac_set_tile_shape.  Tile shapes with one lane per ray produce the same
pixels bit for bit; more lanes per ray composite each row of scan points by
a scan, which changes FP32 rounding only (every setting reproduces its own
image bit for bit).
"""

from __future__ import annotations

import json
import math
import os
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

from . import binding

WAVE_W = (1, 2, 4, 8, 16, 32, 64)
WAVES_X = (1, 2, 4)
UNROLL = (1, 2)
LANES = (1, 2, 4, 8, 16, 32, 64)
MIN_WAVES = (0, 4)
POOLED = (0, 1)
DEFAULT = (8, 2, 1, 1, 0, 0)


def size_class(width: int, height: int) -> int:
    m = max(width, height)
    return min(15, max(0, math.ceil(math.log2(m)) if m > 1 else 0))


def candidates(unrolls: Sequence[int] = UNROLL, lanes: Sequence[int] = LANES, wave_ws: Sequence[int] = WAVE_W,
               waves_xs: Sequence[int] = WAVES_X, min_waves: Sequence[int] = MIN_WAVES,
               pooled: Sequence[int] = POOLED) -> List[Tuple]:
    """Valid (wave_w, waves_x, unroll, lanes_per_ray, min_waves, pooled) settings.

    The pooled schedule ignores the tile shape, so it is tried once per lane count."""
    out = []
    for g in lanes:
        for u in (unrolls if g == 1 else (1,)):
            for m in min_waves:
                if m and (g == 2 or g >= 32 or u == 2):
                    continue
                if 0 in pooled:
                    for w in wave_ws:
                        if w <= 64 // g and (w >= 8 or w == 64 // g):
                            for x in waves_xs:
                                out.append((w, x, u, g, m, 0))
                if 1 in pooled and 2 <= g <= 16 and u == 1:
                    out.append((min(8, 64 // g), 2, 1, g, m, 1))
    return out


def signature(scene) -> str:
    parts = [f"{s.dtype}x{s.f_dim}" for s in scene.sources if s.enabled]
    return f"{'tri' if scene.interpolation else 'near'}:" + ",".join(parts)


def cache_key(arch: str, cls: int, sig: str) -> str:
    return f"{arch}|{cls}|{sig}"


def load_cache(path: str) -> Dict[str, list]:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    return {k: list(v) for k, v in data.items()}


def save_cache(path: str, table: Dict[str, list]) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def pick(times: Dict[Tuple, float]) -> Tuple:
    """Fastest candidate; ties go to the earlier (smaller) shape."""
    return min(sorted(times), key=lambda c: times[c])


def time_candidate(ctx: binding.Context, jobs: Sequence[binding.RenderDesc], cls: int,
                   cand: Tuple, reps: int = 3, flags: int = 0) -> float:
    ctx.set_tile_shape(cls, *cand)
    ctx.render(list(jobs), flags)               # warm-up (and graph capture for batches)
    ctx.timing()
    for _ in range(reps):
        ctx.render(list(jobs), flags | binding.TIMING)
    ms, n = ctx.timing()
    return ms / max(n, 1)


def tune(ctx: binding.Context, jobs_by_class: Dict[int, Sequence[binding.RenderDesc]], arch: str = "gfx950",
         sig: str = "", cands: Optional[Iterable[Tuple]] = None, reps: int = 3,
         cache: Optional[Dict[str, list]] = None, flags: int = 0, log=None) -> Dict[int, Tuple]:
    """Tune each size class on its jobs; returns {class: (wave_w, waves_x, unroll, lanes_per_ray, min_waves)} and applies it."""
    cands = list(cands) if cands is not None else candidates()
    best = {}
    for cls, jobs in sorted(jobs_by_class.items()):
        key = cache_key(arch, cls, sig)
        if cache is not None and key in cache:
            best[cls] = tuple(cache[key])
            ctx.set_tile_shape(cls, *best[cls])
            continue
        times = {c: time_candidate(ctx, jobs, cls, c, reps, flags) for c in cands}
        best[cls] = pick(times)
        if log:
            log(f"autotune class {cls}: best {best[cls]} {times[best[cls]]:.4f} ms "
                f"(default {times.get(DEFAULT, float('nan')):.4f} ms)")
        ctx.set_tile_shape(cls, *best[cls])
        if cache is not None:
            cache[key] = list(best[cls])
    return best


def class_shapes(lanes: int) -> List[Tuple[int, int]]:
    """(wave_w, waves_x) tile shapes a size class can take at a given lanes-per-ray count."""
    return [(w, x) for w in WAVE_W if w <= 64 // lanes and (w >= 8 or w == 64 // lanes) for x in WAVES_X]


def refine_per_class(ctx: binding.Context, classes: Sequence[int], base: Tuple, time_batch,
                     cache: Optional[Dict[str, list]] = None, arch: str = "gfx950", sig: str = "",
                     log=None) -> Dict[int, Tuple]:
    """Tile shape per size class inside one batched launch.

    The jobs of a batch share one kernel variant (lanes per ray, unroll,
    min_waves and the schedule are common to the launch), but every job keeps
    its own tile shape, so each size class can take the (wave_w, waves_x) that
    suits its image size.  Starting from `base` for every class, each class in
    turn tries every tile shape with the other classes at their current shape,
    keeping the fastest whole-batch time (`time_batch()`, ms).  Cached per class
    under the signature `sig`."""
    shapes = {c: tuple(base) for c in classes}
    keys = {c: cache_key(arch, c, sig) for c in classes}
    if cache is not None and all(k in cache for k in keys.values()):
        for c in classes:
            shapes[c] = tuple(cache[keys[c]])
            ctx.set_tile_shape(c, *shapes[c])
        return shapes
    for c in classes:
        ctx.set_tile_shape(c, *shapes[c])
    for c in classes:
        times = {}
        for w, x in class_shapes(base[3]):
            cand = (w, x) + tuple(base[2:])
            ctx.set_tile_shape(c, *cand)
            times[cand] = time_batch()
        shapes[c] = pick(times)
        ctx.set_tile_shape(c, *shapes[c])
        if log:
            log(f"autotune batch class {c}: {shapes[c]} {times[shapes[c]]:.4f} ms "
                f"(shared shape {tuple(base)}: {times.get(tuple(base), float('nan')):.4f} ms)")
    if cache is not None:
        for c in classes:
            cache[keys[c]] = list(shapes[c])
    return shapes

