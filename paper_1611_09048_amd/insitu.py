"""In situ rendering of a running simulation on the same device and stream.

The library visualizes fields that a simulation keeps in device memory, read
in place through their accessors (zero copy, Sec. 3.1); the simulation and
the renderer share the accelerator, so the simulation pauses while a frame
is rendered, and a frame may be rendered only every n-th time step when a
step is short (Sec. 3.6, the Petri net of the render cycle).  Before each
render the library calls every source's update() (Sec. 3.2), which here
derives a secondary field into a scratch buffer; that source is declared
non-persistent, so the library copies it before the next source's update
could reuse the buffer.

`FieldSimulation` stands in for the host application (the paper couples the
renderer to a particle-in-cell code, Sec. 4): an electric and a magnetic
field advanced by a leapfrog curl update on a collocated grid with central
differences, and a density relaxed by diffusion, all with one periodic guard
layer.  Its arithmetic is plain torch on the device; it is the application,
not part of the rendering path.  The secondary field is the curl of B (a
current-density-like quantity), computed in update().
"""

from __future__ import annotations

import ctypes
import dataclasses
import time
from typing import List, Optional

import numpy as np
import torch

from . import binding


class FieldSimulation:
    """E, B (3 x FP32, interleaved) and a density (FP32) on an n^3 grid with one guard layer."""

    def __init__(self, n: int = 128, seed: int = 7, device: str = "cuda", dt: float = 0.2,
                 diffusion: float = 0.05):
        from scenes import fields
        ss = np.random.SeedSequence(seed).spawn(3)
        rng_e, rng_b, rng_d = (np.random.default_rng(s) for s in ss)
        dims = (n, n, n)
        self.n, self.dt, self.kappa = n, dt, diffusion
        self.E = torch.from_numpy(fields.divergence_free_sinusoids(rng_e, dims, 1)).to(device).contiguous()
        self.B = torch.from_numpy(fields.divergence_free_sinusoids(rng_b, dims, 1)).to(device).contiguous()
        self.rho = torch.from_numpy(fields.lognormal_wake(rng_d, dims, 1)).to(device).contiguous()
        self.J = torch.zeros_like(self.E)          # scratch of the secondary field
        self.steps = 0

    @staticmethod
    def _curl(F: torch.Tensor) -> torch.Tensor:
        """Central-difference curl of an interleaved [z][y][x][3] field, on the interior."""
        def d(axis, c):
            if axis == 0:
                return (F[1:-1, 1:-1, 2:, c] - F[1:-1, 1:-1, :-2, c]) * 0.5
            if axis == 1:
                return (F[1:-1, 2:, 1:-1, c] - F[1:-1, :-2, 1:-1, c]) * 0.5
            return (F[2:, 1:-1, 1:-1, c] - F[:-2, 1:-1, 1:-1, c]) * 0.5
        return torch.stack([d(1, 2) - d(2, 1), d(2, 0) - d(0, 2), d(0, 1) - d(1, 0)], dim=-1)

    @staticmethod
    def _fill_guards(F: torch.Tensor) -> None:
        """Periodic guard layers (edges and corners through the sequential axes)."""
        for axis in (0, 1, 2):
            F.narrow(axis, 0, 1).copy_(F.narrow(axis, F.shape[axis] - 2, 1))
            F.narrow(axis, F.shape[axis] - 1, 1).copy_(F.narrow(axis, 1, 1))

    def step(self) -> None:
        inner = (slice(1, -1),) * 3
        self.B[inner] -= self.dt * self._curl(self.E)
        self._fill_guards(self.B)
        self.E[inner] += self.dt * self._curl(self.B)
        self._fill_guards(self.E)
        r = self.rho
        lap = (r[1:-1, 1:-1, 2:] + r[1:-1, 1:-1, :-2] + r[1:-1, 2:, 1:-1] + r[1:-1, :-2, 1:-1] +
               r[2:, 1:-1, 1:-1] + r[:-2, 1:-1, 1:-1] - 6.0 * r[1:-1, 1:-1, 1:-1])
        r[inner] += self.kappa * lap
        self._fill_guards(r)
        self.steps += 1

    def derive_current(self) -> None:
        """The secondary field: curl B into the scratch buffer, guards periodic."""
        self.J[(slice(1, -1),) * 3] = self._curl(self.B)
        self._fill_guards(self.J)


def _accessor(t: torch.Tensor, f_dim: int):
    """(per-component device addresses of interior voxel (0,0,0), byte strides x, y, z)."""
    es = t.element_size()
    s = t.stride()
    stride = (s[2] * es, s[1] * es, s[0] * es)
    base = t.data_ptr() + (s[0] + s[1] + s[2]) * es
    return [base + c * es for c in range(f_dim)], stride


@dataclasses.dataclass
class InSituStats:
    steps: int
    frames: int
    every: int
    total_s: float
    render_s: float

    @property
    def overhead(self) -> float:
        """Share of the run spent rendering (the paper's measure, Sec. 4.1)."""
        return self.render_s / self.total_s if self.total_s > 0 else 0.0


class InSituRenderer:
    """Registers the simulation's fields as sources and renders every n-th step.

    The context must enqueue on the stream the simulation runs on (torch's
    current stream, the binding's default), so a render waits for the step
    before it and the next step waits for the render."""

    def __init__(self, ctx: binding.Context, sim: FieldSimulation, volume_id: int = 0,
                 tfs: Optional[List[list]] = None, weights=(0.6, 0.8, 0.9),
                 chains=("", "length", "length | mul(2) | pow(0.5)")):
        self.ctx, self.sim, self.vid = ctx, sim, volume_id
        self.updates: List[tuple] = []
        self._cb = binding.UPDATE_FN(self._update)
        n = sim.n
        descs = []
        for name, t, f_dim, persistent, chain, w in (("density", sim.rho, 1, True, chains[0], weights[0]),
                                                      ("E", sim.E, 3, True, chains[1], weights[1]),
                                                      ("J", sim.J, 3, False, chains[2], weights[2])):
            comp, stride = _accessor(t, f_dim)
            d = binding.source_desc(name=name, f_dim=f_dim, dtype="f32", comp=comp, stride=stride, guard=1,
                                    chain=chain, weight=w, persistent=persistent)
            d.update = self._cb
            d.user = len(descs)
            descs.append(d)
        ctx.set_sources(volume_id, (n, n, n), descs)
        if tfs is None:
            from scenes import configs
            rng = np.random.default_rng(np.random.SeedSequence(11).spawn(1)[0])
            tfs = [configs.random_tf(rng, 8, 0.03) for _ in range(3)]
        self.tfs = tfs
        self.handles = [ctx.set_transfer(volume_id, s, tf) for s, tf in enumerate(tfs)]

    def _update(self, user, enabled, pointer) -> None:
        # called by the library before each render, once per source, in source order
        src = int(user or 0)
        self.updates.append((src, int(enabled)))
        if src == 2 and enabled:
            # enqueued on torch's current stream, which the context shares (its default),
            # so the library's copy of this source, next on that stream, reads the result
            self.sim.derive_current()

    def render(self, desc: binding.RenderDesc) -> None:
        self.ctx.render([desc])

    def run(self, steps: int, every: int, make_desc, sync=torch.cuda.synchronize) -> InSituStats:
        """Advance `steps` steps, rendering after every `every`-th (0: never)."""
        render_s = 0.0
        frames = 0
        sync()
        t0 = time.perf_counter()
        for k in range(1, steps + 1):
            self.sim.step()
            if every and k % every == 0:
                sync()
                r0 = time.perf_counter()
                self.render(make_desc(frames))
                render_s += time.perf_counter() - r0
                frames += 1
        sync()
        return InSituStats(steps=steps, frames=frames, every=every, total_s=time.perf_counter() - t0,
                           render_s=render_s)
