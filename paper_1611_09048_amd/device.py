"""Device-memory helpers (torch is used only to own device buffers and streams).

upload_volume() copies a scene's raw source bytes into device tensors as
they are laid out on the host (no re-layout) and describes them to the
library by address and byte strides; render_job() fills one render
descriptor for a scene's camera and settings.  Scene objects are duck-typed:
anything with the attributes of scenes.Scene / scenes.SourceSpec works.
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import torch

from . import binding


@dataclasses.dataclass
class DeviceVolume:
    volume_id: int
    dims: tuple
    tensors: list                 # device buffers holding the source bytes
    descs: list                   # SourceDesc structs as passed to the library
    tf_handles: List[int]

    def nbytes(self) -> int:
        return int(sum(t.numel() * t.element_size() for t in self.tensors))


def upload_source_bytes(src, device) -> tuple:
    """(device tensors, component addresses) for one source."""
    tensors = [torch.from_numpy(np.ascontiguousarray(b)).to(device) for b in src.buffers]
    comp = [tensors[bi].data_ptr() + int(off) for bi, off in src.comp]
    return tensors, comp


def upload_volume(ctx: binding.Context, scene, volume_id: int = 0, device: str = "cuda",
                  update=None) -> DeviceVolume:
    tensors, descs, handles = [], [], []
    for s in scene.sources:
        t, comp = upload_source_bytes(s, device)
        tensors.extend(t)
        descs.append(binding.source_desc(name=s.name, f_dim=s.f_dim, dtype=s.dtype, comp=comp, stride=s.strides,
                                         guard=s.guard, chain=s.chain, weight=s.weight, enabled=s.enabled,
                                         persistent=s.persistent, update=update))
    torch.cuda.synchronize()
    ctx.set_sources(volume_id, scene.dims, descs)
    for k, s in enumerate(scene.sources):
        handles.append(ctx.set_transfer(volume_id, k, s.tf))
    return DeviceVolume(volume_id, tuple(scene.dims), tensors, descs, handles)


def render_job(scene, volume_id: int, out: torch.Tensor, samples: Optional[torch.Tensor] = None,
               **overrides) -> binding.RenderDesc:
    """Descriptor rendering `scene` (camera, image size, step, interpolation, clip, threshold) into `out`."""
    cam = scene.camera
    kw = dict(volume_id=volume_id, width=scene.width, height=scene.height, eye=cam.eye, center=cam.center,
              up=cam.up, fovy_deg=cam.fovy_deg,
              projection=binding.ORTHOGRAPHIC if cam.projection == "orthographic" else binding.PERSPECTIVE,
              ortho_height=cam.ortho_height, step=scene.step, interpolation=scene.interpolation, clip=scene.clip,
              ert_threshold=float(scene.ert_threshold), out_rgba=out.data_ptr(),
              out_samples=samples.data_ptr() if samples is not None else 0)
    if scene.mode == "iso":
        kw.update(mode=binding.ISO, iso_values=[s.iso for s in scene.sources])
    kw.update(overrides)
    return binding.render_desc(**kw)


def new_image(scene, device: str = "cuda", fill: float = float("nan")) -> torch.Tensor:
    return torch.full((scene.height, scene.width, 4), fill, dtype=torch.float32, device=device)


def new_counts(scene, device: str = "cuda") -> torch.Tensor:
    return torch.full((scene.height, scene.width), -1, dtype=torch.int32, device=device)


def render_scene(ctx: binding.Context, scene, volume_id: int = 0, count: bool = True, flags: int = 0,
                 device: str = "cuda", **overrides):
    """Upload, render once, return (image, counts) as host numpy arrays (for tests)."""
    vol = upload_volume(ctx, scene, volume_id, device)
    img = new_image(scene, device)
    cnt = new_counts(scene, device) if count else None
    ctx.render([render_job(scene, volume_id, img, cnt, **overrides)], flags)
    torch.cuda.synchronize()
    out = img.cpu().numpy(), (cnt.cpu().numpy() if cnt is not None else None)
    del vol
    return out
