"""Seeded synthetic inputs for the ISAAC volume ray caster.

This package is shared by the GPU library's tests/benchmark and by the CPU
oracle's tests.  It only *produces inputs*: simulation-shaped fields stored in
strided, guarded, padded device-style layouts, transfer-function control
points, functor-chain strings, cameras, clipping planes and request streams.
None of the ray-casting arithmetic (ray generation, sampling, functor
evaluation, classification, compositing) lives here.
"""

from .layout import (DTYPE_SIZE, Camera, SourceSpec, Scene, make_source, store_field,
                     logical_values, relayout, f32_to_bf16_bits, bf16_bits_to_f32)
from . import fields, configs

__all__ = ["DTYPE_SIZE", "Camera", "SourceSpec", "Scene", "make_source", "store_field", "logical_values",
           "relayout", "f32_to_bf16_bits", "bf16_bits_to_f32", "fields", "configs"]
