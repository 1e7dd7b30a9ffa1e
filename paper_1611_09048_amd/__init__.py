"""MI355X (gfx950) volume ray caster for in situ visualization (ISAAC's per-pixel hot path).

The compute path is the HIP library libisaac_mi355x.so (C ABI in
include/isaac_mi355x.h); `binding` marshals Python arguments onto it and
`device` keeps source fields and images in torch device tensors.  There is
no CPU fallback: calls fail if the library is not built.
"""

from .binding import (ASYNC, DERIVE, DIRECT, ISO, NEAREST, NO_GRAPH, ORTHOGRAPHIC, PERSPECTIVE, TIMING, TRILINEAR,
                      VOLUME, Context, IsaacError, check_functor_chain, load, render_desc, source_desc)

__all__ = ["ASYNC", "DERIVE", "DIRECT", "ISO", "NEAREST", "NO_GRAPH", "ORTHOGRAPHIC", "PERSPECTIVE", "TIMING",
           "TRILINEAR", "VOLUME", "Context", "IsaacError", "check_functor_chain", "load", "render_desc", "source_desc"]
