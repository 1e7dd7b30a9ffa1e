"""FP64 CPU oracle of the ISAAC volume ray caster.

TEST INFRASTRUCTURE ONLY.  Imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark; the GPU library never imports, links or
calls anything here.

  isaac_oracle.c  the single-threaded FP64 renderer (C, built to liboracle.so)
  oracle.py       ctypes marshalling of a scenes.Scene into the C structs
  brute.py        an independent pure-Python per-sample loop for tiny grids

Parity unpinned: none of the readings the paper leaves open (cell-centred
samples, the half-step grid anchored at the box entry, the order of functor
chain and interpolation, premultiplied weighted mixing of sources, the
early-termination threshold) can be checked against a value the paper prints;
they are pinned by closed forms and brute force in tests/.
"""

from .oracle import build, load, render, render_pixels, chain_eval, tf_table, ray, encode_rgba8  # noqa: F401
