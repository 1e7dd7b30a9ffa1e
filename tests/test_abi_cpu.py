"""CPU checks of the C ABI: exports, struct layouts, host-only chain parsing, error paths.

No GPU is used: the library is loaded but no device call is made except the
init path, which must fail cleanly when no device is visible.
"""

import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_1611_09048_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "isaac_mi355x.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(isaac_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = binding.load()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(binding.EXPORTS) == names
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (isaac_\w+)", out))
    assert set(names) <= exported


def test_struct_layouts_match_the_header():
    """Compile the header with gcc and compare sizeof/offsetof with the ctypes mirrors."""
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "isaac_mi355x.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("isaac_init_desc %zu\n", sizeof(isaac_init_desc));
  printf("isaac_source_desc %zu\n", sizeof(isaac_source_desc));
  printf("isaac_tf_point %zu\n", sizeof(isaac_tf_point));
  printf("isaac_clip_plane %zu\n", sizeof(isaac_clip_plane));
  printf("isaac_render_desc %zu\n", sizeof(isaac_render_desc));
  P(isaac_source_desc, comp) P(isaac_source_desc, stride) P(isaac_source_desc, functor_chain)
  P(isaac_source_desc, weight) P(isaac_source_desc, update) P(isaac_source_desc, user)
  P(isaac_render_desc, eye) P(isaac_render_desc, step) P(isaac_render_desc, clip)
  P(isaac_render_desc, ert_threshold) P(isaac_render_desc, out_rgba) P(isaac_render_desc, update_pointer)
  P(isaac_render_desc, brick_origin) P(isaac_render_desc, out_depth) P(isaac_render_desc, mode)
  P(isaac_render_desc, iso_values)
  P(isaac_init_desc, mem_budget_bytes) P(isaac_init_desc, flags)
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "l")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(line.rsplit(" ", 1) for line in lines if line)
    mirrors = {"isaac_init_desc": binding.InitDesc, "isaac_source_desc": binding.SourceDesc,
               "isaac_tf_point": binding.TfPoint, "isaac_clip_plane": binding.ClipPlane,
               "isaac_render_desc": binding.RenderDesc}
    for name, cls in mirrors.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
    for key, val in got.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(mirrors[t], f).offset == int(val), key


def test_functor_chain_parser():
    # the paper's examples (Sec. 3.3)
    assert binding.check_functor_chain("mul(2,3,4) | add(1) | length", 3) == (1, 3)
    assert binding.check_functor_chain("mul(0,1,0) | sum", 3) == (1, 2)
    assert binding.check_functor_chain("", 3) == (3, 0)
    assert binding.check_functor_chain("mul(2,3,4) | add(1)", 3) == (3, 2)
    # host simplification: exact identities are dropped, pow(0.5)/pow(2) rewritten
    assert binding.check_functor_chain("length | mul(2) | pow(0.5)", 3) == (1, 3)
    assert binding.check_functor_chain("mul(1) | add(0) | pow(1)", 2) == (2, 0)
    assert binding.check_functor_chain("mul(1,1,1,1) | add(0,0,0,0)", 4) == (4, 0)
    assert binding.check_functor_chain("  length  |  sum ", 4) == (1, 2)
    for bad, f in (("foo", 1), ("add(1,2)", 3), ("length(2)", 3), ("add()", 1), ("mul(1) |", 1),
                   ("add(1 2)", 1), ("sum | add(1,2)", 2), (" | ".join(["add(1)"] * 9), 1), ("add(1,)", 1),
                   ("length", 5), ("| length", 1), ("add(x)", 1)):
        with pytest.raises(binding.IsaacError) as e:
            binding.check_functor_chain(bad, f)
        assert e.value.code == -2, bad


def test_chain_acceptance_matches_oracle():
    """The library's parser and the oracle's accept exactly the same chains."""
    rng = np.random.default_rng(3)
    from scenes import configs
    pieces = ["add(1)", "mul(2,3)", "pow(0.5)", "length", "sum", "mul(1,2,3)", "add(1,2,3,4)", "foo", "add()",
              "sum(1)", "pow(2)"]
    for _ in range(400):
        f_dim = int(rng.integers(1, 5))
        if rng.random() < 0.5:
            chain = configs.random_chain(rng, f_dim)
        else:
            chain = " | ".join(rng.choice(pieces, size=int(rng.integers(1, 5))))
        try:
            oracle.chain_eval(chain, f_dim, [0.5, 0.5, 0.5, 0.5])
            ok_oracle = True
        except ValueError:
            ok_oracle = False
        try:
            binding.check_functor_chain(chain, f_dim)
            ok_lib = True
        except binding.IsaacError:
            ok_lib = False
        assert ok_oracle == ok_lib, (chain, f_dim)


def test_init_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(binding.IsaacError) as e:
        binding.Context(device=0)
    assert e.value.code in (-7, -1)
