"""The C ABI from a C99 program (tests/c/abi_slab.c): no Python between the
caller and the library.  On the CPU the program must compile against
include/isaac_mi355x.h with warnings on and link against the built library;
on the GPU it renders a constant slab and checks every pixel against the
closed form of compositing n equal samples (it exits non-zero otherwise)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "abi_slab.c")
PKG = os.path.join(ROOT, "paper_1611_09048_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(out_dir) -> str:
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    if not os.path.exists(os.path.join(PKG, "libisaac_mi355x.so")):
        pytest.skip("library not built")
    exe = os.path.join(str(out_dir), "abi_slab")
    cmd = [gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), SRC,
           "-L", PKG, "-lisaac_mi355x", "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm",
           f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}", "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    return exe


def test_c_caller_compiles_and_links(tmp_path):
    assert os.path.exists(build(tmp_path))


@pytest.mark.gpu
def test_c_caller_renders_the_closed_form(tmp_path):
    exe = build(tmp_path)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(res.stdout, res.stderr)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "with 32 scan points" in res.stdout
