"""Compile the HIP library for gfx950 into the package directory.

    python -m paper_1611_09048_amd.build [--asm DIR]

Produces paper_1611_09048_amd/libisaac_mi355x.so from csrc/ with hipcc.
Packed FP32 instructions are disabled for all device code.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libisaac_mi355x.so")
SOURCES = ["raycast.hip", "jpeg.hip", "jpeg_tables.cpp", "host_logic.cpp", "isaac_api.cpp"]
ARCH = "gfx950"

DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build(verbose: bool = False, asm_dir: str | None = None) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-command-line-argument", "-Wno-unused-value", *DEVICE_FLAGS,
           "-I", os.path.join(ROOT, "include"), *srcs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(line for line in (res.stdout + res.stderr).splitlines()
                    if "packed-fp32-ops" not in line)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out.strip():
        print(out)
    os.replace(tmp, LIB)
    if asm_dir:
        dump_asm(asm_dir)
    return LIB


def dump_asm(out_dir: str) -> str:
    """Device assembly of the kernels (for reading register use and instruction mix)."""
    os.makedirs(out_dir, exist_ok=True)
    out = os.path.join(out_dir, "raycast.s")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-S", "--cuda-device-only",
           "-Wno-unused-command-line-argument", *DEVICE_FLAGS, "-I", os.path.join(ROOT, "include"),
           os.path.join(CSRC, "raycast.hip"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


if __name__ == "__main__":
    asm = None
    if "--asm" in sys.argv:
        asm = sys.argv[sys.argv.index("--asm") + 1]
    print(build(verbose=True, asm_dir=asm))
