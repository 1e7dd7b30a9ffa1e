"""The library's host-only logic (functor-chain compiler, transfer-table bake,
camera basis, screen rectangle: csrc/host_logic.cpp) under AddressSanitizer
and UndefinedBehaviorSanitizer on the CPU: tests/c/host_fuzz.cpp feeds it
seeded random and hostile inputs (malformed and overlong chains, NaN/inf and
unsorted transfer points, degenerate cameras) and checks the invariants of
every accepted input; any sanitizer report aborts the run."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_logic_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_fuzz")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-Wall", "-Wextra", "-Werror",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1611_09048_amd", "csrc"),
           os.path.join(ROOT, "tests", "c", "host_fuzz.cpp"),
           os.path.join(ROOT, "paper_1611_09048_amd", "csrc", "host_logic.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "host fuzz: 0 failures" in res.stdout
