"""Host-side logic of the library, checked without a GPU."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_serving_arena_allocator(tmp_path):
    """First-fit allocation never overlaps, refuses only when no free run is
    large enough, keeps its accounting, and coalesces back to one block
    (compiled with g++ under AddressSanitizer/UBSan on the host)."""
    exe = tmp_path / "arena_check"
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                           os.path.join(HERE, "arena_check.cpp"), "-o", str(exe)])
    for seed in (1, 2, 3):
        out = subprocess.run([str(exe), str(seed)], capture_output=True, text=True, timeout=120)
        assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
