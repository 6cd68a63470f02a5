"""Host checks of the server's workspace arena (paper_1408_1664_amd/csrc/
bn_arena.h): block rounding, carving and coalescing, best fit, the byte
limit, release of empty chunks, and allocation failures, over a counting
host allocator (tests/native/arena_check.cpp, built with g++ here)."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_arena_checks():
    src = os.path.join(HERE, "native", "arena_check.cpp")
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "arena_check")
        subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-fsanitize=address,undefined",
                        "-o", exe, src], check=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "FAIL" not in r.stdout
    assert r.stdout.count("ok  ") >= 18
