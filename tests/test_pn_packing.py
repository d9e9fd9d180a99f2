"""The pn kernel's gather lists, read from the tables libfotci builds on the
host, satisfy the invariants its read-modify-write order relies on (every
jump once, chunks per lane ending in a flush, no two chunks of a destination
flushing in one pair of rounds): tests/native/pack_check.cpp, built with g++
against the library, no device needed."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1801_08432_amd")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(os.path.join(PKG, "libfotci.so")),
                    reason="g++ or the built library missing")
@pytest.mark.parametrize("Z,N", [(2, 2), (3, 4), (4, 4), (5, 5)])
def test_gather_list_invariants(tmp_path, Z, N):
    exe = str(tmp_path / "pack_check")
    cmd = ["g++", "-std=c++17", "-O2", "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           os.path.join(ROOT, "tests", "native", "pack_check.cpp"), "-o", exe, "-L", PKG, "-lfotci",
           "-Wl,-rpath," + PKG]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([exe, str(Z), str(N)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert " 0 violations" in r.stdout
