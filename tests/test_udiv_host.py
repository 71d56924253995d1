"""Host check of the tile decoders' division by invariant integers
(paper_2506_11586_amd/csrc/udiv.h): the header compiled as plain C++
(tests/host_shim stands in for the HIP runtime header) against C's division
for divisors from 1 to powers of two, their neighbours, primes and the
largest 31-bit values."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CXX = "/opt/rocm/llvm/bin/clang++" if os.path.exists("/opt/rocm/llvm/bin/clang++") else shutil.which("clang++")

DIVISORS = [1, 2, 3, 5, 6, 7, 11, 16, 17, 31, 32, 33, 48, 63, 64, 65, 96, 100, 127, 255, 256, 257, 1000, 1023, 1024,
            1025, 4095, 65535, 65536, 65537, 999983, (1 << 24) - 1, (1 << 24) + 1, (1 << 30) - 1, 1 << 30,
            (1 << 30) + 1, (1 << 31) - 1, 1 << 31]


def test_udiv_matches_division(tmp_path):
    if CXX is None:
        pytest.skip("no clang++ for the host build")
    out = str(tmp_path / "udiv_host")
    subprocess.run([CXX, "-O2", "-std=c++17", "-I", os.path.join(HERE, "host_shim"), "-I",
                    os.path.join(ROOT, "paper_2506_11586_amd", "csrc"), os.path.join(HERE, "udiv_host.cpp"), "-o", out],
                   check=True)
    r = subprocess.run([out] + [str(d) for d in DIVISORS], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
