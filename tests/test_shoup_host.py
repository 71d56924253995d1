"""Host check of the inverse transform's twiddle product (modarith.h,
mul_shoup_2q) and its lazy bound: the library's own header compiled as plain
C++ (tests/host_shim stands in for the HIP runtime header) and run against
exact 128-bit arithmetic on random and extreme operands, for the three
primes of the N = 8192 workloads, a 50-bit prime and the largest prime
below 2^60 (the bound's worst case: 6q closest to 2^62.6)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CXX = "/opt/rocm/llvm/bin/clang++" if os.path.exists("/opt/rocm/llvm/bin/clang++") else shutil.which("clang++")

PRIMES = [1152921504606830593, 1152921504606748673, 1152921504606683137, 1125899906826241, 1152921504606846577]


@pytest.fixture(scope="module")
def shoup_bin(tmp_path_factory):
    if CXX is None:
        pytest.skip("no clang++ for the host build")
    out = str(tmp_path_factory.mktemp("shoup") / "shoup_host")
    subprocess.run([CXX, "-O2", "-std=c++17", "-I", os.path.join(HERE, "host_shim"), "-I",
                    os.path.join(ROOT, "paper_2506_11586_amd", "csrc"), os.path.join(HERE, "shoup_host.cpp"), "-o", out],
                   check=True)
    return out


@pytest.mark.parametrize("q", PRIMES)
def test_mul_shoup_2q_and_inverse_bound(shoup_bin, q):
    r = subprocess.run([shoup_bin, str(q), "400000"], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
