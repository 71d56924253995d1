"""Host check of the MAC's fold for primes 2^60 - delta (modarith.h,
fold30_pm): the library's own header compiled as plain C++ (tests/host_shim
stands in for the HIP runtime header) and run against exact 128-bit
arithmetic on millions of accumulator sets built as the MAC builds them,
plus every accumulator at its bound.  The primes are the three of the
N = 8192 workloads and the largest delta the fast fold accepts."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CXX = "/opt/rocm/llvm/bin/clang++" if os.path.exists("/opt/rocm/llvm/bin/clang++") else shutil.which("clang++")

PRIMES = [1152921504606830593, 1152921504606748673, 1152921504606683137, 1152921504605847553]


@pytest.fixture(scope="module")
def fold_bin(tmp_path_factory):
    if CXX is None:
        pytest.skip("no clang++ for the host build")
    out = str(tmp_path_factory.mktemp("fold") / "fold_host")
    subprocess.run([CXX, "-O2", "-std=c++17", "-I", os.path.join(HERE, "host_shim"), "-I",
                    os.path.join(ROOT, "paper_2506_11586_amd", "csrc"), os.path.join(HERE, "fold_host.cpp"), "-o", out],
                   check=True)
    return out


@pytest.mark.parametrize("q", PRIMES)
def test_fold30_pm_exact(fold_bin, q):
    delta = 2 ** 60 - q
    assert 0 < delta < 2 ** 20
    r = subprocess.run([fold_bin, str(q), str(delta), "600000"], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
