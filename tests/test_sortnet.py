"""The comparator networks the kernels sort with (csrc/sortnet.h), built and
checked on the host: 0-1 principle exhaustively for N <= 20, random inputs
with ties against std::sort for N = 1..64."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2109_03296_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_sorting_networks(tmp_path):
    exe = tmp_path / "sortnet_check"
    subprocess.run(["g++", "-std=c++17", "-O2", f"-I{CSRC}", "-o", str(exe),
                    os.path.join(HERE, "native", "sortnet_check.cpp")], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    lines = res.stdout.split("\n")
    assert res.returncode == 0, [l for l in lines if "FAIL" in l]
    assert sum(1 for l in lines if l.endswith(" ok")) == 64
    ops = {int(l.split()[0]): int(l.split()[1]) for l in lines if l.strip()}
    assert ops[1] == 0 and ops[2] == 1 and ops[3] == 1   # one 3-sorter
