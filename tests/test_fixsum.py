"""The order-independent fixed-point summation of the adjoint's scattered
probe-velocity adjoints, against 128-bit integer and long double sums on the
host: compiled from the library's internal header with hipcc."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_13726_amd", "csrc")


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not found")
def test_fixed_point_sum_is_order_independent_and_accurate(tmp_path):
    exe = tmp_path / "fixsum_check"
    subprocess.run(["hipcc", "-O2", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "native", "fixsum_check.cpp"),
                    "-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "failures 0" in r.stdout
