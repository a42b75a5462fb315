"""The quotient by an invariant divisor (multiply-high and shifts) that the
sweep kernels use for their tile order, against plain integer division on
the host: compiled from the library's internal header with hipcc."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_13726_amd", "csrc")


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not found")
def test_invariant_division_matches_plain_division(tmp_path):
    exe = tmp_path / "udiv_check"
    subprocess.run(["hipcc", "-O2", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "native", "udiv_check.cpp"),
                    "-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "mismatches 0" in r.stdout
