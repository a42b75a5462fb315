"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
code, g++) and driven through its C interface on a small case that reaches
every phase: no report, normal exit."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    cmd = ["g++", "-O1", "-g", "-fopenmp", "-std=c++17", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", os.path.join(ORACLE, "hlbm_oracle.cpp"),
           os.path.join(ORACLE, "hlbm_oracle_adjoint.cpp"), os.path.join(ROOT, "tests", "native", "oracle_sanitize.cpp"),
           "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout, r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "done" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
