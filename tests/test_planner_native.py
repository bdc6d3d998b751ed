"""The host planner under AddressSanitizer and UBSan (g++, host code only):
table sizes at the edges, the core quadrature, the Jacobi eigen/SVD routines
and both compression routes; the SVD reproduces a rectangular matrix."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_planner_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "planner_asan"
    csrc = os.path.join(ROOT, "paper_2202_03655_amd", "csrc")
    r = subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover",
                        "-I", csrc, os.path.join(ROOT, "tests", "native", "planner_asan_main.cpp"),
                        os.path.join(csrc, "planner.cpp"), "-o", str(exe)],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    r = subprocess.run([str(exe)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout
