"""The host planner under AddressSanitizer and UBSan, and ThreadSanitizer (g++, host code only):
table sizes at the edges, the core quadrature, the Jacobi eigen/SVD routines
and both compression routes; the SVD reproduces a rectangular matrix."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("sanitizers", ["address,undefined", "thread"])
def test_planner_under_sanitizers(tmp_path, sanitizers):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "planner_san"
    csrc = os.path.join(ROOT, "paper_2202_03655_amd", "csrc")
    r = subprocess.run([gxx, "-O1", "-g", "-std=c++17", f"-fsanitize={sanitizers}", "-fno-sanitize-recover",
                        "-I", csrc, os.path.join(ROOT, "tests", "native", "planner_asan_main.cpp"),
                        os.path.join(csrc, "planner.cpp"), "-o", str(exe), "-lpthread"],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    r = subprocess.run([str(exe)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout


# The placement of the pass-1 wave items is built twice: with the library's own host compiler and
# optimisation level (hipcc -O3; an earlier form of its capacity count, a nested increment loop over
# compile-time constants, gave wrong capacities there with the loop vectoriser on and right ones
# under the sanitizers) and under the sanitizers.
PLACEMENT_BUILDS = {
    "hipcc_O3": ["/opt/rocm/bin/hipcc", "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-O3"],
    "gxx_sanitizers": ["g++", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover"],
}


@pytest.mark.parametrize("build", list(PLACEMENT_BUILDS))
def test_wave_item_placement(tmp_path, build):
    cmd = PLACEMENT_BUILDS[build]
    if shutil.which(cmd[0]) is None and not os.path.exists(cmd[0]):
        pytest.skip(f"{cmd[0]} not available")
    exe = tmp_path / f"placement_{build}"
    csrc = os.path.join(ROOT, "paper_2202_03655_amd", "csrc")
    r = subprocess.run([*cmd, "-std=c++17", "-I", csrc, os.path.join(ROOT, "tests", "native", "placement_main.cpp"),
                        os.path.join(csrc, "planner.cpp"), "-o", str(exe)],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    r = subprocess.run([str(exe)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout
