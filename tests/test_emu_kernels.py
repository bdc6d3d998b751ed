"""The HIP kernels and the C ABI on a CPU emulation of the device, under ASan/UBSan.

A memory-safety net for the device path, not a parity claim for it (the
GPU tests run the real library on the device).  tests/emu/translate.py
rewrites kernels.hip, krr_kernels.hip, mf_kernels.hip and scratch.hip
mechanically into C++ (launches,
__shared__ variables, the dynamic LDS array); tests/emu/emu_rt.cpp runs every
HIP thread as a fiber with __syncthreads, __syncthreads_count, lane shuffles
and the 16x16x4 MFMA as collectives, and implements the HIP runtime calls of
capi.cpp and krr.cpp on host memory.  capi.cpp, krr.cpp and planner.cpp are
compiled unchanged.  tests/emu/run_cases.py
drives the Python binding (device tensors in guarded host memory) and compares
every result with the oracle.

Two runs: (1) pointer provenance, guard regions flush after every buffer and
input/output tensor, NaN-filled device memory and LDS, random thread order;
(2) ASan redzones, garbage-filled memory, reverse thread order.  Locals are
pattern-initialised in both (-ftrivial-auto-var-init=pattern).  Any
out-of-bounds access, use after free, misaligned vector access, host pointer
passed to a kernel, divergent barrier or partial-wave MFMA aborts the run.
"""
import importlib.util
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("emu_build", os.path.join(HERE, "emu", "build.py"))
emu_build = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(emu_build)

pytestmark = pytest.mark.skipif(not emu_build.available(), reason="clang++ with the ASan runtime not found")

MODES = {
    "provenance_guard_nan_random": dict(EMU_STRICT="1", EMU_GUARD="1", EMU_FILL="0xff", EMU_ORDER="2"),
    "redzones_garbage_reverse": dict(EMU_FILL="0xbe", EMU_ORDER="1"),
}


@pytest.fixture(scope="module")
def emu_lib():
    return emu_build.build()


@pytest.mark.parametrize("mode", list(MODES))
def test_kernels_on_emulated_device(emu_lib, mode):
    env = dict(os.environ, LD_PRELOAD=emu_build.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", EMU_STACK_KB="64", **MODES[mode])
    r = subprocess.run([sys.executable, os.path.join(HERE, "emu", "run_cases.py"), emu_lib],
                       env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + "\n" + "\n".join(l for l in r.stderr.splitlines() if "ASan doesn't fully" not in l)
    assert r.returncode == 0, out[-8000:]
    assert "FAIL" not in r.stdout and r.stdout.count("ok  ") >= 40, out[-4000:]
