"""Builds the HIP shared library libhdf.so in-tree (gfx950)."""
import concurrent.futures
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libhdf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled in every device compilation.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose=False):
    os.makedirs(LIBDIR, exist_ok=True)
    objdir = os.path.join(LIBDIR, "obj")
    os.makedirs(objdir, exist_ok=True)
    cmds = []
    for src in ("planner.cpp", "capi.cpp", "krr.cpp"):
        o = os.path.join(objdir, src + ".o")
        cmds.append((o, [HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", *COMMON, "-c",
                         os.path.join(CSRC, src), "-o", o]))
    for src in ("mf_kernels.hip", "kernels.hip", "krr_kernels.hip", "scratch.hip"):
        o = os.path.join(objdir, src + ".o")
        cmds.append((o, [HIPCC, *DEVICE_FLAGS, *COMMON, "-c", os.path.join(CSRC, src), "-o", o]))
    # the translation units are independent: compile them concurrently
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
        outs = list(ex.map(lambda c: _run(c[1]), cmds))
    if verbose:
        for out in outs:
            if out:
                print(out)
    objs = [o for o, _ in cmds]
    tmp = LIB + ".tmp"
    _run([HIPCC, *DEVICE_FLAGS, "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
