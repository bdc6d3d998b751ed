"""Build the CPU-emulated library (libhdf_emu.so) under ASan/UBSan.

The product sources (capi.cpp, planner.cpp, krr.cpp, and kernels.hip,
krr_kernels.hip, mf_kernels.hip and scratch.hip through translate.py) are compiled unchanged for the host, with the device-allocation
cache off (-DHDF_ALLOC_CACHE=0: exact-size allocations keep ASan's redzones tight).  The build lands in tests/emu/_build/<hash>
and is reused while sources and flags are unchanged.
"""
import concurrent.futures
import hashlib
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2202_03655_amd", "csrc")
CXX = os.environ.get("EMU_CXX", "/opt/rocm/llvm/bin/clang++")
FLAGS = ["-std=c++17", "-g", "-O1", "-fPIC", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined", "-ftrivial-auto-var-init=pattern",
         "-DHDF_ALLOC_CACHE=0",
         "-Wno-psabi", "-Wno-unused-value", "-I", os.path.join(HERE, "shim"), "-I", CSRC]
SOURCES = [os.path.join(CSRC, f) for f in ("kernels.hip", "kernels.hpp", "capi.cpp", "planner.cpp", "planner.hpp",
                                            "krr_kernels.hip", "krr_kernels.hpp", "krr.cpp", "status.hpp",
                                            "scratch.hip", "mf_kernels.hip")] + \
          [os.path.join(ROOT, "include", "hdf.h")] + \
          [os.path.join(HERE, f) for f in ("emu_hip.h", "emu_rt.cpp", "translate.py", "build.py")]


def available():
    return os.path.exists(CXX) and os.path.exists(asan_runtime() or "")


def asan_runtime():
    if not os.path.exists(CXX):
        return None
    r = subprocess.run([CXX, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if os.path.isabs(p) else None


def build():
    h = hashlib.sha1(" ".join(FLAGS).encode())
    for s in SOURCES:
        h.update(open(s, "rb").read())
    out = os.path.join(HERE, "_build", h.hexdigest()[:12])
    lib = os.path.join(out, "libhdf_emu.so")
    if os.path.exists(lib):
        return lib
    tmp = out + ".tmp"
    shutil.rmtree(tmp, ignore_errors=True)
    os.makedirs(tmp)
    import importlib.util
    spec = importlib.util.spec_from_file_location("emu_translate", os.path.join(HERE, "translate.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    translate = mod.translate
    kern = os.path.join(tmp, "kernels_emu.cpp")
    open(kern, "w").write(translate(open(os.path.join(CSRC, "kernels.hip")).read()))
    kern2 = os.path.join(tmp, "krr_kernels_emu.cpp")
    open(kern2, "w").write(translate(open(os.path.join(CSRC, "krr_kernels.hip")).read(), "krr_kernels.hpp"))
    kern3 = os.path.join(tmp, "scratch_emu.cpp")
    open(kern3, "w").write(translate(open(os.path.join(CSRC, "scratch.hip")).read()))
    kern4 = os.path.join(tmp, "mf_kernels_emu.cpp")
    open(kern4, "w").write(translate(open(os.path.join(CSRC, "mf_kernels.hip")).read()))
    units = [kern, kern2, kern3, kern4, os.path.join(CSRC, "capi.cpp"), os.path.join(CSRC, "planner.cpp"),
             os.path.join(CSRC, "krr.cpp"), os.path.join(HERE, "emu_rt.cpp")]

    def compile_one(src):
        obj = os.path.join(tmp, os.path.basename(src) + ".o")
        r = subprocess.run([CXX, *FLAGS, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError(f"emulator build failed for {src}:\n{r.stderr[-4000:]}")
        return obj
    with concurrent.futures.ThreadPoolExecutor(len(units)) as ex:
        objs = list(ex.map(compile_one, units))
    r = subprocess.run([CXX, "-shared", "-fsanitize=address,undefined", *objs, "-o", os.path.join(tmp, "libhdf_emu.so")],
                       capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError("emulator link failed:\n" + r.stderr[-4000:])
    shutil.rmtree(out, ignore_errors=True)
    os.replace(tmp, out)
    return lib


if __name__ == "__main__":
    print(build())
