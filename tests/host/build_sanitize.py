"""Build tests/host/abi_sanitize: the library's host code (engine.cpp,
serve.cpp) compiled with AddressSanitizer and UndefinedBehaviorSanitizer on
the host pass only (every -fsanitize= behind -Xarch_host: the GPU code is
built as in the product), linked with the product's kernel objects and the
driver program abi_sanitize.cpp.  Test infrastructure: run by the GPU test
tests/test_gpu_sanitize.py, built here on the CPU by __graft_entry__.build()
after the library (whose kernel objects it reuses)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1709_06924_amd", "csrc")
OBJ = os.path.join(ROOT, "paper_1709_06924_amd", "_build")
EXE = os.path.join(HERE, "abi_sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
KERNEL_OBJS = ["grid.hip.o", "cells.hip.o", "lbfgs.hip.o", "mesh.hip.o", "round.hip.o"]
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def build():
    out = os.path.join(HERE, "_san")
    os.makedirs(out, exist_ok=True)
    common = ["-O1", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
              "-Wno-unused-result"]
    objs = []
    for src in ("engine.cpp", "serve.cpp"):
        obj = os.path.join(out, src + ".o")
        subprocess.run([HIPCC] + common + HOST_SAN + ["-x", "hip", "-c", os.path.join(CSRC, src),
                                                     "-o", obj],
                       check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        objs.append(obj)
    drv = os.path.join(out, "abi_sanitize.o")
    subprocess.run([CLANG, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-c", os.path.join(HERE, "abi_sanitize.cpp"),
                    "-o", drv], check=True)
    kern = [os.path.join(OBJ, o) for o in KERNEL_OBJS]
    tmp = EXE + ".tmp%d" % os.getpid()
    subprocess.run([CLANG, "-fsanitize=address,undefined", "-o", tmp, drv] + objs + kern +
                   ["-L/opt/rocm/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx", "-lpthread",
                    "-Wl,-rpath,/opt/rocm/lib"], check=True)
    os.replace(tmp, EXE)
    return EXE


if __name__ == "__main__":
    print(build())
