"""Build the test-side CPU executor of the HIP kernels (tests/emu/libgzemu.so).

The kernel and host sources of the device path are compiled for the CPU
against tests/emu/include/hip/hip_runtime.h, a stand-in that runs every GPU
thread as a fiber with lockstep wave intrinsics.  Test use only.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1905_07224_amd", "csrc")
LIB = os.path.join(HERE, "libgzemu.so")
# stage2_diff.cpp includes gz_kernels.hip (one translation unit for the kernels)
SRCS = [os.path.join(HERE, "stage2_diff.cpp"), os.path.join(CSRC, "gz_dna.hip"), os.path.join(CSRC, "gz_api.cpp"),
        os.path.join(CSRC, "gz_serve.cpp"), os.path.join(HERE, "emu_rt.cpp")]
CXX = "/opt/rocm/lib/llvm/bin/clang++" if os.path.exists("/opt/rocm/lib/llvm/bin/clang++") else "clang++"


def build(opt="-O1", extra=()):
    deps = SRCS + [os.path.join(CSRC, "gz_kernels.hip"), os.path.join(HERE, "include", "hip", "hip_runtime.h")] + [
        os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    if os.path.exists(LIB) and os.path.getmtime(LIB) >= max(os.path.getmtime(d) for d in deps) and not extra:
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [CXX, "-std=c++17", opt, "-g", "-fPIC", "-shared", "-Wno-unused-function",
           "-I", os.path.join(HERE, "include"), "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-DGZ_GLOBAL=", "-DGZ_WRITELANE=__builtin_amdgcn_writelane", "-x", "c++"] + SRCS + list(extra) + ["-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
