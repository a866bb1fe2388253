"""Test infrastructure: build ``tests/emu/_build/libvpm_emu.so``, the rollout
library's sources compiled for the CPU against the emulation header in
``tests/emu/hip`` (see its header comment). Only the CPU tests use it."""
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2509_16079_amd", "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libvpm_emu.so")
FILES = ["host.cpp", "sampling.cpp", "api.hip", "rollout.hip", "solve_mppi.hip", "policy.hip",
         "replan.hip", "plate_system.cpp", "host_common.h", "vpm_internal.h", "wave_ops.h"]


def build():
    src_dir = os.path.join(OUT_DIR, "src")
    os.makedirs(src_dir, exist_ok=True)
    for f in FILES:
        s = open(os.path.join(CSRC, f)).read()
        # dynamic LDS becomes the emulated block's buffer
        s = re.sub(r"extern __shared__ __align__\(\d+\) unsigned char (\w+)\[\];",
                   r"unsigned char *\1 = emu_blk->dyn;", s)
        # kernel arguments are the kernel function's own parameter (no
        # kernarg segment on the CPU)
        s = re.sub(r"__device__ inline const KArgs &fresh_args\(const KArgs &\) \{.*?\n\}",
                   "__device__ inline const KArgs &fresh_args(const KArgs &a) { return a; }",
                   s, flags=re.S)
        open(os.path.join(src_dir, f), "w").write(s)
    cmd = ["g++", "-std=c++20", "-O1", "-fPIC", "-shared", "-pthread", "-fvisibility=hidden",
           "-I", HERE, "-I", os.path.join(ROOT, "include"), "-I", src_dir, "-o", LIB + ".tmp",
           "-x", "c++"] + [os.path.join(src_dir, f) for f in FILES if not f.endswith(".h")]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())
    sys.exit(0)
