"""Build the HIP library in-tree for gfx950.

    python -m paper_2607_00790_amd.build

Produces (next to this file):
  libbmhss.so            -- the product library (C-ABI of include/bmhss.h)
  libbmhss_hostcheck.so  -- host-compiled instances of the device math, loaded
                            only by the CPU unit tests
  libbmhss_probe.so      -- the benchmark's FP64 FMA-rate probe (benchsrc/), loaded
                            only by bench.py and its test
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libbmhss.so")
HOSTCHECK = os.path.join(HERE, "libbmhss_hostcheck.so")
PROBE = os.path.join(HERE, "libbmhss_probe.so")

ARCH = "gfx950"
COMMON = ["-std=c++17", "-O3", "-fPIC", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
# Packed FP32 instructions are disabled for every HIP object.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> None:
    srcs = sorted(s for s in glob.glob(os.path.join(CSRC, "*.hip")) if not s.endswith("hostcheck.hip"))
    objs = []
    tmpdir = os.path.join(HERE, "_build")
    os.makedirs(tmpdir, exist_ok=True)
    for s in srcs:
        o = os.path.join(tmpdir, os.path.basename(s) + ".o")
        _run([hipcc(), f"--offload-arch={ARCH}", *COMMON, *DEVICE_FLAGS, "-c", s, "-o", o])
        objs.append(o)
    tmp = LIB + ".tmp"
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    _run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, f"-L{rocm_lib}", "-lrocblas",
          f"-Wl,-rpath,{rocm_lib}", "-o", tmp])
    os.replace(tmp, LIB)
    tmp = HOSTCHECK + ".tmp"
    _run([hipcc(), f"--offload-arch={ARCH}", *COMMON, *DEVICE_FLAGS, "-shared",
          os.path.join(CSRC, "hostcheck.hip"), "-o", tmp])
    os.replace(tmp, HOSTCHECK)
    tmp = PROBE + ".tmp"
    _run([hipcc(), f"--offload-arch={ARCH}", *COMMON, *DEVICE_FLAGS, "-shared",
          os.path.join(HERE, "benchsrc", "fma_probe.hip"), "-o", tmp])
    os.replace(tmp, PROBE)


if __name__ == "__main__":
    build()
    sys.exit(0)
