"""Build the gfx950 HIP library liblkp.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "liblkp.so")
LATTICES = ["d1q5", "d1q9", "d1q13", "d2q5", "d2q9", "d2q25", "d2q81", "d2q169", "d3q111",
            "d2q37", "d2q77"]
# largest first so the parallel build finishes early
SOURCES = (["sweep_d2q169.hip", "sweep_d3q111.hip", "sweep_d2q81.hip"]
           + [f"sweep_{l}.hip" for l in LATTICES if l not in ("d2q169", "d3q111", "d2q81")]
           + ["sweep.hip", "dev.hip", "lkp.cpp", "group.cpp", "constants.cpp"])
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]
DEVICE = ["--offload-arch=gfx950",
          # packed FP32 instructions stay off: the compiler may not form them
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC, *COMMON, *DEVICE, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    subprocess.check_call(cmd)
    return obj


def build(jobs: int = 8) -> str:
    """Compile every source for gfx950 and link liblkp.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs,
                           "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else 8))
