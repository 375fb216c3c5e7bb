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
LATTICES = ["D2Q169", "D3Q111", "D3Q107", "D2Q81", "D2Q77", "D2Q37", "D1Q13", "D2Q25", "D1Q9", "D2Q9",
            "D1Q5", "D2Q5"]
# (source, defines, object): every velocity set is compiled in eight parts
# (dispatch + deviation sweep, one part per population-sweep precision mode,
# one per stencil-form mode),
# largest sets first so that the parallel build finishes early
JOBS = ([("sweep_tu.hip", [f"-DLKP_TU_LATTICE={l}", f"-DLKP_TU_MODE={m}"], f"sweep_{l.lower()}_{m + 1}")
         for l in LATTICES for m in (0, 1, 3, 10, 11, 2, 12, -1)]
        + [(src, [], src) for src in ("sweep.hip", "dev.hip", "lkp.cpp", "group.cpp", "constants.cpp",
                                   "noalloc.cpp", "validate.cpp")])
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]
DEVICE = ["--offload-arch=gfx950",
          # packed FP32 instructions stay off: the compiler may not form them
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(job) -> str:
    src, defines, name = job
    obj = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC, *COMMON, *DEVICE, *defines, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    subprocess.check_call(cmd)
    return obj


def build(jobs: int = 8) -> str:
    """Compile every source for gfx950 and link liblkp.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, JOBS))
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs,
                           "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else 8))
