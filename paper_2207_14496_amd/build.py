"""Build ``libfslbm.so`` (HIP, gfx950) in the package directory with hipcc.

Each translation unit is compiled in its own process (they are independent),
then linked into one shared library.  Run ``python -m paper_2207_14496_amd.build``.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfslbm.so")
BUILD_DIR = os.path.join(HERE, "_build")

# Translation units: (source, extra defines).  The step kernels are split by
# PDF storage type so the four instantiations compile in parallel.
UNITS = [
    ("api.hip", []),
    ("step_kernels.hip", ["-DFSLBM_UNIT_STORAGE=0"]),
    ("step_kernels.hip", ["-DFSLBM_UNIT_STORAGE=1"]),
    ("step_kernels.hip", ["-DFSLBM_UNIT_STORAGE=2"]),
    ("step_kernels.hip", ["-DFSLBM_UNIT_STORAGE=3"]),
    ("step_kernels.hip", ["-DFSLBM_UNIT_DISPATCH=1"]),
    ("adjoint_kernels.hip", []),
    ("adjoint_api.hip", []),
    ("bubble.hip", []),
]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         # no packed FP32 instructions anywhere in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(idx_unit):
    idx, (src, defs) = idx_unit
    obj = os.path.join(BUILD_DIR, f"{os.path.splitext(src)[0]}_{idx}.o")
    cmd = [HIPCC, *FLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src} {defs}:\n{r.stderr[-4000:]}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(UNITS), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(_compile, enumerate(UNITS)))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
