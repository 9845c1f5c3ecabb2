"""Build libpic.so (hand-written HIP for gfx950) in-tree with hipcc.

Each translation unit is compiled to an object in ``_build/`` (in parallel), then linked into
``paper_2501_07465_amd/libpic.so``.  Compile flags:

* ``--offload-arch=gfx950`` only;
* ``-Xclang -target-feature -Xclang -packed-fp32-ops``: no packed FP32 instructions;
* the FP64 form (``pic_k64.hip``) is compiled without FMA contraction so its arithmetic
  rounds like the plain-C reference it is checked against.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libpic.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "--offload-arch=gfx950", "-fPIC", "-std=c++17", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
UNITS = {
    "pic_k32.hip": [],
    "pic_k64.hip": ["-ffp-contract=off"],
    "pic_sort.hip": [],
    "pic_host.hip": [],
}
DEPS = ["pic_internal.h", "pic_sort.h", "pic_kernels.inc"]


def _compile(unit: str, extra: list[str]) -> str:
    obj = os.path.join(BUILD, unit.replace(".hip", ".o"))
    cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, unit), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {unit}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(UNITS)) as ex:
        objs = list(ex.map(lambda kv: _compile(*kv), UNITS.items()))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
