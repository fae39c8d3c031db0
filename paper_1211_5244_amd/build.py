"""Build libpoisson.so for gfx950 in place with hipcc.

Usage: python -m paper_1211_5244_amd.build [-j N]

Every call compiles all sources again (objects go to paper_1211_5244_amd/_build)
and links paper_1211_5244_amd/libpoisson.so.
"""

from __future__ import annotations

import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libpoisson.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are switched off for all device code.
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]

SOURCES = ["plan.cpp", "api.cpp", "kernel_build.hip", "kernel_isf.hip", "queue.hip"]
# the pass kernels are split by FFT length so they compile in parallel
PASS_LENGTHS = [4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024]


def _compile(src, obj, extra=()):
    cmd = [HIPCC, *COMMON, *extra, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs=None, verbose=False):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    tasks = []
    for s in SOURCES:
        tasks.append((os.path.join(CSRC, s), os.path.join(BUILD, s.rsplit(".", 1)[0] + ".o"), ()))
    # one object per length group, each instantiating the launchers for its lengths
    for L in PASS_LENGTHS:
        for mode in (0, 1, 2):  # float32, split fp16, split bf16
            # split modes: matrix-core results straight into VGPRs (no
            # accumulator-register reads after every product)
            extra = ("-mllvm", "-amdgpu-mfma-vgpr-form=1") if mode else ()
            tasks.append((os.path.join(CSRC, "passes.hip"), os.path.join(BUILD, f"passes_{L}_{mode}.o"),
                          (f"-DPSN_ONLY_LENGTH={L}", f"-DPSN_ONLY_MODE={mode}", *extra)))
    tasks.append((os.path.join(CSRC, "passes.hip"), os.path.join(BUILD, "passes_dispatch.o"),
                  ("-DPSN_DISPATCH_ONLY=1",)))
    for mode in (0, 1, 2):  # the small-grid plane kernel, one object per precision
        extra = ("-mllvm", "-amdgpu-mfma-vgpr-form=1") if mode else ()
        tasks.append((os.path.join(CSRC, "passes.hip"), os.path.join(BUILD, f"passes_plane_{mode}.o"),
                      ("-DPSN_PLANE_ONLY=1", f"-DPSN_ONLY_MODE={mode}", *extra)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda t: _compile(*t), tasks))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    a = ap.parse_args()
    try:
        build(a.j, verbose=True)
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
