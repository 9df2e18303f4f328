"""Build libnasg.so (HIP kernels + C ABI) for gfx950 with hipcc.

Each translation unit is compiled to an object in parallel, then linked into
paper_2303_08064_amd/libnasg.so. Usage: python -m paper_2303_08064_amd.build
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libnasg.so")
SOURCES = ["query.hip", "records.hip", "train.hip", "large.hip", "large_paper.hip", "api.hip"]
# per-file code generation options: the query kernels and the large network's
# kernels keep MFMA accumulators in VGPRs (no accumulator-register reads in
# their VALU-bound epilogues; the large backward kernels run two waves per
# SIMD, which leaves no accumulator registers anyway); the fused training
# kernel needs the accumulator registers for its gradient tiles
EXTRA = {"query.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
         "large.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
         "large_paper.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}
ARCH = os.environ.get("NASG_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 VALU ops stay off: ordinary float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _compile(src, verbose):
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [_hipcc(), *FLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
