"""Build the HIP library libttrbki.so for gfx950 (MI355X) in-tree.

Every translation unit under csrc/ is compiled with hipcc for --offload-arch=gfx950
(packed FP32 instructions disabled) and linked into paper_2308_01480_amd/libttrbki.so.
"""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libttrbki.so")
SOURCES = ["plan.cpp", "stream_kernels.hip", "bf16_kernels.hip", "small_kernels.hip", "sweep.hip", "grad.hip", "block_orth.hip"]
ARCH = "gfx950"


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain (ROCm) is required to build libttrbki.so")


# Matrix-core accumulators in ordinary VGPRs for these units: without it the float32 /
# float64 streaming loops (the wide A^T Z and carry kernels above all) copied their
# accumulators between AGPRs and VGPRs on every iteration.  The bf16 units measured no
# better with it.
VGPR_FORM = {"stream_kernels.hip", "block_orth.hip"}


def _flags(src: str = ""):
    f = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wall", "-Wno-unused-result", "-Wno-unused-function"]
    if src in VGPR_FORM:
        f += ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]
    return f


def build(verbose: bool = False) -> str:
    """Compile every source and link the shared library; returns its path."""
    hipcc = _hipcc()
    os.makedirs(OBJ, exist_ok=True)

    def compile_one(src):
        out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *_flags(src), "-c", os.path.join(CSRC, src), "-o", out]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling {src} failed:\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr)
        return out

    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libttrbki.so failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
