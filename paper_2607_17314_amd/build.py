"""Build libisdfxtc.so for gfx950 with hipcc (in-tree; no JIT cache).

    python -m paper_2607_17314_amd.build [-v]

Every .hip file under csrc/ is compiled to an object in _build/ (in parallel),
then linked into paper_2607_17314_amd/libisdfxtc.so. The build always runs
(no staleness check), so the library matches the sources after every call.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "libisdfxtc.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = os.environ.get("XTC_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-I", INCLUDE, "-I", CSRC,
    # packed FP32 VALU forms are kept out of the device code on purpose
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]

# Per-file additions: MFMA accumulators in VGPRs. In the default (AGPR) form the
# compiler copies the generic FP64 GEMM's accumulators out of and back into AGPRs
# around every k-tile's MFMAs (the VGPR form is 10-20% faster at the fit's shapes,
# bitwise the same results), and shuttles the adjoint kernels' values between the
# two register files (fewer registers and spills in the VGPR form: EE adjoint 8%,
# BH adjoint 22% faster). The option is not applied globally: it crashes the
# compiler on the FP64 stage-1 kernels.
FILE_FLAGS = {
    "gemm_f64.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
    "grad.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
}


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))

    def compile_one(src):
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        cmd = [hipcc, *FLAGS, *FILE_FLAGS.get(os.path.basename(src), []), "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        msg = "\n".join(line for line in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops" not in line)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
        if verbose and msg.strip():
            print(msg)
        return obj

    with ThreadPoolExecutor(min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = OUT + f".tmp{os.getpid()}"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
