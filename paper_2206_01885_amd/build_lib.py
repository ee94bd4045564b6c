"""Build the HIP shared library libh2.so for gfx950 (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libh2.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Sources whose arithmetic must round exactly as written (geometry,
# DataReduct, the ID and its calibration) are compiled without FMA
# contraction.
EXACT = {"tree.hip", "lists.hip", "hidr.hip", "basis.hip", "calib.hip"}
# Sources whose matrix-core loops keep their accumulators in VGPRs: with the
# default AGPR form the compiler copies every accumulator out and back at
# each loop iteration.
MFMA_VGPR = {"matvec.hip"}
SOURCES = ["alloc.hip", "scan.hip", "tree.hip", "lists.hip", "hidr.hip", "calib.hip", "basis.hip", "blocks.hip",
           "matvec.hip", "api.hip"]
COMMON = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(HERE, "..", "include")]


def _compile(src: str, outdir: str) -> str:
    obj = os.path.join(outdir, src.replace(".hip", ".o"))
    flags = list(COMMON)
    flags.append("-ffp-contract=off" if src in EXACT else "-ffp-contract=fast")
    if src in MFMA_VGPR:
        flags += ["-mllvm", "-amdgpu-mfma-vgpr-form"]
    cmd = [HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(jobs: int = 8) -> str:
    outdir = os.path.join(HERE, "_build")
    os.makedirs(outdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, outdir), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
