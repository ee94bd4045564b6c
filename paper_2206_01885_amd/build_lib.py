"""Build the HIP shared library libh2.so for gfx950 (in-tree)."""
from __future__ import annotations

import json
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libh2.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Launch parameters measured by autotune.py (csrc/tuning.h holds the
# defaults and their meaning); absent file: the defaults.
TUNING = os.path.join(HERE, "tuning.json")


def tuning_params(path: str = TUNING) -> dict:
    """The H2_TUNE_* values of tuning.json ({} when there is none)."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return {k: int(v) for k, v in json.load(f)["params"].items()}

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


def _compile(src: str, outdir: str, params: dict) -> str:
    obj = os.path.join(outdir, src.replace(".hip", ".o"))
    flags = list(COMMON) + [f"-D{k}={v}" for k, v in sorted(params.items())]
    flags.append("-ffp-contract=off" if src in EXACT else "-ffp-contract=fast")
    if src in MFMA_VGPR:
        flags += ["-mllvm", "-amdgpu-mfma-vgpr-form"]
    cmd = [HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(jobs: int = 8, out: str = LIB, params: dict | None = None) -> str:
    """Compile every source and link `out`; params: H2_TUNE_* values (default:
    tuning.json)."""
    if params is None:
        params = tuning_params()
    outdir = os.path.join(HERE, "_build", os.path.basename(out).replace(".so", ""))
    os.makedirs(outdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, outdir, params), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
