"""Build libfslbm.so (HIP kernels + C ABI) for gfx950 with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfslbm.so")
BUILD = os.path.join(HERE, "_build")

ARCH = os.environ.get("FSLBM_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", f"-I{INCLUDE}", f"-I{CSRC}",
          # packed FP32 instructions stay off (not emitted from plain float code)
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# No FMA contraction in any precision: every kernel body computes in the
# operation order of its source, so a domain gives bit-identical results
# whether it is launched alone or in a batch (where the compiler would
# otherwise contract differently), and the FP64 form keeps the operation
# order of its definition.
UNITS = {
    "k_fp64.hip": ["-ffp-contract=off"],
    "k_fp32.hip": ["-ffp-contract=off"],
    "k_fp16.hip": ["-ffp-contract=off"],
    "api.hip": [],
}


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def _compile(src: str, extra: list) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile every unit and link libfslbm.so next to this file."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, len(UNITS))) as ex:
        futs = {ex.submit(_compile, s, e): s for s, e in UNITS.items()}
        objs = [f.result() for f in futs]
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *sorted(objs)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
