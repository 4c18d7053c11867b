"""Build the HIP library libvfp.so in-tree for gfx950 (hipcc, no GPU needed).

Usage: python -m paper_2501_05110_amd.build   (or build() from Python).
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libvfp.so")

ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-mcode-object-version=5",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
# packed FP32 instructions stay disabled in every HIP translation unit
DEVICE = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics", "-ffp-contract=fast"]
SOURCES = ["shtab.cpp", "vfp.cpp", "stage.hip", "stage_gen_1f.hip", "stage_gen_1a.hip", "stage_gen_2f.hip",
           "stage_gen_2a.hip", "stage_gen_3f.hip", "stage_gen_3a.hip", "stage_shock.hip", "stage_shock_shapes.hip", "stage_batch.hip", "stage_batch_shapes.hip", "field_grad.hip",
           "krylov.hip", "reconstruct.hip", "noalloc.hip", "resident.hip", "xline.hip"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str, extra=()) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + "".join(extra).replace("-", "_").replace("=", "") + ".o")
    cmd = [_hipcc(), *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip"]
        cmd += DEVICE
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True, out: str = LIB, extra=()) -> str:
    """Compile every source (with optional extra flags) and link `out`."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(int(os.environ.get("MAX_JOBS", "8")), len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, tuple(extra)), SOURCES))
    tmp = out + ".tmp"
    cmd = [_hipcc(), "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    try:
        build()
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
