"""Build the HIP library ``libgplhr.so`` for gfx950 in-tree (hipcc).

Usage: ``python -m paper_1506_06829_amd.build`` (or ``build()`` from Python).
Always recompiles; objects go to ``_build/`` at the repository root.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "libgplhr.so"

SOURCES = ["kernels.hip", "driver.hip", "capi.cpp", "memory.cpp", "small_dense.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{ROOT / 'include'}", f"-I{CSRC}",
]
# -fcx-limited-range: textbook complex multiply/divide (no NaN/Inf recovery
# calls); the small dense step never sees magnitudes near the overflow range
HOST_ONLY = ["-O3", "-std=c++17", "-fPIC", "-march=x86-64-v3", "-fcx-limited-range", f"-I{CSRC}"]


def _compile(src: str, build_dir: Path) -> Path:
    obj = build_dir / (src + ".o")
    if src == "small_dense.cpp":
        cmd = ["g++", *HOST_ONLY, "-c", str(CSRC / src), "-o", str(obj)]
    elif src.endswith(".cpp"):
        cmd = [HIPCC, *COMMON, "-x", "hip", "-c", str(CSRC / src), "-o", str(obj)]
    else:
        cmd = [HIPCC, *COMMON, "-c", str(CSRC / src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compilation of {src} failed:\n{' '.join(cmd)}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> Path:
    if shutil.which(HIPCC) is None and not Path(HIPCC).exists():
        raise RuntimeError("hipcc not found")
    build_dir = ROOT / "_build"
    build_dir.mkdir(exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir), SOURCES))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
