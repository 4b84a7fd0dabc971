"""Build libpc2.so (HIP kernels + C ABI) for gfx950, in-tree.

    python -m paper_2601_14980_amd.build

Compiles each translation unit in parallel with hipcc and links the shared
library next to this file.  Every call rebuilds (the objects are cheap to
compare against sources, but a forced rebuild is what a build check wants).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
OUT = PKG / "libpc2.so"
BUILD = PKG / "_build"

ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed fp32 instructions are disabled in all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
UNITS = {
    "kernels_paillier.hip": [],
    "kernels_batch.hip": [],
    "kernels_mfma.hip": [],
    "kernels_matvec.hip": [],
    "kernels_quant.hip": ["-ffp-contract=off"],
    "kernels_admm.hip": ["-ffp-contract=off"],
    "kernels_colsplit.hip": ["-ffp-contract=off"],
    "static_scratch.hip": [],
    "api.cpp": [],
    "serve.cpp": [],
}


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and Path(cand).exists():
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, extra: list[str]) -> Path:
    obj = BUILD / (src.replace(".", "_") + ".o")
    cmd = [hipcc(), *COMMON, *extra, "-c", str(CSRC / src), "-o", str(obj)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> Path:
    BUILD.mkdir(exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(UNITS)) as ex:
        futs = {ex.submit(_compile, s, e): s for s, e in UNITS.items()}
        objs = [f.result() for f in futs]
    tmp = OUT.with_suffix(".so.tmp")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp),
           *[str(o) for o in objs]]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
