"""Build libpfista.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2204_10252_amd.build          # or: python paper_2204_10252_amd/build.py

Cross-compiles on a machine without a GPU.  Packed FP32 instructions are
disabled for all device code.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "pfista_lib.hip")
OUT = os.path.join(HERE, "libpfista.so")
ARCH = os.environ.get("PFISTA_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def command(out: str = OUT) -> list:
    return [
        hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
        "-I", os.path.join(ROOT, "include"),
        SRC, "-o", out,
    ]


def build(verbose: bool = True) -> str:
    tmp = OUT + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with code {res.returncode}")
    noisy = [ln for ln in res.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if verbose and noisy:
        sys.stderr.write("\n".join(noisy) + "\n")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build()
