"""Build libpfista.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2204_10252_amd.build          # or: python paper_2204_10252_amd/build.py

Cross-compiles on a machine without a GPU.  Packed FP32 instructions are
disabled for all device code.  ``build(sanitize=True, out=...)`` builds a copy
whose host code carries AddressSanitizer and UndefinedBehaviorSanitizer (device
code unchanged); it needs the clang ASan runtime preloaded into the process
that loads it (``asan_runtime()``) and is meant for CPU-only checks of the
host-side validation paths.
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


def command(out: str = OUT, sanitize: bool = False) -> list:
    # sanitizers apply to the host code only (each flag behind -Xarch_host)
    san = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-shared-libasan"] if sanitize else []
    return [
        hipcc(), f"--offload-arch={ARCH}", "-O1" if sanitize else "-O3", "-std=c++17", "-fPIC", "-shared",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
        *san, "-I", os.path.join(ROOT, "include"),
        SRC, "-o", out,
    ]


def asan_runtime():
    """Path of the clang ASan runtime that a sanitized build needs preloaded, or None."""
    import glob
    llvm = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(hipcc()))), "llvm")
    for base in (llvm, "/opt/rocm/llvm"):
        hits = sorted(glob.glob(os.path.join(base, "lib", "clang", "*", "lib", "linux",
                                             "libclang_rt.asan-x86_64.so")))
        if hits:
            return hits[-1]
    return None


def build(verbose: bool = True, sanitize: bool = False, out: str = OUT) -> str:
    tmp = out + ".tmp"
    cmd = command(tmp, sanitize)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with code {res.returncode}")
    noisy = [ln for ln in res.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if verbose and noisy:
        sys.stderr.write("\n".join(noisy) + "\n")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build()
