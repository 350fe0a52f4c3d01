"""Build libzolo.so (all HIP kernels + host code) for gfx950 with hipcc.

Usage: python -m paper_1701_08935_amd.build  (or build() from Python).
Objects go to paper_1701_08935_amd/_build/, the library next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libzolo.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = ["planner.cpp", "symbolic.cpp", "capi.cpp", "serve.cpp", "gemm.hip", "front.hip", "sparse.hip", "krylov.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wno-unused-result",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") or src in ("capi.cpp", "serve.cpp") else []
    cmd = [HIPCC] + COMMON + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-pthread", "-o", OUT + ".tmp"] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    # every symbol of the library's own namespace must be defined (a missing
    # template instantiation would otherwise only show when the library loads)
    nm = subprocess.run(["nm", "-C", "-u", OUT + ".tmp"], capture_output=True, text=True)
    missing = [ln.strip() for ln in nm.stdout.splitlines() if "zolo::" in ln]
    if missing:
        raise RuntimeError("undefined symbols in libzolo.so:\n" + "\n".join(missing))
    os.replace(OUT + ".tmp", OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
