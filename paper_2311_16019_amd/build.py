"""Build ``libskrylov.so`` (HIP, gfx950) in-tree with hipcc.

Usage: ``python -m paper_2311_16019_amd.build`` or ``build()`` from Python.  Every call
recompiles all sources (object files go to ``paper_2311_16019_amd/_build``).

``--sanitize`` builds ``libskrylov_asan.so`` instead, with AddressSanitizer on the host code
only (the device code is compiled as usual), for checking the library's host paths on the
CPU: load it with the clang ASan runtime preloaded and ``SKR_LIBRARY`` pointing at it.
"""
from __future__ import annotations

import shlex
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libskrylov.so")
ARCH = "gfx950"

SOURCES = ["runtime.hip", "op.hip", "blockstep.hip", "block_cgs.hip", "whiten.hip", "sorth.hip", "srht.hip", "dense.hip", "gauss_jordan.hip", "proj.hip", "solver.hip", "api.hip"]

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-fvisibility=hidden",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-result",
    # packed FP32 instructions are disabled for every device kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}",
    f"-I{CSRC}",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the HIP library)")


# host-only AddressSanitizer (each -fsanitize= right after -Xarch_host: device code unchanged)
ASAN_HOST_FLAGS = shlex.split("-Xarch_host -fsanitize=address -Xarch_host -fno-omit-frame-pointer")
ASAN_LINK_FLAGS = shlex.split("-Xarch_host -fsanitize=address -Xarch_host -shared-libasan")


def _compile(src: str, verbose: bool, sanitize: bool = False) -> str:
    obj = os.path.join(BUILD + ("_asan" if sanitize else ""), os.path.splitext(src)[0] + ".o")
    extra = ASAN_HOST_FLAGS if sanitize else []
    cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{proc.stdout}\n{proc.stderr}")
    if verbose and proc.stderr.strip():
        print(proc.stderr, file=sys.stderr)
    return obj


def build(verbose: bool = False, jobs: int | None = None, sanitize: bool = False) -> str:
    """Compile every source for gfx950 and link ``libskrylov.so`` (``libskrylov_asan.so`` with
    ``sanitize``); returns its path."""
    os.makedirs(BUILD + ("_asan" if sanitize else ""), exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 2) - 1))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, sanitize), SOURCES))
    lib = os.path.join(PKG, "libskrylov_asan.so") if sanitize else LIB
    tmp = lib + ".tmp"
    # rocBLAS for the large plain FP64 products; at run time the loader resolves its soname to
    # the copy PyTorch has already loaded (as for the HIP runtime)
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-L/opt/rocm/lib", "-lrocblas",
           *(ASAN_LINK_FLAGS if sanitize else [])]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"link failed:\n{proc.stdout}\n{proc.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
