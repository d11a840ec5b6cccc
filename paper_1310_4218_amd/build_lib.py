"""Build liblbgrid.so in-tree with hipcc for gfx950.

    python -m paper_1310_4218_amd.build_lib [-v]

Every source is compiled for gfx950 only, with packed FP32 instructions
disabled (-packed-fp32-ops), native FP64 atomics (-munsafe-fp-atomics; the
workspace is ordinary device memory) and the atomic optimizer off (claims are
single-lane atomics read late).  Objects go to ``_build/`` at the
repository root; the library lands next to this file.
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
OUT = os.path.join(HERE, "liblbgrid.so")
BUILD = os.path.join(ROOT, "_build")
SOURCES = ["kernels.hip", "runtime.cpp", "balance.cpp"]
ARCH = "gfx950"
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          f"-I{os.path.join(ROOT, 'include')}"]
# -amdgpu-atomic-optimizer-strategy=None: a claim is one lane's atomic whose
# result is needed only later in the item; the optimizer would rewrite it as a
# wave-wide atomic and wait for its reply on the spot.
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics", "-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise FileNotFoundError("hipcc not found (ROCm is required to build liblbgrid)")


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, src + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [hipcc(), *DEVICE, *COMMON, "-c", path, "-o", obj]
    else:  # host-only C++ (HIP runtime API headers, no device code)
        cmd = [hipcc(), *COMMON, "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", "-x", "c++", "-c",
               path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source (always) and link liblbgrid.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = OUT + f".tmp{os.getpid()}"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv[1:]))
