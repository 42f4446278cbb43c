"""Build libvgicp.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2109_07073_amd.build

Every source under csrc/ is compiled to an object with hipcc and the objects
are linked into paper_2109_07073_amd/libvgicp.so; then the plain C client
tests/c/vgicp_example.c is built against it with gcc.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libvgicp.so")
ARCH = os.environ.get("VGICP_OFFLOAD_ARCH", "gfx950")

SOURCES = ["runtime.hip", "voxelize.hip", "linearize.hip", "server.hip", "reorder.hip",
           "mapping.hip", "noalloc.hip"]

COMMON = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # code object v5: loadable by the HIP runtime that PyTorch-ROCm bundles
    "-mcode-object-version=5",
    # packed FP32 instructions stay off on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    build_c_example(verbose)
    return LIB


EXAMPLE_SRC = os.path.join(ROOT, "tests", "c", "vgicp_example.c")
EXAMPLE_BIN = os.path.join(ROOT, "tests", "c", "vgicp_example")


def build_c_example(verbose: bool = False) -> str:
    """A plain C client of the C ABI (gcc, C99, linked against libvgicp.so
    and the HIP runtime of /opt/rocm), used by the tests."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"),
           EXAMPLE_SRC, "-o", EXAMPLE_BIN, "-L", HERE, "-lvgicp",
           "-L", os.path.join(rocm, "lib"), "-lamdhip64",
           f"-Wl,-rpath,{HERE}", f"-Wl,-rpath,{os.path.join(rocm, 'lib')}"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"C example build failed:\n{res.stdout}\n{res.stderr}")
    return EXAMPLE_BIN


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
