"""Build libftv.so (gfx950 HIP kernels + C ABI) in-tree with hipcc.

    python -m paper_1405_2912_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(ROOT, "_build", "ftv")
LIB = os.path.join(PKG, "libftv.so")

SOURCES = ["ftv_vote_f32.hip", "ftv_vote_f64.hip", "ftv_vote_i32.hip", "ftv_vote_i64.hip", "ftv_vote_batch.hip",
           "ftv_vote_noalloc.hip",
           "ftv_hash.hip", "ftv_blocks.hip", "ftv_copy.hip", "ftv_api.cpp", "ftv_server.cpp", "ftv_units.cpp", "ftv_mm.cpp",
           "ftv_run.cpp", "ftv_host.cpp", "ftv_place.cpp"]

ARCH = "gfx950"
# -ffp-contract=off and no flush-to-zero: the relative tolerance test must be
# the IEEE binary64 computation, identical on every device.  Packed fp32 ops
# are disabled for every HIP translation unit.
DEVICE_FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
                "-fno-gpu-flush-denormals-to-zero", "-Wall", "-Wno-unused-function",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-D__HIP_PLATFORM_AMD__", "-fopenmp"]


def _hipcc() -> str:
    for cand in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: cannot build the gfx950 library")


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJ, src + ".o")
    if src.endswith(".hip"):
        cmd = [_hipcc(), *DEVICE_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", "-c", path, "-o", obj]
    else:
        cmd = [_hipcc(), *HOST_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", "-c", path, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{res.stderr[-4000:]}")
    return obj


def build(jobs: int = 4) -> str:
    """Compile every source (always) and link libftv.so next to this file."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    # only the C ABI (ftv_*) is exported; internal C++ symbols stay local
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread", "-fopenmp",
           f"-Wl,--version-script={os.path.join(CSRC, 'ftv.map')}"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"linking libftv.so failed:\n{res.stderr[-4000:]}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else 4))
