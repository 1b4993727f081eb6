"""Build librrf.so (the HIP kernels and the C-ABI) in-tree for gfx950.

Usage: ``python paper_2106_13402_amd/build.py`` or ``build()`` (run as a
script or loaded by path: importing the package would load the library). Every source
is compiled with hipcc for gfx950 (cross-compiles without a GPU) and linked
into ``paper_2106_13402_amd/librrf.so``. Packed-FP32 instruction selection is
disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "librrf.so")
BENCH_BIN = os.path.join(PKG, "rrf_bench")
BUILD_DIR = os.path.join(ROOT, "_build")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-function",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (needs ROCm)")


def _compile(hipcc: str, src: str) -> tuple[str, str]:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = [hipcc, *HIPCC_FLAGS, "-c", src, "-o", obj]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{proc.stdout}\n{proc.stderr}")
    noise = "\n".join(l for l in proc.stderr.splitlines() if "packed-fp32-ops" not in l)
    return obj, noise


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link librrf.so; returns its path."""
    hipcc = _hipcc()
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    objs = []
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        for obj, noise in ex.map(lambda s: _compile(hipcc, s), srcs):
            objs.append(obj)
            if verbose and noise.strip():
                print(noise, file=sys.stderr)
    tmp = OUT + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{proc.stdout}\n{proc.stderr}")
    os.replace(tmp, OUT)
    # stand-alone C-ABI client used for profiling without Python in the process
    drv = os.path.join(PKG, "driver", "rrf_bench.cpp")
    cmd = [hipcc, "-O2", "-std=c++17", f"-I{INCLUDE}", drv, "-o", BENCH_BIN + ".tmp",
           f"-L{PKG}", "-lrrf", "-Wl,-rpath,$ORIGIN"]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"driver build failed: {' '.join(cmd)}\n{proc.stdout}\n{proc.stderr}")
    os.replace(BENCH_BIN + ".tmp", BENCH_BIN)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
