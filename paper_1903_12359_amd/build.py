"""Build libpgcp.so in-tree with hipcc for gfx950.

    python -m paper_1903_12359_amd.build

Device code is compiled with packed FP32 instructions disabled.  Host C++
(partition, weld, C ABI) uses OpenMP.  The weld uses plain complex multiply
and divide (-fcx-limited-range): every point at infinity is carried as an
explicit flag, so no operation there meets an infinite or NaN operand.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpgcp.so")

ARCH = os.environ.get("PGCP_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-fPIC", "-std=c++17", "-fopenmp", "-Wno-unused-result"]
DEVICE_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-munsafe-fp-atomics"]
HOST_SOURCES = ["partition.cpp", "weld.cpp", "api.cpp"]
HOST_EXTRA = {"weld.cpp": ["-fcx-limited-range"]}
DEVICE_EXTRA = {"weld_dev.hip": ["-fcx-limited-range"]}
DEVICE_SOURCES = ["device.hip", "lpc.hip", "weld_dev.hip", "area.hip"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    """Compile every source (in parallel, one compiler per source) and link."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src in DEVICE_SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        jobs.append((obj, [hipcc, *COMMON, *DEVICE_FLAGS, *DEVICE_EXTRA.get(src, []), "-c",
                           os.path.join(CSRC, src), "-o", obj]))
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src.replace(".cpp", ".o"))
        jobs.append((obj, [hipcc, *COMMON, *HOST_EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for f in [ex.submit(_run, cmd) for _, cmd in jobs]:
            f.result()
    objs = [obj for obj, _ in jobs]
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fopenmp", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
