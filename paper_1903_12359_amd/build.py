"""Build libpgcp.so in-tree with hipcc for gfx950.

    python -m paper_1903_12359_amd.build              # libpgcp.so
    python -m paper_1903_12359_amd.build --sanitize   # libpgcp_asan.so (host ASan + UBSan)

Device code is compiled with packed FP32 instructions disabled.  Host C++
(partition, weld, C ABI) uses OpenMP; each C-ABI call opens a roctx range
(librocprofiler-sdk-roctx).  The weld uses plain complex multiply
and divide (-fcx-limited-range): every point at infinity is carried as an
explicit flag, so no operation there meets an infinite or NaN operand.
"""
from __future__ import annotations

import os
import re
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


# The batched-CG kernels run as persistent cooperative grids whose workgroups
# wait for each other at every iteration, so all of them must be resident at
# once.  A kernel that needs scratch memory may have fewer of its waves running
# than the grid holds (the hardware hands out scratch per wave), and the
# missing workgroups would never reach the barriers: device.hip is compiled
# with the compiler's resource-usage remarks and the build fails if the
# streaming CG kernel (the one every batch can fall back to) uses scratch.
NO_SCRATCH_KERNELS = ("k_pcg_stream",)


def _check_scratch(remarks: str) -> None:
    name = None
    for line in remarks.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"remark:\s+ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name and any(k in name for k in NO_SCRATCH_KERNELS) and int(m.group(1)) > 0:
            raise RuntimeError(f"{name} uses {m.group(1)} bytes of scratch per lane; a persistent "
                               "cooperative kernel must not spill")


def _run_checked(cmd):
    print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd + ["-Rpass-analysis=kernel-resource-usage"], capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise subprocess.CalledProcessError(r.returncode, cmd)
    _check_scratch(r.stderr)


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
        for f in [ex.submit(_run_checked if cmd[-3].endswith("device.hip") else _run, cmd) for _, cmd in jobs]:
            f.result()
    objs = [obj for obj, _ in jobs]
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fopenmp", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lrocprofiler-sdk-roctx"])
    os.replace(tmp, LIB)
    return LIB


# Host sanitizers (AddressSanitizer + UndefinedBehaviorSanitizer) on the host
# code: partition, weld and the C ABI are rebuilt instrumented and linked with
# the device objects of the normal build into libpgcp_asan.so, a test build
# that a process loads with clang's ASan runtime preloaded (see
# sanitizer_env()).  Device code is not instrumented.
ASAN_BUILD = os.path.join(HERE, "_build_asan")
ASAN_LIB = os.path.join(HERE, "libpgcp_asan.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def build_sanitized(verbose: bool = True) -> str:
    from concurrent.futures import ThreadPoolExecutor
    hipcc = _hipcc()
    os.makedirs(ASAN_BUILD, exist_ok=True)
    dev_objs = [os.path.join(BUILD, src.replace(".hip", ".o")) for src in DEVICE_SOURCES]
    if not all(os.path.exists(o) for o in dev_objs):
        build(verbose)
    jobs = []
    for src in HOST_SOURCES:
        obj = os.path.join(ASAN_BUILD, src.replace(".cpp", ".o"))
        jobs.append([hipcc, *COMMON, *SAN_FLAGS, *HOST_EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        for f in [ex.submit(_run, cmd) for cmd in jobs]:
            f.result()
    objs = [os.path.join(ASAN_BUILD, src.replace(".cpp", ".o")) for src in HOST_SOURCES] + dev_objs
    tmp = ASAN_LIB + ".tmp"
    _run([hipcc, "-shared", "-fopenmp", f"--offload-arch={ARCH}", "-Xarch_host", "-fsanitize=address",
          "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", "-o", tmp, *objs, "-lrocprofiler-sdk-roctx"])
    os.replace(tmp, ASAN_LIB)
    return ASAN_LIB


def sanitizer_env() -> dict:
    """Environment for a process that loads libpgcp_asan.so: the ASan runtime
    preloaded, leaks of the interpreter itself not reported, the first error
    fatal."""
    rt = subprocess.run([_hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], check=True,
                        capture_output=True, text=True).stdout.strip()
    env = dict(os.environ)
    env["LD_PRELOAD"] = rt
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=24"
    return env


if __name__ == "__main__":
    if "--sanitize" in sys.argv[1:]:
        build_sanitized()
    else:
        build()
    sys.exit(0)
