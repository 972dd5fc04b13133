"""Build libnw.so (HIP for gfx950) in-tree, one object per translation unit in parallel.

Usage: python -m paper_2509_01654_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnw.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

DEVICE_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed fp32 VALU forms are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _la_splits():
    text = open(os.path.join(CSRC, "nw_kernels.h"), encoding="utf-8").read()
    m = re.search(r"#define NW_LA_SPLITS (.*)", text)
    return [(int(a), int(b)) for a, b in re.findall(r"X\((\d+), (\d+)\)", m.group(1))]


def _class8():
    text = open(os.path.join(CSRC, "nw_kernels.h"), encoding="utf-8").read()
    m = re.search(r"#define NW_CLASS8 (.*)", text)
    return [(int(a), int(b)) for a, b in re.findall(r"X\((\d+), (\d+)\)", m.group(1))]


def _units():
    units = [
        ("nw_api", os.path.join(CSRC, "nw_api.cpp"), []),
        ("nw_server", os.path.join(CSRC, "nw_server.cpp"), []),
        ("nw_batch", os.path.join(CSRC, "nw_batch.cpp"), []),
        ("nw_export", os.path.join(CSRC, "nw_export.cpp"), []),
        ("nw_graph", os.path.join(CSRC, "nw_graph.hip"), []),
        ("k_peak", os.path.join(CSRC, "k_peak.hip"), []),
        ("k_launch", os.path.join(CSRC, "k_launch.hip"), []),
        ("nw_noalloc", os.path.join(CSRC, "nw_noalloc.hip"), []),
    ]
    for lo, hi in _la_splits():
        units.append((f"k_inst_{lo}_{hi}", os.path.join(CSRC, "k_inst.hip"),
                      [f"-DNW_LA_LO={lo}", f"-DNW_LA_HI={hi}"]))
    for lo, hi in _class8():
        units.append((f"k_batch_inst_{lo}_{hi}", os.path.join(CSRC, "k_batch_inst.hip"),
                      [f"-DNW_CLASS_LO={lo}", f"-DNW_CLASS_HI={hi}"]))
    return units


def _compile(unit):
    name, src, extra = unit
    obj = os.path.join(OUT_DIR, name + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC] + DEVICE_FLAGS + extra + lang + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    """Compile every HIP/C++ unit for gfx950 and link libnw.so (always rebuilds)."""
    os.makedirs(OUT_DIR, exist_ok=True)
    units = _units()
    jobs = jobs or min(len(units), max(1, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, units))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(objs)} objects", file=sys.stderr)
    return LIB


# Host code with AddressSanitizer + UBSan (every report fatal).  Each flag is
# scoped to the host compilation: device code is never built with them.
HOST_SAN_FLAGS = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
                  "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
HOST_SAN_LIB = os.path.join(OUT_DIR, "libnw_hostsan.so")
# the units that hold only host code: argument checks, layouts, schedulers
HOST_UNITS = ["nw_api", "nw_server", "nw_batch", "nw_export"]


def build_host_sanitized(verbose: bool = False) -> str:
    """libnw with its host-only units built under AddressSanitizer and UBSan.

    The other units' objects come from the last build() (run it first).  A
    process loads the result with the sanitizer runtime preloaded
    (LD_PRELOAD = hipcc's libclang_rt.asan-x86_64.so) and NW_LIBRARY set to
    the returned path."""
    units = {u[0]: u for u in _units()}
    objs = []
    for name, src, extra in units.values():
        obj = os.path.join(OUT_DIR, name + ".o")
        if name in HOST_UNITS:
            obj = os.path.join(OUT_DIR, name + ".hostsan.o")
            cmd = [HIPCC] + DEVICE_FLAGS + HOST_SAN_FLAGS + extra + ["-c", src, "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        elif not os.path.exists(obj):
            raise RuntimeError(f"{obj} is missing: run build() first")
        objs.append(obj)
    tmp = HOST_SAN_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address,undefined",
           "-Xarch_host", "-shared-libsan", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, HOST_SAN_LIB)
    if verbose:
        print(f"built {HOST_SAN_LIB}", file=sys.stderr)
    return HOST_SAN_LIB


def asan_runtime() -> str:
    """hipcc's shared AddressSanitizer runtime (to preload into Python)."""
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        import glob
        hits = glob.glob("/opt/rocm*/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        if not hits:
            raise RuntimeError("no libclang_rt.asan-x86_64.so found")
        path = hits[0]
    return path


if __name__ == "__main__":
    build()
