"""Build libafqmc.so (the HIP kernels and the C ABI) in-tree for gfx950.

    python -m paper_2406_16238_amd.build

Every .hip file under csrc/ is compiled by hipcc, every host-only .cpp file by
g++, into _build/, in parallel, and linked into paper_2406_16238_amd/libafqmc.so.
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libafqmc.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
GXX = shutil.which("g++") or "/usr/bin/g++"

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def _check_defined(lib: str) -> None:
    """Fail when the library references a symbol of its own namespace that no
    object defines: the host pass can drop a kernel's launch stub without a
    diagnostic, which would otherwise surface only when the library is loaded."""
    nm = shutil.which("nm") or "/usr/bin/nm"
    r = subprocess.run([nm, "-D", "--undefined-only", lib], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"nm failed on {lib}:\n{r.stderr}")
    missing = [ln.split()[-1] for ln in r.stdout.splitlines() if "_ZN5afqmc" in ln]
    if missing:
        raise RuntimeError("libafqmc.so leaves its own symbols undefined:\n  " + "\n  ".join(missing))


def _compile_host(src: str) -> str:
    """Host-only C++ (no device code) with the system compiler."""
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [GXX, "-O2", "-std=c++17", "-fPIC", "-Wall", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
           "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"g++ failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    host = sorted(glob.glob(os.path.join(CSRC, "*.cpp")))
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs) + len(host))) as ex:
        objs = list(ex.map(_compile, srcs)) + list(ex.map(_compile_host, host))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    _check_defined(tmp)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
