"""Build libprnu.so for gfx950 with hipcc (in-tree, no JIT cache).

    python -m paper_1909_04573_amd.build          # compile + link
    python -m paper_1909_04573_amd.build check    # + the sanitized host check

Every HIP source is compiled with packed-FP32 instructions disabled; the
objects go to ``_build/`` and the library to ``paper_1909_04573_amd/libprnu.so``.

build_host_check() links tests/host_check.cpp with the library's host
sources (the .cpp files: validation, planning, tile table, filter design)
compiled with AddressSanitizer and UndefinedBehaviorSanitizer on their host
code only, and the kernel objects as built for the library; the program
runs on a machine without a GPU.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libprnu.so")
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libprnu.so)")


COMMON = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    f"--offload-arch={ARCH}",
    "-Wall",
    "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}",
    f"-I{CSRC}",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), *COMMON]
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


# sanitizers on the host side of a HIP compile only (never on device code)
SANITIZE = [
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
    "-Xarch_host", "-fno-omit-frame-pointer",
]
HOST_CHECK_SRC = os.path.join(ROOT, "tests", "host_check.cpp")
HOST_CHECK = os.path.join(BUILD, "sanitize", "host_check")


def _run(cmd, what, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{what} failed:\n{r.stdout}\n{r.stderr}")


def build_host_check(verbose: bool = False, jobs: int = 8) -> str:
    """Sanitized host-check program (see the module docstring); reuses the
    library's kernel objects when they are newer than their sources."""
    out = os.path.dirname(HOST_CHECK)
    os.makedirs(out, exist_ok=True)
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", f"-I{INCLUDE}", f"-I{CSRC}"]
    hosts = [s for s in sources() if s.endswith(".cpp")] + [HOST_CHECK_SRC]
    kernels = [s for s in sources() if s.endswith(".hip")]

    def host_obj(src):
        obj = os.path.join(out, os.path.basename(src) + ".o")
        _run([hipcc(), *flags, *SANITIZE, "-x", "hip", "-c", src, "-o", obj], f"hipcc {os.path.basename(src)}",
             verbose)
        return obj

    def kernel_obj(src):
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        if os.path.exists(obj) and os.path.getmtime(obj) >= max(os.path.getmtime(src), _newest_header()):
            return obj
        os.makedirs(BUILD, exist_ok=True)
        return _compile(src, verbose)

    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(hosts) + len(kernels))) as ex:
        objs = list(ex.map(host_obj, hosts)) + list(ex.map(kernel_obj, kernels))
    _run([hipcc(), f"--offload-arch={ARCH}", *SANITIZE, "-o", HOST_CHECK, *objs], "host_check link", verbose)
    return HOST_CHECK


def _newest_header() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hs += [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE) if f.endswith(".h")]
    return max(os.path.getmtime(h) for h in hs)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
    if "check" in sys.argv:
        print(build_host_check(verbose="-v" in sys.argv))
