"""Builds libelbm.so (HIP kernels for gfx950 + the C ABI) and the bandwidth
probe libelbm_probe.so in the package directory, and the plain C client of
the ABI (tests/c/abi_run.c) into _build/abi_run.

Usage: python -m paper_2101_04550_amd.build   (or build() from Python)

Every call recompiles all sources. hipcc cross-compiles for gfx950 without a
GPU. Packed FP32 instructions are disabled for all device code.
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
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libelbm.so")

SOURCES = ["elbm_step.hip", "elbm_aux.hip", "elbm_static.hip", "elbm_faces.hip", "elbm_walls3d.hip",
           "elbm_api.cpp"]
# bandwidth probe of the step's access pattern (measurement only)
PROBE_SOURCES = ["elbm_probe.hip"]
PROBE_LIB = os.path.join(PKG, "libelbm_probe.so")
ARCH = "gfx950"
# a C program that runs the step through the ABI alone (tests/test_gpu_c_client.py)
C_CLIENT = os.path.join(ROOT, "tests", "c", "abi_run.c")
C_CLIENT_EXE = os.path.join(BUILD, "abi_run")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: install ROCm or put hipcc on PATH")
    return exe


def common_flags():
    return [
        "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE, "-I", CSRC,
        "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    ]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), *common_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip() and verbose:
        print(r.stderr, file=sys.stderr)
    return obj


def _link(objs, out, verbose):
    tmp = out + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)


def _c_client(verbose):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("no C compiler for the ABI client")
    cmd = [cc, "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-I", INCLUDE, "-I", os.path.join(ROCM, "include"),
           C_CLIENT, "-o", C_CLIENT_EXE, "-L", PKG, "-l:libelbm.so", f"-Wl,-rpath,{PKG}",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"build of the C client failed:\n{r.stdout}\n{r.stderr}")


def build(verbose: bool = False) -> str:
    """Builds libelbm.so, the bandwidth probe libelbm_probe.so and the C
    client of the ABI."""
    os.makedirs(BUILD, exist_ok=True)
    sources = SOURCES + PROBE_SOURCES
    with cf.ThreadPoolExecutor(max_workers=len(sources)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), sources))
    _link(objs[:len(SOURCES)], LIB, verbose)
    _link(objs[len(SOURCES):], PROBE_LIB, verbose)
    _c_client(verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
