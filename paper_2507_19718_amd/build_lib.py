"""Builds libgsc.so (the HIP kernels and the C-ABI runtime) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgsc.so")
DEBUG_LIB = os.path.join(HERE, "libgsc_debug.so")
SOURCES = ["k_project.hip", "k_sort.hip", "k_bin.hip", "k_splat.hip", "k_trace.hip",
           "k_train.hip", "k_init.hip", "k_probe.hip", "runtime.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# fp32 in program order (no FMA contraction), correctly rounded division and square root,
# fp32 denormals kept, no packed-fp32 instructions.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-fno-fast-math", "-fhip-fp32-correctly-rounded-divide-sqrt",
         "-fno-gpu-flush-denormals-to-zero", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wall", "-Wno-unused-function"]


def _compile(src: str, debug: bool = False) -> str:
    out = os.path.join(BUILD, "debug" if debug else "", src.replace(".hip", ".o"))
    cmd = [HIPCC] + FLAGS + (["-DGSC_DEBUG"] if debug else []) + [
        "-I", os.path.join(HERE, "..", "include"), "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = ("packed-fp32-ops", "ignoring feature")
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if not any(n in l for n in noise))
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
    if msg.strip():
        sys.stderr.write(msg + "\n")
    return out


def build(verbose: bool = True, debug: bool = False) -> str:
    """Compiles every HIP source and links libgsc.so (debug: libgsc_debug.so, with the device
    bounds checks of -DGSC_DEBUG).  Always recompiles."""
    if not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(os.path.join(BUILD, "debug" if debug else ""), exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, debug), SOURCES))
    target = DEBUG_LIB if debug else LIB
    tmp = target + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, target)
    if verbose:
        print(f"built {target}")
    return target


# The host-ASan check: the library's sources and a driver of its C ABI linked into one
# executable whose host code is built with AddressSanitizer (device code as in the library; the
# GPU code itself is not instrumented).  Run by tests/test_gpu_host_asan.py.
ASAN_DIR = os.path.join(BUILD, "asan")
ASAN_EXE = os.path.join(ASAN_DIR, "gsc_host_asan")
ASAN_DRIVER = os.path.join(HERE, "..", "tests", "native", "host_asan_check.hip")
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
              "-Xarch_host", "-g"]


def _compile_asan(src: str) -> str:
    out = os.path.join(ASAN_DIR, os.path.basename(src).replace(".hip", ".o"))
    cmd = [HIPCC] + FLAGS + ASAN_FLAGS + ["-I", os.path.join(HERE, "..", "include"), "-c", src,
                                          "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc (host ASan) failed for {src}:\n{r.stdout + r.stderr}")
    return out


def build_host_asan_check(verbose: bool = True) -> str:
    """Builds the host-ASan check executable (always recompiles)."""
    os.makedirs(ASAN_DIR, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES] + [ASAN_DRIVER]
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile_asan, srcs))
    tmp = ASAN_EXE + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("host ASan link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, ASAN_EXE)
    if verbose:
        print(f"built {ASAN_EXE}")
    return ASAN_EXE


if __name__ == "__main__":
    build()
    if "--debug" in sys.argv[1:]:
        build(debug=True)
    if "--host-asan" in sys.argv[1:]:
        build_host_asan_check()
