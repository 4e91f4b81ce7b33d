"""Build librad.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Every source is compiled to an object file in parallel (one hipcc per source,
objects under _build/), then linked into one shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "librad.so")
OBJ = os.path.join(PKG, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["rad_kernels.hip", "rad_lib.cpp", "rad_static.hip", "mlp_kernels.hip", "mlp_lib.cpp",
           "sampler_kernels.hip", "sampler_lib.cpp", "traj_kernels.hip", "traj_lib.cpp", "peak_kernels.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the GPU code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _compile(src, extra, verbose, tag=""):
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + tag + ".o")
    cmd = [HIPCC] + FLAGS + extra + ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c",
                                     os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False, extra=(), out: str = LIB, tag: str = "") -> str:
    """Compile and link; `extra` flags go to every compile, objects get the suffix `tag`."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, list(extra), verbose, tag), SOURCES))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


# Host code (validation, planning, workspace layout, bindings) with the address and
# undefined-behaviour sanitizers; the GPU code is built as usual.  The library leaves the
# sanitizer runtime to the process: load it with the runtime preloaded (SANITIZER_RUNTIME).
SAN_LIB = os.path.join(OBJ, "librad_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def sanitizer_runtime() -> str:
    """The compiler's shared address-sanitizer runtime (it carries the UB handlers too)."""
    import glob
    hits = sorted(glob.glob(os.path.join(os.path.dirname(os.path.dirname(HIPCC)), "llvm", "lib", "clang", "*",
                                         "lib", "linux", "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise RuntimeError("no libclang_rt.asan-x86_64.so next to %s" % HIPCC)
    return hits[-1]


def build_sanitized(verbose: bool = False) -> str:
    return build(verbose, extra=SAN_FLAGS, out=SAN_LIB, tag="_san")


# The kernels' index checks (RAD_DEBUG; see rad_debug_violations), in-tree beside librad.so.
DEBUG_LIB = os.path.join(PKG, "librad_debug.so")


def build_debug(verbose: bool = False) -> str:
    return build(verbose, extra=["-DRAD_DEBUG=1"], out=DEBUG_LIB, tag="_dbg")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
