"""Build libatsparse.so in-tree: HIP kernels for gfx950 with hipcc, the host
planner and runtime with g++, linked into one shared library."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libatsparse.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
INC = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-munsafe-fp-atomics", "-mllvm", "-disable-promote-alloca-to-lds", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__",
             "-I" + os.path.join(ROCM, "include")]

SOURCES = {
    "kernels.hip": "hip",
    "mpm.hip": "hip",
    "sfg.cpp": "cxx",
    "runtime.cpp": "cxx",
    "jit.cpp": "cxx",
}
HEADERS = ["internal.hpp", "sfg.hpp", "grid_device.hpp"]


def _compile(name: str, kind: str, verbose: bool) -> str:
    src = os.path.join(CSRC, name)
    obj = os.path.join(BUILD, name + ".o")
    if kind == "hip":
        cmd = [os.path.join(ROCM, "bin", "hipcc"), "-c", *HIP_FLAGS, *INC, src, "-o", obj]
    else:
        cmd = ["g++", "-c", *CXX_FLAGS, *INC, src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (name, r.stdout, r.stderr))
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source and link the library (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda kv: _compile(kv[0], kv[1], verbose), SOURCES.items()))
    tmp = LIB + ".tmp"
    cmd = [os.path.join(ROCM, "bin", "hipcc"), "-shared", "-fPIC", "--offload-arch=gfx950", *objs,
           "-o", tmp, "-Wl,-soname,libatsparse.so", "-L" + os.path.join(ROCM, "lib"), "-lhiprtc"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


def built() -> bool:
    if not os.path.exists(LIB):
        return False
    t = os.path.getmtime(LIB)
    srcs = [os.path.join(CSRC, s) for s in list(SOURCES) + HEADERS] + [os.path.join(ROOT, "include", "atsparse.h")]
    return all(os.path.getmtime(s) <= t for s in srcs)


if __name__ == "__main__":
    print(build(verbose=True))
