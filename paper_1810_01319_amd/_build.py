"""Compile the HIP library libamr.so for gfx950 (in-tree, next to this file)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
SO = os.path.join(HERE, "libamr.so")
SOURCES = ["kernels.hip", "adjoint.hip", "tracers.hip", "comoving.hip", "poisson.hip", "composite.hip", "mesh.cpp", "capi.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall",
          "-I" + os.path.join(HERE, "..", "include")]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, "-c", os.path.join(SRC, src), "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = DEVICE
    else:
        cmd[1:1] = ["-D__HIP_PLATFORM_AMD__"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


CORE_SO = os.path.join(HERE, "libamr_core_host.so")


def build_core_host() -> str:
    """Host build of the sweep formulas and their adjoint, for the CPU unit
    tests of the adjoint (g++, no FMA contraction)."""
    tmp = CORE_SO + ".tmp"
    r = subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
                        "-o", tmp, os.path.join(SRC, "core_host.cpp")], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("g++ failed on core_host.cpp:\n" + r.stderr)
    os.replace(tmp, CORE_SO)
    return CORE_SO


def build(force: bool = True) -> str:
    if not force and os.path.exists(SO):
        return SO
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = SO + ".tmp"
    r = subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, SO)
    build_core_host()
    return SO


def build_host_sanitized(path: str) -> str:
    """The library with its host half (mesh.cpp, capi.cpp) compiled by g++
    with AddressSanitizer and UndefinedBehaviorSanitizer (abort on the first
    report) and linked with the device objects of the last build(): for the
    CPU suite's sanitizer run, loaded in place of libamr.so when AMR_LIBRARY
    names it (with the sanitizer runtimes preloaded).  Nothing in the device
    code is sanitized."""
    objs = [os.path.join(BUILD, s + ".o") for s in SOURCES if s.endswith(".hip")]
    missing = [o for o in objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"device objects missing (run build() first): {missing}")
    san = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    out_dir = os.path.dirname(os.path.abspath(path))
    host = []
    for src in ("mesh.cpp", "capi.cpp"):
        obj = os.path.join(out_dir, src + ".san.o")
        r = subprocess.run(["g++", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", *san,
                            "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                            "-I" + os.path.join(HERE, "..", "include"), "-c", os.path.join(SRC, src), "-o", obj],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"g++ failed on {src}:\n{r.stderr}")
        host.append(obj)
    r = subprocess.run(["g++", "-shared", "-fsanitize=address,undefined", "-o", path, *host, *objs,
                        "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("sanitized link failed:\n" + r.stderr)
    return path


if __name__ == "__main__":
    print(build())
