"""Build ``libfamlies.so`` (HIP kernels + planner + C ABI) for gfx950 with
hipcc.  Usage: ``python -m paper_2604_07311_amd.build`` (always rebuilds)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfamlies.so")
OBJDIR = os.path.join(HERE, "_build")

SOURCES = ["abi.hip", "planner.cpp", "table.cpp", "plain_kernels.hip", "split_kernels.hip",
           "batch.hip", "tune.hip", "pack_kernels.hip", "network.cpp", "registry.cpp", "plan_host.cpp", "int8_kernels.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXX = os.environ.get("FAMLIES_CXX", "/opt/rocm/lib/llvm/bin/clang++")
ARCH = "gfx950"
COMMON = ["-O3", "-fPIC", "-std=c++17", "-I" + INCLUDE, "-I" + CSRC, "-Wall",
          "-Wno-unused-parameter", "-Wno-unused-variable"]
# Packed FP32 instructions stay disabled in every device compile.
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _headers_mtime() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    hs += [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE)]
    return max(os.path.getmtime(h) for h in hs)


def _compile(src: str, extra=()) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    # FAMLIES_INCREMENTAL=1 (development only) keeps objects newer than their
    # source and every header; the default rebuilds everything.
    if os.environ.get("FAMLIES_INCREMENTAL") == "1" and not extra and os.path.exists(obj) and \
            os.path.getmtime(obj) > max(os.path.getmtime(path), _headers_mtime()):
        return obj
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip"] + DEVICE + COMMON + list(extra) + ["-c", path, "-o", obj]
    else:  # host-only C++
        cmd = [CXX] + COMMON + ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"] + list(extra) + \
            ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose: bool = False, extra=()) -> str:
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
