"""Build the gfx950 HIP library (libibm.so) in-tree with hipcc.

    python -m paper_2505_17287_amd.build

Flags: -O3, gfx950 only, no floating-point contraction (geometry predicates and the
smoother reproduce a plain sequential evaluation bit for bit), packed-FP32 instructions
disabled for the device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libibm.so")
SOURCES = ["geometry.hip", "sweep.hip", "sweepc.hip", "finepass.hip", "solver.hip", "momentum.hip", "noalloc.hip", "api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
LIBS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]  # named host ranges (roctx)
FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-std=c++17", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(OBJ, src.replace(".hip", ".o"))
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(SRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, *LIBS]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


def build_host_sanitized(out_dir: str) -> str:
    """The library with its host code (argument checks, level planning, workspace layout,
    mesh validation, schedules) built with AddressSanitizer and UndefinedBehaviorSanitizer;
    the device code is built as usual (at -O1) and is not instrumented.  Load it with
    IBM_LIB=<path> in a process that preloads clang's ASan runtime (asan_runtime()); it is
    meant for the host entry points, on a machine without a GPU."""
    os.makedirs(out_dir, exist_ok=True)
    san = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined".split()
    host = ["-O1", "-g", "-fPIC", "-std=c++17", "-ffp-contract=off", "--offload-arch=gfx950",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", *san]

    def compile_one(src):
        obj = os.path.join(out_dir, src.replace(".hip", ".san.o"))
        r = subprocess.run([HIPCC, *host, "-c", os.path.join(SRC, src), "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc (sanitized host) failed for %s:\n%s" % (src, r.stderr))
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    out = os.path.join(out_dir, "libibm_san.so")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *san,
                        "-Xarch_host", "-shared-libsan", "-o", out, *objs, *LIBS], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("sanitized link failed:\n%s" % r.stderr)
    return out


def asan_runtime() -> str:
    """clang's shared ASan runtime of the ROCm toolchain (preloaded for build_host_sanitized)."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise FileNotFoundError("libclang_rt.asan-x86_64.so not found under /opt/rocm/llvm")
    return hits[-1]


if __name__ == "__main__":
    print(build(verbose=True))
