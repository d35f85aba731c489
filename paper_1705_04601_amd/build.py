"""Builds libh2sp.so (HIP for gfx950 + host C++) in this directory.

Every source is compiled by hipcc: the .hip file for the device, the .cpp
files as host C++ against the HIP runtime.  The cluster-tree file is built
with -ffp-contract=off so that the admissibility tests are evaluated one
rounded operation at a time.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libh2sp.so")
OBJ = os.path.join(HERE, "_build")
ARCH = os.environ.get("H2SP_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# host-only translation units: plain C++ against the HIP runtime headers
CXX = os.environ.get("H2SP_CXX", "/opt/rocm/llvm/bin/clang++")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I", os.path.join(HERE, "..", "include")]
HOST = ["-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# the wide GEMM tiles (up to 32 accumulator blocks) need their epilogue fully
# unrolled, or the accumulators move to scratch memory
WIDE = DEVICE + ["-mllvm", "-pragma-unroll-threshold=200000"]

SOURCES = {
    "kernels.hip": DEVICE,
    "gemm_transform.hip": DEVICE,
    "gemm_transform_gen.hip": DEVICE,
    "gemm_factor.hip": DEVICE,
    "gemm_solve.hip": WIDE,
    "gemm_matvec.hip": DEVICE,
    "tune.cpp": [],
    "autotune.cpp": [],
    "runtime.cpp": [],
    "tree.cpp": ["-ffp-contract=off"],
    "h2build.cpp": ["-fopenmp"],
    "matrix.cpp": ["-fopenmp"],
    "sparsify.cpp": ["-fopenmp"],
    "factor.cpp": ["-fopenmp"],
    "solve.cpp": ["-fopenmp"],
    "api.cpp": [],
}


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + res.stdout + res.stderr)
        raise RuntimeError(f"compile failed: {cmd[-1]}")
    return res


def _stale(obj: str, src: str) -> bool:
    """An object is stale when it is missing or older than its source or any
    header of the library."""
    if not os.path.exists(obj):
        return True
    deps = [src] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")] + \
        [os.path.join(HERE, "..", "include", h) for h in os.listdir(os.path.join(HERE, "..", "include"))]
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, force: bool = True) -> str:
    """Compiles every source (force) or only the stale ones, then links."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJ, exist_ok=True)
    objs, cmds = [], []
    for src, extra in SOURCES.items():
        obj = os.path.join(OBJ, src + ".o")
        objs.append(obj)
        if not force and not _stale(obj, os.path.join(CSRC, src)):
            continue
        if src.endswith(".hip"):
            cmd = [HIPCC] + COMMON + extra
        else:
            cmd = [CXX] + COMMON + HOST + extra
        cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        cmds.append(cmd)
    # translation units are independent: compile them side by side
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    if cmds:
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            list(ex.map(_run, cmds))
    tmp = LIB + ".tmp"
    link = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fopenmp", "-o", tmp] + objs + \
        ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/llvm/lib"]
    if verbose:
        print(" ".join(link), flush=True)
    _run(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, force="--changed" not in sys.argv))
