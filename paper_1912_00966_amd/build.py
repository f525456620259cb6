"""Builds libeat.so (gfx950 HIP kernels + C++ host runtime) in place.

Every source is compiled to an object of its own, in parallel (the three
relaxation-kernel sources dominate), then linked into one shared library.

    python -m paper_1912_00966_amd.build
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libeat.so")
OBJ_DIR = os.path.join(HERE, "_build")
SOURCES = ["layout.cpp", "subtrips.cpp", "capi.cpp", "queries.cpp", "variants.cpp", "session.cpp", "tune.cpp",
           "kernels.hip", "batch_static.hip", "journeys.hip", "variant_kernels.hip", "relax_grid.hip", "relax_compact.hip",
           "relax_flat.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found; the library needs ROCm's HIP compiler")
    return p


def _flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            # packed fp32 instructions are kept out of every kernel
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]


def _compile(src, verbose):
    obj = os.path.join(OBJ_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + _flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    return obj, r


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    with ThreadPoolExecutor(max(1, jobs)) as ex:
        results = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    msgs = []
    for (obj, r), src in zip(results, SOURCES):
        out = r.stdout + r.stderr
        if r.returncode != 0:
            raise RuntimeError(f"libeat build failed compiling {src}:\n{out}")
        msgs += [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results] + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("libeat link failed:\n" + r.stdout + r.stderr)
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
