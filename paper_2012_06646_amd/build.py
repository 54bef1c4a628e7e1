"""Build libibops.so (HIP kernels + C-ABI host runtime) for gfx950, in-tree.

Usage: python -m paper_2012_06646_amd.build  (or call build()).
"""
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libibops.so")
OBJDIR = os.path.join(ROOT, "_build")

SOURCES = ["ib_api.cpp", "ib_batch.cpp", "ib_server.cpp", "plan_kernels.hip", "ops_kernels.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("IBOPS_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
         # packed fp32 instructions stay disabled in all device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _compile(src, obj, verbose):
    cmd = [HIPCC] + FLAGS + ["-c", "-x", "hip", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False, jobs: int = 4) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    t0 = time.time()
    from concurrent.futures import ThreadPoolExecutor
    objs = []
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = []
        for s in SOURCES:
            obj = os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o")
            futs.append(ex.submit(_compile, os.path.join(CSRC, s), obj, verbose))
            objs.append(obj)
        for f in futs:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "-pthread", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
