"""Build libhelm.so (HIP, gfx950) in-tree.

    python -m paper_1809_03808_amd.build

Compiles the host FP64 eigen-setup with g++ (OpenMP) and every HIP source
with hipcc for gfx950, then links them into
``paper_1809_03808_amd/libhelm.so`` with an rpath to the ROCm libraries.
"""

import concurrent.futures
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libhelm.so")
BUILD = os.path.join(ROOT, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = os.environ.get("HELM_OFFLOAD_ARCH", "gfx950")

HIP_SOURCES = ["fft.hip", "lines.hip", "boundary.hip", "stencil.hip", "dense.hip", "cap.hip", "eigdev.hip", "solver.hip"]
CXX_SOURCES = ["eig1d.cpp"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose=False):
    """Compile and link; returns the path of the shared library."""
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    jobs = []
    objs = []
    for s in CXX_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        jobs.append(["g++", "-O3", "-std=c++17", "-fPIC", "-fopenmp", "-fcx-fortran-rules", "-Wall", *inc,
                     "-c", os.path.join(CSRC, s), "-o", o])
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        jobs.append([hipcc, *HIPCC_FLAGS, *inc, "-c", os.path.join(CSRC, s), "-o", o])
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = OUT + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp,
          "-lgomp", f"-Wl,-rpath,{ROCM}/lib"])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    p = build(verbose="-v" in sys.argv)
    print(p)
