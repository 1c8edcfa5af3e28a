"""Build libp2m.so in-tree: host C++ with g++ (OpenMP), device code with hipcc
for gfx950, linked into one shared library next to this file."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libp2m.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HOST_SOURCES = ["predicates.cpp", "delaunay.cpp", "convex_cell.cpp", "mesh.cpp", "kdtree.cpp",
                "interception.cpp", "p2m_host.cpp"]
DEVICE_SOURCES = ["p2m_device.hip", "radix_sort.hip", "p2m_batch.hip", "p2m_flood.hip"]
# The device inspection repeats the host builder's FP64 operations exactly:
# no contraction into fused multiply-adds, as in the host build.
EXTRA_FLAGS = {"p2m_flood.hip": ["-ffp-contract=off"]}

HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-fopenmp", "-Wall", "-Wextra", "-Wno-unused-parameter",
              "-ffp-contract=off", f"-I{INCLUDE}"]
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", f"-I{INCLUDE}",
             # packed FP32 instructions are kept out of every HIP build
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + p.stdout)
    return p.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    jobs = []
    for s in HOST_SOURCES:
        jobs.append(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, s), "-o", os.path.join(BUILD, s + ".o")])
    for s in DEVICE_SOURCES:
        jobs.append([hipcc, *HIP_FLAGS, *EXTRA_FLAGS.get(s, []), "-c", os.path.join(CSRC, s), "-o",
                     os.path.join(BUILD, s + ".o")])
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    objs = [os.path.join(BUILD, s + ".o") for s in HOST_SOURCES + DEVICE_SOURCES]
    tmp = LIB + ".tmp"
    _run(["g++", "-shared", "-o", tmp, *objs, "-fopenmp", f"-L{ROCM}/lib", "-lamdhip64",
          f"-Wl,-rpath,{ROCM}/lib"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
