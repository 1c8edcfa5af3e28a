"""The host precompute (mesh checks, KD tree, Delaunay with exact
predicates, Voronoi cells, the filter and flooding with their threads,
packing, save / load) built on its own with AddressSanitizer and
UndefinedBehaviorSanitizer, and with ThreadSanitizer for the threaded
stages, and driven through the C interface on small meshes in every table
mode (tests/host_sanitize/driver.cpp); any sanitizer report fails the test.
CPU only: the device sources are left out (stubs.cpp stands in for the two
device entry points the host code calls)."""
from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

from synth import configs as C
from synth import mesh as M
from tests._helpers import CUBE_F, CUBE_V, TETRA_F, TETRA_V

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2308_16084_amd", "csrc")
HOST = ["predicates.cpp", "delaunay.cpp", "convex_cell.cpp", "mesh.cpp", "kdtree.cpp", "interception.cpp",
        "p2m_host.cpp"]


def _write(path, V, F, S=None):
    V = np.ascontiguousarray(V, np.float32)
    F = np.ascontiguousarray(F if F is not None else np.zeros((0, 3)), np.int32)
    S = np.ascontiguousarray(S if S is not None else np.zeros((0, 2)), np.int32)
    with open(path, "wb") as fh:
        fh.write(np.array([len(V), len(F), len(S)], np.int64).tobytes())
        fh.write(V.tobytes())
        fh.write(F.tobytes())
        fh.write(S.tobytes())


def _meshes(tmp):
    paths = []
    items = [("tetra", TETRA_V, TETRA_F, None), ("cube", CUBE_V, CUBE_F, None)]
    V, F = C.sphere_mesh(2, "uniform", 5)
    items.append(("sphere2", V, F, None))
    Vh, Fh = M.heightfield(10, 3)
    items.append(("heightfield10", Vh, Fh, None))
    # a mixed set: the tetrahedron plus a free segment crossing it
    Vm = np.concatenate([TETRA_V, [[0.2, 0.2, -0.5], [0.3, 0.1, 1.5]]]).astype(np.float32)
    items.append(("mixed", Vm, TETRA_F, np.array([[4, 5]], np.int32)))
    for name, V_, F_, S_ in items:
        p = os.path.join(tmp, name + ".bin")
        _write(p, V_, F_, S_)
        paths.append(p)
    return paths


def _build_and_run(tmp, flags, env_extra, openmp=True):
    exe = os.path.join(tmp, "driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags, "-ffp-contract=off",
           f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
           *[os.path.join(CSRC, s) for s in HOST], os.path.join(HERE, "host_sanitize", "stubs.cpp"),
           os.path.join(HERE, "host_sanitize", "driver.cpp"), "-o", exe, "-lpthread"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, **env_extra)
    env["OMP_NUM_THREADS"] = "4"
    r = subprocess.run([exe, tmp, *_meshes(tmp)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]


def test_host_precompute_asan_ubsan(tmp_path):
    _build_and_run(str(tmp_path), ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                   {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1"})


def test_host_precompute_tsan(tmp_path):
    """The threads of the host build (std::thread work queues; the OpenMP
    loops are compiled serially here: libgomp is not instrumented, so its
    barriers would read as races)."""
    _build_and_run(str(tmp_path), ["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"}, openmp=False)
