"""The C interface: libp2m.so loads and exports every function that
include/p2m.h declares (no device calls)."""
from __future__ import annotations

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "p2m.h")


def declared() -> set[str]:
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b(p2m_[a-z_]+)\s*\(", text))


def test_header_declares_the_interface():
    names = declared()
    for n in ("p2m_mesh_create", "p2m_precompute", "p2m_upload", "p2m_query", "p2m_query_backward",
              "p2m_order_queries", "p2m_nearest_vertex", "p2m_batch_create", "p2m_batch_query",
              "p2m_batch_autotune", "p2m_save", "p2m_load", "p2m_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2308_16084_amd import _lib
    path = _lib.LIB_PATH
    assert os.path.exists(path), "build the library first"
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s+(p2m_\w+)", out))
    missing = declared() - exported
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2308_16084_amd import _lib
    _lib.lib()
    assert declared() == set(_lib.exported_symbols())


def test_errors_without_device():
    """Calls that need an uploaded mesh fail with P2M_ERR_STATE, not a crash."""
    import ctypes

    import numpy as np

    import paper_2308_16084_amd as P
    from paper_2308_16084_amd._lib import lib
    from tests._helpers import TETRA_F, TETRA_V
    m = P.Mesh(TETRA_V, TETRA_F)
    m.precompute()
    z = ctypes.c_void_p(0)
    st = lib().p2m_query(m.handle, z, 4, z, z, z, z, z, z, z, z)
    assert st == -3 and b"upload" in lib().p2m_last_error()
    assert lib().p2m_query(m.handle, z, -1, z, z, z, z, z, z, z, z) == -1
    assert lib().p2m_query_backward(m.handle, z, 4, z, z, z, z, z, z, z, z) == -3
    assert lib().p2m_mesh_create(None, 3, None, 1, ctypes.byref(ctypes.c_void_p())) == -1
    with pytest.raises(P.P2MError):
        P.Mesh(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32))


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures have the size and field offsets the C
    compiler gives the header's structs."""
    import ctypes

    from paper_2308_16084_amd import _lib
    pairs = {"p2m_build_opts": _lib.BuildOpts, "p2m_build_stats": _lib.BuildStats, "p2m_query_opts": _lib.QueryOpts}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "p2m.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'    printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, py in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU; --gpus above 1 exits with a message."""
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout
