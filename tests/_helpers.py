"""Shared test helpers: tiny closed-form meshes and the golden-file parser."""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

CUBE_V = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], dtype=np.float32)
CUBE_F = np.array([[0, 2, 6], [0, 6, 4], [1, 3, 7], [1, 7, 5], [0, 1, 5], [0, 5, 4],
                   [2, 3, 7], [2, 7, 6], [0, 1, 3], [0, 3, 2], [4, 5, 7], [4, 7, 6]], dtype=np.int32)
TETRA_V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float32)
TETRA_F = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], dtype=np.int32)

TYPE_CODE = {"V": 0, "E": 1, "F": 2}


def load_golden(name: str):
    """Rows of (q, [(type, frozenset(vertex ids))], d, c or None)."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            q, prims, d, c = [s.strip() for s in line.split(";")]
            q = np.array([float(x) for x in q.split()], dtype=np.float64)
            plist = []
            for p in prims.split("|"):
                t, ids = p.split(":")
                plist.append((TYPE_CODE[t], frozenset(int(x) for x in ids.split(","))))
            c = None if c == "-" else np.array([float(x) for x in c.split()])
            rows.append((q, plist, float(d), c))
    return rows


def primitive_vertices(F: np.ndarray, E: np.ndarray, ptype: int, pid: int) -> frozenset:
    if ptype == 0:
        return frozenset([int(pid)])
    if ptype == 1:
        return frozenset(int(x) for x in E[pid])
    return frozenset(int(x) for x in F[pid])


def random_tiny_mesh(rng: np.random.Generator, kind: str = "sphere"):
    """A small closed or open mesh with generic coordinates."""
    from synth import mesh as M
    if kind == "sphere":
        V, F = M.icosphere(1)
        V = M.displace_uniform(V, 0.15, int(rng.integers(1 << 30)))
    else:
        V, F = M.heightfield(6, int(rng.integers(1 << 30)), jitter=0.3)
    return V.astype(np.float32), F.astype(np.int32)
