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


def gate_boundary_points(V, F, E, lo, hi, rng, n=400):
    """Points where the list scan's gates decide: on edges (midpoints and near
    the ends), at vertices, on faces, pushed off the surface by tiny and by
    large amounts, and the corners of the box [lo, hi]; clipped to the box."""
    Vd = np.asarray(V, dtype=np.float64)
    tri = Vd[F]
    nrm = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    pts = []
    ke = rng.integers(0, len(E), n)
    for t in (0.5, 1e-4, 1 - 1e-4, 0.0):
        pts.append(Vd[E[ke, 0]] * (1 - t) + Vd[E[ke, 1]] * t)
    kf = rng.integers(0, len(F), n)
    b = rng.dirichlet([1, 1, 1], n)
    on_face = (tri[kf] * b[:, :, None]).sum(1)
    pts.append(on_face)
    diag = float(np.linalg.norm(np.asarray(hi) - np.asarray(lo)))
    for h in (1e-7, 1e-4, 0.05, 0.3):
        pts.append(on_face + h * diag * nrm[kf])
        pts.append(pts[0] + h * diag * rng.normal(size=(n, 3)))
    corners = np.array([[x, y, z] for x in (lo[0], hi[0]) for y in (lo[1], hi[1]) for z in (lo[2], hi[2])])
    pts.append(corners)
    return np.clip(np.concatenate(pts), lo, hi).astype(np.float32)


def margin_points(V, F, E, diag, mu, rng, n=1000):
    """Points within the list scan's gate margin mu of primitive boundaries,
    where a primitive passes its gate with its foot just off it: within
    1e-5 diag of random edges; in a face's plane (or up to 1e-4 diag off it)
    at -3.5 mu .. 3.5 mu from one of its sides; within 5e-5 diag of
    vertices."""
    Vd = np.asarray(V, dtype=np.float64)
    pts = []
    ke = rng.integers(0, len(E), n)
    t = rng.uniform(0, 1, n)
    base = Vd[E[ke, 0]] * (1 - t[:, None]) + Vd[E[ke, 1]] * t[:, None]
    dirs = rng.normal(size=(n, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    pts.append(base + dirs * rng.uniform(0, 1e-5 * diag, (n, 1)))
    tri = Vd[F]
    nrm = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    kf = rng.integers(0, len(F), n)
    side = rng.integers(0, 3, n)
    a, b, c = tri[kf, side], tri[kf, (side + 1) % 3], tri[kf, (side + 2) % 3]
    tt = rng.uniform(0.05, 0.95, n)
    p = a * (1 - tt[:, None]) + b * tt[:, None]
    inward = np.cross(nrm[kf], b - a)
    inward /= np.linalg.norm(inward, axis=1, keepdims=True)
    inward *= np.sign(np.einsum("ij,ij->i", inward, c - p))[:, None]
    s = rng.uniform(-3.5, 3.5, n) * mu
    h = rng.choice([0.0, 1e-7, 1e-6, 1e-5, 1e-4], n) * diag * rng.choice([-1, 1], n)
    pts.append(p + inward * s[:, None] + nrm[kf] * h[:, None])
    kv = rng.integers(0, len(Vd), n)
    pts.append(Vd[kv] + dirs * rng.uniform(0, 5e-5 * diag, (n, 1)))
    return np.concatenate(pts).astype(np.float32)


def odd_meshes(rng: np.random.Generator):
    """Inputs far from a clean surface mesh: a soup of 200 disconnected,
    intersecting triangles; a fan of 64 triangles round one vertex; 150
    slivers (third corner near the opposite side); 300 triangles drawn at
    random over 120 shared vertices (non-manifold, long lists)."""
    def soup(nf):
        return rng.uniform(0, 1, size=(3 * nf, 3)).astype(np.float32), np.arange(3 * nf, dtype=np.int32).reshape(nf, 3)

    out = [("soup200",) + soup(200)]
    a = np.linspace(0, 2 * np.pi, 64, endpoint=False)
    ring = np.stack([np.cos(a), np.sin(a), 0.05 * rng.standard_normal(64)], 1)
    out.append(("fan64", np.vstack([[0.0, 0.0, 0.0], ring]).astype(np.float32),
                np.array([[0, 1 + i, 1 + (i + 1) % 64] for i in range(64)], np.int32)))
    V, F = soup(150)
    V = V.reshape(150, 3, 3)
    V[:, 2] = V[:, 0] + (V[:, 1] - V[:, 0]) * rng.uniform(0.2, 0.8, (150, 1)) + 1e-3 * rng.standard_normal((150, 3))
    out.append(("slivers150", V.reshape(-1, 3).astype(np.float32), F))
    V = rng.uniform(0, 1, size=(120, 3)).astype(np.float32)
    F = np.array([rng.choice(120, 3, replace=False) for _ in range(300)], np.int32)
    out.append(("shared300", V, F))
    return out


def flat_meshes():
    """Meshes whose vertices are coplanar (the Delaunay step meets a flat
    point set): one triangle, two coplanar triangles, planar grids of 8 x 8
    and 30 x 30 vertices, and a nearly collinear strip."""
    def grid(n):
        x, y = np.meshgrid(np.linspace(0, 1, n), np.linspace(0, 1, n))
        V = np.stack([x.ravel(), y.ravel(), np.zeros(n * n)], 1).astype(np.float32)
        F = []
        for i in range(n - 1):
            for j in range(n - 1):
                a = i * n + j
                F += [[a, a + 1, a + n], [a + 1, a + n + 1, a + n]]
        return V, np.array(F, np.int32)

    return [("one triangle", np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32), np.array([[0, 1, 2]], np.int32)),
            ("two coplanar", np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], np.float32),
             np.array([[0, 1, 2], [1, 3, 2]], np.int32)),
            ("grid 8",) + grid(8), ("grid 30",) + grid(30),
            ("strip", np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [0.5, 1e-3, 0], [1.5, 1e-3, 0]], np.float32),
             np.array([[0, 1, 3], [1, 2, 4]], np.int32))]
