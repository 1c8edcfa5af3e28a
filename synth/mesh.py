"""Seeded synthetic triangle meshes (NumPy).

Shapes stand in for the paper's scanned models: displaced spheres (smooth,
closed, with the near-symmetric structure that the paper flags as the worst
case for interception-list length) and heightfields (open surfaces whose
compressed rows give needle triangles, standing in for the poor-triangulation
study).  Every mesh holds one copy of each vertex, as the problem statement
assumes.  Output coordinates are float32, faces int32.
"""
from __future__ import annotations

import numpy as np

from .noise import fbm2, fbm3

_PHI = (1.0 + 5.0 ** 0.5) / 2.0

ICOSA_V = np.array([
    [-1, _PHI, 0], [1, _PHI, 0], [-1, -_PHI, 0], [1, -_PHI, 0],
    [0, -1, _PHI], [0, 1, _PHI], [0, -1, -_PHI], [0, 1, -_PHI],
    [_PHI, 0, -1], [_PHI, 0, 1], [-_PHI, 0, -1], [-_PHI, 0, 1],
], dtype=np.float64)
ICOSA_F = np.array([
    [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
    [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
    [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
    [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
], dtype=np.int64)


def _normalize(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def icosphere(level: int) -> tuple[np.ndarray, np.ndarray]:
    """Unit icosphere by `level` rounds of 1->4 midpoint subdivision.

    Returns float64 unit vertices and int64 faces; V = 10*4^L+2, F = 20*4^L.
    """
    V = _normalize(ICOSA_V.copy())
    F = ICOSA_F.copy()
    for _ in range(level):
        nv = V.shape[0]
        e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0)
        lo = np.minimum(e[:, 0], e[:, 1])
        hi = np.maximum(e[:, 0], e[:, 1])
        key = lo * nv + hi
        uk, inv = np.unique(key, return_inverse=True)
        mid = _normalize(0.5 * (V[uk // nv] + V[uk % nv]))
        m = nv + inv.reshape(3, -1).T  # per face: m01, m12, m20
        a, b, c = F[:, 0], F[:, 1], F[:, 2]
        m01, m12, m20 = m[:, 0], m[:, 1], m[:, 2]
        F = np.concatenate([
            np.stack([a, m01, m20], 1), np.stack([b, m12, m01], 1),
            np.stack([c, m20, m12], 1), np.stack([m01, m12, m20], 1)], axis=0)
        V = np.concatenate([V, mid], axis=0)
    return V, F


def geodesic_sphere(freq: int) -> tuple[np.ndarray, np.ndarray]:
    """Class-I geodesic sphere: each icosahedron face split into freq^2 triangles.

    Points are the barycentric grid of each face projected to the unit sphere.
    Shared edge/corner points get one canonical key (corner ids sorted with
    their integer weights), so the vertex set holds one copy of each point.
    """
    n = int(freq)
    assert n >= 1
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    sel = ii + jj <= n
    gi, gj = ii[sel], jj[sel]
    gk = n - gi - gj
    npf = gi.size
    local_index = -np.ones((n + 1, n + 1), dtype=np.int64)
    local_index[gi, gj] = np.arange(npf)
    keys = []
    for f in ICOSA_F:
        cw = np.stack([np.broadcast_to(f[0], gi.shape), gi,
                       np.broadcast_to(f[1], gi.shape), gj,
                       np.broadcast_to(f[2], gi.shape), gk], axis=1)
        # canonical: zero weights get corner -1, then sort pairs by corner id
        c = cw[:, 0::2].copy()
        w = cw[:, 1::2].copy()
        c[w == 0] = -1
        order = np.argsort(c, axis=1, kind="stable")
        c = np.take_along_axis(c, order, 1)
        w = np.take_along_axis(w, order, 1)
        keys.append(np.concatenate([c, w], axis=1))
    keys = np.concatenate(keys, axis=0)
    uk, inv = np.unique(keys, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    cid = uk[:, :3]
    wts = uk[:, 3:].astype(np.float64)
    P = np.zeros((uk.shape[0], 3))
    for t in range(3):
        valid = cid[:, t] >= 0
        P[valid] += wts[valid, t:t + 1] * ICOSA_V[cid[valid, t]]
    V = _normalize(P)
    tris = []
    for a in range(n):
        for b in range(n - a):
            tris.append((local_index[a, b], local_index[a + 1, b], local_index[a, b + 1]))
            if a + b + 1 < n:
                tris.append((local_index[a + 1, b], local_index[a + 1, b + 1], local_index[a, b + 1]))
    tris = np.array(tris, dtype=np.int64)
    F = np.concatenate([inv[fi * npf + tris] for fi in range(20)], axis=0)
    # orient outward
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    flip = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def displace_uniform(Vunit: np.ndarray, amp: float, seed: int) -> np.ndarray:
    """r_i = 1 + U[-amp, amp] iid per vertex; v <- r_i * v_hat."""
    rng = np.random.default_rng(seed)
    r = 1.0 + rng.uniform(-amp, amp, size=Vunit.shape[0])
    return Vunit * r[:, None]


def displace_fbm(Vunit: np.ndarray, amp: float, seed: int, octaves: int = 4,
                 base_freq: float = 4.0) -> np.ndarray:
    """r = 1 + amp * fbm(v_hat); v <- r * v_hat."""
    r = 1.0 + amp * fbm3(Vunit, seed, octaves=octaves, base_freq=base_freq)
    return Vunit * r[:, None]


def heightfield(n: int, seed: int, amp: float = 0.2, jitter: float = 0.45,
                compress_every: int = 7, compress_factor: float = 20.0,
                octaves: int = 6, base_freq: float = 8.0) -> tuple[np.ndarray, np.ndarray]:
    """n x n heightfield over [0,1]^2 with compressed rows and in-plane jitter.

    The gap after every row j = 0 (mod compress_every) is compress_factor
    times smaller than the others (needle triangles); rows are renormalised
    to [0,1].  x is jittered by up to jitter*dx, y by up to jitter times the
    smaller adjacent row gap.  Quads are split on the (i,j)-(i+1,j+1) diagonal.
    z = amp * fbm2(x, y).
    """
    rng = np.random.default_rng(seed)
    gaps = np.ones(n - 1)
    gaps[np.arange(n - 1) % compress_every == 0] = 1.0 / compress_factor
    y = np.concatenate([[0.0], np.cumsum(gaps)])
    y /= y[-1]
    gaps = np.diff(y)
    x = np.linspace(0.0, 1.0, n)
    dx = 1.0 / (n - 1)
    adj = np.empty(n)
    adj[0] = gaps[0]
    adj[-1] = gaps[-1]
    adj[1:-1] = np.minimum(gaps[:-1], gaps[1:])
    X, Y = np.meshgrid(x, y, indexing="xy")  # X[j, i], Y[j, i]; row j = y index
    jx = rng.uniform(-1.0, 1.0, size=X.shape) * jitter * dx
    jy = rng.uniform(-1.0, 1.0, size=Y.shape) * jitter * adj[:, None]
    # keep the outer boundary on the unit square
    jx[:, 0] = 0.0
    jx[:, -1] = 0.0
    jy[0, :] = 0.0
    jy[-1, :] = 0.0
    jj, ii = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="ij")
    v00 = (jj * n + ii).ravel()
    v10 = v00 + 1
    v01 = v00 + n
    v11 = v00 + n + 1
    F = np.concatenate([np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)], axis=0)
    # nominal (unjittered) area of each triangle: half a cell of its row
    nominal = np.tile(0.5 * dx * np.repeat(gaps, n - 1), 2)
    jx = jx.ravel()
    jy = jy.ravel()
    X0 = X.ravel()
    Y0 = Y.ravel()
    # Halve the jitter of every vertex of a triangle whose xy area fell below
    # 5% of its nominal area (or inverted) until no such triangle remains.
    for _ in range(60):
        xy = np.stack([X0 + jx, Y0 + jy], axis=1)
        bad = signed_xy_area(xy, F) <= 0.05 * nominal
        if not bad.any():
            break
        vb = np.unique(F[bad].ravel())
        jx[vb] *= 0.5
        jy[vb] *= 0.5
    else:
        raise RuntimeError("heightfield jitter did not converge")
    Z = amp * fbm2(xy, seed + 7, octaves=octaves, base_freq=base_freq)
    V = np.concatenate([xy, Z[:, None]], axis=1)
    return V, F


def signed_xy_area(V: np.ndarray, F: np.ndarray) -> np.ndarray:
    a, b, c = V[F[:, 0], :2], V[F[:, 1], :2], V[F[:, 2], :2]
    return 0.5 * ((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))


def triangle_quality(V: np.ndarray, F: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Per-triangle quality Q = (6/sqrt 3) S / (p h) (S area, p half-perimeter,
    h longest edge) and minimum angle in degrees (the paper's mesh-quality
    measure, Sec. 5.5)."""
    V = V.astype(np.float64)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    la = np.linalg.norm(b - c, axis=1)
    lb = np.linalg.norm(c - a, axis=1)
    lc = np.linalg.norm(a - b, axis=1)
    S = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    p = 0.5 * (la + lb + lc)
    h = np.maximum(np.maximum(la, lb), lc)
    Q = (6.0 / np.sqrt(3.0)) * S / (p * h)
    cosA = np.clip((lb ** 2 + lc ** 2 - la ** 2) / (2 * lb * lc), -1, 1)
    cosB = np.clip((la ** 2 + lc ** 2 - lb ** 2) / (2 * la * lc), -1, 1)
    cosC = np.clip((la ** 2 + lb ** 2 - lc ** 2) / (2 * la * lb), -1, 1)
    ang = np.degrees(np.arccos(np.stack([cosA, cosB, cosC], 1)))
    return Q, ang.min(axis=1)
