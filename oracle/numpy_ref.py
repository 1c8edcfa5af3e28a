"""TEST ORACLE (NumPy twin) -- test infrastructure only.

A second, separately written implementation of the same brute-force
definition as p2m_oracle.c, vectorised over primitives, for tiny meshes:
the answer is the minimum over every vertex, open edge and open face of the
gated distances (problem statement Sec. 4.1; gated tests of Algorithm A.2),
ties broken by (d, dim, id).
"""
from __future__ import annotations

import numpy as np


def canonical_edges(F: np.ndarray) -> np.ndarray:
    """Undirected (min,max) side pairs, deduplicated, sorted lexicographically."""
    F = np.asarray(F, dtype=np.int64)
    s = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0)
    s = np.sort(s, axis=1)
    return np.unique(s, axis=0).astype(np.int32)


def query(V, F, Q):
    """Return (type, id, closest, dist) for every query (FP64)."""
    V = np.asarray(V, dtype=np.float32).astype(np.float64)
    F = np.asarray(F, dtype=np.int64)
    Q = np.asarray(Q, dtype=np.float32).astype(np.float64).reshape(-1, 3)
    E = canonical_edges(F).astype(np.int64)
    n = Q.shape[0]
    out_t = np.zeros(n, np.int32)
    out_i = np.zeros(n, np.int64)
    out_c = np.zeros((n, 3))
    out_d = np.zeros(n)
    A, B = V[E[:, 0]], V[E[:, 1]]
    AB = B - A
    abab = np.einsum("ij,ij->i", AB, AB)
    Fa, Fb, Fc = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    N = np.cross(Fb - Fa, Fc - Fa)
    NN = np.einsum("ij,ij->i", N, N)
    for i in range(n):
        q = Q[i]
        dv = np.linalg.norm(V - q, axis=1)
        t = np.einsum("ij,ij->i", q - A, AB) / abab
        fe = A + t[:, None] * AB
        de = np.where((t > 0) & (t < 1), np.linalg.norm(q - fe, axis=1), np.inf)
        s = np.einsum("ij,ij->i", q - Fa, N) / NN
        P = q - s[:, None] * N
        wa = np.einsum("ij,ij->i", np.cross(Fb - P, Fc - P), N) / NN
        wb = np.einsum("ij,ij->i", np.cross(Fc - P, Fa - P), N) / NN
        wc = np.einsum("ij,ij->i", np.cross(Fa - P, Fb - P), N) / NN
        inside = (wa > 0) & (wb > 0) & (wc > 0)
        df = np.where(inside, np.linalg.norm(q - P, axis=1), np.inf)
        best = (np.inf, 3, -1)
        for dim, arr in ((0, dv), (1, de), (2, df)):
            if arr.size == 0:
                continue
            k = int(np.argmin(arr))  # first index among equal minima
            cand = (float(arr[k]), dim, k)
            if cand < best:
                best = cand
        d, dim, k = best
        out_t[i], out_i[i], out_d[i] = dim, k, d
        out_c[i] = V[k] if dim == 0 else (fe[k] if dim == 1 else P[k])
    return out_t, out_i, out_c, out_d
