"""TEST ORACLE (derivatives) -- test infrastructure only.

The paper defines no derivative.  For d(q, V) = |q - c| with c the closest
mesh point, c = sum_k w_k v_k over the vertices of the closest primitive
(weights: 1 for a vertex; (1-t, t) for an edge; barycentrics for a face),
the envelope theorem gives

  dd/dq   =  (q - c) / d
  dd/dv_k = -w_k (q - c) / d

and 0 where d = 0 (the subgradient 0 is taken).  Here w and c come from the
FP64 brute-force answer.
"""
from __future__ import annotations

import numpy as np

from . import EDGE, FACE, VERTEX


def weights(om, ptype: int, pid: int, c) -> tuple[np.ndarray, np.ndarray]:
    """Vertex ids and weights reproducing the closest point c on the primitive."""
    V = om.V
    c = np.asarray(c, dtype=np.float64)
    if ptype == VERTEX:
        return np.array([pid]), np.array([1.0])
    if ptype == EDGE:
        a, b = om.E[pid]
        ab = V[b] - V[a]
        t = float(np.dot(c - V[a], ab) / np.dot(ab, ab))
        return np.array([a, b]), np.array([1.0 - t, t])
    if ptype == FACE:
        ia, ib, ic = om.F[pid]
        a, b, cc = V[ia], V[ib], V[ic]
        n = np.cross(b - a, cc - a)
        nn = float(np.dot(n, n))
        wa = np.dot(np.cross(b - c, cc - c), n) / nn
        wb = np.dot(np.cross(cc - c, a - c), n) / nn
        wc = np.dot(np.cross(a - c, b - c), n) / nn
        return np.array([ia, ib, ic]), np.array([wa, wb, wc])
    raise ValueError(ptype)


def gradients(om, Q, ans, gbar) -> tuple[np.ndarray, np.ndarray]:
    """grad_q [n,3] and grad_V [nv,3] for upstream gradient gbar [n] of the distances."""
    Q = om._widen(Q).reshape(-1, 3)
    gbar = np.asarray(gbar, dtype=np.float64)
    gq = np.zeros_like(Q)
    gV = np.zeros_like(om.V)
    for i in range(Q.shape[0]):
        d = float(ans["dist"][i])
        if not (d > 0.0):
            continue
        u = (Q[i] - ans["closest"][i]) / d
        gq[i] = gbar[i] * u
        ids, w = weights(om, int(ans["type"][i]), int(ans["id"][i]), ans["closest"][i])
        for k, wk in zip(ids, w):
            gV[k] -= gbar[i] * wk * u
    return gq, gV
