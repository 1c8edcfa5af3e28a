"""Acceptance rule for a P2M answer against the FP64 brute-force oracle.

With tol = 1e-5 x the mesh AABB diagonal (float32 storage of coordinates):
  * |d - d*| <= tol + 2 float32 spacings at d* and d >= 0 (d is reported
    in float32: for a query hundreds of diagonals away a spacing alone
    exceeds tol; near the mesh the term is negligible);
  * the reported primitive is the oracle's best, or belongs to the oracle's
    near-optimal set (primitives whose distance under tolerance-relaxed
    gates is within tol of d*): exact or rounding-level ties may go either
    way, so only a genuinely worse primitive is a failure;
  * | |q - c| - d | <= tol + e (+ the two spacings at d*) and c lies within
    tol + e of the reported (closed) primitive;
  * when the near-optimal set is a single primitive, |c - c*| <= tol + e;
where e = sqrt(3)/2 x the float32 spacing at c's largest coordinate: c is
reported in float32, which cannot place it closer than half a spacing per
coordinate (negligible beside tol for a mesh near the origin; for a mesh far
from it, the distance is still held to tol alone).
"""
from __future__ import annotations

import numpy as np


def prim_split(prim):
    p = np.asarray(prim).astype(np.int64) & 0xFFFFFFFF
    return p >> 30, p & 0x3FFFFFFF


def check_answers(om, Q, ans, prim, closest, dist, tol=None, idx=None, max_report=5):
    """Returns a list of failure strings (empty when all rows pass).

    om: oracle.OracleMesh; Q [n,3] float32 queries; ans: om.query(Q);
    prim/closest/dist: the answers under test for the same rows.
    """
    if tol is None:
        tol = 1e-5 * om.diag
    Q = np.asarray(Q, dtype=np.float32).astype(np.float64).reshape(-1, 3)
    typ, pid = prim_split(prim)
    closest = np.asarray(closest, dtype=np.float64).reshape(-1, 3)
    dist = np.asarray(dist, dtype=np.float64)
    fails = []

    def bad(i, why):
        if len(fails) < max_report:
            j = i if idx is None else idx[i]
            fails.append(f"row {j}: {why} (q={Q[i].tolist()}, got {(int(typ[i]), int(pid[i]))} d={dist[i]!r}, "
                         f"oracle {(int(ans['type'][i]), int(ans['id'][i]))} d*={ans['dist'][i]!r})")
        else:
            fails.append("...")

    dd = np.abs(dist - ans["dist"])
    with np.errstate(invalid="ignore"):
        dtol = tol + 2.0 * np.spacing(np.abs(ans["dist"]).astype(np.float32)).astype(np.float64)
    for i in np.nonzero(~(dd <= dtol))[0]:
        bad(i, f"|d-d*|={dd[i]:.3g} > tol={dtol[i]:.3g}")
    for i in np.nonzero(~(dist >= 0))[0]:
        bad(i, "negative or NaN distance")
    with np.errstate(invalid="ignore"):
        e = 0.5 * np.sqrt(3.0) * np.spacing(np.abs(closest).max(axis=1).astype(np.float32)).astype(np.float64)
    ctol = tol + np.where(np.isfinite(e), e, 0.0)
    qc = np.linalg.norm(Q - closest, axis=1)
    for i in np.nonzero(~(np.abs(qc - dist) <= ctol + (dtol - tol)))[0]:
        bad(i, f"| |q-c| - d | = {abs(qc[i]-dist[i]):.3g}")
    same = (typ == ans["type"]) & (pid == ans["id"])
    for i in range(Q.shape[0]):
        on = om.point_to_primitive(int(typ[i]), int(pid[i]), closest[i])
        if not (on <= ctol[i]):
            bad(i, f"closest point is {on:.3g} off the reported primitive")
        if not same[i] or np.linalg.norm(closest[i] - ans["closest"][i]) > ctol[i]:
            ns = om.near_set(Q[i], ans["dist"][i], tol)
            if not same[i] and (int(typ[i]), int(pid[i])) not in ns:
                bad(i, "primitive not in the oracle's near-optimal set")
            if len(ns) == 1 and np.linalg.norm(closest[i] - ans["closest"][i]) > ctol[i]:
                bad(i, "closest point differs from the unique optimum")
    return fails
