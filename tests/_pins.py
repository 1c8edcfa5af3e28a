"""Pin functions for the FP64 brute-force oracle, from outside the oracle itself.

Each check uses something the oracle does not compute the same way: closed
forms on a unit cube, a corner tetrahedron and a convex icosphere; dense
surface sampling; an independent clamped point-triangle formula; a separately
written NumPy twin; and invariants (distance >= 0, |q-c| = d, c on the
reported primitive, surface points at distance 0, 1-Lipschitz).
"""
from __future__ import annotations

import numpy as np
import oracle
from oracle import numpy_ref
from synth import mesh as M
from synth import queries as SQ
from tests._helpers import (CUBE_F, CUBE_V, TETRA_F, TETRA_V, load_golden,
                            primitive_vertices, random_tiny_mesh)


def _check_golden(V, F, name, library):
    om = oracle.OracleMesh(V, F, library)
    rows = load_golden(name)
    Q = np.array([r[0] for r in rows], dtype=np.float32)
    ans = om.query(Q)
    for i, (q, prims, d, c) in enumerate(rows):
        got = (int(ans["type"][i]), primitive_vertices(om.F, om.E, ans["type"][i], ans["id"][i]))
        assert got in prims, (name, q, got, prims)
        assert abs(ans["dist"][i] - d) <= 1e-7, (name, q, ans["dist"][i], d)
        if c is not None:
            assert np.allclose(ans["closest"][i], c, atol=1e-7), (name, q, ans["closest"][i], c)


def pin_golden_tetrahedron(library=None):
    _check_golden(TETRA_V, TETRA_F, "tetra.txt", library)


def pin_golden_cube(library=None):
    _check_golden(CUBE_V, CUBE_F, "cube.txt", library)


def pin_cube_closed_form_random(library=None):
    """Outside: d = |q - clamp(q)|, type from the number of clamped axes;
    inside: d = min_k min(q_k, 1-q_k) and the face of that axis."""
    rng = np.random.default_rng(5)
    Q = rng.uniform(-1.0, 2.0, size=(3000, 3)).astype(np.float32)
    om = oracle.OracleMesh(CUBE_V, CUBE_F, library)
    ans = om.query(Q)
    Qd = Q.astype(np.float64)
    for i in range(Q.shape[0]):
        q = Qd[i]
        c = np.clip(q, 0.0, 1.0)
        nclamp = int(np.sum(c != q))
        if nclamp:
            d = np.linalg.norm(q - c)
            etype = {3: 0, 2: 1, 1: 2}[nclamp]
        else:
            m = np.minimum(q, 1.0 - q)
            k = int(np.argmin(m))
            d = m[k]
            c = q.copy()
            c[k] = 0.0 if q[k] < 1.0 - q[k] else 1.0
            etype = 2
        assert abs(ans["dist"][i] - d) <= 1e-12
        assert np.allclose(ans["closest"][i], c, atol=1e-12)
        assert ans["type"][i] == etype
        if etype == 0:
            assert np.allclose(om.V[ans["id"][i]], c)
        # the reported primitive contains the closed-form closest point
        assert om.point_to_primitive(ans["type"][i], ans["id"][i], c) <= 1e-12


def pin_tetra_vertex_regions(library=None):
    """Points beyond a corner inside its normal cone: nearest primitive is that vertex."""
    om = oracle.OracleMesh(TETRA_V, TETRA_F, library)
    rng = np.random.default_rng(7)
    # corner (1,0,0): q = (1,0,0) + t*(1, -a, -b) with a,b in (0,1) lies in its normal cone
    ab = rng.uniform(0.05, 0.95, size=(200, 2))
    t = rng.uniform(0.1, 2.0, size=200)
    Q = np.stack([1 + t, -t * ab[:, 0], -t * ab[:, 1]], 1).astype(np.float32)
    ans = om.query(Q)
    assert np.all(ans["type"] == 0) and np.all(ans["id"] == 1)
    ref = np.linalg.norm(Q.astype(np.float64) - np.array([1.0, 0, 0]), axis=1)
    assert np.allclose(ans["dist"], ref, atol=1e-12)


def pin_convex_icosphere_plane_distance(library=None):
    """Undisplaced icosphere is convex: inside, d = min over faces of the plane
    distance; outside with the foot inside the face whose plane q is beyond,
    d = that plane distance."""
    V, F = M.icosphere(2)
    V = V.astype(np.float32)
    om = oracle.OracleMesh(V, F, library)
    Vd = om.V
    a, b, c = Vd[F[:, 0]], Vd[F[:, 1]], Vd[F[:, 2]]
    n = np.cross(b - a, c - a)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    n *= np.sign(np.einsum("ij,ij->i", n, a))[:, None]  # outward
    rng = np.random.default_rng(11)
    # interior points
    Q = rng.uniform(-0.55, 0.55, size=(400, 3)).astype(np.float32)  # inside the inscribed ball
    Qd = Q.astype(np.float64)
    ans = om.query(Q)
    pd = np.einsum("fj,fj->f", n, a)[None, :] - Qd @ n.T  # distance inside each plane
    assert np.all(pd > 0)
    assert np.allclose(ans["dist"], pd.min(1), atol=1e-12)
    # exterior points above face centroids along the face normal
    f = rng.integers(0, F.shape[0], 400)
    w = rng.dirichlet([4, 4, 4], size=400)
    foot = w[:, :1] * a[f] + w[:, 1:2] * b[f] + w[:, 2:] * c[f]
    Q = (foot + rng.uniform(0.01, 0.5, size=(400, 1)) * n[f]).astype(np.float32)
    Qd = Q.astype(np.float64)
    ans = om.query(Q)
    plane = np.einsum("ij,ij->i", Qd - a[f], n[f])
    assert np.allclose(ans["dist"], plane, atol=1e-12)
    assert np.all(ans["type"] == 2) and np.all(ans["id"] == f)


def pin_gated_equals_clamped(library=None):
    for kind in ("sphere", "heightfield"):
        _gated_equals_clamped(kind, library)


def _gated_equals_clamped(kind, library):
    """Two independent formulas: min over open primitives with gates vs min
    over closed triangles of the clamped distance."""
    rng = np.random.default_rng(3 if kind == "sphere" else 4)
    V, F = random_tiny_mesh(rng, kind)
    om = oracle.OracleMesh(V, F, library)
    lo, hi = SQ.aabb(V)
    Q = SQ.uniform_in_box(2000, *SQ.scaled_box(lo, hi, 1.6), rng)
    ans = om.query(Q)
    dc = om.dist_clamped(Q)
    assert np.max(np.abs(ans["dist"] - dc)) <= 1e-12 * om.diag


def pin_numpy_twin_agrees(library=None):
    rng = np.random.default_rng(21)
    for kind in ("sphere", "heightfield"):
        V, F = random_tiny_mesh(rng, kind)
        om = oracle.OracleMesh(V, F, library)
        assert np.array_equal(om.E, numpy_ref.canonical_edges(F))
        lo, hi = SQ.aabb(V)
        Q = SQ.uniform_in_box(300, *SQ.scaled_box(lo, hi, 1.5), rng)
        ans = om.query(Q)
        t, i, c, d = numpy_ref.query(V, F, Q)
        assert np.allclose(ans["dist"], d, rtol=0, atol=1e-13)
        same = (ans["type"] == t) & (ans["id"] == i)
        # identical arithmetic order is not promised; differences must be exact ties
        for k in np.nonzero(~same)[0]:
            assert abs(ans["runner_up"][k] - ans["dist"][k]) <= 1e-13


def pin_dense_surface_sampling(library=None):
    """Brute force from the other side: the distance to a dense point sample
    of the surface bounds the oracle from above, and from below up to the
    sample spacing."""
    rng = np.random.default_rng(8)
    V, F = random_tiny_mesh(rng, "sphere")
    om = oracle.OracleMesh(V, F, library)
    Vd = om.V
    k = 60
    ii, jj = np.meshgrid(np.arange(k + 1), np.arange(k + 1), indexing="ij")
    sel = ii + jj <= k
    w1, w2 = ii[sel] / k, jj[sel] / k
    w0 = 1 - w1 - w2
    S = (w0[None, :, None] * Vd[om.F[:, 0]][:, None] + w1[None, :, None] * Vd[om.F[:, 1]][:, None]
         + w2[None, :, None] * Vd[om.F[:, 2]][:, None]).reshape(-1, 3)
    emax = max(np.linalg.norm(Vd[om.E[:, 0]] - Vd[om.E[:, 1]], axis=1))
    h = emax / k  # every surface point is within h of a sample
    lo, hi = SQ.aabb(V)
    Q = SQ.uniform_in_box(200, *SQ.scaled_box(lo, hi, 1.4), rng)
    ans = om.query(Q)
    for i in range(Q.shape[0]):
        ds = np.min(np.linalg.norm(S - Q[i].astype(np.float64), axis=1))
        assert ans["dist"][i] <= ds + 1e-12
        assert ans["dist"][i] >= ds - h


def pin_invariants_random_meshes(library=None):
    rng = np.random.default_rng(13)
    for kind in ("sphere", "heightfield"):
        V, F = random_tiny_mesh(rng, kind)
        om = oracle.OracleMesh(V, F, library)
        lo, hi = SQ.aabb(V)
        Q = SQ.uniform_in_box(500, *SQ.scaled_box(lo, hi, 1.5), rng)
        ans = om.query(Q)
        Qd = Q.astype(np.float64)
        assert np.all(ans["dist"] >= 0)
        assert np.allclose(np.linalg.norm(Qd - ans["closest"], axis=1), ans["dist"], atol=1e-12)
        for i in range(Q.shape[0]):
            assert om.point_to_primitive(ans["type"][i], ans["id"][i], ans["closest"][i]) <= 1e-12
        # 1-Lipschitz
        D = np.abs(ans["dist"][:, None] - ans["dist"][None, :])
        P = np.linalg.norm(Qd[:, None] - Qd[None, :], axis=2)
        assert np.all(D <= P + 1e-12)
        # surface samples lie at distance ~0 (fp32 rounding of the sample only)
        S = SQ.surface_samples(om.V, om.F, 300, rng).astype(np.float32)
        ds = om.query(S)["dist"]
        assert np.all(ds <= 1e-6 * om.diag)


def pin_near_set_contains_best_and_ties(library=None):
    om = oracle.OracleMesh(TETRA_V, TETRA_F, library)
    q = np.array([0.5, 0.5, -1.0], np.float32)
    ans = om.query(q[None])
    ns = om.near_set(q, ans["dist"][0], 1e-6)
    assert (int(ans["type"][0]), int(ans["id"][0])) in ns
    # the z=0 face is equidistant up to the boundary and belongs to the set
    assert (2, 0) in ns


# Exact near-optimal sets (tol 1e-6), derived by hand from the definition of
# the set: a primitive belongs when its foot lies on it or within tol of it
# (edge parameter in [-tol/|e|, 1+tol/|e|]; face foot within tol of the
# closed triangle) and its line / plane distance is within tol of d*.  Every
# other primitive is absent: farther, or its foot lies a finite distance
# off it.  Rows: query, d*, members as (type, sorted vertex ids).
_TETRA_NEAR = [
    ((0.1, 0.2, 0.3), 0.1, {"F:0,2,3"}),
    ((1, 1, 1), 2 / np.sqrt(3), {"F:1,2,3"}),
    ((-1, -1, -1), np.sqrt(3), {"V:0"}),
    # the edges at vertex 1 have their feet at t = 2 or t = -1/2; the faces
    # at it have their feet 1 (or more) off them
    ((2, 0, 0), 1.0, {"V:1"}),
    ((0.5, -1, -1), np.sqrt(2), {"E:0,1"}),
    ((0.25, 0.25, -1), 1.0, {"F:0,1,2"}),
    # the z=0 face's foot (0.5,0.5,0) lies on its side (1,2): a tie at the boundary
    ((0.5, 0.5, -1), 1.0, {"E:1,2", "F:0,1,2"}),
    # on the edge (0,3): both faces at it have their foot on their boundary
    ((0, 0, 0.5), 0.0, {"E:0,3", "F:0,2,3", "F:0,1,3"}),
    ((0.2, 0.2, 0.2), 0.2, {"F:0,1,2", "F:0,1,3", "F:0,2,3"}),
    ((0.25, 0.25, 0.25), 0.25 / np.sqrt(3), {"F:1,2,3"}),
    # the x-axis edge (0,1) has its foot exactly at t = 0 (vertex 0), inside
    # the relaxed gate, at the same distance sqrt(2) as vertex 0
    ((0, -1, -1), np.sqrt(2), {"V:0", "E:0,1"}),
]
_CUBE_NEAR = [
    # the face diagonals (1,7), (2,7) have their feet at t = 1, at 0.866 > d*
    ((1.5, 1.5, 0.5), np.sqrt(0.5), {"E:3,7"}),
    ((2, 2, 2), np.sqrt(3), {"V:7"}),
    ((0.2, 0.3, 0.6), 0.2, {"F:0,4,6"}),
    # the other z=0 triangle's foot is 0.05/sqrt(2) off it
    ((0.3, 0.25, -0.5), 0.5, {"F:0,1,3"}),
    # on the z=0 diagonal: both triangles have their foot on their boundary
    ((0.5, 0.5, -2), 2.0, {"E:0,3", "F:0,1,3", "F:0,3,2"}),
    ((-1, 0.5, 2), np.sqrt(2), {"E:4,6"}),
    ((0.9, 0.6, 0.55), 0.1, {"F:1,3,7"}),
    # the centre: all 12 triangles (feet at the square centres, on their
    # diagonals) and the 6 diagonals at 0.5; the cube edges are at sqrt(0.5)
    ((0.5, 0.5, 0.5), 0.5, {"F:0,2,6", "F:0,6,4", "F:1,3,7", "F:1,7,5", "F:0,1,5", "F:0,5,4", "F:2,3,7",
                            "F:2,7,6", "F:0,1,3", "F:0,3,2", "F:4,5,7", "F:4,7,6", "E:0,6", "E:1,7",
                            "E:0,5", "E:2,7", "E:0,3", "E:4,7"}),
]


def _named_set(om, ns):
    out = set()
    for t, i in ns:
        vs = sorted(primitive_vertices(om.F, om.E, t, i))
        out.add("VEF"[t] + ":" + ",".join(str(v) for v in vs))
    return out


def _check_near(V, F, rows, library):
    om = oracle.OracleMesh(V, F, library)
    for q, dstar, want in rows:
        want = {w[:2] + ",".join(str(v) for v in sorted(int(x) for x in w[2:].split(","))) for w in want}
        got = _named_set(om, om.near_set(np.array(q, np.float64), float(dstar), 1e-6))
        assert got == want, (q, sorted(got), sorted(want))


def pin_near_set_exact_tetrahedron(library=None):
    """The near-optimal set holds exactly the hand-derived members: the best,
    its rounding-level ties at a boundary, and nothing farther or off."""
    _check_near(TETRA_V, TETRA_F, _TETRA_NEAR, library)


def pin_near_set_exact_cube(library=None):
    _check_near(CUBE_V, CUBE_F, _CUBE_NEAR, library)


def pin_point_to_primitive_off_primitive(library=None):
    """Distance from points off a closed primitive, against closed forms on
    the unit cube: a vertex |x - v|; an axis-parallel cube edge along axis k
    at fixed coordinates c_j (j != k): sqrt(sum_j (x_j - c_j)^2 + (x_k -
    clamp(x_k, 0, 1))^2); a square face at x_a = s, split in two triangles:
    the smaller of the two triangle distances equals sqrt((x_a - s)^2 +
    sum_{j != a} (x_j - clamp(x_j, 0, 1))^2)."""
    om = oracle.OracleMesh(CUBE_V, CUBE_F, library)
    rng = np.random.default_rng(41)
    X = rng.uniform(-1.0, 2.0, size=(400, 3))
    Vd = CUBE_V.astype(np.float64)
    edge_id = {tuple(e): k for k, e in enumerate(om.E.tolist())}
    for x in X:
        for v in range(8):
            assert abs(om.point_to_primitive(0, v, x) - np.linalg.norm(x - Vd[v])) <= 1e-12
        for (a, b), k in edge_id.items():
            diff = np.abs(Vd[a] - Vd[b])
            if diff.sum() != 1.0:
                continue  # a face diagonal
            ax = int(np.argmax(diff))
            r = x - Vd[a]
            r[ax] = x[ax] - np.clip(x[ax], 0.0, 1.0)
            assert abs(om.point_to_primitive(1, k, x) - np.linalg.norm(r)) <= 1e-12, (a, b, x)
        for f0 in range(0, 12, 2):
            ax = int(np.argmin(np.ptp(Vd[CUBE_F[f0]], axis=0)))
            s = Vd[CUBE_F[f0][0], ax]
            r = x - np.clip(x, 0.0, 1.0)
            r[ax] = x[ax] - s
            d = min(om.point_to_primitive(2, f0, x), om.point_to_primitive(2, f0 + 1, x))
            assert abs(d - np.linalg.norm(r)) <= 1e-12, (f0, x)
    # tetrahedron: (2,0,0) is 1 from the slanted face (its closest point is
    # the corner (1,0,0)), 2 from vertex 0, sqrt(2) from the edge (0,0,1)-(0,1,0)
    ot = oracle.OracleMesh(TETRA_V, TETRA_F, library)
    x = np.array([2.0, 0.0, 0.0])
    assert abs(ot.point_to_primitive(2, 3, x) - 1.0) <= 1e-12
    assert abs(ot.point_to_primitive(0, 0, x) - 2.0) <= 1e-12
    e23 = [k for k, e in enumerate(ot.E.tolist()) if e == [2, 3]][0]
    assert abs(ot.point_to_primitive(1, e23, x) - np.sqrt(4.5)) <= 1e-12


_NOF = np.zeros((0, 3), np.int32)


def pin_single_segment_closed_form(library=None):
    """One free segment (Sec. 5.5's mixed sets): distance to the closed
    segment by projection and clamping; the end vertex when clamped."""
    rng = np.random.default_rng(31)
    V = np.array([[0.1, -0.2, 0.3], [0.9, 0.4, -0.1]], np.float32)
    om = oracle.OracleMesh(V, _NOF, library, segments=[[0, 1]])
    Q = rng.uniform(-1.0, 2.0, size=(400, 3)).astype(np.float32)
    ans = om.query(Q)
    a, b = V.astype(np.float64)
    e = b - a
    for i, q in enumerate(Q.astype(np.float64)):
        t = (q - a) @ e / (e @ e)
        c = a + min(max(t, 0.0), 1.0) * e
        assert abs(ans["dist"][i] - np.linalg.norm(q - c)) <= 1e-12
        assert ans["type"][i] == (1 if 0.0 < t < 1.0 else 0), (q, t, ans["type"][i])


def pin_wireframe_cube_closed_form(library=None):
    """The 12 edges of the unit cube as free segments: the nearest edge
    parallel to axis k is at squared distance sum over j != k of
    min(x_j^2, (x_j - 1)^2), plus the clamp along k."""
    rng = np.random.default_rng(32)
    S = np.array([[a, b] for a in range(8) for b in range(a + 1, 8)
                  if np.abs(CUBE_V[a] - CUBE_V[b]).sum() == 1.0], np.int32)
    assert len(S) == 12
    om = oracle.OracleMesh(CUBE_V, _NOF, library, segments=S)
    Q = rng.uniform(-0.5, 1.5, size=(600, 3))
    ans = om.query(Q.astype(np.float32))
    Qd = Q.astype(np.float32).astype(np.float64)
    near = np.minimum(Qd ** 2, (Qd - 1.0) ** 2)
    along = (Qd - np.clip(Qd, 0.0, 1.0)) ** 2
    d = np.sqrt(np.min([near.sum(1) - near[:, k] + along[:, k] for k in range(3)], axis=0))
    assert np.max(np.abs(ans["dist"] - d)) <= 1e-12
    assert set(np.unique(ans["type"])) <= {0, 1}


def pin_mixed_set_is_min_of_parts(library=None):
    """A mixed set's distance is the smaller of its triangles' and its
    segments' distances (the primitive set is their union)."""
    rng = np.random.default_rng(33)
    V1, F1 = random_tiny_mesh(rng, "sphere")
    V2, F2 = random_tiny_mesh(rng, "sphere")
    V2 = (0.5 * V2 + np.array([0.6, 0.1, 0.0], np.float32)).astype(np.float32)
    S2 = np.unique(np.sort(np.concatenate([F2[:, [0, 1]], F2[:, [1, 2]], F2[:, [2, 0]]]), axis=1), axis=0)
    V = np.concatenate([V1, V2])
    mixed = oracle.OracleMesh(V, F1, library, segments=S2 + len(V1))
    tri = oracle.OracleMesh(V1, F1, library)
    seg = oracle.OracleMesh(V2, _NOF, library, segments=S2)
    Q = rng.uniform(-1.5, 1.5, size=(500, 3)).astype(np.float32)
    d = mixed.query(Q)["dist"]
    assert np.array_equal(d, np.minimum(tri.query(Q)["dist"], seg.query(Q)["dist"]))


PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
