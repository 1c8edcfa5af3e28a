"""Host side (no GPU): mesh validation, KD tree, Voronoi neighbours, the
interception table's properties, and the full query through the host model
of the kernel (same tree, table and float32 code), checked against the
FP64 brute-force oracle."""
from __future__ import annotations

import os
import tempfile

import numpy as np
import pytest

import oracle
import paper_2308_16084_amd as P
from synth import configs as C
from synth import queries as SQ
from tests._accept import check_answers
from tests._helpers import (CUBE_F, CUBE_V, TETRA_F, TETRA_V, gate_boundary_points, margin_points,
                            random_tiny_mesh)


def _mesh(V, F, domain=None, mode=P.TABLE_FLOODING, scale=1.5):
    m = P.Mesh(V, F)
    if domain is None:
        lo, hi = SQ.aabb(V)
        domain = SQ.scaled_box(lo, hi, scale)
    st = m.precompute(domain=domain, table_mode=mode)
    return m, st, domain


@pytest.mark.parametrize("bad,msg", [
    ("oob", "out of range"), ("repeat", "repeats"), ("zero_area", "zero area"), ("nan", "non-finite"),
    ("dup", "coincide")])
def test_mesh_validation(bad, msg):
    V = TETRA_V.copy()
    F = TETRA_F.copy()
    if bad == "oob":
        F[1, 2] = 7
    elif bad == "repeat":
        F[1, 2] = F[1, 0]
    elif bad == "zero_area":
        V = np.concatenate([V, [[0.5, 0, 0]]]).astype(np.float32)
        F = np.concatenate([F, [[0, 1, 4]]]).astype(np.int32)
    elif bad == "nan":
        V[2, 1] = np.nan
    elif bad == "dup":
        V = np.concatenate([V, V[2:3]]).astype(np.float32)
    with pytest.raises(P.P2MError) as e:
        P.Mesh(V, F)
    assert e.value.status == -2 and msg in str(e.value)


def test_state_errors():
    m = P.Mesh(TETRA_V, TETRA_F)
    with pytest.raises(P.P2MError) as e:
        m.table()
    assert e.value.status == -3
    with pytest.raises(P.P2MError):
        m.query_host(np.zeros((1, 3), np.float32))
    with pytest.raises(P.P2MError) as e:
        m.precompute(domain=([0, 0, 0], [0, 1, 1]))
    assert e.value.status == -1


def test_edges_match_oracle():
    rng = np.random.default_rng(0)
    V, F = random_tiny_mesh(rng, "heightfield")
    m = P.Mesh(V, F)
    assert np.array_equal(m.edges(), oracle.OracleMesh(V, F).E)


def test_kdtree_is_a_kd_tree():
    rng = np.random.default_rng(1)
    V = rng.random((1000, 3)).astype(np.float32)
    F = np.array([[0, 1, 2]], np.int32)
    m = P.Mesh(V, F)
    m.precompute()
    xyz, vid = m.kdtree()
    assert sorted(vid.tolist()) == list(range(1000))
    assert np.array_equal(xyz, V[vid])
    n = len(vid)

    def check(node, depth, lo, hi):
        if node >= n:
            return
        d = depth % 3
        assert np.all(xyz[node] >= lo) and np.all(xyz[node] <= hi)
        s = xyz[node, d]
        hl = hi.copy(); hl[d] = s
        lr = lo.copy(); lr[d] = s
        check(2 * node + 1, depth + 1, lo, hl)
        check(2 * node + 2, depth + 1, lr, hi)

    check(0, 0, np.full(3, -np.inf, np.float32), np.full(3, np.inf, np.float32))


def test_voronoi_neighbours_match_qhull():
    """Delaunay edges whose Voronoi facet meets the domain are all present:
    every pair of nearest and second-nearest vertices of a point in D is a
    neighbour pair; and (away from the hull) the graph equals Qhull's."""
    from scipy.spatial import Delaunay, cKDTree
    rng = np.random.default_rng(2)
    V, F = random_tiny_mesh(rng, "sphere")
    m, st, (lo, hi) = _mesh(V, F)
    off, nb = m.neighbors()
    mine = {(i, int(j)) for i in range(len(V)) for j in nb[off[i]:off[i + 1]]}
    assert all((j, i) in mine for i, j in mine)
    d = Delaunay(V.astype(np.float64))
    qh = set()
    for t in d.simplices:
        for a in range(4):
            for b in range(4):
                if a != b:
                    qh.add((int(t[a]), int(t[b])))
    assert mine <= qh
    X = rng.uniform(lo, hi, size=(20000, 3))
    _, ii = cKDTree(V.astype(np.float64)).query(X, k=2)
    assert all((int(a), int(b)) in mine for a, b in ii)


@pytest.mark.parametrize("name", ["tetra", "cube", "sphere", "heightfield", "c1"])
def test_voronoi_walk_reaches_nearest_vertex(name):
    """Greedy descent over the neighbour graph (the device's Voronoi-walk
    traversal) ends at an exact nearest vertex from any start, for every
    point of D: a point outside Cell(v) is closer to some neighbour of v."""
    rng = np.random.default_rng(5)
    if name == "tetra":
        V, F = TETRA_V, TETRA_F
    elif name == "cube":
        V, F = CUBE_V, CUBE_F
    elif name == "c1":
        w = C.c1()
        V, F = w.V, w.F
    else:
        V, F = random_tiny_mesh(rng, name)
    m, st, (lo, hi) = _mesh(V, F, scale=3.0)
    off, nb = m.neighbors()
    Vd = V.astype(np.float64)
    X = rng.uniform(lo, hi, size=(3000, 3))
    X[:8] = np.array([[lo[0], lo[1], lo[2]], [hi[0], hi[1], hi[2]], [lo[0], hi[1], lo[2]], [hi[0], lo[1], hi[2]],
                      [lo[0], lo[1], hi[2]], [hi[0], hi[1], lo[2]], [lo[0], hi[1], hi[2]], [hi[0], lo[1], lo[2]]])
    start = rng.integers(0, len(V), size=len(X))
    for x, v in zip(X, start):
        dv = ((x - Vd[v]) ** 2).sum()
        while True:
            ns = nb[off[v]:off[v + 1]]
            if len(ns) == 0:
                break
            d = ((x - Vd[ns]) ** 2).sum(1)
            k = int(d.argmin())
            if d[k] >= dv:
                break
            v, dv = int(ns[k]), d[k]
        best = ((x - Vd) ** 2).sum(1).min()
        assert dv <= best * (1 + 1e-12), (name, x)


@pytest.mark.parametrize("name", ["tetra", "cube", "sphere", "heightfield", "c1"])
def test_entry_boxes_hold_their_polytopes(name):
    """Every entry (v,p) whose Space-perp(p) holds a point x of D with nearest
    vertex v has x inside its box (the box bounds Cell(v) n Space-perp(p) n
    D); boxes of the table lie inside the 16-bit frame and are not all full."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(13)
    if name == "tetra":
        V, F = TETRA_V, TETRA_F
    elif name == "cube":
        V, F = CUBE_V, CUBE_F
    elif name == "c1":
        w = C.c1()
        V, F = w.V, w.F
    else:
        V, F = random_tiny_mesh(rng, name)
    m, st, (lo, hi) = _mesh(V, F, scale=2.0)
    off, ent = m.table()
    box = m.table_boxes().astype(np.int64)
    assert box.shape == (len(ent), 6)
    assert np.all(box[:, :3] <= box[:, 3:]) and np.any(box[:, :3] > 0)
    E = m.edges()
    Vd = V.astype(np.float64)
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    # Space-perp(e) (Eq. 4): the foot on the line inside e, and q not on the
    # face side of the plane through e perpendicular to an adjacent face
    adj = {}
    for f, tri in enumerate(F):
        for i in range(3):
            a, b = sorted((int(tri[i]), int(tri[(i + 1) % 3])))
            adj.setdefault((a, b), []).append(int(tri[(i + 2) % 3]))
    X = rng.uniform(lo, hi, size=(1000 if name == "c1" else 3000, 3))
    _, nn = cKDTree(Vd).query(X)
    U = (X - lo) * (65535.0 / (hi - lo))
    checked = 0
    for x, u, v in zip(X, U, nn):
        for k in range(off[2 * v], off[2 * v + 2]):
            pid = ent[k]
            if k < off[2 * v + 1]:
                a, b = Vd[E[pid, 0]], Vd[E[pid, 1]]
                t = (x - a) @ (b - a) / ((b - a) @ (b - a))
                inside = 0 < t < 1
                for c in adj[(int(E[pid, 0]), int(E[pid, 1]))]:
                    nf = np.cross(b - a, Vd[c] - a)
                    mm = np.cross(b - a, nf)
                    if mm @ (Vd[c] - a) < 0:
                        mm = -mm
                    inside &= mm @ (x - a) < 0
            else:
                a, b, c = Vd[F[pid]]
                n = np.cross(b - a, c - a)
                p = x - ((x - a) @ n) / (n @ n) * n
                w = [np.cross(c - b, p - b) @ n, np.cross(a - c, p - c) @ n, np.cross(b - a, p - a) @ n]
                inside = min(w) > 0
            if inside:
                checked += 1
                assert np.all(u >= box[k, :3]) and np.all(u <= box[k, 3:]), (name, x, v, k)
    assert checked > 100


def test_table_contains_incident_primitives():
    """Theorem 2: every vertex intercepts its incident edges and faces."""
    rng = np.random.default_rng(3)
    V, F = random_tiny_mesh(rng, "sphere")
    m, _, _ = _mesh(V, F)
    off, ent = m.table()
    E = m.edges()
    for v in range(len(V)):
        edges = set(ent[off[2 * v]:off[2 * v + 1]].tolist())
        faces = set(ent[off[2 * v + 1]:off[2 * v + 2]].tolist())
        assert {e for e in range(len(E)) if v in E[e]} <= edges
        assert {f for f in range(len(F)) if v in F[f]} <= faces
        assert sorted(edges) == ent[off[2 * v]:off[2 * v + 1]].tolist()


def test_flooding_subset_of_all_pairs():
    """Flooding only visits what the all-pairs filter would accept (Theorem 7
    says it finds all of them; the equality is checked too)."""
    rng = np.random.default_rng(4)
    for kind in ("sphere", "heightfield"):
        V, F = random_tiny_mesh(rng, kind)
        m1, _, dom = _mesh(V, F)
        m2, _, _ = _mesh(V, F, domain=dom, mode=P.TABLE_ALL_PAIRS)
        o1, e1 = m1.table()
        o2, e2 = m2.table()
        for v in range(len(V)):
            a = set(e1[o1[2 * v]:o1[2 * v + 1]].tolist()), set(e1[o1[2 * v + 1]:o1[2 * v + 2]].tolist())
            b = set(e2[o2[2 * v]:o2[2 * v + 1]].tolist()), set(e2[o2[2 * v + 1]:o2[2 * v + 2]].tolist())
            assert a[0] <= b[0] and a[1] <= b[1]
            assert a == b


@pytest.mark.parametrize("name,V,F", [("tetra", TETRA_V, TETRA_F), ("cube", CUBE_V, CUBE_F)])
def test_host_query_closed_forms(name, V, F):
    m, _, dom = _mesh(V, F, scale=4.0)
    rng = np.random.default_rng(5)
    Q = rng.uniform(dom[0], dom[1], size=(4000, 3)).astype(np.float32)
    om = oracle.OracleMesh(V, F)
    ans = om.query(Q)
    h = m.query_host(Q)
    assert check_answers(om, Q, ans, h["prim"], h["closest"], h["dist"]) == []


@pytest.mark.parametrize("mode", [P.TABLE_FLOODING, P.TABLE_ALL_PAIRS, P.TABLE_EVERYTHING])
def test_host_query_tiny_meshes(mode):
    rng = np.random.default_rng(6 + mode)
    for kind in ("sphere", "heightfield"):
        V, F = random_tiny_mesh(rng, kind)
        m, _, dom = _mesh(V, F, mode=mode)
        Q = rng.uniform(dom[0], dom[1], size=(3000, 3)).astype(np.float32)
        om = oracle.OracleMesh(V, F)
        h = m.query_host(Q)
        assert check_answers(om, Q, om.query(Q), h["prim"], h["closest"], h["dist"]) == []


def test_host_query_c1_all_queries():
    """Workload C1 (icosphere level 4, 10^4 queries): every query accepted."""
    w = C.c1()
    m, st, _ = _mesh(w.V, w.F, domain=(w.domain_lo, w.domain_hi))
    om = oracle.OracleMesh(w.V, w.F)
    h = m.query_host(w.Q)
    assert check_answers(om, w.Q, om.query(w.Q), h["prim"], h["closest"], h["dist"]) == []
    assert st["nv"] == 2562 and st["nf"] == 5120 and st["ne"] == 7680


@pytest.mark.parametrize("name", ["c1", "needles"])
def test_host_query_gate_boundaries(name):
    """Points where the list scan's gates decide: on edges (midpoints and
    near the ends), at vertices, on faces, pushed off the surface by tiny
    and by large amounts, and the far corners of the domain; on C1 and on a
    heightfield with needle rows."""
    from synth import mesh as M
    rng = np.random.default_rng(9)
    if name == "c1":
        w = C.c1()
        V, F = w.V, w.F
    else:
        V, F = M.heightfield(24, 77)
        V, F = V.astype(np.float32), F.astype(np.int32)
    m, st, (lo, hi) = _mesh(V, F, scale=1.5)
    om = oracle.OracleMesh(V, F)
    Q = gate_boundary_points(V, F, om.E, lo, hi, rng)
    h = m.query_host(Q)
    assert np.all(h["status"] == 0)
    assert check_answers(om, Q, om.query(Q), h["prim"], h["closest"], h["dist"]) == []


@pytest.mark.parametrize("name,scale", [("c1", 1.5), ("c1", 10.0), ("c1", 12.0), ("fbm5", 10.0),
                                        ("needles", 10.0)])
def test_host_query_within_gate_margin(name, scale):
    """Points within the gate margin mu (2^-20 of the domain diagonal) of
    primitive boundaries, where a primitive passes its gate with its foot
    just off it and its line / plane distance undercuts the true distance:
    the answer stays the exact minimum (|d - d*| <= tol / 4) at any domain
    size, the default 10x AABB included."""
    from synth import mesh as M
    rng = np.random.default_rng(12)
    if name == "c1":
        V, F = C.c1().V, C.c1().F
    elif name == "fbm5":
        V, F = C.sphere_mesh(5, "fbm", 17)
    else:
        V, F = M.heightfield(24, 77)
        V, F = V.astype(np.float32), F.astype(np.int32)
    m, st, (lo, hi) = _mesh(V, F, scale=scale)
    om = oracle.OracleMesh(V, F)
    mu = 2.0 ** -20 * float(np.linalg.norm(np.asarray(hi) - np.asarray(lo)))
    Q = margin_points(V, F, om.E, om.diag, mu, rng)
    h = m.query_host(Q)
    ans = om.query(Q)
    assert check_answers(om, Q, ans, h["prim"], h["closest"], h["dist"]) == []
    err = np.abs(h["dist"].astype(np.float64) - ans["dist"])
    assert err.max() <= 0.25e-5 * om.diag, err.max() / om.diag


def test_table_completeness_dense_sampling():
    """Completeness by dense sampling: for many random points of D, the
    oracle's optimal primitive (or a member of its near-optimal set) is the
    nearest vertex itself or in that vertex's list."""
    rng = np.random.default_rng(9)
    V, F = random_tiny_mesh(rng, "heightfield")
    m, _, dom = _mesh(V, F)
    off, ent = m.table()
    om = oracle.OracleMesh(V, F)
    Q = rng.uniform(dom[0], dom[1], size=(20000, 3)).astype(np.float32)
    ans = om.query(Q)
    nn = np.argmin(((Q[:, None, :].astype(np.float64) - om.V[None]) ** 2).sum(-1), axis=1)
    tol = 1e-5 * om.diag
    for i in range(Q.shape[0]):
        v, t, p = int(nn[i]), int(ans["type"][i]), int(ans["id"][i])
        ok = (t == 0 and p == v) or (t == 1 and p in ent[off[2 * v]:off[2 * v + 1]]) or \
             (t == 2 and p in ent[off[2 * v + 1]:off[2 * v + 2]])
        if not ok:
            ns = om.near_set(Q[i], ans["dist"][i], tol)
            ok = any((tt == 0 and pp == v) or (tt == 1 and pp in ent[off[2 * v]:off[2 * v + 1]]) or
                     (tt == 2 and pp in ent[off[2 * v + 1]:off[2 * v + 2]]) for tt, pp in ns)
        assert ok, (i, Q[i], v, t, p)


def test_out_of_domain_and_nonfinite_flags():
    m, _, dom = _mesh(TETRA_V, TETRA_F, scale=2.0)
    Q = np.array([[0.2, 0.2, 0.2], [50, 0, 0], [np.nan, 0, 0], [1e20, 0, 0]], np.float32)
    h = m.query_host(Q)
    assert h["status"].tolist() == [0, P.OUT_OF_DOMAIN, P.NONFINITE, P.OUT_OF_DOMAIN]
    # squared distances overflow float32 here; the answer is still a vertex
    assert P.prim_type(h["prim"][3]) == P.VERTEX
    assert np.isnan(h["dist"][2]) and P.prim_type(h["prim"][2]) == P.NONE
    assert abs(h["dist"][1] - 49.0) < 1e-4  # still a valid distance (to vertex (1,0,0))


def test_save_load_roundtrip():
    rng = np.random.default_rng(10)
    V, F = random_tiny_mesh(rng, "sphere")
    m, _, dom = _mesh(V, F)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "m.p2m")
        m.save(path)
        m2 = P.Mesh.load(path)
        for a, b in zip(m.table(), m2.table()):
            assert np.array_equal(a, b)
        Q = rng.uniform(dom[0], dom[1], size=(500, 3)).astype(np.float32)
        h1, h2 = m.query_host(Q), m2.query_host(Q)
        assert np.array_equal(h1["prim"], h2["prim"]) and np.array_equal(h1["dist"], h2["dist"])
        with open(path, "r+b") as fh:
            fh.seek(40)
            fh.write(b"\x00\x01\x02\x03")
        with pytest.raises(P.P2MError):
            P.Mesh.load(path)


# ------------------------------------------------ mixed primitive sets (Sec. 5.5)

def _wire(F):
    return np.unique(np.sort(np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]]), axis=1), axis=0)


@pytest.mark.parametrize("S,msg", [
    ([[0, 9]], "out of range"),
    ([[2, 2]], "repeats"),
    ([[-1, 0]], "out of range"),
])
def test_mixed_validation(S, msg):
    with pytest.raises(P.P2MError, match=msg):
        P.Mesh(TETRA_V, TETRA_F, segments=S)


def test_mixed_needs_a_primitive():
    with pytest.raises(P.P2MError, match="at least one"):
        P.Mesh(TETRA_V, np.zeros((0, 3), np.int32), segments=np.zeros((0, 2), np.int32))


def test_mixed_edges_union_and_duplicates():
    """A segment that is also a face side is that edge; the others are new
    edges, all numbered in lexicographic (min, max) order."""
    m = P.Mesh(TETRA_V, TETRA_F[:1], segments=[[3, 0], [2, 0], [1, 3]])
    E = m.edges()
    assert [tuple(e) for e in E.tolist()] == sorted({(0, 1), (0, 2), (1, 2), (0, 3), (1, 3)})


@pytest.mark.parametrize("name", ["wireframe", "c6"])
def test_mixed_host_query(name):
    """Segment-only and mixed sets through the host model of the kernel:
    every answer accepted by the FP64 oracle over the same primitive set,
    including points on segments, near their ends and pushed off them."""
    from synth import mesh as M
    rng = np.random.default_rng(71)
    if name == "wireframe":
        V, F0 = random_tiny_mesh(rng, "sphere")
        F, S = np.zeros((0, 3), np.int32), _wire(F0)
        m, st, (lo, hi) = None, None, SQ.scaled_box(*SQ.aabb(V), 1.5)
        Q = [rng.uniform(lo, hi, size=(2000, 3))]
    else:
        w = C.c6(n_queries=3000)
        V, F, S = w.V, w.F, w.S
        lo, hi = w.domain_lo, w.domain_hi
        Q = [w.Q.astype(np.float64)]
    m = P.Mesh(V, F, segments=S)
    m.precompute(domain=(lo, hi))
    Vd = V.astype(np.float64)
    k = rng.integers(0, len(S), 300)
    for t in (0.5, 1e-4, 1 - 1e-4, 0.0):
        P0 = Vd[S[k, 0]] * (1 - t) + Vd[S[k, 1]] * t
        Q.append(P0)
        Q.append(P0 + 1e-3 * rng.normal(size=P0.shape))
    Q = np.clip(np.concatenate(Q), lo, hi).astype(np.float32)
    om = oracle.OracleMesh(V, F, segments=S)
    h = m.query_host(Q)
    assert check_answers(om, Q, om.query(Q), h["prim"], h["closest"], h["dist"]) == []


def test_mixed_save_load_roundtrip():
    rng = np.random.default_rng(72)
    V, F0 = random_tiny_mesh(rng, "sphere")
    S = _wire(F0)[::2]
    m = P.Mesh(V, F0[: len(F0) // 2], segments=S)
    lo, hi = SQ.scaled_box(*SQ.aabb(V), 1.5)
    m.precompute(domain=(lo, hi))
    Q = rng.uniform(lo, hi, size=(500, 3)).astype(np.float32)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mixed.p2m")
        m.save(path)
        m2 = P.Mesh.load(path)
    assert np.array_equal(m.edges(), m2.edges())
    a, b = m.query_host(Q), m2.query_host(Q)
    assert np.array_equal(a["prim"], b["prim"]) and np.array_equal(a["dist"], b["dist"])


@pytest.mark.parametrize("kw,msg", [(dict(table_mode=4), "bad table_mode"),
                                    (dict(table_mode=P.TABLE_FLOODING_DEVICE, device_visit_cap=513), "device_visit_cap"),
                                    (dict(table_mode=P.TABLE_FLOODING_DEVICE, device_visit_cap=-1), "device_visit_cap")])
def test_precompute_option_validation(kw, msg):
    """Build options are checked before any work, on the host."""
    m = P.Mesh(TETRA_V, TETRA_F)
    with pytest.raises(P.P2MError, match=msg):
        m.precompute(**kw)


def test_list_statistics():
    """Table 1's list statistics: Avg^1 and the maxima from the table itself;
    Avg^2 (weighted by Voronoi-cell volume in D) against an independent
    estimate: uniform random points of D, their nearest vertex by brute
    force, the mean of its list lengths (within 4 standard errors)."""
    rng = np.random.default_rng(14)
    V, F = random_tiny_mesh(rng, "sphere")
    m, st, (lo, hi) = _mesh(V, F, scale=2.0)
    off, _ = m.table()
    ne = (off[1::2][:len(V)] - off[0::2][:len(V)]).astype(np.float64)
    nf = (off[2::2] - off[1::2][:len(V)]).astype(np.float64)
    assert abs(st["avg_edges"] - ne.mean()) < 1e-12 and abs(st["avg_faces"] - nf.mean()) < 1e-12
    assert st["max_edges"] == ne.max() and st["max_faces"] == nf.max()
    assert st["max_list"] == (ne + nf).max()
    Q = rng.uniform(lo, hi, size=(200_000, 3))
    nn = np.argmin(((Q[:, None, :] - V.astype(np.float64)[None]) ** 2).sum(-1), axis=1)
    for key, per in (("avg_edges_volw", ne), ("avg_faces_volw", nf), ("avg_list_volw", ne + nf)):
        x = per[nn]
        se = x.std() / np.sqrt(len(x))
        assert abs(st[key] - x.mean()) <= 4 * se + 0.01, (key, st[key], x.mean(), se)
    assert st["flood_visits"] == st["flood_tests"] + 2 * st["ne"] + 3 * st["nf"]


def test_host_odd_meshes():
    """Triangle soups, a high-valence fan, slivers and a non-manifold set
    (tests/_helpers.odd_meshes) through the host model, every answer against
    the oracle; flooding (Algorithm 1) gives the table that testing every
    vertex-primitive pair gives (Theorem 7), on these inputs too."""
    from tests._helpers import odd_meshes
    rng = np.random.default_rng(7)
    for name, V, F in odd_meshes(rng):
        lo, hi = SQ.aabb(V)
        dom = SQ.scaled_box(lo, hi, 1.5)
        m, _, _ = _mesh(V, F, domain=dom)
        Q = rng.uniform(dom[0], dom[1], size=(2000, 3)).astype(np.float32)
        om = oracle.OracleMesh(V, F)
        out = m.query_host(Q)
        assert check_answers(om, Q, om.query(Q), out["prim"], out["closest"], out["dist"]) == [], name
        m2, _, _ = _mesh(V, F, domain=dom, mode=P.TABLE_ALL_PAIRS)
        o1, e1 = m.table()
        o2, e2 = m2.table()
        for v in range(len(V)):
            for r in (0, 1):
                a = set(e1[o1[2 * v + r]:o1[2 * v + r + 1]].tolist())
                b = set(e2[o2[2 * v + r]:o2[2 * v + r + 1]].tolist())
                assert a == b, (name, v, r)


@pytest.mark.parametrize("scale,offset", [(1.0, 1e3), (1.0, 1e4), (1.0, -3e4), (1e-3, 5.0), (1e3, 0.0)])
def test_host_far_from_origin(scale, offset):
    """A mesh far from the origin (or tiny, or large): the distance keeps the
    tolerance because an edge's or face's closest point is formed relative to
    the domain centre; the reported float32 point carries its own rounding
    (tests/_accept.py)."""
    w = C.c1(n_queries=2000)
    V = (w.V.astype(np.float64) * scale + offset).astype(np.float32)
    Q = (w.Q.astype(np.float64) * scale + offset).astype(np.float32)
    m, _, _ = _mesh(V, w.F)
    om = oracle.OracleMesh(V, w.F)
    out = m.query_host(Q)
    assert check_answers(om, Q, om.query(Q), out["prim"], out["closest"], out["dist"]) == []


def _odd_domains(V):
    lo, hi = SQ.aabb(V)
    c, e = 0.5 * (lo + hi), hi - lo
    return [("inner half", c - 0.25 * e, c + 0.25 * e), ("one octant", c, hi),
            ("thin slab", np.array([lo[0], lo[1], c[2] - 1e-3]), np.array([hi[0], hi[1], c[2] + 1e-3])),
            ("far box", hi + 2 * e, hi + 3 * e), ("exact box", lo, hi)]


def test_host_domains_not_holding_the_mesh():
    """Query domains that hold only part of the mesh, a thin slab, a box
    away from it, the mesh's own box: answers in D stay exact (the cells are
    clipped to D, the primitives are not)."""
    w = C.c1(n_queries=10)
    rng = np.random.default_rng(3)
    om = oracle.OracleMesh(w.V, w.F)
    for name, dlo, dhi in _odd_domains(w.V):
        m, _, _ = _mesh(w.V, w.F, domain=(dlo, dhi))
        Q = rng.uniform(dlo, dhi, size=(2000, 3)).astype(np.float32)
        out = m.query_host(Q)
        assert check_answers(om, Q, om.query(Q), out["prim"], out["closest"], out["dist"]) == [], name


def test_host_domain_1000x():
    """A domain 1,000 times the mesh's box, queries over all of it (up to
    hundreds of diagonals from the mesh): answers exact to the float32
    output (the distance within two float32 spacings of the exact one,
    tests/_accept.py), and within tol near the mesh."""
    w = C.c1(n_queries=10)
    lo, hi = SQ.aabb(w.V)
    m, _, dom = _mesh(w.V, w.F, scale=1000.0)
    om = oracle.OracleMesh(w.V, w.F)
    rng = np.random.default_rng(5)
    for qs in (1.2, 1000.0):
        b = SQ.scaled_box(lo, hi, qs)
        Q = rng.uniform(b[0], b[1], size=(2000, 3)).astype(np.float32)
        out = m.query_host(Q)
        ans = om.query(Q)
        assert check_answers(om, Q, ans, out["prim"], out["closest"], out["dist"]) == [], qs
        if qs < 2:
            assert np.max(np.abs(out["dist"].astype(np.float64) - ans["dist"])) <= 1e-5 * om.diag


def test_host_flat_meshes():
    """Coplanar vertex sets (tests/_helpers.flat_meshes) with a padded domain
    and with the default one: every answer against the oracle."""
    from tests._helpers import flat_meshes
    rng = np.random.default_rng(1)
    for name, V, F in flat_meshes():
        lo, hi = SQ.aabb(V)
        for dom in ((lo - 0.5, hi + 0.5), None):
            m = P.Mesh(V, F)
            m.precompute(domain=dom)
            qlo, qhi = (lo - 0.5, hi + 0.5)
            Q = rng.uniform(qlo, qhi, size=(1500, 3)).astype(np.float32)
            om = oracle.OracleMesh(V, F)
            out = m.query_host(Q)
            assert check_answers(om, Q, om.query(Q), out["prim"], out["closest"], out["dist"]) == [], (name, dom)
