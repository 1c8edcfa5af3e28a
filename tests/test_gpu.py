"""GPU parity: the HIP path through the C interface against the FP64
brute-force oracle (acceptance rule in tests/_accept.py), and the query
ordering against its definition, bit for bit."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import morton as OM
from synth import configs as C
from synth import queries as SQ
from tests._accept import check_answers
from tests._helpers import CUBE_F, CUBE_V, TETRA_F, TETRA_V, random_tiny_mesh

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _build(V, F, domain, mode=0):
    import paper_2308_16084_amd as P
    m = P.Mesh(V, F)
    m.precompute(domain=domain, table_mode=mode)
    m.upload(0)
    return m


def _run(m, Q, **kw):
    torch = _torch()
    q = torch.from_numpy(np.ascontiguousarray(Q, dtype=np.float32)).cuda()
    out = m.query(q, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.fixture(scope="module")
def c1():
    w = C.c1()
    m = _build(w.V, w.F, (w.domain_lo, w.domain_hi))
    om = oracle.OracleMesh(w.V, w.F)
    return w, m, om, om.query(w.Q)


def test_c1_all_queries(c1):
    """Workload C1: icosphere level 4, all 10^4 queries, sorted launch."""
    w, m, om, ans = c1
    print("case: c1 sorted", flush=True)
    out = _run(m, w.Q, sort=True)
    assert check_answers(om, w.Q, ans, out["prim"], out["closest"], out["dist"]) == []
    assert np.all(out["status"] == 0)


def test_c1_unsorted_and_block_sizes_identical(c1):
    """Ordering and launch shape change which lane runs a query, never its answer."""
    w, m, om, ans = c1
    ref = _run(m, w.Q)
    for kw in ({"sort": True}, {"sort": False}, {"block_size": 64}, {"block_size": 64, "sort": True},
               {"block_size": 128, "sort": False}, {"traversal": 1},
               {"traversal": 1, "lds_levels": 4}, {"traversal": 1, "lds_levels": 9, "block_size": 64},
               {"traversal": 1, "lds_levels": 8, "sort": False},
               {"traversal": 2}, {"traversal": 2, "sort": False}, {"traversal": 3},
               {"traversal": 3, "sort": False, "block_size": 64}, {"lds_levels": 9}):
        print("case: c1", kw, flush=True)
        out = _run(m, w.Q, **kw)
        for k in ("prim", "closest", "dist"):
            assert np.array_equal(out[k], ref[k]), (kw, k)


def test_default_ordering_by_batch_size(c1):
    """The default orders a batch from 2^19 queries on and leaves smaller
    ones in input order; the profile's ordering time is zero exactly when no
    ordering ran, and the answers are those of an explicit choice."""
    torch = _torch()
    w, m, om, ans = c1
    rng = np.random.default_rng(5)
    for n in (1000, (1 << 19) - 1, 1 << 19):
        print("case: default ordering n =", n, flush=True)
        Q = w.Q[rng.integers(0, len(w.Q), n)]
        q = torch.from_numpy(np.ascontiguousarray(Q, dtype=np.float32)).cuda()
        out = m.query(q, profile=True)
        order_ms, query_ms, finish_ms = m.query_profile()
        ordered = n >= (1 << 19)
        assert (order_ms > 0) == ordered and (finish_ms > 0) == ordered and query_ms > 0, (n, order_ms, finish_ms)
        ref = m.query(q, sort=ordered)
        for k in ("prim", "closest", "dist", "status"):
            assert torch.equal(out[k], ref[k]), (n, k)


def test_c1_matches_host_model(c1):
    """Same tree, table and float32 code on host and device: same primitive,
    distances equal to a few ulps (the device may fuse multiply-adds)."""
    w, m, om, ans = c1
    out = _run(m, w.Q)
    h = m.query_host(w.Q)
    assert np.mean(out["prim"] == h["prim"]) > 0.999
    assert np.max(np.abs(out["dist"] - h["dist"])) <= 1e-6


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_tiny_meshes(mode):
    rng = np.random.default_rng(40 + mode)
    meshes = [(TETRA_V, TETRA_F), (CUBE_V, CUBE_F), random_tiny_mesh(rng, "sphere"),
              random_tiny_mesh(rng, "heightfield")]
    for k, (V, F) in enumerate(meshes):
        lo, hi = SQ.aabb(V)
        dom = SQ.scaled_box(lo, hi, 3.0)
        print(f"case: tiny mesh {k} mode {mode}", flush=True)
        m = _build(V, F, dom, mode)
        Q = rng.uniform(dom[0], dom[1], size=(5000, 3)).astype(np.float32)
        om = oracle.OracleMesh(V, F)
        ans = om.query(Q)
        # the staged tree top may hold the whole tree (4 to a few hundred vertices)
        for kw in ({}, {"traversal": 3}, {"traversal": 1, "lds_levels": 9}, {"traversal": 1, "lds_levels": 1}):
            out = _run(m, Q, **kw)
            assert check_answers(om, Q, ans, out["prim"], out["closest"], out["dist"]) == [], kw


def test_odd_meshes_on_device():
    """Triangle soups, a high-valence fan, slivers and a non-manifold set
    with lists of 500 entries: every answer against the oracle, the
    traversals and the ordering change no answer, and the inspection on the
    device builds the host's table."""
    from tests._helpers import odd_meshes
    rng = np.random.default_rng(7)
    for name, V, F in odd_meshes(rng):
        lo, hi = SQ.aabb(V)
        dom = SQ.scaled_box(lo, hi, 1.5)
        print(f"case: odd mesh {name}", flush=True)
        m = _build(V, F, dom)
        tri = V.astype(np.float64)[F]
        b = rng.dirichlet([1, 1, 1], 1000)
        near = (tri[rng.integers(0, len(F), 1000)] * b[:, :, None]).sum(1) + 1e-3 * rng.standard_normal((1000, 3))
        Q = np.concatenate([rng.uniform(dom[0], dom[1], size=(3000, 3)), near]).astype(np.float32)
        om = oracle.OracleMesh(V, F)
        ans = om.query(Q)
        ref = _run(m, Q)
        assert check_answers(om, Q, ans, ref["prim"], ref["closest"], ref["dist"]) == [], name
        for kw in ({"traversal": 1}, {"traversal": 2}, {"sort": True}):
            out = _run(m, Q, **kw)
            for k in ref:
                assert np.array_equal(out[k], ref[k]), (name, kw, k)
        # the inspection on the device builds the host's table, entry for entry
        import paper_2308_16084_amd as P
        md = P.Mesh(V, F)
        md.precompute(domain=dom, table_mode=P.TABLE_FLOODING_DEVICE)
        assert all(np.array_equal(a, c) for a, c in zip(md.table(), m.table())), name
        assert np.array_equal(md.table_boxes(), m.table_boxes()), name


def test_domains_not_holding_the_mesh_on_device():
    """The host suite's odd domains (part of the mesh, a thin slab, a box
    away from it, the mesh's own box) through the device path, ordered and
    in input order, against the oracle."""
    from tests.test_host import _odd_domains
    w = C.c1(n_queries=10)
    rng = np.random.default_rng(3)
    om = oracle.OracleMesh(w.V, w.F)
    for name, dlo, dhi in _odd_domains(w.V):
        print("case: domain", name, flush=True)
        m = _build(w.V, w.F, (dlo, dhi))
        Q = rng.uniform(dlo, dhi, size=(3000, 3)).astype(np.float32)
        ans = om.query(Q)
        for sort in (True, False):
            out = _run(m, Q, sort=sort)
            assert check_answers(om, Q, ans, out["prim"], out["closest"], out["dist"]) == [], (name, sort)
            assert np.all(out["status"] == 0), name


def test_domain_1000x_on_device():
    """D 1,000 times the mesh's box (the walk's second seed grid covers the
    mesh), queries near the mesh and over all of D, ordered and in input
    order: exact to the float32 output (tests/_accept.py)."""
    w = C.c1(n_queries=10)
    lo, hi = SQ.aabb(w.V)
    m = _build(w.V, w.F, SQ.scaled_box(lo, hi, 1000.0))
    om = oracle.OracleMesh(w.V, w.F)
    rng = np.random.default_rng(5)
    for qs in (1.2, 30.0, 1000.0):
        b = SQ.scaled_box(lo, hi, qs)
        Q = rng.uniform(b[0], b[1], size=(3000, 3)).astype(np.float32)
        ans = om.query(Q)
        for sort in (True, False):
            print("case: D 1000x, queries in", qs, "sort", sort, flush=True)
            out = _run(m, Q, sort=sort)
            assert check_answers(om, Q, ans, out["prim"], out["closest"], out["dist"]) == [], (qs, sort)


def test_flat_meshes_on_device():
    """Coplanar vertex sets (tests/_helpers.flat_meshes) through the device
    path, ordered and in input order, against the oracle."""
    from tests._helpers import flat_meshes
    rng = np.random.default_rng(1)
    for name, V, F in flat_meshes():
        lo, hi = SQ.aabb(V)
        print("case: flat mesh", name, flush=True)
        m = _build(V, F, (lo - 0.5, hi + 0.5))
        Q = rng.uniform(lo - 0.5, hi + 0.5, size=(2000, 3)).astype(np.float32)
        om = oracle.OracleMesh(V, F)
        ans = om.query(Q)
        for sort in (True, False):
            out = _run(m, Q, sort=sort)
            assert check_answers(om, Q, ans, out["prim"], out["closest"], out["dist"]) == [], (name, sort)
        # the inspection on the device builds the host's table here too
        import paper_2308_16084_amd as P
        md = P.Mesh(V, F)
        md.precompute(domain=(lo - 0.5, hi + 0.5), table_mode=P.TABLE_FLOODING_DEVICE)
        assert all(np.array_equal(a, c) for a, c in zip(md.table(), m.table())), name


def test_far_mesh_device_table():
    """C1 moved 10^4 units from the origin: the inspection on the device
    builds the host's table, entry for entry."""
    import paper_2308_16084_amd as P
    w = C.c1(n_queries=10)
    V = (w.V.astype(np.float64) + 1e4).astype(np.float32)
    lo, hi = SQ.aabb(V)
    dom = SQ.scaled_box(lo, hi, 1.5)
    h = P.Mesh(V, w.F)
    h.precompute(domain=dom)
    d = P.Mesh(V, w.F)
    d.precompute(domain=dom, table_mode=P.TABLE_FLOODING_DEVICE)
    assert all(np.array_equal(a, c) for a, c in zip(d.table(), h.table()))
    assert np.array_equal(d.table_boxes(), h.table_boxes())


def test_golden_points_on_device():
    from tests._helpers import load_golden, primitive_vertices
    for V, F, name in ((TETRA_V, TETRA_F, "tetra.txt"), (CUBE_V, CUBE_F, "cube.txt")):
        rows = load_golden(name)
        Q = np.array([r[0] for r in rows], np.float32)
        lo, hi = SQ.aabb(V)
        m = _build(V, F, SQ.scaled_box(lo, hi, 8.0))
        out = _run(m, Q)
        om = oracle.OracleMesh(V, F)
        for i, (q, prims, d, c) in enumerate(rows):
            t = int((np.int64(out["prim"][i]) & 0xFFFFFFFF) >> 30)
            pid = int(out["prim"][i] & 0x3FFFFFFF)
            # the golden primitive (type and vertex set), or one of its listed
            # exact ties; where the golden closest point lies on a side or
            # corner of a face (its foot on the face's boundary), float32
            # rounding may report that face: it must contain the golden
            # primitive, and the closest point must be the golden one
            got = (t, primitive_vertices(om.F, om.E, t, pid))
            if got not in prims:
                assert t == 2 and c is not None and any(got[1] >= pv for _, pv in prims), (name, q, got, prims)
            assert abs(out["dist"][i] - d) <= 1e-6
            if c is not None:
                assert np.allclose(out["closest"][i], c, atol=1e-6), (name, q, out["closest"][i], c)


@pytest.mark.parametrize("n", [1, 2, 255, 4096, 4097, 70001, 1 << 20, (1 << 24) + 4097])
def test_order_bit_exact(c1, n):
    """Morton keys and their stable sort equal the definition exactly (the
    largest size has more than 16 count tiles per column-scan thread, the
    column scan's looped form)."""
    torch = _torch()
    w, m, _, _ = c1
    rng = np.random.default_rng(n)
    lo, hi = w.domain_lo, w.domain_hi
    Q = rng.uniform(lo - 0.2, hi + 0.2, size=(n, 3)).astype(np.float32)
    if n > 100:
        Q[10:60] = Q[3]                 # runs of equal keys
        Q[70] = np.nan                  # non-finite -> cell 0
    keys, perm = m.order_queries(torch.from_numpy(Q).cuda())
    torch.cuda.synchronize()
    rk, rp = OM.order(Q, lo, hi)
    assert np.array_equal(keys.cpu().numpy().view(np.uint32), rk)
    assert np.array_equal(perm.cpu().numpy(), rp)
    if n > 100:
        # already in key order: whole wavefronts share their high digits
        Qs = np.ascontiguousarray(Q[rp])
        keys, perm = m.order_queries(torch.from_numpy(Qs).cuda())
        torch.cuda.synchronize()
        rk2, rp2 = OM.order(Qs, lo, hi)
        assert np.array_equal(rp2, np.arange(n))
        assert np.array_equal(keys.cpu().numpy().view(np.uint32), rk2)
        assert np.array_equal(perm.cpu().numpy(), rp2)
    # queries at an address that is not 16-byte aligned (the key kernel's
    # scalar form): the same keys and permutation
    buf = torch.zeros(3 * n + 1, dtype=torch.float32, device="cuda")
    buf[1:] = torch.from_numpy(Q.reshape(-1)).cuda()
    qu = buf[1:].view(n, 3)
    assert qu.data_ptr() % 16 != 0
    keys, perm = m.order_queries(qu)
    torch.cuda.synchronize()
    assert np.array_equal(keys.cpu().numpy().view(np.uint32), rk)
    assert np.array_equal(perm.cpu().numpy(), rp)


@pytest.mark.parametrize("traversal", [1, 2, 3])
@pytest.mark.parametrize("ordered", [False, True])
def test_nearest_vertex_brute_force(c1, traversal, ordered):
    """Every traversal returns the exact nearest vertex, on scattered and on
    Morton-ordered batches, inside and outside the query domain."""
    torch = _torch()
    w, m, om, _ = c1
    rng = np.random.default_rng(11)
    lo, hi = w.domain_lo, w.domain_hi
    Q = np.concatenate([w.Q, rng.uniform(lo - 0.5 * (hi - lo), hi + 0.5 * (hi - lo), size=(3000, 3)),
                        np.array([lo, hi, [lo[0], hi[1], lo[2]]])]).astype(np.float32)
    if ordered:
        Q = Q[OM.order(Q, w.domain_lo, w.domain_hi)[1]]
    vid, d2 = m.nearest_vertex(torch.from_numpy(np.ascontiguousarray(Q)).cuda(), traversal=traversal)
    torch.cuda.synchronize()
    vid = vid.cpu().numpy()
    D = ((Q.astype(np.float64)[:, None, :] - om.V[None]) ** 2).sum(-1)
    best = D.min(1)
    got = D[np.arange(len(Q)), vid]
    # exact nearest, or a tie within float64 rounding of the squared distance
    assert np.all(got <= best * (1 + 1e-12) + 1e-300)


def test_edge_cases(c1):
    torch = _torch()
    import paper_2308_16084_amd as P
    w, m, om, _ = c1
    out = _run(m, np.zeros((0, 3), np.float32))
    assert out["dist"].shape == (0,)
    Q = np.array([[0.1, 0.2, 0.3], [np.nan, 0, 0], [0, np.inf, 0], [30.0, 0, 0]], np.float32)
    out = _run(m, Q)
    # the ordered path (keys, sort, staged answers, write-out) on a tiny batch: same answers
    for n in (0, 1, 4):
        o = _run(m, Q[:n], sort=True)
        for k in out:
            assert np.array_equal(o[k], out[k][:n], equal_nan=o[k].dtype.kind == "f"), (n, k)
    assert out["status"].tolist() == [0, P.NONFINITE, P.NONFINITE, P.OUT_OF_DOMAIN]
    assert np.isnan(out["dist"][1]) and np.isnan(out["dist"][2])
    assert P.prim_type(out["prim"][1]) == P.NONE
    a = om.query(Q[[0, 3]])
    assert abs(out["dist"][0] - a["dist"][0]) <= 1e-5 * om.diag
    assert out["dist"][3] >= a["dist"][1] - 1e-5 * om.diag  # an upper bound outside the domain
    with pytest.raises(TypeError):
        m.query(torch.zeros((4, 3), dtype=torch.float64, device="cuda"))
    with pytest.raises(P.P2MError):
        m.query(torch.zeros((4, 3), dtype=torch.float32, device="cuda"), block_size=1024)
    for bad in (-1, 10):
        with pytest.raises(P.P2MError):
            m.query(torch.zeros((4, 3), dtype=torch.float32, device="cuda"), traversal=1, lds_levels=bad)
    with pytest.raises(P.P2MError):
        P.Mesh(TETRA_V, TETRA_F).upload(0)  # before precompute


def _sampled_parity(w, m, n_sample, seed):
    """n_sample seeded rows, stratified: half from the uniform rows, half from
    the near-surface rows of the workload."""
    om = oracle.OracleMesh(w.V, w.F)
    out = _run(m, w.Q)
    rng = np.random.default_rng(seed)
    near = w.meta["near"]
    idx = np.sort(np.concatenate([rng.choice(np.nonzero(~near)[0], size=n_sample // 2, replace=False),
                                  rng.choice(np.nonzero(near)[0], size=n_sample - n_sample // 2, replace=False)]))
    print(f"case: oracle on {len(idx)} sampled rows", flush=True)
    ans = om.query(w.Q[idx])
    fails = check_answers(om, w.Q[idx], ans, out["prim"][idx], out["closest"][idx], out["dist"][idx], idx=idx)
    err = np.abs(out["dist"][idx].astype(np.float64) - ans["dist"]) / (1e-5 * om.diag)
    print(f"worst |d - d*| = {err.max():.3f} tol", flush=True)
    return fails, out


@pytest.fixture(scope="module")
def c2_full():
    print("case: building c2 (655,362 V / 1,310,720 F)", flush=True)
    import os
    import paper_2308_16084_amd as P
    w = C.c2()
    m, _ = P.Mesh.cached(w.V, w.F, (w.domain_lo, w.domain_hi), os.environ.get("P2M_CACHE_DIR") or None)
    m.upload(0)
    return w, m


def test_c2_full_size_sampled(c2_full):
    """Workload C2 at full size (10^7 queries, one sorted launch as timed by
    the benchmark); 10^4 seeded rows (5,000 uniform, 5,000 near-surface)
    checked against the oracle; all distances finite and non-negative; no
    row flagged out of domain."""
    w, m = c2_full
    print("case: c2 sampled parity", flush=True)
    fails, out = _sampled_parity(w, m, 10_000, 77)
    assert fails == []
    out1 = _run(m, w.Q[:200_000], traversal=1)
    # the tree's top eight levels read from LDS: the same answers, bit for bit
    out1s = _run(m, w.Q[:200_000], traversal=1, lds_levels=8)
    for k in ("prim", "closest", "dist", "status"):
        assert np.array_equal(out1s[k], out1[k]), k
    # the traversals agree on the nearest vertex up to float64 ties
    for t in (2, 3):
        out2 = _run(m, w.Q[:200_000], traversal=t)
        assert np.mean(out1["prim"] == out2["prim"]) > 0.9999, t
        assert np.max(np.abs(out1["dist"] - out2["dist"])) <= 1e-5 * 3.8, t
    assert np.all(np.isfinite(out["dist"])) and np.all(out["dist"] >= 0)
    assert np.all(out["status"] == 0)


def test_c2_traversals_same_vertex(c2_full):
    """All 10^7 C2 queries in the query kernel's order (stable by the top 24
    Morton bits): the per-lane tree search, the wavefront tree walk and the
    Voronoi walk return the same nearest vertex for every query.  The batch
    holds the wavefront whose lanes 23 and 41 (input rows 1,314,140 and
    6,265,676) the wavefront tree walk once answered with their
    second-nearest vertex: returning from a node's near child it tested the
    near child's box where the far child's was meant, and a lane whose near
    box sat at its bound by one rounding let the far child go for all."""
    torch = _torch()
    w, m = c2_full
    k = OM.morton_keys(w.Q, w.domain_lo, w.domain_hi) >> 6
    perm = np.argsort(k, kind="stable")
    q = torch.from_numpy(np.ascontiguousarray(w.Q[perm])).cuda()
    vids = {}
    for t in (1, 2, 3):
        print("case: c2 nearest vertex, traversal", t, flush=True)
        vid, _ = m.nearest_vertex(q, traversal=t)
        torch.cuda.synchronize()
        vids[t] = vid.cpu().numpy()
    for t in (2, 3):
        diff = np.nonzero(vids[1] != vids[t])[0]
        assert len(diff) == 0, (t, len(diff), perm[diff[:5]].tolist())
    pos = np.empty(len(perm), np.int64)
    pos[perm] = np.arange(len(perm))
    V = w.V.astype(np.float64)
    for r in (1_314_140, 6_265_676):
        D = ((V - w.Q[r].astype(np.float64)) ** 2).sum(1)
        assert vids[2][pos[r]] == int(np.argmin(D)), r
