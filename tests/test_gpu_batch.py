"""Batched P2M: many meshes of uneven size in one persistent, graph-captured
launch, against the oracle and against one plain launch per mesh."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import morton as OM
from synth import configs as C
from tests._accept import check_answers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch_setup():
    import torch

    import paper_2308_16084_amd as P
    plan = C.c4_plan(count=12, tri_hi=2e4, q_hi=2e4)
    works = [C.c4_mesh(e) for e in plan]
    works[3].Q = works[3].Q[:0]            # a mesh with no queries
    meshes = []
    for w in works:
        m = P.Mesh(w.V, w.F)
        m.precompute(domain=(w.domain_lo, w.domain_hi))
        meshes.append(m)
    b = P.Batch(meshes, 0)
    Q = np.concatenate([w.Q for w in works])
    off = np.concatenate([[0], np.cumsum([len(w.Q) for w in works])]).astype(np.int64)
    q = torch.from_numpy(Q).cuda()
    return works, meshes, b, Q, off, q


def _np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def test_batch_against_oracle(batch_setup):
    import torch
    works, meshes, b, Q, off, q = batch_setup
    out = _np(b.query(q, off))
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    for k, w in enumerate(works):
        if len(w.Q) == 0:
            continue
        print(f"case: batch mesh {k} ({w.name}, {len(w.Q)} queries)", flush=True)
        idx = np.sort(rng.choice(len(w.Q), size=min(64, len(w.Q)), replace=False))
        rows = off[k] + idx
        om = oracle.OracleMesh(w.V, w.F)
        ans = om.query(w.Q[idx])
        assert check_answers(om, w.Q[idx], ans, out["prim"][rows], out["closest"][rows], out["dist"][rows]) == []


def test_batch_equals_plain_launches(batch_setup):
    import torch
    works, meshes, b, Q, off, q = batch_setup
    ref = _np(b.query(q, off))
    for k, (w, m) in enumerate(zip(works, meshes)):
        if len(w.Q) == 0:
            continue
        m.upload(0)
        o = _np(m.query(q[off[k]:off[k + 1]].contiguous(), traversal=1))
        sl = slice(off[k], off[k + 1])
        assert np.mean(o["prim"] == ref["prim"][sl]) > 0.999
        assert np.max(np.abs(o["dist"] - ref["dist"][sl])) <= 1e-5 * w.diag


def test_graph_replays_match_eager(batch_setup):
    """Replay the captured graph several times, with eager work and
    synchronisation in between; every replay equals the eager result."""
    import torch
    works, meshes, b, Q, off, q = batch_setup
    eager = _np(b.query(q, off, graph=False))
    torch.cuda.synchronize()
    out = None
    for r in range(4):
        out = b.query(q, off, out=out)
        torch.cuda.synchronize()
        got = _np(out)
        for key in ("prim", "closest", "dist"):
            assert np.array_equal(got[key], eager[key]), (r, key)
        junk = torch.randn(1 << 20, device="cuda") * 2.0   # unrelated eager work between replays
        junk.sum().item()
        for v in out.values():
            v.fill_(-1)


# (64, 8, 3) and (128, 5, 3): a tile's rounds regrouped in several groups of
# up to 256 queries, the last one partial
@pytest.mark.parametrize("shape", [(64, 1, 1), (128, 2, 2), (256, 4, 1), (192, 3, 2), (64, 2, 3), (256, 1, 3),
                                   (64, 8, 3), (128, 5, 3)])
def test_launch_shapes_give_same_answers(batch_setup, shape):
    works, meshes, b, Q, off, q = batch_setup
    b.set_shape(256, 1, 1)
    ref = _np(b.query(q, off))
    b.set_shape(*shape)
    got = _np(b.query(q, off))
    assert np.mean(got["prim"] == ref["prim"]) > 0.999
    assert np.max(np.abs(got["dist"] - ref["dist"])) <= 1e-5 * max(w.diag for w in works)


def test_persistent_schedule_same_answers(batch_setup):
    """One workgroup per tile (the default) and persistent workgroups taking
    tiles from a counter give the same answers, bit for bit, graph and eager."""
    works, meshes, b, Q, off, q = batch_setup
    assert b.schedule() is False
    ref = _np(b.query(q, off))
    try:
        b.set_schedule(True)
        assert b.schedule() is True
        for graph in (True, False):
            got = _np(b.query(q, off, graph=graph))
            for k in ref:
                assert np.array_equal(got[k], ref[k]), (k, graph)
    finally:
        b.set_schedule(False)


def test_lds_levels_same_answers(batch_setup):
    """The per-lane tree search with the top of each tile's mesh's tree
    staged in LDS gives the answers of the unstaged search, bit for bit,
    graph and eager (meshes smaller than the staged levels included)."""
    import paper_2308_16084_amd as P
    works, meshes, b, Q, off, q = batch_setup
    shape = b.shape()
    assert b.lds_levels() == 0
    try:
        b.set_shape(128, 2, 1)
        ref = _np(b.query(q, off))
        for lv in (3, 9):
            b.set_lds_levels(lv)
            assert b.lds_levels() == lv
            for graph in (True, False):
                got = _np(b.query(q, off, graph=graph))
                for k in ref:
                    assert np.array_equal(got[k], ref[k]), (lv, k, graph)
        for bad in (-1, 10):
            with pytest.raises(P.P2MError):
                b.set_lds_levels(bad)
    finally:
        b.set_lds_levels(0)
        b.set_shape(*shape)


def test_autotune_and_layout_change(batch_setup):
    import torch
    works, meshes, b, Q, off, q = batch_setup
    ref = _np(b.query(q, off))
    shape = b.autotune(q, off)
    assert shape[0] in (64, 128, 256) and shape[1] in (1, 2, 4) and shape[2] in (1, 2, 3)
    assert b.lds_levels() in ((0, 8) if shape[2] == 1 else (0,))
    got = _np(b.query(q, off))
    assert np.mean(got["prim"] == ref["prim"]) > 0.999
    # a different split of the same rows between meshes: only mesh 0 and 1 swap sizes
    half = np.concatenate([[0], np.cumsum([len(w.Q) // 2 for w in works])]).astype(np.int64)
    q2 = torch.cat([q[off[k]:off[k] + len(works[k].Q) // 2] for k in range(len(works))]).contiguous()
    out2 = _np(b.query(q2, half))
    for k in range(len(works)):
        n2 = len(works[k].Q) // 2
        assert np.array_equal(out2["dist"][half[k]:half[k] + n2], got["dist"][off[k]:off[k] + n2]) or \
            np.max(np.abs(out2["dist"][half[k]:half[k] + n2] - got["dist"][off[k]:off[k] + n2])) <= 1e-6


def test_batch_status_flags(batch_setup):
    """Per-query status bits from the batched launch: out of the mesh's
    domain and non-finite queries are flagged as by the plain launch."""
    import torch

    import paper_2308_16084_amd as P
    works, meshes, b, Q, off, q = batch_setup
    Q2 = Q.copy()
    k = 1
    r0 = int(off[k])
    Q2[r0] = works[k].domain_hi + 1.0          # outside mesh k's domain
    Q2[r0 + 1] = np.nan                         # non-finite
    q2 = torch.from_numpy(Q2).cuda()
    for graph in (True, False):
        out = _np(b.query(q2, off, graph=graph))
        assert out["status"][r0] == P.OUT_OF_DOMAIN and out["status"][r0 + 1] == P.NONFINITE
        rest = np.ones(len(Q2), bool)
        rest[[r0, r0 + 1]] = False
        assert np.all(out["status"][rest] == 0)
        assert np.isnan(out["dist"][r0 + 1]) and P.prim_type(out["prim"][r0 + 1]) == P.NONE
        m = meshes[k]
        m.upload(0)
        o = _np(m.query(q2[r0:r0 + 2].contiguous()))
        assert o["status"].tolist() == out["status"][r0:r0 + 2].tolist()


def test_batch_outside_domain_nearest_vertex(batch_setup):
    """Queries in a box twice each mesh's domain (seven in eight outside D,
    where the walk hands over to the wavefront tree walk): the batched launch
    flags and answers them as a plain launch does (primitives equal up to
    0.1 %, as inside D), the plain launch's three traversals agree bit for
    bit, and the wavefront tree walk's vertex is the brute-force nearest one
    (outside D the answer itself is only an upper bound)."""
    import torch
    works, meshes, b, Q, off, q = batch_setup
    rng = np.random.default_rng(21)
    parts = []
    for w in works:
        ext = w.domain_hi - w.domain_lo
        parts.append(rng.uniform(w.domain_lo - 0.5 * ext, w.domain_hi + 0.5 * ext,
                                 size=(len(w.Q), 3)).astype(np.float32))
    Q2 = np.concatenate(parts)
    q2 = torch.from_numpy(Q2).cuda()
    out = _np(b.query(q2, off))
    for k, (w, m) in enumerate(zip(works, meshes)):
        if len(w.Q) == 0:
            continue
        print(f"case: batch mesh {k} outside-domain queries", flush=True)
        sl = slice(off[k], off[k + 1])
        m.upload(0)
        qk = q2[sl].contiguous()
        ref = _np(m.query(qk))
        for t in (1, 2):
            o = _np(m.query(qk, traversal=t))
            for key in ref:
                assert np.array_equal(o[key], ref[key]), (k, t, key)
        assert np.array_equal(out["status"][sl], ref["status"])
        assert np.mean(out["prim"][sl] == ref["prim"]) > 0.999
        vid, _ = m.nearest_vertex(qk, traversal=2)
        idx = rng.choice(len(w.Q), size=min(500, len(w.Q)), replace=False)
        vid = vid.cpu().numpy()[idx]
        D = ((Q2[sl][idx].astype(np.float64)[:, None, :] - w.V.astype(np.float64)[None]) ** 2).sum(-1)
        assert np.all(D[np.arange(len(vid)), vid] <= D.min(1) * (1 + 1e-12)), k
    assert np.any(out["status"] == 0) and np.any(out["status"] != 0)


def test_batch_order_bit_exact(batch_setup):
    """The batched query's ordering equals its definition: per mesh, the top
    24 bits of the Morton key in the mesh's own domain and a stable sort of
    the mesh's rows, in place (an empty mesh included); also with runs of
    equal keys and a non-finite query."""
    import torch
    works, meshes, b, Q, off, q = batch_setup
    Q2 = Q.copy()
    k1 = 1
    Q2[off[k1]:off[k1] + 40] = Q2[off[k1]]      # a run of equal keys
    Q2[off[k1] + 50] = np.nan                    # non-finite: cell 0
    for Qx in (Q, Q2):
        keys, perm = b.order_queries(torch.from_numpy(Qx).cuda(), off)
        torch.cuda.synchronize()
        keys, perm = keys.cpu().numpy().view(np.uint32), perm.cpu().numpy()
        for k, w in enumerate(works):
            rk = OM.morton_keys(Qx[off[k]:off[k + 1]], w.domain_lo, w.domain_hi) >> 6
            rp = np.argsort(rk, kind="stable")
            assert np.array_equal(keys[off[k]:off[k + 1]], rk[rp]), k
            assert np.array_equal(perm[off[k]:off[k + 1]], rp + off[k]), k


def test_far_from_origin_single_and_batched():
    """C1 moved 10^4 units from the origin: the plain launch, ordered and in
    input order, and a batch of it with the mesh at its own place, all against
    the oracle (the write-outs rebuild the distance from the point staged
    relative to each mesh's domain centre)."""
    import torch

    import paper_2308_16084_amd as P
    from synth import queries as SQ
    w = C.c1(n_queries=4000)
    works = []
    for off in (0.0, 1e4):
        V = (w.V.astype(np.float64) + off).astype(np.float32)
        Q = (w.Q.astype(np.float64) + off).astype(np.float32)
        works.append((V, Q))
    meshes = []
    for V, Q in works:
        lo, hi = SQ.aabb(V)
        m = P.Mesh(V, w.F)
        m.precompute(domain=SQ.scaled_box(lo, hi, 1.5))
        meshes.append(m)
    V, Q = works[1]
    om = oracle.OracleMesh(V, w.F)
    ans = om.query(Q)
    meshes[1].upload(0)
    q = torch.from_numpy(Q).cuda()
    for sort in (True, False):
        print("case: far mesh, sort", sort, flush=True)
        out = _np(meshes[1].query(q, sort=sort))
        assert check_answers(om, Q, ans, out["prim"], out["closest"], out["dist"]) == [], sort
    b = P.Batch(meshes, 0)
    Qb = np.concatenate([x[1] for x in works])
    off = np.array([0, len(works[0][1]), len(Qb)], np.int64)
    out = _np(b.query(torch.from_numpy(Qb).cuda(), off))
    sl = slice(int(off[1]), int(off[2]))
    assert check_answers(om, Q, ans, out["prim"][sl], out["closest"][sl], out["dist"][sl]) == []


def test_many_small_meshes():
    """1,500 small meshes (tetrahedra, cubes, displaced icospheres, each at
    its own place) with 0 to 60 queries each in one batch: answers against
    the oracle on a sample of meshes, the batched ordering against its
    definition, and the status bits as plain launches give them."""
    import torch

    import paper_2308_16084_amd as P
    from synth import queries as SQ
    from tests._helpers import CUBE_F, CUBE_V, TETRA_F, TETRA_V, random_tiny_mesh
    rng = np.random.default_rng(12)
    tiny = random_tiny_mesh(rng, "sphere")
    shapes = [(TETRA_V, TETRA_F), (CUBE_V, CUBE_F), tiny]
    meshes, works = [], []
    for k in range(1500):
        V0, F = shapes[k % 3]
        V = (V0.astype(np.float64) * rng.uniform(0.5, 2.0) + rng.uniform(-50, 50, 3)).astype(np.float32)
        lo, hi = SQ.aabb(V)
        dom = SQ.scaled_box(lo, hi, 2.0)
        nq = int(rng.integers(0, 61))
        Q = rng.uniform(dom[0], dom[1], size=(nq, 3)).astype(np.float32)
        works.append((V, F, Q, dom))
    print("case: precomputing 1,500 meshes", flush=True)
    meshes = P.precompute_many([(V, F, dom) for V, F, Q, dom in works], None)
    b = P.Batch(meshes, 0)
    Qb = np.concatenate([x[2] for x in works]).astype(np.float32)
    off = np.concatenate([[0], np.cumsum([len(x[2]) for x in works])]).astype(np.int64)
    qd = torch.from_numpy(Qb).cuda()
    out = _np(b.query(qd, off))
    keys, perm = b.order_queries(qd, off)
    torch.cuda.synchronize()
    keys, perm = keys.cpu().numpy().view(np.uint32), perm.cpu().numpy()
    for k, (V, F, Q, dom) in enumerate(works):
        sl = slice(int(off[k]), int(off[k + 1]))
        rk = OM.morton_keys(Q, dom[0], dom[1]) >> 6
        rp = np.argsort(rk, kind="stable")
        assert np.array_equal(keys[sl], rk[rp]) and np.array_equal(perm[sl], rp + off[k]), k
    for k in range(0, 1500, 50):
        V, F, Q, dom = works[k]
        if len(Q) == 0:
            continue
        sl = slice(int(off[k]), int(off[k + 1]))
        om = oracle.OracleMesh(V, F)
        assert check_answers(om, Q, om.query(Q), out["prim"][sl], out["closest"][sl], out["dist"][sl]) == [], k
        meshes[k].upload(0)
        o = _np(meshes[k].query(qd[sl].contiguous()))
        assert np.array_equal(o["status"], out["status"][sl]), k
