"""Full-size workloads on the GPU: C3 (needle heightfield, 10^7 queries) and
the batched C4 plan (all 256 meshes, as benchmarked), sampled against the
FP64 oracle; C5 (10^6 near-surface queries on the C2 mesh) forward and
backward against the oracle's closest points and gradients."""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from oracle import morton as OM
from oracle import grad as OG
from synth import configs as C
from tests._accept import check_answers

pytestmark = pytest.mark.gpu

CACHE = os.environ.get("P2M_CACHE_DIR") or None


def _np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.fixture(scope="module")
def c3_mesh():
    import paper_2308_16084_amd as P
    print("case: c3 build", flush=True)
    w = C.c3()
    m, _ = P.Mesh.cached(w.V, w.F, (w.domain_lo, w.domain_hi), CACHE, table_mode=P.TABLE_FLOODING_DEVICE)
    m.upload(0)
    return w, m


def test_c3_full_size_sampled(c3_mesh):
    """Heightfield 1024 x 1024 with compressed rows (needles; table built with
    the inspection on the device), 10^7 queries in one sorted launch; 10^4
    seeded rows against the oracle."""
    import torch
    w, m = c3_mesh
    q = torch.from_numpy(w.Q).cuda()
    out = _np(m.query(q))
    torch.cuda.synchronize()
    assert np.all(np.isfinite(out["dist"])) and np.all(out["status"] == 0)
    print("case: c3 oracle sample", flush=True)
    rng = np.random.default_rng(33)
    idx = np.sort(rng.choice(len(w.Q), size=10_000, replace=False))
    om = oracle.OracleMesh(w.V, w.F)
    ans = om.query(w.Q[idx])
    assert check_answers(om, w.Q[idx], ans, out["prim"][idx], out["closest"][idx], out["dist"][idx], idx=idx) == []
    err = np.abs(out["dist"][idx].astype(np.float64) - ans["dist"]) / (1e-5 * om.diag)
    print(f"c3: worst |d - d*| = {err.max():.3f} tol", flush=True)


def test_c3_traversals_and_ordering_identical(c3_mesh):
    """Which traversal finds the nearest vertex, and whether the batch is
    ordered, never changes an answer: 10^6 of the C3 queries and 10^6 seeded
    points in a box twice D's size (seven in eight of them outside D, where every
    traversal ends in the wavefront tree walk), bit for bit."""
    import torch
    w, m = c3_mesh
    ext = w.domain_hi - w.domain_lo
    Qo = np.random.default_rng(9).uniform(w.domain_lo - 0.5 * ext, w.domain_hi + 0.5 * ext, size=(1_000_000, 3))
    for name, Q in (("c3 queries", w.Q[:1_000_000]), ("c3 wide box", Qo)):
        q = torch.from_numpy(np.ascontiguousarray(Q, dtype=np.float32)).cuda()
        ref = _np(m.query(q))
        for kw in ({"traversal": 1}, {"traversal": 2}, {"sort": False}, {"sort": True}):
            print("case:", name, kw, flush=True)
            out = _np(m.query(q, **kw))
            for k in ref:
                assert np.array_equal(out[k], ref[k]), (name, kw, k)


def test_c3_backward_large_mesh(c3_mesh):
    """Backward on the 1,048,576-vertex heightfield (10^6 of its queries,
    loss = sum d^2): at this size every 1,024-vertex bucket of the vertex
    gradient is summed by one block that updates grad_V four floats at a
    time; the result equals a float64 accumulation of the same per-query
    contributions -(dL/dd) w_k (q - c)/d built on the host from the
    forward's outputs."""
    import torch
    w, m = c3_mesh
    assert m.nv > 1023 * 1024
    q = torch.from_numpy(w.Q[:1_000_000]).cuda()
    fwd = m.query(q, for_backward=True, status=False)
    g = 2.0 * fwd["dist"]
    gV = torch.zeros((m.nv, 3), dtype=torch.float32, device="cuda")
    gq, gV = m.query_backward(q, fwd, g, grad_q=True, grad_V=gV)
    torch.cuda.synchronize()
    Q = w.Q[:1_000_000].astype(np.float64)
    c = fwd["closest"].cpu().numpy().astype(np.float64)
    d = fwd["dist"].cpu().numpy().astype(np.float64)
    bary = fwd["bary"].cpu().numpy().astype(np.float64)
    pvid = fwd["pvid"].cpu().numpy()
    u = np.where(d[:, None] > 0, (Q - c) / np.maximum(d, 1e-30)[:, None], 0.0)
    ref = np.zeros((m.nv, 3))
    for k in range(3):
        ok = (pvid[:, k] >= 0) & (bary[:, k] != 0)
        np.add.at(ref, pvid[ok, k], -(2.0 * d[ok] * bary[ok, k])[:, None] * u[ok])
    got = gV.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"c3 backward: |gV - ref| / |ref| = {rel:.2e}", flush=True)
    assert rel <= 1e-5
    assert np.allclose(gq.cpu().numpy(), 2.0 * d[:, None] * u, atol=1e-5)


def test_c4_batched_sampled():
    """All 256 meshes of the seeded C4 plan (tables built with the inspection
    on the device) in one graph launch at the autotuned launch shape; 64
    sampled queries per mesh against the oracle; the persistent schedule at
    that shape gives the same answers."""
    from concurrent.futures import ThreadPoolExecutor

    import torch

    import paper_2308_16084_amd as P
    print("case: c4 build", flush=True)
    with ThreadPoolExecutor(max_workers=16) as ex:
        works = list(ex.map(C.c4_mesh, C.c4_plan()))
    meshes = P.precompute_many([(x.V, x.F, (x.domain_lo, x.domain_hi)) for x in works], CACHE,
                               table_mode=P.TABLE_FLOODING_DEVICE)
    b = P.Batch(meshes, 0)
    Q = np.concatenate([x.Q for x in works])
    off = np.concatenate([[0], np.cumsum([len(x.Q) for x in works])]).astype(np.int64)
    qd = torch.from_numpy(Q).cuda()
    # the launch shape the benchmark times: the autotuner's pick
    shape = b.autotune(qd, off)
    print(f"case: c4 at the autotuned shape {shape}", flush=True)
    out = _np(b.query(qd, off))
    torch.cuda.synchronize()
    assert np.all(out["status"] == 0)  # every query lies in its mesh's domain
    rng = np.random.default_rng(44)
    for k, x in enumerate(works):
        idx = np.sort(rng.choice(len(x.Q), size=min(64, len(x.Q)), replace=False))
        rows = off[k] + idx
        om = oracle.OracleMesh(x.V, x.F)
        fails = check_answers(om, x.Q[idx], om.query(x.Q[idx]), out["prim"][rows], out["closest"][rows],
                              out["dist"][rows], idx=rows)
        assert fails == [], (k, x.name, fails)
    # the batch's ordering (37.9 M queries, segments of up to a few hundred
    # sort tiles) against its definition, bit for bit
    print("case: c4 ordering", flush=True)
    keys, perm = b.order_queries(qd, off)
    torch.cuda.synchronize()
    keys, perm = keys.cpu().numpy().view(np.uint32), perm.cpu().numpy()
    for k, x in enumerate(works):
        rk = OM.morton_keys(x.Q, x.domain_lo, x.domain_hi) >> 6
        rp = np.argsort(rk, kind="stable")
        assert np.array_equal(keys[off[k]:off[k + 1]], rk[rp]), k
        assert np.array_equal(perm[off[k]:off[k + 1]], rp + off[k]), k
    # the persistent schedule at the same shape: the same answers, bit for bit
    print("case: c4 persistent schedule", flush=True)
    try:
        b.set_schedule(True)
        got = _np(b.query(qd, off))
        torch.cuda.synchronize()
        for key in out:
            assert np.array_equal(got[key], out[key]), key
    finally:
        b.set_schedule(False)


def _star_fd(om64, q, k, axis, h, faces_of):
    """d(q)^2 with vertex k moved by +h and -h along axis, from an FP64 brute
    force over the faces incident to k (their edges and vertices included):
    the primitives a move of v_k changes.  Valid where every other
    primitive is at least 10h farther than the closest (a runner-up gap of
    at least 10h), so the minimum stays within k's star."""
    from oracle import OracleMesh
    Fk = om64.F[faces_of[k]]
    vs, local = np.unique(Fk, return_inverse=True)
    out = []
    for sgn in (1.0, -1.0):
        Vs = om64.V[vs].copy()
        Vs[np.searchsorted(vs, k), axis] += sgn * h
        star = OracleMesh(Vs, local.reshape(-1, 3).astype(np.int32), promote=False)
        out.append(star.query(np.asarray(q, np.float64)[None])["dist"][0])
    return (out[0] ** 2 - out[1] ** 2) / (2 * h)


def test_c5_forward_backward_vs_oracle():
    """C5 backward check: the C2 mesh, 10^6 near-surface queries; on 1,000
    sampled queries (the forward accepted by the oracle), the queries whose
    oracle runner-up gap is at least 10h (h = 1e-6; the others sit at a
    non-smooth point and are counted) are checked for the subset loss
    sum d^2:
      * grad_q per query against the oracle gradient 2(q - c*) and against
        FP64 central finite differences of the brute-force distance;
      * each query's vertex contributions -2 w_k (q - c) against the
        oracle's weights and against FP64 central differences in every
        vertex of the closest primitive (re-evaluated over that vertex's
        star of faces);
      * the vertex gradient of the subset loss against the oracle gradient,
        |dgV| / |gV| <= 1e-4.
    Per-query tolerance: 1e-5 diag + 1e-4 |g|."""
    import torch

    import paper_2308_16084_amd as P
    print("case: c5 build", flush=True)
    w = C.c5()
    m, _ = P.Mesh.cached(w.V, w.F, (w.domain_lo, w.domain_hi), CACHE)
    m.upload(0)
    qd = torch.from_numpy(w.Q).cuda()
    fwd = {k: v.cpu().numpy() for k, v in m.query(qd, for_backward=True).items()}
    rng = np.random.default_rng(55)
    S = np.sort(rng.choice(len(w.Q), size=1000, replace=False))
    om = oracle.OracleMesh(w.V, w.F)
    print("case: c5 oracle sample", flush=True)
    ans = om.query(w.Q[S])
    assert check_answers(om, w.Q[S], ans, fwd["prim"][S], fwd["closest"][S], fwd["dist"][S], idx=S) == []
    h = 1e-6
    keep = (ans["runner_up"] - ans["dist"]) >= 10 * h
    Sk = S[keep]
    ansk = {k: v[keep] for k, v in ans.items()}
    print(f"c5 backward: {keep.sum()} of {len(S)} sampled queries checked, {len(S) - keep.sum()} excluded "
          f"(runner-up gap < 10h)", flush=True)
    assert keep.sum() >= 300
    diag = om.diag
    # GPU gradients of the subset loss (upstream gradient masked to Sk)
    q = qd.clone().requires_grad_(True)
    Vt = torch.from_numpy(w.V).cuda().requires_grad_(True)
    d, _, _ = P.p2m_distance(q, Vt, m)
    mask = torch.zeros(len(w.Q), device="cuda")
    mask[torch.from_numpy(Sk).cuda()] = 1.0
    (d * d * mask).sum().backward()
    torch.cuda.synchronize()
    gq = q.grad.cpu().numpy().astype(np.float64)[Sk]
    gV = Vt.grad.cpu().numpy().astype(np.float64)
    ogq, ogV = OG.gradients(om, w.Q[Sk], ansk, 2.0 * ansk["dist"])
    gmag = np.linalg.norm(ogq, axis=1)
    qtol = 1e-5 * diag + 1e-4 * gmag
    assert np.all(np.linalg.norm(gq - ogq, axis=1) <= qtol)
    # each query's vertex contributions: GPU weights vs the oracle's
    Qd = w.Q.astype(np.float64)
    contrib_gpu, contrib_orc = [], []
    for j, i in enumerate(Sk):
        u2 = 2.0 * (Qd[i] - fwd["closest"][i].astype(np.float64))
        cg = {int(v): -float(wt) * u2 for v, wt in zip(fwd["pvid"][i], fwd["bary"][i]) if v >= 0 and wt != 0}
        ids, wts = OG.weights(om, int(ansk["type"][j]), int(ansk["id"][j]), ansk["closest"][j])
        co = {int(v): -float(wt) * 2.0 * (Qd[i] - ansk["closest"][j]) for v, wt in zip(ids, wts)}
        for v in set(cg) | set(co):
            dv = cg.get(v, np.zeros(3)) - co.get(v, np.zeros(3))
            assert np.linalg.norm(dv) <= qtol[j], (i, v, cg, co)
        contrib_gpu.append(cg)
        contrib_orc.append(co)
    # the subset's vertex gradient
    rel = np.linalg.norm(gV - ogV) / np.linalg.norm(ogV)
    print(f"c5 backward: |dgV|/|gV| = {rel:.2e}", flush=True)
    assert rel <= 1e-4, rel
    # FP64 central differences in q (brute force over the whole mesh)
    print("case: c5 finite differences in q", flush=True)
    om64 = oracle.OracleMesh(w.V.astype(np.float64), w.F, promote=False)
    E3 = np.eye(3)
    Qp = np.concatenate([Qd[Sk] + h * E3[a] for a in range(3)] + [Qd[Sk] - h * E3[a] for a in range(3)])
    dd = om64.query(Qp)["dist"].reshape(6, len(Sk))
    fdq = np.stack([(dd[a] ** 2 - dd[3 + a] ** 2) / (2 * h) for a in range(3)], axis=1)
    errq = np.linalg.norm(fdq - gq, axis=1)
    print(f"c5 backward: worst |FD(q) - grad_q| / tol = {np.max(errq / qtol):.3f}", flush=True)
    assert np.all(errq <= qtol)
    # FP64 central differences in every vertex of each query's closest primitive
    print("case: c5 finite differences in the vertices", flush=True)
    faces_of = {}
    touched = sorted({v for co in contrib_orc for v in co})
    tset = set(touched)
    for f, tri in enumerate(om64.F.tolist()):
        for v in tri:
            if v in tset:
                faces_of.setdefault(v, []).append(f)
    # vertices the GPU touched outside the oracle's primitives: their central
    # difference is 0 (the runner-up gap keeps their stars farther than d)
    touched = sorted(tset | {v for cg in contrib_gpu for v in cg})
    fd_sum = {v: np.zeros(3) for v in touched}
    worst = 0.0
    for j, i in enumerate(Sk):
        for v in contrib_orc[j]:
            fd = np.array([_star_fd(om64, Qd[i], v, a, h, faces_of) for a in range(3)])
            fd_sum[v] += fd
            err = np.linalg.norm(fd - contrib_gpu[j].get(v, np.zeros(3)))
            worst = max(worst, err / qtol[j])
            assert err <= qtol[j], (i, v, fd, contrib_gpu[j].get(v))
    print(f"c5 backward: worst |FD(v) - contribution| / tol = {worst:.3f} over {len(touched)} vertices", flush=True)
    T = np.array(touched)
    fdV = np.stack([fd_sum[v] for v in touched])
    relfd = np.linalg.norm(gV[T] - fdV) / np.linalg.norm(fdV)
    print(f"c5 backward: |gV - FD| / |FD| over the touched vertices = {relfd:.2e}", flush=True)
    assert relfd <= 1e-4, relfd
    # no other vertex received a gradient
    others = np.ones(len(gV), bool)
    others[T] = False
    assert np.all(gV[others] == 0.0)


def test_c5_vertex_gradient_reduction_dense():
    """Full C5 loss: the vertex gradient (bucketed reduction on a mesh this
    size) equals a float64 accumulation of the same per-query contributions
    -(dL/dd) w_k (q - c)/d built on the host from the forward's outputs."""
    import torch

    import paper_2308_16084_amd as P
    print("case: c5 dense vertex gradient", flush=True)
    w = C.c5()
    m, _ = P.Mesh.cached(w.V, w.F, (w.domain_lo, w.domain_hi), CACHE)
    m.upload(0)
    q = torch.from_numpy(w.Q).cuda()
    fwd = m.query(q, for_backward=True, status=False)
    g = 2.0 * fwd["dist"]
    gV = torch.zeros((m.nv, 3), dtype=torch.float32, device="cuda")
    gq, gV = m.query_backward(q, fwd, g, grad_q=True, grad_V=gV)
    torch.cuda.synchronize()
    Q = w.Q.astype(np.float64)
    c = fwd["closest"].cpu().numpy().astype(np.float64)
    d = fwd["dist"].cpu().numpy().astype(np.float64)
    bary = fwd["bary"].cpu().numpy().astype(np.float64)
    pvid = fwd["pvid"].cpu().numpy()
    u = np.where(d[:, None] > 0, (Q - c) / np.maximum(d, 1e-30)[:, None], 0.0)
    ref = np.zeros((m.nv, 3))
    for k in range(3):
        ok = (pvid[:, k] >= 0) & (bary[:, k] != 0)
        np.add.at(ref, pvid[ok, k], -(2.0 * d[ok] * bary[ok, k])[:, None] * u[ok])
    got = gV.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)
    assert np.allclose(gq.cpu().numpy(), 2.0 * d[:, None] * u, atol=1e-5)


def test_c6_mixed_primitives_sampled():
    """C6 (Sec. 5.5 mixed set: triangles + a crossing wireframe of free
    segments), 10^6 queries in one ordered launch: 1,500 sampled rows
    against the oracle over the same primitive set; the other traversals
    give the same answers; served as one mesh of a batch with a triangle
    mesh, it gives the plain launch's answers."""
    import torch

    import paper_2308_16084_amd as P
    print("case: c6 build", flush=True)
    w = C.c6()
    m, _ = P.Mesh.cached(w.V, w.F, (w.domain_lo, w.domain_hi), CACHE, segments=w.S)
    m.upload(0)
    q = torch.from_numpy(w.Q).cuda()
    out = {k: v.cpu().numpy() for k, v in m.query(q).items()}
    rng = np.random.default_rng(66)
    S = np.sort(rng.choice(len(w.Q), size=1500, replace=False))
    om = oracle.OracleMesh(w.V, w.F, segments=w.S)
    ans = om.query(w.Q[S])
    assert check_answers(om, w.Q[S], ans, out["prim"][S], out["closest"][S], out["dist"][S], idx=S) == []
    assert np.all(out["status"] == 0)
    for t in (1, 2):
        o = {k: v.cpu().numpy() for k, v in m.query(q[:200_000], traversal=t).items()}
        assert np.mean(o["prim"] == out["prim"][:200_000]) > 0.9999, t
    w1 = C.c1()
    m1 = P.Mesh(w1.V, w1.F)
    m1.precompute(domain=(w1.domain_lo, w1.domain_hi))
    b = P.Batch([m1, m], 0)
    qb = torch.cat([torch.from_numpy(w1.Q).cuda(), q[:300_000]]).contiguous()
    off = np.array([0, len(w1.Q), len(w1.Q) + 300_000], np.int64)
    ob = {k: v.cpu().numpy() for k, v in b.query(qb, off).items()}
    sl = slice(len(w1.Q), None)
    assert np.mean(ob["prim"][sl] == out["prim"][:300_000]) > 0.9999
    assert np.max(np.abs(ob["dist"][sl] - out["dist"][:300_000])) <= 1e-5 * om.diag
