"""Full-size workloads on the GPU: C3 (needle heightfield, 10^7 queries) and
the batched C4 plan (all 256 meshes, as benchmarked), sampled against the
FP64 oracle; C5 (10^6 near-surface queries on the C2 mesh) forward and
backward against the oracle's closest points and gradients."""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from oracle import grad as OG
from synth import configs as C
from tests._accept import check_answers

pytestmark = pytest.mark.gpu

CACHE = os.environ.get("P2M_CACHE_DIR") or None


def _np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def test_c3_full_size_sampled():
    """Heightfield 1024 x 1024 with compressed rows (needles; table built with
    the inspection on the device), 10^7 queries in one sorted launch; 1,200
    sampled rows against the oracle."""
    import torch

    import paper_2308_16084_amd as P
    print("case: c3 build", flush=True)
    w = C.c3()
    m, _ = P.Mesh.cached(w.V, w.F, (w.domain_lo, w.domain_hi), CACHE, table_mode=P.TABLE_FLOODING_DEVICE)
    m.upload(0)
    q = torch.from_numpy(w.Q).cuda()
    out = _np(m.query(q))
    torch.cuda.synchronize()
    assert np.all(np.isfinite(out["dist"])) and np.all(out["status"] == 0)
    print("case: c3 oracle sample", flush=True)
    rng = np.random.default_rng(33)
    idx = np.sort(rng.choice(len(w.Q), size=1200, replace=False))
    om = oracle.OracleMesh(w.V, w.F)
    ans = om.query(w.Q[idx])
    assert check_answers(om, w.Q[idx], ans, out["prim"][idx], out["closest"][idx], out["dist"][idx], idx=idx) == []


def test_c4_batched_sampled():
    """All 256 meshes of the seeded C4 plan (tables built with the inspection
    on the device) in one graph launch; 64 sampled queries per mesh against
    the oracle."""
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
    out = _np(b.query(torch.from_numpy(Q).cuda(), off))
    torch.cuda.synchronize()
    rng = np.random.default_rng(44)
    for k, x in enumerate(works):
        idx = np.sort(rng.choice(len(x.Q), size=min(64, len(x.Q)), replace=False))
        rows = off[k] + idx
        om = oracle.OracleMesh(x.V, x.F)
        fails = check_answers(om, x.Q[idx], om.query(x.Q[idx]), out["prim"][rows], out["closest"][rows],
                              out["dist"][rows], idx=rows)
        assert fails == [], (k, x.name, fails)


def test_c5_forward_backward_vs_oracle():
    """C5: the C2 mesh, 10^6 near-surface queries, loss = sum of d^2.  On 1,000
    sampled queries: forward accepted by the oracle, grad_q = 2(q - c*) and
    the vertex gradient of the sampled subset equal to the oracle gradient."""
    import torch

    import paper_2308_16084_amd as P
    print("case: c5 build", flush=True)
    w = C.c5()
    m, _ = P.Mesh.cached(w.V, w.F, (w.domain_lo, w.domain_hi), CACHE)
    m.upload(0)
    q = torch.from_numpy(w.Q).cuda().requires_grad_(True)
    Vt = torch.from_numpy(w.V).cuda().requires_grad_(True)
    d, prim, c = P.p2m_distance(q, Vt, m)
    (d * d).sum().backward()
    torch.cuda.synchronize()
    rng = np.random.default_rng(55)
    S = np.sort(rng.choice(len(w.Q), size=1000, replace=False))
    om = oracle.OracleMesh(w.V, w.F)
    print("case: c5 oracle sample", flush=True)
    ans = om.query(w.Q[S])
    dn, pn, cn = d.detach().cpu().numpy(), prim.cpu().numpy(), c.detach().cpu().numpy()
    assert check_answers(om, w.Q[S], ans, pn[S], cn[S], dn[S], idx=S) == []
    tol = 1e-5 * om.diag
    gq = q.grad.cpu().numpy().astype(np.float64)[S]
    ogq, _ = OG.gradients(om, w.Q[S], ans, 2.0 * ans["dist"])
    assert np.max(np.abs(gq - ogq)) <= 4 * tol
    # vertex gradient of the subset loss: upstream gradient masked to S
    q2 = torch.from_numpy(w.Q).cuda().requires_grad_(True)
    V2 = torch.from_numpy(w.V).cuda().requires_grad_(True)
    d2, _, _ = P.p2m_distance(q2, V2, m)
    mask = torch.zeros(len(w.Q), device="cuda")
    mask[torch.from_numpy(S).cuda()] = 1.0
    (d2 * d2 * mask).sum().backward()
    gV = V2.grad.cpu().numpy().astype(np.float64)
    _, ogV = OG.gradients(om, w.Q[S], ans, 2.0 * ans["dist"])
    # near-ties (a face vs. its side) may pick either primitive; the gradient
    # is continuous across them, so the whole vertex gradient is compared
    rel = np.linalg.norm(gV - ogV) / np.linalg.norm(ogV)
    assert rel <= 5e-3, rel


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
