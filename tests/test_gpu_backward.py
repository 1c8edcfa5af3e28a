"""GPU backward: d dist / d q and d dist / d V from the hand-written kernel
against the oracle's gradient (FP64, from the brute-force closest point) and
against FP64 central finite differences of the brute-force distance."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import grad as OG
from synth import configs as C
from synth import queries as SQ

pytestmark = pytest.mark.gpu


def test_backward_small_mesh_fd_and_oracle():
    import torch
    import paper_2308_16084_amd as P
    V, F = C.sphere_mesh(3, "fbm", 17)
    lo, hi = SQ.aabb(V)
    dom = SQ.scaled_box(lo, hi, 1.5)
    m = P.Mesh(V, F)
    m.precompute(domain=dom)
    m.upload(0)
    rng = np.random.default_rng(3)
    diag = float(np.linalg.norm(hi - lo))
    Q = SQ.near_surface(V, F, 2000, 0.02 * diag, rng)
    q = torch.from_numpy(Q).cuda().requires_grad_(True)
    Vt = torch.from_numpy(V).cuda().requires_grad_(True)
    d, prim, c = P.p2m_distance(q, Vt, m)
    loss = (d * d).sum()
    loss.backward()
    torch.cuda.synchronize()
    gq = q.grad.cpu().numpy().astype(np.float64)
    gV = Vt.grad.cpu().numpy().astype(np.float64)
    om = oracle.OracleMesh(V, F)
    ans = om.query(Q)
    ogq, ogV = OG.gradients(om, Q, ans, 2.0 * ans["dist"])
    tol = 1e-5 * diag
    # closed form dL/dq = 2 (q - c)
    assert np.max(np.abs(gq - ogq)) <= 4 * tol + 1e-4 * np.abs(ogq).max()
    rel = np.linalg.norm(gV - ogV) / np.linalg.norm(ogV)
    assert rel <= 1e-3, rel
    # finite differences on queries away from non-smooth points
    h = 1e-6
    om64 = oracle.OracleMesh(V.astype(np.float64), F, promote=False)
    keep = np.nonzero((ans["runner_up"] - ans["dist"]) > 100 * h)[0][:200]
    for i in keep:
        x = Q[i].astype(np.float64)
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            dp = om64.query(x + e)["dist"][0]
            dm = om64.query(x - e)["dist"][0]
            fd = (dp * dp - dm * dm) / (2 * h)
            assert abs(fd - gq[i, a]) <= 1e-4 + 1e-3 * abs(fd), (i, a, fd, gq[i, a])


def test_backward_translation_invariance():
    import torch
    import paper_2308_16084_amd as P
    V, F = C.sphere_mesh(3, "uniform", 5)
    lo, hi = SQ.aabb(V)
    m = P.Mesh(V, F)
    m.precompute(domain=SQ.scaled_box(lo, hi, 1.5))
    m.upload(0)
    rng = np.random.default_rng(8)
    Q = SQ.uniform_in_box(3000, *SQ.scaled_box(lo, hi, 1.4), rng)
    q = torch.from_numpy(Q).cuda().requires_grad_(True)
    Vt = torch.from_numpy(V).cuda().requires_grad_(True)
    d, _, _ = P.p2m_distance(q, Vt, m)
    d.sum().backward()
    # moving q and every vertex together leaves each distance unchanged
    s = q.grad.sum(0) + Vt.grad.sum(0)
    assert torch.all(torch.abs(s) <= 1e-3 * q.grad.abs().sum(0) + 1e-4)


def test_backward_odd_meshes():
    """The backward on triangle soups, a high-valence fan, slivers and a
    non-manifold set (tests/_helpers.odd_meshes): dL/dq and dL/dV of
    L = sum d^2 over queries whose runner-up primitive is clearly farther
    (ties excluded, where d is not differentiable) against the oracle's
    gradients."""
    import torch

    import paper_2308_16084_amd as P
    from tests._helpers import odd_meshes
    rng = np.random.default_rng(8)
    for name, V, F in odd_meshes(rng):
        lo, hi = SQ.aabb(V)
        dom = SQ.scaled_box(lo, hi, 1.5)
        m = P.Mesh(V, F)
        m.precompute(domain=dom)
        m.upload(0)
        diag = float(np.linalg.norm(hi - lo))
        tri = V.astype(np.float64)[F]
        b = rng.dirichlet([1, 1, 1], 3000)
        Q = ((tri[rng.integers(0, len(F), 3000)] * b[:, :, None]).sum(1)
             + 0.02 * diag * rng.standard_normal((3000, 3))).astype(np.float32)
        om = oracle.OracleMesh(V, F)
        ans = om.query(Q)
        tol = 1e-5 * diag
        keep = (ans["runner_up"] - ans["dist"]) > 10 * tol
        print(f"case: backward on {name}, {int(keep.sum())} of {len(Q)} queries away from ties", flush=True)
        q = torch.from_numpy(Q).cuda().requires_grad_(True)
        Vt = torch.from_numpy(V).cuda().requires_grad_(True)
        d, prim, c = P.p2m_distance(q, Vt, m)
        w = torch.from_numpy(keep.astype(np.float32)).cuda()
        (w * d * d).sum().backward()
        torch.cuda.synchronize()
        gq = q.grad.cpu().numpy().astype(np.float64)
        gV = Vt.grad.cpu().numpy().astype(np.float64)
        ogq, ogV = OG.gradients(om, Q, ans, 2.0 * ans["dist"] * keep)
        assert np.max(np.abs(gq[keep] - ogq[keep])) <= 4 * tol + 1e-4 * np.abs(ogq).max(), name
        assert np.all(gq[~keep] == 0), name
        rel = np.linalg.norm(gV - ogV) / max(np.linalg.norm(ogV), 1e-30)
        assert rel <= 1e-3, (name, rel)
