"""GPU parity at the library's default query domain (D = the AABB scaled
10x, the paper's query box in Sec. 5) and at the gate boundaries: the
device answers stay within a quarter of the tolerance of the FP64 oracle for
points inside the list scan's gate margin, where a primitive passes its gate
with its foot just off it, and for the near/far sweep's boxes (Sec. 5.3)."""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from synth import configs as C
from synth import queries as SQ
from tests._accept import check_answers
from tests._helpers import gate_boundary_points, margin_points

pytestmark = pytest.mark.gpu

CACHE = os.environ.get("P2M_CACHE_DIR") or None
SWEEP_BOXES = (1.0, 1.5, 2.0, 3.0, 5.0, 10.0)


def _run(m, Q, **kw):
    import torch
    q = torch.from_numpy(np.ascontiguousarray(Q, dtype=np.float32)).cuda()
    out = m.query(q, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _check(om, Q, out, what):
    ans = om.query(Q)
    fails = check_answers(om, Q, ans, out["prim"], out["closest"], out["dist"])
    assert fails == [], (what, fails)
    err = np.abs(out["dist"].astype(np.float64) - ans["dist"]) / (1e-5 * om.diag)
    print(f"{what}: {len(Q)} rows, worst |d - d*| = {err.max():.3f} tol", flush=True)
    assert err.max() <= 0.25, (what, err.max())
    return err


@pytest.fixture(scope="module")
def c2_default_domain():
    import paper_2308_16084_amd as P
    print("case: c2 mesh, default 10x domain, device inspection", flush=True)
    w = C.c2(n_queries=16)
    m, _ = P.Mesh.cached(w.V, w.F, None, CACHE, table_mode=P.TABLE_FLOODING_DEVICE)
    m.upload(0)
    return w, m, oracle.OracleMesh(w.V, w.F)


def test_c2_default_domain_margin_and_sweep(c2_default_domain):
    """C2 mesh precomputed for D = 10x AABB: 3,000 points inside the gate
    margin of edges, face sides and vertices, 1,000 near-surface points and
    6,000 uniform points of the near/far sweep's boxes (1x .. 10x AABB), 10^4
    rows against the oracle, in one sorted launch; worst |d - d*| <= tol/4."""
    w, m, om = c2_default_domain
    lo, hi = SQ.aabb(w.V)
    dlo, dhi = SQ.scaled_box(lo, hi, 10.0)
    mu = 2.0 ** -20 * float(np.linalg.norm(dhi - dlo))
    rng = np.random.default_rng(101)
    parts = [margin_points(w.V, w.F, om.E, om.diag, mu, rng),
             SQ.near_surface(w.V, w.F, 1000, 0.01 * om.diag, rng)]
    parts += [SQ.uniform_in_box(1000, *SQ.scaled_box(lo, hi, s), rng) for s in SWEEP_BOXES]
    Q = np.concatenate(parts)
    print("case: c2 10x domain query", flush=True)
    out = _run(m, Q)
    assert np.all(out["status"] == 0)
    _check(om, Q, out, "c2 10x domain")
    # unsorted, and the tree traversals, give the same answers
    for kw in ({"sort": False}, {"traversal": 2}):
        o2 = _run(m, Q, **kw)
        assert np.mean(o2["prim"] == out["prim"]) > 0.999, kw
        assert np.max(np.abs(o2["dist"] - out["dist"])) <= 0.25e-5 * om.diag, kw


@pytest.mark.parametrize("name,scale", [("c1", 1.5), ("needles", 1.5), ("c1", 10.0), ("needles", 10.0)])
def test_gate_boundaries_on_device(name, scale):
    """Device twin of the host gate-boundary checks: points on edges, at
    vertices, on faces, off the surface by 1e-7 .. 0.3 diag, the domain's
    corners, and points inside the gate margin, on C1 and on a heightfield
    with needle rows, at D = 1.5x and 10x AABB."""
    import paper_2308_16084_amd as P
    from synth import mesh as M
    rng = np.random.default_rng(9)
    if name == "c1":
        w = C.c1()
        V, F = w.V, w.F
    else:
        V, F = M.heightfield(24, 77)
        V, F = V.astype(np.float32), F.astype(np.int32)
    lo, hi = SQ.aabb(V)
    dlo, dhi = SQ.scaled_box(lo, hi, scale)
    print(f"case: gate boundaries {name} {scale}x", flush=True)
    m = P.Mesh(V, F)
    m.precompute(domain=(dlo, dhi))
    m.upload(0)
    om = oracle.OracleMesh(V, F)
    mu = 2.0 ** -20 * float(np.linalg.norm(dhi - dlo))
    Q = np.concatenate([gate_boundary_points(V, F, om.E, dlo, dhi, rng),
                        margin_points(V, F, om.E, om.diag, mu, rng)])
    out = _run(m, Q)
    assert np.all(out["status"] == 0)
    _check(om, Q, out, f"{name} {scale}x")
