"""Pins for the oracle's query-ordering definition and its gradient."""
from __future__ import annotations

import numpy as np

import oracle
from oracle import grad as OG
from oracle import morton as OM
from tests._helpers import random_tiny_mesh
from synth import queries as SQ


def _interleave_py(cx, cy, cz):
    key = 0
    for b in range(10):
        key |= ((cx >> b) & 1) << (3 * b + 2)
        key |= ((cy >> b) & 1) << (3 * b + 1)
        key |= ((cz >> b) & 1) << (3 * b)
    return key


def test_morton_hand_values():
    lo, hi = np.zeros(3), np.full(3, 1024.0)
    Q = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [3, 3, 3], [1023.5, 1023.5, 1023.5],
                  [-5, 2000, 0.5], [np.nan, 0, 0]], np.float32)
    k = OM.morton_keys(Q, lo, hi)
    assert k.tolist() == [4, 2, 1, 63, (1 << 30) - 1, sum(1 << (3 * b + 1) for b in range(10)), 0]


def test_morton_order_brute_force():
    rng = np.random.default_rng(0)
    lo, hi = np.array([-1.3, -0.2, 0.7]), np.array([2.1, 0.9, 1.9])
    Q = rng.uniform(lo - 0.1, hi + 0.1, size=(3000, 3)).astype(np.float32)
    Q[100:200] = Q[0]  # many equal keys: order must be stable
    keys, perm = OM.order(Q, lo, hi)
    # brute force: python ints from the same float32 quantisation, sorted on (key, index)
    c = OM.quantise(Q, lo, hi)
    ref = sorted(range(len(Q)), key=lambda i: (_interleave_py(*map(int, c[i])), i))
    assert perm.tolist() == ref
    assert np.all(np.diff(keys.astype(np.int64)) >= 0)


def test_grad_matches_central_differences():
    """FP64 central differences of the brute-force distance, on queries whose
    runner-up is well separated (the distance is smooth there)."""
    rng = np.random.default_rng(2)
    V, F = random_tiny_mesh(rng, "sphere")
    V = V.astype(np.float64)
    om = oracle.OracleMesh(V, F, promote=False)
    lo, hi = SQ.aabb(V)
    Q = rng.uniform(*SQ.scaled_box(lo, hi, 1.4), size=(60, 3))
    ans = om.query(Q)
    g = rng.uniform(0.5, 2.0, size=Q.shape[0])
    gq, gV = OG.gradients(om, Q, ans, g)
    h = 1e-6
    keep = (ans["runner_up"] - ans["dist"]) > 100 * h
    assert keep.sum() > 30
    for i in np.nonzero(keep)[0]:
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            dp = om.query(Q[i] + e)["dist"][0]
            dm = om.query(Q[i] - e)["dist"][0]
            assert abs(g[i] * (dp - dm) / (2 * h) - gq[i, a]) <= 1e-6
    # vertex gradients of the loss sum_i g_i d_i over the kept queries
    sel = np.nonzero(keep)[0]
    gq_s, gV_s = OG.gradients(om, Q[sel], {k: v[sel] for k, v in ans.items()}, g[sel])
    touched = np.unique(np.nonzero(np.abs(gV_s).sum(1))[0])
    for k in touched[:25]:
        for a in range(3):
            Vp = V.copy(); Vp[k, a] += h
            Vm = V.copy(); Vm[k, a] -= h
            Lp = np.dot(g[sel], oracle.OracleMesh(Vp, F, promote=False).query(Q[sel])["dist"])
            Lm = np.dot(g[sel], oracle.OracleMesh(Vm, F, promote=False).query(Q[sel])["dist"])
            assert abs((Lp - Lm) / (2 * h) - gV_s[k, a]) <= 1e-5


def test_grad_translation_invariance():
    """Moving the query and the whole mesh together leaves d unchanged, so the
    per-query vertex gradient sums to -grad_q."""
    rng = np.random.default_rng(4)
    V, F = random_tiny_mesh(rng, "heightfield")
    om = oracle.OracleMesh(V, F)
    lo, hi = SQ.aabb(V)
    Q = SQ.uniform_in_box(40, *SQ.scaled_box(lo, hi, 1.5), rng)
    ans = om.query(Q)
    for i in range(Q.shape[0]):
        gq, gV = OG.gradients(om, Q[i:i + 1], {k: v[i:i + 1] for k, v in ans.items()}, np.ones(1))
        assert np.allclose(gV.sum(0), -gq[0], atol=1e-12)
