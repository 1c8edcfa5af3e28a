"""The allocation-free query (p2m_query_noalloc) through the C interface:
on two calls in a row, the second with fewer queries (the fixed scratch then
holds the first call's contents), its answers equal those of p2m_query bit
for bit; beyond its limit it refuses with P2M_ERR_ARG."""
from __future__ import annotations

import numpy as np
import pytest

from synth import configs as C
from synth import queries as SQ

pytestmark = pytest.mark.gpu


def _np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def test_noalloc_equals_query_two_calls():
    import torch

    import paper_2308_16084_amd as P
    print("case: no-alloc query, level-6 sphere", flush=True)
    V, F = C.sphere_mesh(6, "fbm", 71)
    lo, hi = SQ.aabb(V)
    m = P.Mesh(V, F)
    m.precompute(domain=SQ.scaled_box(lo, hi, 1.5))
    m.upload(0)
    rng = np.random.default_rng(72)
    for n, extras in ((600_000, True), (90_001, False)):
        Q = SQ.mixed(V, F, n, 1.5, 0.01, rng)
        q = torch.from_numpy(Q).cuda()
        ref = _np(m.query(q, for_backward=extras))
        out = {k: torch.full_like(v, -7) for k, v in m.query(q, for_backward=extras).items()}
        torch.cuda.synchronize()
        got = _np(m.query(q, for_backward=extras, out=out, noalloc=True))
        torch.cuda.synchronize()
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (n, k)
        print(f"case: {n} queries (bary/pvid: {extras}) equal to p2m_query", flush=True)
    with pytest.raises(P.P2MError) as e:
        m.query(torch.zeros(((1 << 20) + 1, 3), dtype=torch.float32, device="cuda"), noalloc=True)
    assert e.value.status == -1
    with pytest.raises(P.P2MError) as e:
        m.query(torch.zeros((16, 3), dtype=torch.float32, device="cuda"), noalloc=True, profile=True)
    assert e.value.status == -1
