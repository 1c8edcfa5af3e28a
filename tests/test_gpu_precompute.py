"""Device inspection (filter + flooding, Sec. 4.4-4.5, Algorithm 1, on the
GPU): the table, its entry boxes and the build counters must be those of the
host build entry for entry, on closed meshes, a heightfield with needles, a
mixed triangle + segment set and the default 10x domain; with the device's
visit capacity cut down, the primitives handed back to the host must still
give the same table; queries on the device-built mesh are checked against
the FP64 oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_2308_16084_amd as P
from synth import configs as C
from synth import mesh as SM
from synth import queries as SQ
from tests._accept import check_answers

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "c1":
        w = C.c1(2000)
        return w.V, w.F, None, (w.domain_lo, w.domain_hi)
    if name == "sphere5_fbm_10x":
        V, F = C.sphere_mesh(5, "fbm", 77)
        return V, F, None, None
    if name == "heightfield48":
        V, F = SM.heightfield(48, 5)
        V = V.astype(np.float32)
        return V, F.astype(np.int32), None, C.heightfield_domain(V)
    if name == "mixed":
        w = C.c6(1000, level=3, wire_level=2)
        return w.V, w.F, w.S, (w.domain_lo, w.domain_hi)
    raise ValueError(name)


def _tables(V, F, S, dom, **kw):
    h = P.Mesh(V, F, segments=S)
    sh = h.precompute(dom, table_mode=P.TABLE_FLOODING)
    d = P.Mesh(V, F, segments=S)
    sd = d.precompute(dom, table_mode=P.TABLE_FLOODING_DEVICE, **kw)
    return h, sh, d, sd


def _same(h, sh, d, sd):
    oh, eh = h.table()
    od, ed = d.table()
    assert np.array_equal(oh, od)
    assert np.array_equal(eh, ed)
    assert np.array_equal(h.table_boxes(), d.table_boxes())
    for k in ("nnz_edges", "nnz_faces", "max_list", "flood_tests", "flood_hits", "quick_rejects", "skipped_clips"):
        assert sh[k] == sd[k], k


@pytest.mark.parametrize("name", ["c1", "sphere5_fbm_10x", "heightfield48", "mixed"])
def test_device_table_equals_host(name):
    print(f"case: device inspection {name}", flush=True)
    V, F, S, dom = _case(name)
    h, sh, d, sd = _tables(V, F, S, dom)
    _same(h, sh, d, sd)
    # a working polytope of more than 64 corners sends its primitive back
    assert sd["device_redo"] <= max(4, 1e-3 * (sh["ne"] + sh["nf"]))


def test_device_handback_to_host():
    """A visit capacity of 40 sends every primitive whose flood grows past 40
    vertices (about half of C1's) back to the host; entries the device wrote
    for them are dropped and the host's replace them."""
    print("case: device inspection hand-back", flush=True)
    V, F, S, dom = _case("c1")
    h, sh, d, sd = _tables(V, F, S, dom, device_visit_cap=40)
    assert 0 < sd["device_redo"] < sh["ne"] + sh["nf"]
    _same(h, sh, d, sd)


def test_device_built_mesh_queries():
    """Queries on the mesh whose table the device built, against the oracle."""
    import torch

    print("case: device-built mesh queries", flush=True)
    w = C.c1(3000)
    m = P.Mesh(w.V, w.F)
    m.precompute((w.domain_lo, w.domain_hi), table_mode=P.TABLE_FLOODING_DEVICE)
    m.upload(0)
    out = {k: v.cpu().numpy() for k, v in m.query(torch.from_numpy(w.Q).cuda()).items()}
    om = oracle.OracleMesh(w.V, w.F)
    ans = om.query(w.Q)
    assert check_answers(om, w.Q, ans, out["prim"], out["closest"], out["dist"]) == []


def test_device_table_equals_host_with_host_built_cells():
    """A level-6 C2-style sphere (40,962 vertices): some Voronoi cells have
    more than 64 corners and are built on the host into the second cell
    allocation; the table must still equal the host build's."""
    print("case: device inspection, host-built cells", flush=True)
    w = C.c2(1000, level=6)
    h, sh, d, sd = _tables(w.V, w.F, None, (w.domain_lo, w.domain_hi))
    print("cells built on the host:", sd["device_cells_back"], flush=True)
    assert sd["device_cells_back"] > 0
    _same(h, sh, d, sd)
