"""Benchmark: P2M queries/sec on one MI355X.

Workload (the headline configuration): icosphere level 8 (655,362 vertices,
1,310,720 triangles) displaced by 4-octave value-noise fbm, float32; 10^7
queries, half uniform in the 1.5x AABB and half near the surface.  One step
is one pass of the whole query path over the batch with the inputs resident
in HBM: Morton keys + stable radix sort of the queries, then the query
kernel (nearest vertex by a walk over the Voronoi neighbour graph, the
interception-list scan with its entry boxes and gated point-line /
point-plane tests, the winner resolved exactly: primitive, closest point,
distance), then the write-out of the answers in input order.  The host
precompute is timed separately and never counted.

The roofline of the query kernel counts the method's algorithmic bytes per
query (the query and its answer, the nearest-vertex candidates, the list
range, 4 bytes per scanned entry, the vertices of every tested edge and
face), measured per query by the host model over the same structures, over
the kernel's duration from HIP events on its stream; the HBM traffic, L2 hit
rate and VALU figures come from committed rocprofv3 summaries of the same
kernel source (null when the kernel has changed since).

Also reported on the same GPU: the ordering's bytes and bandwidth; the batch
in input order (no ordering); the small icosphere and the needle heightfield
workloads; Table 1's list statistics (Avg^1, Avg^2, max) per workload;
forward+backward on 10^6 near-surface queries of the same mesh (loss = sum of
squared distances) and the backward kernels alone; the mixed primitive set;
the interception table built on the device; the near/far sweep (Sec. 5.3:
the mesh precomputed for the default 10x domain, uniform queries in boxes of
1x..10x AABB); the 256-mesh batch in one graph launch against 256 plain
launches; the FP64 brute-force oracle on a bounded sample of the workload's
queries (host cores) and the CPU P2M query over the same tree and table, on
all host threads and on one.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_query_c2.txt")
SQ_FILE = os.path.join(ROOT, "profiles", "k_query_c2_counters.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("query_core.hpp", "nearest.hpp", "wave_kdtree.hpp", "wave_scan.hpp", "device_common.hpp", "regroup.hpp",
              "p2m_device.hip"):
        with open(os.path.join(ROOT, "paper_2308_16084_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _summary(path: str, n_queries: int):
    """key: value lines of a committed rocprofv3 counter summary, if it was
    taken on the current kernel source at this batch size."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash() or int(vals.get("queries", -1)) != n_queries:
        return None
    return vals


def b_alg(visits: float, entries: float, edge_forms: float, face_forms: float) -> float:
    """Algorithmic bytes per query of the method (what it must touch, no
    caching credit): the query in (12) and the answer out (primitive,
    closest point, distance: 20); 16 per nearest-vertex candidate (a
    vertex's position and id); the list range of the nearest vertex (8);
    4 per list entry scanned (its id); per edge tested (an entry whose box
    holds q) 4 + 8 + 24 (id, its two vertex ids and positions), per face
    tested 4 + 12 + 36."""
    return 12 + 20 + 16 * visits + 8 + 4 * entries + 36 * edge_forms + 52 * face_forms


def touched_bytes(visits: float, steps: float, entries: float, edge_forms: float, face_forms: float) -> float:
    """Bytes this implementation's layout reads and writes per query, every
    L2 / Infinity-Cache hit counted as if it came from HBM: query in (12) +
    results out (20) + the walk (seed record 16, per step the neighbour-list
    offsets 8, per neighbour its record 16) + the list head (32) + 8 per list
    entry (id + box; runs padded to even length) + per entry whose box holds
    q its forms (edge 32, face 48) + the winner's exact re-evaluation (48)."""
    return 12 + 20 + 16 + 8 * steps + 16 * visits + 32 + 8 * entries + 32 * edge_forms + 48 * face_forms + 48


def list_stats(st: dict):
    """Table 1's list statistics (edges, faces) from the build statistics."""
    if "avg_edges" not in st:
        return None
    return {"avg1": [round(st["avg_edges"], 2), round(st["avg_faces"], 2)],
            "avg2": [round(st["avg_edges_volw"], 2), round(st["avg_faces_volw"], 2)],
            "max": [int(st["max_edges"]), int(st["max_faces"])], "avg_list": round(st["avg_list"], 2),
            "avg_list_volw": round(st["avg_list_volw"], 2), "max_list": int(st["max_list"])}


def host_counts(mesh, Q, k=200_000, seed=123):
    """Per-query counts of the host model over the same structures (a sample)."""
    rng = np.random.default_rng(seed)
    sub = Q[rng.choice(len(Q), size=min(len(Q), k), replace=False)]
    hs = mesh.query_host(sub)
    per = {key: hs[key] / len(sub) for key in ("nodes", "steps", "edges", "faces", "edge_forms", "face_forms",
                                               "rescans")}
    return per


def alt_legs(args, mesh, q, out, n, ms_step, result):
    """The headline batch without the ordering step, and with the other
    nearest-vertex traversals: the per-lane tree search (with and without
    its top levels staged in LDS) and the wavefront tree walk."""
    ms_uns = time_steps(lambda: mesh.query(q, out=out, sort=False), args.steps, args.warmup)
    result["unsorted"] = {"value": round(n / (ms_uns / 1e3), 1), "unit": "queries/s", "ms_per_step": round(ms_uns, 4),
                          "workload": "the headline batch in input order (no Morton ordering)"}
    log(f"[bench] unsorted: {ms_uns:.3f} ms/step, {n / (ms_uns / 1e3) / 1e9:.3f} Gq/s")

    trav = {}
    for name, tv, lv in (("kd_per_lane", 1, 0), ("kd_per_lane_lds8", 1, 8), ("kd_wavefront", 2, 0)):
        ms_t = time_steps(lambda: mesh.query(q, out=out, traversal=tv, lds_levels=lv), args.steps, args.warmup)
        trav[name] = round(ms_t, 4)
    trav["voronoi_walk"] = round(ms_step, 4)
    result["traversals_ms"] = trav
    log("[bench] traversals (ms/step): " + ", ".join(f"{k} {v:.3f}" for k, v in trav.items()))


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--queries", type=int, default=10_000_000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baselines")
    ap.add_argument("--no-bwd", action="store_true", help="skip the forward+backward leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched leg")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-primitive (triangles + segments) leg")
    ap.add_argument("--no-configs", action="store_true", help="skip the C1 and C3 legs")
    ap.add_argument("--no-sweep", action="store_true", help="skip the near/far sweep leg")
    ap.add_argument("--no-alt", action="store_true",
                    help="skip the unsorted and alternative-traversal legs on the headline batch")
    ap.add_argument("--no-precompute", action="store_true",
                    help="skip the device-inspection leg (the C2 table built with the filter and flooding on the GPU)")
    ap.add_argument("--sweep-queries", type=int, default=1_000_000,
                    help="queries per box of the near/far sweep (the C2 mesh precomputed for the default domain, "
                         "D = 10x AABB; uniform queries in boxes of 1x..10x AABB)")
    ap.add_argument("--batched-meshes", type=int, default=256,
                    help="batched leg on the first N meshes of the seeded 256-mesh plan (default: all 256)")
    ap.add_argument("--breakdown", action="store_true",
                    help="also time the nearest-vertex step alone and the query kernel on pre-sorted queries "
                         "(extra launches of the same kernel; off by default so profiles average the step only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB-in / 1 GiB-out elementwise copy kernel (counter calibration)")
    ap.add_argument("--cache", default=os.environ.get("P2M_CACHE_DIR", ""),
                    help="directory to save/load the precomputed mesh (default $P2M_CACHE_DIR; empty: none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU: --gpus must be 1 (the queries of a batch are "
                                   "independent, so more GPUs would each take a share of the sorted batch)"}))
        sys.exit(2)

    import torch

    import paper_2308_16084_amd as P
    from synth import configs as C
    from synth import queries as SQ

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")

    t0 = time.time()
    w = C.c2(n_queries=args.queries)
    log(f"[bench] workload generated in {time.time() - t0:.1f}s: {w.V.shape[0]} V, {w.F.shape[0]} F, {len(w.Q)} queries")
    t0 = time.time()
    mesh, stats = P.Mesh.cached(w.V, w.F, (w.domain_lo, w.domain_hi), args.cache or None)
    t_pre = time.time() - t0
    if "avg_list" not in stats:
        off, _ = mesh.table()
        stats["avg_list"] = float(off[-1]) / mesh.nv
    log(f"[bench] host precompute {t_pre:.1f}s {json.dumps({k: stats[k] for k in stats if k.startswith('t_') or k in ('avg_list', 'max_list', 'flood_tests')})}")
    t0 = time.time()
    dev_bytes = mesh.upload(0)
    torch.cuda.synchronize()
    t_upload = time.time() - t0
    q = torch.from_numpy(w.Q).to(dev)
    n = q.shape[0]
    out = {"prim": torch.empty(n, dtype=torch.int32, device=dev),
           "closest": torch.empty((n, 3), dtype=torch.float32, device=dev),
           "dist": torch.empty(n, dtype=torch.float32, device=dev),
           "status": torch.empty(n, dtype=torch.uint8, device=dev)}
    torch.cuda.synchronize()

    def step(profile=False):
        mesh.query(q, out=out, profile=profile)

    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    wall0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = e0.elapsed_time(e1) / args.steps
    qps = n / (ms_step / 1e3)
    log(f"[bench] forward: {ms_step:.3f} ms/step ({wall / args.steps * 1e3:.3f} ms wall), {qps / 1e9:.3f} Gq/s")

    # live per-kernel timing of the dominant (query) kernel over profiled steps
    order_ms, query_ms, finish_ms = [], [], []
    for _ in range(args.steps):
        step(profile=True)
        a, b, c = mesh.query_profile()
        order_ms.append(a)
        query_ms.append(b)
        finish_ms.append(c)
    order_avg, query_avg, finish_avg = (float(np.mean(x)) for x in (order_ms, query_ms, finish_ms))
    log(f"[bench] stage times: ordering {order_avg:.3f} ms, query kernel {query_avg:.3f} ms, "
        f"answer write-out {finish_avg:.3f} ms")

    # cost breakdown: nearest vertex alone vs the whole query kernel, both on
    # the Morton-ordered batch without the ordering step, default traversal
    breakdown = None
    if args.breakdown:
        _, perm = mesh.order_queries(q)
        qs = q[perm.long()].contiguous()
        nv_ms, full_ms = [], []
        for _ in range(args.steps):
            e0.record()
            mesh.nearest_vertex(qs)
            e1.record()
            torch.cuda.synchronize()
            nv_ms.append(e0.elapsed_time(e1))
            e0.record()
            mesh.query(qs, out=out, sort=False)
            e1.record()
            torch.cuda.synchronize()
            full_ms.append(e0.elapsed_time(e1))
        del qs, perm
        breakdown = {"nearest_vertex_only_ms": round(float(np.mean(nv_ms)), 4),
                     "query_presorted_ms": round(float(np.mean(full_ms)), 4)}
        log(f"[bench] breakdown on pre-sorted queries: nearest vertex {breakdown['nearest_vertex_only_ms']:.3f} ms, "
            f"whole query {breakdown['query_presorted_ms']:.3f} ms")

    # algorithmic bytes per query from the same structures (host model counts)
    rng = np.random.default_rng(123)
    per = host_counts(mesh, w.Q)
    entries = per["edges"] + per["faces"]
    balg = b_alg(per["nodes"], entries, per["edge_forms"], per["face_forms"])
    btouch = touched_bytes(per["nodes"], per["steps"], entries, per["edge_forms"], per["face_forms"])
    achieved = balg * n / (query_avg / 1e3) / 1e9
    tr = _summary(TRAFFIC_FILE, n)
    sq = _summary(SQ_FILE, n)
    traffic = float(tr["hbm_bytes_per_launch"]) if tr else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_query", "kernel_ms": round(query_avg, 4),
                "b_alg_bytes_per_query": round(balg, 1),
                # from the committed rocprofv3 counter summaries of this kernel source (null when stale)
                "counter_hbm_GBps": round(traffic / (query_avg / 1e3) / 1e9, 1) if traffic else None,
                "counter_hbm_frac": round(traffic / (query_avg / 1e3) / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
                "l2_hit_rate": float(tr["l2_hit_rate"]) if tr else None,
                "valu_issue_frac": float(sq["valu_issue_frac"]) if sq else None,
                "lanes_active_frac": float(sq["lanes_active_frac"]) if sq else None,
                "valu_insts_per_wave": float(sq["valu_insts_per_wave"]) if sq else None,
                # bytes of this layout touched per query, cache hits counted as HBM reads
                "touched_bytes_per_query": round(btouch, 1),
                "touched_GBps": round(btouch * n / (query_avg / 1e3) / 1e9, 1),
                "per_query": {"walk_vertices": round(per["nodes"], 2), "walk_steps": round(per["steps"], 2),
                              "edge_entries": round(per["edges"], 2), "face_entries": round(per["faces"], 2),
                              "edge_forms_read": round(per["edge_forms"], 2),
                              "face_forms_read": round(per["face_forms"], 2),
                              "second_scans": per["rescans"]}}
    log(f"[bench] roofline: B_alg {balg:.0f} B/query -> {achieved:.0f} GB/s ({achieved / HBM_PEAK_GBS:.3f} of HBM); "
        f"touched {btouch:.0f} B/query; counters {'current' if tr else 'stale or missing'}")

    result = {"metric": "P2M queries/sec at 1.3M tris (fwd, fwd+bwd, batched); % of HBM peak",
              "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "dtype": "f32",
              "data": "synthetic (seeded displaced icosphere; generated queries)",
              "config": {"workload": "icosphere level 8 + 4-octave fbm displacement (655,362 V, 1,310,720 F), "
                                     "1e7 queries: 50% uniform in 1.5x AABB, 50% near-surface (sigma 1% diag)",
                         "queries": n, "ordering": "morton30+radix", "host_precompute_s": round(t_pre, 1),
                         "precompute_cached": "loaded_from" in stats,
                         "avg_list": round(float(stats.get("avg_list", 0.0)), 2),
                         "device_bytes": dev_bytes, "upload_s": round(t_upload, 3)},
              "roofline": roofline,
              "stages_ms": {"ordering": round(order_avg, 4), "query": round(query_avg, 4),
                            "write_out": round(finish_avg, 4)}}
    # the ordering: Morton keys (12 B in, 4 out per query) and three 8-bit
    # passes (count: 4 B; scatter: key + value in and out, 16 B, except
    # that the first pass reads no values and the last writes no keys)
    ord_bytes = 16 + (4 + 12) + (4 + 16) + (4 + 12)
    result["ordering"] = {"bytes_per_query": ord_bytes, "ms": round(order_avg, 4),
                          "GBps": round(ord_bytes * n / (order_avg / 1e3) / 1e9, 1),
                          "frac": round(ord_bytes * n / (order_avg / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    result["list_stats"] = {"c2": list_stats(stats)}
    if breakdown:
        result["breakdown"] = breakdown

    # the unsorted and alternative-traversal legs
    if not args.no_alt:
        alt_legs(args, mesh, q, out, n, ms_step, result)

    if not args.no_configs:
        # the small icosphere (C1) and the needle heightfield (C3): q/s, list statistics
        for name, make, mode in (("c1", C.c1, P.TABLE_FLOODING), ("c3", C.c3, P.TABLE_FLOODING_DEVICE)):
            log(f"[bench] {name}: generating and precomputing")
            t0 = time.time()
            wk = make()
            mk, sk = P.Mesh.cached(wk.V, wk.F, (wk.domain_lo, wk.domain_hi), args.cache or None, table_mode=mode)
            t_pk = time.time() - t0
            mk.upload(0)
            qk = torch.from_numpy(wk.Q).to(dev)
            ok = mk.query(qk)
            ms_k = time_steps(lambda: mk.query(qk, out=ok), args.steps, args.warmup)
            nk = qk.shape[0]
            pk = host_counts(mk, wk.Q, k=100_000)
            bk = b_alg(pk["nodes"], pk["edges"] + pk["faces"], pk["edge_forms"], pk["face_forms"])
            result[name] = {"value": round(nk / (ms_k / 1e3), 1), "unit": "queries/s", "ms_per_step": round(ms_k, 4),
                            "queries": nk, "b_alg_bytes_per_query": round(bk, 1),
                            "achieved_GBps_whole_step": round(bk * nk / (ms_k / 1e3) / 1e9, 1),
                            "workload": wk.name, "setup_s": round(t_pk, 1)}
            result["list_stats"][name] = list_stats(sk)
            log(f"[bench] {name}: {ms_k:.3f} ms/step, {nk / (ms_k / 1e3) / 1e9:.3f} Gq/s")
            del mk, qk, ok

    if not args.no_bwd:
        w5 = C.c5()
        q5 = torch.from_numpy(w5.Q).to(dev)
        Vt = torch.from_numpy(w.V).to(dev)
        n5 = q5.shape[0]

        def fb():
            qq = q5.detach().requires_grad_(True)
            VV = Vt.detach().requires_grad_(True)
            d, _, _ = P.p2m_distance(qq, VV, mesh)
            (d * d).sum().backward()
            return qq.grad, VV.grad

        ms_fb = time_steps(fb, args.steps, args.warmup)
        # the backward kernels alone: per query q, c, d, upstream gradient,
        # weights and vertex ids in (56 B), grad_q out (12 B), and a
        # read-modify-write of one grad_V row (24 B) per nonzero weight
        f5 = mesh.query(q5, for_backward=True, status=False)
        g5 = 2.0 * f5["dist"]
        gV5 = torch.zeros((mesh.nv, 3), dtype=torch.float32, device=dev)
        ms_bwd = time_steps(lambda: mesh.query_backward(q5, f5, g5, grad_q=True, grad_V=gV5), args.steps, args.warmup)
        nz = float((f5["bary"] != 0).sum().item()) / n5
        bb = 56 + 12 + 24 * nz
        result["fwd_bwd"] = {"value": round(n5 / (ms_fb / 1e3), 1), "unit": "queries/s", "ms_per_step": round(ms_fb, 4),
                             "workload": "same mesh, 1e6 near-surface queries, loss = sum d^2, grads wrt q [1e6,3] and V [655362,3]",
                             "backward_kernels": {"ms": round(ms_bwd, 4), "b_alg_bytes_per_query": round(bb, 1),
                                                  "achieved_GBps": round(bb * n5 / (ms_bwd / 1e3) / 1e9, 1),
                                                  "frac": round(bb * n5 / (ms_bwd / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                                                  "weights_per_query": round(nz, 3)}}
        log(f"[bench] fwd+bwd: {ms_fb:.3f} ms/step, {n5 / (ms_fb / 1e3) / 1e9:.3f} Gq/s; backward kernels {ms_bwd:.3f} ms")
        del f5, g5, gV5

    if not args.no_mixed:
        t0 = time.time()
        w6 = C.c6()
        m6, _ = P.Mesh.cached(w6.V, w6.F, (w6.domain_lo, w6.domain_hi), args.cache or None, segments=w6.S)
        t_pre6 = time.time() - t0
        m6.upload(0)
        q6 = torch.from_numpy(w6.Q).to(dev)
        out6 = m6.query(q6)
        for _ in range(args.warmup):
            m6.query(q6, out=out6)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            m6.query(q6, out=out6)
        e1.record()
        torch.cuda.synchronize()
        ms6 = e0.elapsed_time(e1) / args.steps
        n6 = q6.shape[0]
        result["mixed"] = {"value": round(n6 / (ms6 / 1e3), 1), "unit": "queries/s", "ms_per_step": round(ms6, 4),
                           "workload": f"mixed primitive set: {len(w6.F)} triangles + {len(w6.S)} free segments "
                                       f"({len(w6.V)} V), {n6} queries (half uniform in 1.5x AABB, half near "
                                       f"the triangles / segments)",
                           "host_precompute_s": round(t_pre6, 1)}
        log(f"[bench] mixed (triangles + segments): {ms6:.3f} ms/step, {n6 / (ms6 / 1e3) / 1e9:.3f} Gq/s")
        del m6, q6, out6

    if not args.no_precompute:
        # The C2 table again, with the inspection (filter + flooding) on the
        # device; it must equal the host-built table used above.
        t0 = time.time()
        md = P.Mesh(w.V, w.F)
        sd = md.precompute((w.domain_lo, w.domain_hi), table_mode=P.TABLE_FLOODING_DEVICE)
        t_dev = time.time() - t0
        oh, eh = mesh.table()
        od, ed = md.table()
        same = bool(np.array_equal(oh, od) and np.array_equal(eh, ed) and
                    np.array_equal(mesh.table_boxes(), md.table_boxes()))
        host_stages = {k: round(stats[k], 3) for k in ("t_delaunay", "t_cells", "t_flood", "t_pack") if k in stats}
        result["precompute_device"] = {
            "total_s": round(t_dev, 2),
            "stages_s": {"delaunay": round(sd["t_delaunay"], 3), "cells": round(sd["t_cells"], 3),
                         "inspection": round(sd["t_flood"], 3), "upload": round(sd["t_dev_upload"], 3),
                         "kernel": round(sd["t_dev_kernel"], 3), "download": round(sd["t_dev_download"], 3),
                         "pack": round(sd["t_pack"], 3)},
            "host_build_stages_s": host_stages or None,
            "host_threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
            "primitives_finished_on_host": int(sd["device_redo"]), "filter_tests": int(sd["flood_tests"]),
            "identical_to_host_table": same,
            "workload": "C2 mesh (655,362 V, 1,966,080 E, 1,310,720 F), D = 1.5x AABB"}
        log(f"[bench] device inspection: total {t_dev:.1f}s, kernel {sd['t_dev_kernel']:.2f}s, inspection "
            f"{sd['t_flood']:.2f}s (host build: {host_stages or 'loaded from cache'}), "
            f"{int(sd['device_redo'])} primitives finished on the host, identical table: {same}")
        assert same, "device-built interception table differs from the host-built one"
        del md

    if not args.no_sweep:
        # Sec. 5.3's near/far study: the C2 mesh precomputed for the library's
        # default domain (10x AABB), uniform queries in boxes of 1x..10x AABB
        log("[bench] sweep: precomputing the mesh for the default 10x domain")
        t0 = time.time()
        lo2, hi2 = SQ.aabb(w.V)
        m10, st10 = P.Mesh.cached(w.V, w.F, None, args.cache or None, table_mode=P.TABLE_FLOODING_DEVICE)
        t_pre10 = time.time() - t0
        m10.upload(0)
        rows = []
        ns_ = args.sweep_queries
        for scale in (1.0, 1.5, 2.0, 3.0, 5.0, 10.0):
            blo, bhi = SQ.scaled_box(lo2, hi2, scale)
            Qs = SQ.uniform_in_box(ns_, blo, bhi, np.random.default_rng(2100 + int(10 * scale)))
            qs_t = torch.from_numpy(Qs).to(dev)
            o = m10.query(qs_t)
            ms = time_steps(lambda: m10.query(qs_t, out=o), args.steps, args.warmup)
            hc = host_counts(m10, Qs, k=100_000)
            rows.append({"box_scale": scale, "queries_per_s": round(ns_ / (ms / 1e3), 1), "ms_per_step": round(ms, 4),
                         "walk_vertices": round(hc["nodes"], 2), "walk_steps": round(hc["steps"], 2),
                         "list_entries": round(hc["edges"] + hc["faces"], 2),
                         "forms_read": round(hc["edge_forms"] + hc["face_forms"], 2),
                         "second_scans": hc["rescans"]})
            log(f"[bench] sweep box {scale}x: {ms:.3f} ms per {ns_}, entries {rows[-1]['list_entries']}, "
                f"forms {rows[-1]['forms_read']}")
        result["near_far_sweep"] = {"domain": "10x AABB (default)", "queries_per_box": ns_,
                                    "setup_s": round(t_pre10, 1), "list_stats": list_stats(st10), "rows": rows}
        del m10

    if not args.no_batched:
        from concurrent.futures import ThreadPoolExecutor
        count = max(1, min(256, args.batched_meshes))
        log(f"[bench] batched: generating and precomputing {count} meshes")
        t0 = time.time()
        plan = C.c4_plan()[:count]
        with ThreadPoolExecutor(max_workers=max(1, len(os.sched_getaffinity(0)))) as ex:
            works = list(ex.map(C.c4_mesh, plan))
        t_gen = time.time() - t0
        log(f"[bench] batched: {count} meshes generated in {t_gen:.1f}s")
        t0 = time.time()
        # inspection on the device (the table is the host build's), 32 meshes
        # at a time with a progress line after each group
        meshes = []
        for k0 in range(0, count, 32):
            part = works[k0:k0 + 32]
            meshes += P.precompute_many([(x.V, x.F, (x.domain_lo, x.domain_hi)) for x in part], args.cache or None,
                                        table_mode=P.TABLE_FLOODING_DEVICE)
            log(f"[bench] batched: {len(meshes)} of {count} meshes precomputed ({time.time() - t0:.1f}s)")
        t_pre4 = time.time() - t0
        Qb = np.concatenate([x.Q for x in works])
        offb = np.concatenate([[0], np.cumsum([len(x.Q) for x in works])]).astype(np.int64)
        nb = int(offb[-1])
        qb = torch.from_numpy(Qb).to(dev)
        batch = P.Batch(meshes, 0)
        outb = batch.query(qb, offb, graph=False)
        torch.cuda.synchronize()
        shape = batch.autotune(qb, offb, out=outb)
        for _ in range(args.warmup):
            batch.query(qb, offb, out=outb)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            batch.query(qb, offb, out=outb)
        e1.record()
        torch.cuda.synchronize()
        ms_b = e0.elapsed_time(e1) / args.steps
        # the persistent schedule (workgroups claiming tiles from a counter) at the same shape
        batch.set_schedule(True)
        ms_pers = time_steps(lambda: batch.query(qb, offb, out=outb), args.steps, args.warmup)
        batch.set_schedule(False)
        # the same work as one plain launch sequence per mesh
        for m_ in meshes:
            m_.upload(0)
        outs = [{"prim": outb["prim"][offb[k]:offb[k + 1]], "closest": outb["closest"][offb[k]:offb[k + 1]],
                 "dist": outb["dist"][offb[k]:offb[k + 1]]} for k in range(count)]
        qsl = [qb[offb[k]:offb[k + 1]] for k in range(count)]

        def plain_all():
            for k in range(count):
                if offb[k + 1] > offb[k]:
                    meshes[k].query(qsl[k], out=outs[k])

        for _ in range(args.warmup):
            plain_all()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            plain_all()
        e1.record()
        torch.cuda.synchronize()
        ms_p = e0.elapsed_time(e1) / args.steps
        ntri = int(sum(len(x.F) for x in works))
        # algorithmic bytes over the batch: host-model counts on every 16th query of each mesh
        tot = 0.0
        for k, m_ in enumerate(meshes):
            Qk = works[k].Q[::16]
            if len(Qk) == 0:
                continue
            hk = m_.query_host(Qk)
            bk = b_alg(hk["nodes"] / len(Qk), (hk["edges"] + hk["faces"]) / len(Qk), hk["edge_forms"] / len(Qk),
                       hk["face_forms"] / len(Qk))
            tot += bk * len(works[k].Q)
        result["batched_roofline"] = {"b_alg_bytes_per_query": round(tot / nb, 1),
                                      "achieved_GBps_whole_launch": round(tot / (ms_b / 1e3) / 1e9, 1),
                                      "frac": round(tot / (ms_b / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                                      "note": "over the whole graph launch (keys, sort, query, write-out)"}
        result["batched"] = {"value": round(nb / (ms_b / 1e3), 1), "unit": "queries/s", "ms_per_step": round(ms_b, 4),
                             "plain_launches": {"value": round(nb / (ms_p / 1e3), 1), "ms_per_step": round(ms_p, 4),
                                                "launches": count},
                             "speedup_vs_plain": round(ms_p / ms_b, 3),
                             "persistent_schedule_ms": round(ms_pers, 4),
                             "shape": {"block": shape[0], "queries_per_lane": shape[1],
                                       "traversal": {1: "kd per-lane", 2: "kd wavefront", 3: "voronoi walk"}[shape[2]],
                                       "lds_levels": batch.lds_levels()},
                             "workload": (f"{'all' if count == 256 else 'first'} {count} meshes of the seeded 256-mesh plan "
                                          f"(displaced geodesic spheres / heightfields, log-uniform sizes): {ntri} triangles, "
                                          f"{nb} queries (log-uniform per mesh, mixed uniform/near-surface); one graph launch"),
                             "precompute_s": round(t_pre4, 1), "precompute": "host Delaunay + cells, inspection on the GPU",
                             "generate_s": round(t_gen, 1)}
        log(f"[bench] batched ({count} meshes, {ntri} tris, {nb} queries): {ms_b:.3f} ms graph vs {ms_p:.3f} ms "
            f"for {count} plain launches; persistent schedule {ms_pers:.3f} ms; shape {shape}; precompute {t_pre4:.1f}s")
        del batch, meshes, qb, outb, outs, qsl

    if not args.no_cpu:
        import oracle
        om = oracle.OracleMesh(w.V, w.F)
        # a bounded sample: chunks of 500 queries until about 12 s of CPU time
        pool = w.Q[rng.choice(n, size=10_000, replace=False)]
        ns, dt = 0, 0.0
        t0 = time.perf_counter()
        while ns < len(pool) and dt < 12.0:
            om.query(pool[ns:ns + 500])
            ns += 500
            dt = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": round(ns / dt, 2), "unit": "queries/s", "cores": oracle.num_threads(),
                                  "kind": "oracle",
                                  "sample": f"{ns} queries drawn from the workload's 1e7 (seed 123), FP64 brute force "
                                            f"over all V, E, F, in chunks of 500 until 12 s had passed; {dt:.1f}s"}
        log(f"[bench] oracle: {ns / dt:.1f} q/s on {oracle.num_threads()} threads ({dt:.1f}s)")
        sub2 = w.Q[:1_000_000]
        nth = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        mesh.query_host(sub2, threads=nth)
        dt = time.perf_counter() - t0
        sub1 = w.Q[:100_000]
        t0 = time.perf_counter()
        mesh.query_host(sub1, threads=1)
        dt1 = time.perf_counter() - t0
        result["cpu_p2m"] = {"value": round(len(sub2) / dt, 1), "unit": "queries/s", "threads": nth,
                             "kind": "multi-threaded CPU P2M query, same structures and float32 code as the default device path",
                             "sample": "first 1e6 queries of the workload",
                             "one_thread": {"value": round(len(sub1) / dt1, 1), "us_per_query": round(dt1 / len(sub1) * 1e6, 3),
                                            "sample": "first 1e5 queries of the workload"}}
        log(f"[bench] CPU P2M: {len(sub2) / dt:.0f} q/s on {nth} threads, {len(sub1) / dt1:.0f} q/s on one")

    print(json.dumps(result))


if __name__ == "__main__":
    main()
