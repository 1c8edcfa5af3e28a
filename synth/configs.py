"""The synthetic workloads (seeded), as plain arrays.

C1  icosphere level 4 (2,562 V / 5,120 F), radial U[-0.05,0.05] noise,
    10^4 queries uniform in the 1.2x AABB.
C2  icosphere level 8 (655,362 V / 1,310,720 F), radial 4-octave value-noise
    fbm (amplitude 0.1, base frequency 4), 10^7 queries: half uniform in the
    1.5x AABB, half near-surface (sigma = 1% of the AABB diagonal).
C3  1024 x 1024 heightfield (1,048,576 V / 2,093,058 F), fbm heights
    (amplitude 0.2), in-plane jitter up to 0.45 cell, every 7th row gap
    compressed 20x; 10^7 queries uniform in the AABB grown 0.1 in z.
C4  256 displaced spheres / heightfields, triangle counts log-uniform in
    [1e3, 2e5], query counts log-uniform in [1e3, 1e6] (mixed as C2).
C5  the C2 mesh with 10^6 near-surface queries (loss = sum of d^2).
C6  a mixed primitive set: the triangles of a displaced icosphere level 6
    (40,962 V / 81,920 F) and, as free segments, the edge wireframe of a
    displaced icosphere level 5 of radius 0.6 centred at (0.55, 0.1, -0.05)
    (10,242 V / 30,720 segments), intersecting it; 10^6 queries: half uniform
    in the 1.5x AABB, a quarter near the triangles and a quarter near the
    segments (sigma = 1% of the AABB diagonal).

Each workload also fixes the query domain box D that the precompute clips
Voronoi cells to: the box the queries are drawn from.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import mesh as M
from . import queries as Q

MESH_SEED = 1000
QUERY_SEED = 2000


@dataclass
class Workload:
    name: str
    V: np.ndarray            # float32 [nv,3]
    F: np.ndarray            # int32 [nf,3]
    Q: np.ndarray            # float32 [n,3]
    domain_lo: np.ndarray    # float64 [3]
    domain_hi: np.ndarray    # float64 [3]
    meta: dict = field(default_factory=dict)
    S: np.ndarray | None = None  # int32 [ns,2] free segments (mixed primitive sets)

    @property
    def diag(self) -> float:
        lo, hi = Q.aabb(self.V)
        return float(np.linalg.norm(hi - lo))


def _finish(name, V, F, Qp, dlo, dhi, **meta) -> Workload:
    return Workload(name, np.ascontiguousarray(V, dtype=np.float32),
                    np.ascontiguousarray(F, dtype=np.int32),
                    np.ascontiguousarray(Qp, dtype=np.float32),
                    np.asarray(dlo, dtype=np.float64), np.asarray(dhi, dtype=np.float64), meta)


def sphere_mesh(level: int, noise: str, seed: int) -> tuple[np.ndarray, np.ndarray]:
    Vu, F = M.icosphere(level)
    if noise == "uniform":
        V = M.displace_uniform(Vu, 0.05, seed)
    elif noise == "fbm":
        V = M.displace_fbm(Vu, 0.1, seed)
    elif noise == "none":
        V = Vu
    else:
        raise ValueError(noise)
    return V.astype(np.float32), F.astype(np.int32)


def c1(n_queries: int = 10_000) -> Workload:
    V, F = sphere_mesh(4, "uniform", MESH_SEED + 1)
    lo, hi = Q.aabb(V)
    dlo, dhi = Q.scaled_box(lo, hi, 1.2)
    rng = np.random.default_rng(QUERY_SEED + 1)
    return _finish("c1_icosphere4_uniform", V, F, Q.uniform_in_box(n_queries, dlo, dhi, rng), dlo, dhi)


def c2(n_queries: int = 10_000_000, level: int = 8) -> Workload:
    V, F = sphere_mesh(level, "fbm", MESH_SEED + 2)
    lo, hi = Q.aabb(V)
    dlo, dhi = Q.scaled_box(lo, hi, 1.5)
    rng = np.random.default_rng(QUERY_SEED + 2)
    Qp, near = Q.mixed(V, F, n_queries, 1.5, 0.01, rng, return_near=True)
    return _finish(f"c2_icosphere{level}_fbm", V, F, Qp, dlo, dhi, near=near)


def heightfield_domain(V: np.ndarray, pad_z: float = 0.1):
    lo, hi = Q.aabb(V)
    lo = lo.copy()
    hi = hi.copy()
    lo[2] -= pad_z
    hi[2] += pad_z
    return lo, hi


def c3(n_queries: int = 10_000_000, n: int = 1024) -> Workload:
    V, F = M.heightfield(n, MESH_SEED + 3)
    V = V.astype(np.float32)
    dlo, dhi = heightfield_domain(V)
    rng = np.random.default_rng(QUERY_SEED + 3)
    return _finish(f"c3_heightfield{n}", V, F, Q.uniform_in_box(n_queries, dlo, dhi, rng), dlo, dhi)


def c5(n_queries: int = 1_000_000, level: int = 8) -> Workload:
    V, F = sphere_mesh(level, "fbm", MESH_SEED + 2)
    lo, hi = Q.aabb(V)
    dlo, dhi = Q.scaled_box(lo, hi, 1.5)
    rng = np.random.default_rng(QUERY_SEED + 5)
    diag = float(np.linalg.norm(hi - lo))
    return _finish(f"c5_icosphere{level}_fbm_near", V, F,
                   Q.near_surface(V, F, n_queries, 0.01 * diag, rng), dlo, dhi)


def c4_plan(count: int = 256, seed: int = MESH_SEED + 4, tri_lo: float = 1e3, tri_hi: float = 2e5,
            q_lo: float = 1e3, q_hi: float = 1e6) -> list[dict]:
    """Per-mesh kind, size parameter and query count (log-uniform draws)."""
    rng = np.random.default_rng(seed)
    plan = []
    for k in range(count):
        kind = "sphere" if rng.random() < 0.5 else "heightfield"
        T = float(np.exp(rng.uniform(np.log(tri_lo), np.log(tri_hi))))
        nq = int(round(np.exp(rng.uniform(np.log(q_lo), np.log(q_hi)))))
        if kind == "sphere":
            size = max(1, int(round((T / 20.0) ** 0.5)))
        else:
            size = int(round((T / 2.0) ** 0.5)) + 1
        plan.append({"kind": kind, "size": size, "queries": nq, "seed": seed * 1000 + k})
    return plan


def c4_mesh(entry: dict, query_scale: float = 1.0) -> Workload:
    s = entry["seed"]
    if entry["kind"] == "sphere":
        Vu, F = M.geodesic_sphere(entry["size"])
        V = M.displace_fbm(Vu, 0.1, s).astype(np.float32)
    else:
        V, F = M.heightfield(entry["size"], s)
        V = V.astype(np.float32)
    lo, hi = Q.aabb(V)
    dlo, dhi = Q.scaled_box(lo, hi, 1.5)
    rng = np.random.default_rng(s + 1)
    nq = max(1, int(round(entry["queries"] * query_scale)))
    return _finish(f"c4_{entry['kind']}{entry['size']}", V, F.astype(np.int32),
                   Q.mixed(V, F, nq, 1.5, 0.01, rng), dlo, dhi, kind=entry["kind"])


def c4(count: int = 256, query_scale: float = 1.0, tri_hi: float = 2e5) -> list[Workload]:
    return [c4_mesh(e, query_scale) for e in c4_plan(count, tri_hi=tri_hi)]


def c6(n_queries: int = 1_000_000, level: int = 6, wire_level: int = 5) -> Workload:
    """Mixed primitive set: triangles of one displaced sphere, the edge
    wireframe of another (free segments) crossing it."""
    V1, F1 = sphere_mesh(level, "fbm", MESH_SEED + 6)
    V2u, F2 = M.icosphere(wire_level)
    V2 = (0.6 * M.displace_fbm(V2u, 0.1, MESH_SEED + 7) + np.array([0.55, 0.1, -0.05])).astype(np.float32)
    S2 = np.unique(np.sort(np.concatenate([F2[:, [0, 1]], F2[:, [1, 2]], F2[:, [2, 0]]]), axis=1), axis=0)
    V = np.concatenate([V1, V2]).astype(np.float32)
    S = (S2 + len(V1)).astype(np.int32)
    lo, hi = Q.aabb(V)
    dlo, dhi = Q.scaled_box(lo, hi, 1.5)
    diag = float(np.linalg.norm(hi - lo))
    rng = np.random.default_rng(QUERY_SEED + 6)
    nu = n_queries // 2
    nt = (n_queries - nu) // 2
    Qp = np.concatenate([Q.uniform_in_box(nu, dlo, dhi, rng),
                         Q.near_surface(V, F1, nt, 0.01 * diag, rng),
                         Q.near_segments(V, S, n_queries - nu - nt, 0.01 * diag, rng)])
    Qp = Qp[rng.permutation(n_queries)]
    w = _finish(f"c6_mixed_icosphere{level}_wire{wire_level}", V, F1, Qp, dlo, dhi)
    w.S = S
    return w
