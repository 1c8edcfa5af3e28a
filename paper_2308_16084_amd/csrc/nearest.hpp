// Nearest-vertex step of the query (Algorithm A.2): the three device
// traversals and the seed grid of the Voronoi walk.
#pragma once

#include <hip/hip_runtime.h>

#include "query_core.hpp"
#include "wave_kdtree.hpp"

namespace p2m {

// Nearest-vertex search used by a query kernel.
enum Walk { WALK_LANE = 0, WALK_WAVE = 1, WALK_VORONOI = 2 };

// WALK_LANE: every lane searches the KD tree on its own.  WALK_WAVE: the
// wavefront-coherent tree walk (dense, Morton-ordered batches).
// WALK_VORONOI: greedy walk over the Voronoi neighbour graph from the grid
// seed for queries in D (where it is exact); the queries of a wavefront that
// lie outside D then take the wavefront tree walk together, so that every
// traversal returns the same vertex.  All lanes of the wavefront must call
// this (inactive ones with active = false).
// WALK_LANE reads nodes below ntop from `top` (a copy of the tree's top
// levels in LDS) when ntop > 0.
template <int kWalk>
__device__ __forceinline__ Nearest nearest_vertex(const MeshView& m, float qx, float qy, float qz, bool active,
                                                  uint64_t& visits, uint64_t& steps, const KdNode* top = nullptr,
                                                  int32_t ntop = 0) {
    Nearest b;
    b.d2 = INFINITY;
    b.px = b.py = b.pz = 0.f;
    b.vid = -1;
    if (kWalk == WALK_WAVE) return kdt_nearest_wave(m.node, m.nv, qx, qy, qz, active);
    if (kWalk == WALK_LANE) {
        if (!active) return b;
        if (ntop <= 0) return kdt_nearest(m.node, m.nv, qx, qy, qz, visits);
        const KdNode* node = m.node;
        return kdt_nearest_f([node, top, ntop](int32_t i) { return i < ntop ? top[i] : node[i]; }, m.nv, qx, qy, qz,
                             visits);
    }
    const bool inside = active && domain_status(m, qx, qy, qz) == 0;
    if (inside) b = voronoi_walk(m, qx, qy, qz, visits, steps);
    const bool outside = active && !inside;
    if (__any(outside)) {
        const Nearest t = kdt_nearest_wave(m.node, m.nv, qx, qy, qz, outside);
        if (outside) b = t;
    }
    return b;
}

// The top `levels` levels of a KD tree of nv nodes: the nodes a staged copy
// holds (at most 2^levels - 1, and no more than the tree has).
__host__ __device__ inline int32_t top_nodes(int levels, int32_t nv) {
    const int32_t t = levels > 0 ? (int32_t)((1u << levels) - 1u) : 0;
    return t < nv ? t : nv;
}

// Copies nodes [0, ntop) into LDS (`top`) with the whole block; the caller
// synchronises before reading them.
__device__ __forceinline__ void stage_top(const KdNode* __restrict__ node, int32_t ntop, KdNode* top) {
    const float4* src = reinterpret_cast<const float4*>(node);
    float4* dst = reinterpret_cast<float4*>(top);
    for (int32_t i = (int32_t)threadIdx.x; i < 4 * ntop; i += (int32_t)blockDim.x) dst[i] = src[i];
}

// Side of the seed grid of the Voronoi walk: about 27 cells per vertex over
// D, between 8^3 and 256^3 cells.
int32_t walk_grid_side(int64_t nv);

// Fills m.grid^3 seeds (nearest vertex of every cell centre: position, id
// bits) on `st`; m points to device arrays (its seed field is ignored).
hipError_t launch_seed_grid(const MeshView& m, float4* seed, hipStream_t st);

}  // namespace p2m
