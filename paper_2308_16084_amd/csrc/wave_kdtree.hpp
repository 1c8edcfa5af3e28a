// Wavefront-coherent KD-tree nearest-vertex search (device only).
//
// The 64 lanes of a wavefront hold Morton-ordered, hence nearby, queries and
// walk the tree together.  A node is entered when at least one lane's box
// bound (squared distance from its query to the subtree box, within the
// 2^-20 tie margin of its own best) allows it, so each lane still sees every
// node its own exact search would see, and lanes only ever test extra points
// -- each lane's result is its exact nearest vertex.  Node indices are
// wave-uniform, so nodes are read with scalar loads, and the walk needs no
// stack: in the implicit tree the parent of node i is (i-1)/2, a step that
// arrives from the parent is a descent, and the child order at a node is
// fixed by the box distances of one reference query (the first active
// lane's), so returning from the near child can tell whether the far one
// is still owed.
#pragma once

#include <hip/hip_runtime.h>

#include "query_core.hpp"

namespace p2m {

__device__ __forceinline__ int32_t wave_uniform(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ float child_box_d2(float qx, float qy, float qz, const KdNode& nd, bool left) {
    return left ? box_d2(qx, qy, qz, nd.b0.x, nd.b0.y, nd.b0.z, nd.b0.w, nd.b1.x, nd.b1.y)
                : box_d2(qx, qy, qz, nd.b1.z, nd.b1.w, nd.b2.x, nd.b2.y, nd.b2.z, nd.b2.w);
}

// `active`: the lane holds a finite query that takes part.  Inactive lanes
// never ask for a node and their result is undefined.
//
// Per step: descending into a node tests its point and both child boxes for
// every lane; the child order (the reference lane's nearer box first) is
// kept in a wave-uniform bit per depth, so a return from the near child
// re-reads the node only for the far child's box and a return from the far
// child costs neither a load nor arithmetic.
__device__ __forceinline__ Nearest kdt_nearest_wave(const KdNode* __restrict__ node, int32_t n, float qx, float qy,
                                                    float qz, bool active) {
    Nearest b;
    b.d2 = INFINITY;
    b.px = b.py = b.pz = 0.f;
    b.vid = -1;
    const unsigned long long am = __ballot(active);
    if (am == 0ull) return b;
    const int src = __ffsll((long long)am) - 1;
    uint32_t right_first = 0;  // bit d: at depth d the right child was taken first
    int32_t prev = -1, cur = 0;
    int depth = 0;
    while (cur >= 0) {
        cur = wave_uniform(cur);
        prev = wave_uniform(prev);
        const int32_t parent = (cur - 1) >> 1;
        int32_t next;
        if (prev < cur) {  // arrived from the parent: test the point and both children
            const KdNode nd = node[cur];
            if (active) {
                const float dx = qx - nd.p.x, dy = qy - nd.p.y, dz = qz - nd.p.z;
                consider(b, qx, qy, qz, dx * dx + dy * dy + dz * dz, nd.p);
            }
            const float dl = child_box_d2(qx, qy, qz, nd, true);
            const float dr = child_box_d2(qx, qy, qz, nd, false);
            const bool right_near = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dr), src)) <
                                    __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dl), src));
            right_first = right_near ? (right_first | (1u << depth)) : (right_first & ~(1u << depth));
            const int32_t cn = 2 * cur + (right_near ? 2 : 1);
            const int32_t cf = 2 * cur + (right_near ? 1 : 2);
            const float dn = right_near ? dr : dl, df = right_near ? dl : dr;
            const float lim = b.d2 * kTieHi;
            const bool wn = active && cn < n && dn <= lim;
            const bool wf = active && cf < n && df <= lim;
            if (__ballot(wn)) {
                next = cn;
                ++depth;
            } else if (__ballot(wf)) {
                next = cf;
                ++depth;
            } else {
                next = parent;
                --depth;
            }
        } else {
            const bool right_near = (right_first >> depth) & 1u;
            const int32_t cn = 2 * cur + (right_near ? 2 : 1);
            const int32_t cf = 2 * cur + (right_near ? 1 : 2);
            next = parent;
            if (prev == cn) {  // back from the near child: is the far one still owed?
                // (the far child is the left one exactly when the near one is the right)
                const KdNode nd = node[cur];
                const bool wf = active && cf < n &&
                                child_box_d2(qx, qy, qz, nd, right_near) <= b.d2 * kTieHi;
                if (__ballot(wf)) next = cf;
            }
            depth += next == parent ? -1 : 1;
        }
        prev = cur;
        cur = next;
    }
    return b;
}

}  // namespace p2m
