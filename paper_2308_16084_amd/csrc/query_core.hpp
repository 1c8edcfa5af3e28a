// Per-query arithmetic of the P2M query (Appendix, Algorithm A.2), shared by
// the device kernels and the host CPU baseline (compiled by hipcc only).
//
//  1. nearest vertex v by the KD tree (float32 distances; candidates whose
//     squared distances agree to within 2^-20 relative are decided in
//     float64, then by vertex id; subtrees are pruned only when their lower
//     bound exceeds the best squared distance by more than 2^-20 relative);
//  2. d_min <- d(q, v);
//  3. for every edge and face in v's interception list, the distance to the
//     closed segment / triangle.  The paper gates each primitive by
//     Space-perp and then takes the line / plane distance; the clamped test
//     returns the same value whenever the gate passes and otherwise a
//     distance to a point of the primitive's boundary, which never
//     undercuts the true minimum.  So the minimum is unchanged in exact
//     arithmetic, and rounding in a gate cannot drop the true answer.  The
//     clamp region tells whether the closest point is inside the face, on
//     one of its sides or at a corner, which names the primitive returned.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace p2m {

#define P2M_HD __host__ __device__ __forceinline__

constexpr float kTieLo = 0.99999904632568359375f;  // 1 - 2^-20
constexpr float kTieHi = 1.00000095367431640625f;  // 1 + 2^-20
constexpr int kMaxDepth = 32;

enum : int { KIND_VERTEX = 0, KIND_EDGE = 1, KIND_FACE = 2, KIND_NONE = 3 };

struct MeshView {
    const struct KdNode* node;  // [nv] KD-tree nodes (point + child boxes)
    int32_t nv;
    const uint32_t* off;    // [2nv+1]
    const int32_t* ent;     // [nnz]
    const float4* seg;      // [2ne]
    const float4* tri;      // [3nf]
    const int32_t* fedge;   // [4nf]
    float dlo[3], dhi[3];   // query domain rounded outward to float
};

P2M_HD int depth_of(int32_t node) { return 31 - __builtin_clz((unsigned)(node + 1)); }

P2M_HD int as_int(float f) {
    union {
        float f;
        int i;
    } u;
    u.f = f;
    return u.i;
}

P2M_HD bool finite3(float x, float y, float z) {
    return ((as_int(x) & 0x7f800000) != 0x7f800000) && ((as_int(y) & 0x7f800000) != 0x7f800000) &&
           ((as_int(z) & 0x7f800000) != 0x7f800000);
}

struct Nearest {
    float d2;
    float px, py, pz;
    int32_t vid;
};

P2M_HD double d2_f64(float qx, float qy, float qz, float px, float py, float pz) {
    double dx = (double)qx - (double)px, dy = (double)qy - (double)py, dz = (double)qz - (double)pz;
    return dx * dx + dy * dy + dz * dz;
}

P2M_HD void consider(Nearest& b, float qx, float qy, float qz, float d2, const float4& p) {
    const int32_t vid = as_int(p.w);
    bool take;
    if (d2 < b.d2 * kTieLo) {
        take = true;
    } else if (d2 <= b.d2 * kTieHi) {
        double D = d2_f64(qx, qy, qz, p.x, p.y, p.z);
        double Db = d2_f64(qx, qy, qz, b.px, b.py, b.pz);
        take = D < Db || (D == Db && vid < b.vid);
    } else {
        take = false;
    }
    if (take) {
        b.d2 = d2;
        b.px = p.x;
        b.py = p.y;
        b.pz = p.z;
        b.vid = vid;
    }
}

// Nearest vertex by the implicit KD tree.  `visits` counts node loads.
//
// Node i (children 2i+1, 2i+2) is four float4: its point and vertex id, then
// the bounding boxes of its left and right subtrees (an absent child has an
// empty box: lo = +inf, hi = -inf).  Depth-first search, nearer child box
// first; a subtree is skipped when the squared distance from q to its box
// exceeds the best squared distance by more than 2^-20 relative.
struct KdNode {
    float4 p;   // x, y, z, vertex id bits
    float4 b0;  // left lo.xyz, left hi.x
    float4 b1;  // left hi.yz, right lo.xy
    float4 b2;  // right lo.z, right hi.xyz
};

P2M_HD float box_d2(float qx, float qy, float qz, float lx, float ly, float lz, float hx, float hy, float hz) {
    const float dx = fmaxf(fmaxf(lx - qx, qx - hx), 0.f);
    const float dy = fmaxf(fmaxf(ly - qy, qy - hy), 0.f);
    const float dz = fmaxf(fmaxf(lz - qz, qz - hz), 0.f);
    return dx * dx + dy * dy + dz * dz;
}

P2M_HD Nearest kdt_nearest(const KdNode* __restrict__ node, int32_t n, float qx, float qy, float qz,
                           uint64_t& visits) {
    Nearest b;
    b.d2 = INFINITY;
    b.px = b.py = b.pz = 0.f;
    b.vid = 0x7fffffff;
    int32_t st_node[kMaxDepth];
    float st_d[kMaxDepth];
    int sp = 0;
    int32_t cur = 0;
    while (cur >= 0) {
        while (cur >= 0) {
            const KdNode nd = node[cur];
            ++visits;
            const float dx = qx - nd.p.x, dy = qy - nd.p.y, dz = qz - nd.p.z;
            consider(b, qx, qy, qz, dx * dx + dy * dy + dz * dz, nd.p);
            const float dl = box_d2(qx, qy, qz, nd.b0.x, nd.b0.y, nd.b0.z, nd.b0.w, nd.b1.x, nd.b1.y);
            const float dr = box_d2(qx, qy, qz, nd.b1.z, nd.b1.w, nd.b2.x, nd.b2.y, nd.b2.z, nd.b2.w);
            const bool left_first = dl <= dr;
            const int32_t c0 = 2 * cur + (left_first ? 1 : 2), c1 = 2 * cur + (left_first ? 2 : 1);
            const float d0 = left_first ? dl : dr, d1 = left_first ? dr : dl;
            const float lim = b.d2 * kTieHi;
            if (d1 <= lim && sp < kMaxDepth) {
                st_node[sp] = c1;
                st_d[sp] = d1;
                ++sp;
            }
            cur = d0 <= lim ? c0 : -1;
        }
        while (sp > 0) {
            --sp;
            if (st_d[sp] <= b.d2 * kTieHi) {
                cur = st_node[sp];
                break;
            }
        }
    }
    return b;
}

// Closest point on the closed segment (a,b).  region: 0 inside, 1 at a, 2 at b.
P2M_HD float seg_d2(float qx, float qy, float qz, const float4& a, const float4& b, float& t, int& region) {
    const float ex = b.x - a.x, ey = b.y - a.y, ez = b.z - a.z;
    const float wx = qx - a.x, wy = qy - a.y, wz = qz - a.z;
    const float ee = ex * ex + ey * ey + ez * ez;
    t = (wx * ex + wy * ey + wz * ez) / ee;
    region = 0;
    if (!(t > 0.f)) {
        t = 0.f;
        region = 1;
    } else if (!(t < 1.f)) {
        t = 1.f;
        region = 2;
    }
    const float cx = wx - t * ex, cy = wy - t * ey, cz = wz - t * ez;
    return cx * cx + cy * cy + cz * cz;
}

// Closest point on the closed triangle (a,b,c).
// region: 0 inside; 1,2,3 on side ab, bc, ca; 4,5,6 at corner a, b, c.
// w: barycentric weights of the closest point.
P2M_HD float tri_d2(float qx, float qy, float qz, const float4& a, const float4& b, const float4& c, float w[3],
                    int& region) {
    const float abx = b.x - a.x, aby = b.y - a.y, abz = b.z - a.z;
    const float acx = c.x - a.x, acy = c.y - a.y, acz = c.z - a.z;
    const float nx = aby * acz - abz * acy, ny = abz * acx - abx * acz, nz = abx * acy - aby * acx;
    const float nn = nx * nx + ny * ny + nz * nz;
    const float aqx = qx - a.x, aqy = qy - a.y, aqz = qz - a.z;
    const float bqx = qx - b.x, bqy = qy - b.y, bqz = qz - b.z;
    const float cqx = qx - c.x, cqy = qy - c.y, cqz = qz - c.z;
    // signed areas of the sub-triangles seen along the normal (scaled by nn)
    const float ua = (bqy * cqz - bqz * cqy) * nx + (bqz * cqx - bqx * cqz) * ny + (bqx * cqy - bqy * cqx) * nz;
    const float ub = (cqy * aqz - cqz * aqy) * nx + (cqz * aqx - cqx * aqz) * ny + (cqx * aqy - cqy * aqx) * nz;
    const float uc = (aqy * bqz - aqz * bqy) * nx + (aqz * bqx - aqx * bqz) * ny + (aqx * bqy - aqy * bqx) * nz;
    if (ua >= 0.f && ub >= 0.f && uc >= 0.f) {
        const float h = aqx * nx + aqy * ny + aqz * nz;
        const float inv = 1.f / nn;
        w[0] = ua * inv;
        w[1] = ub * inv;
        w[2] = uc * inv;
        region = 0;
        return h * h * inv;
    }
    float t0, t1, t2;
    int r0, r1, r2;
    const float d0 = seg_d2(qx, qy, qz, a, b, t0, r0);
    const float d1 = seg_d2(qx, qy, qz, b, c, t1, r1);
    const float d2 = seg_d2(qx, qy, qz, c, a, t2, r2);
    float d = d0, t = t0;
    int side = 0, r = r0;
    if (d1 < d) {
        d = d1;
        t = t1;
        side = 1;
        r = r1;
    }
    if (d2 < d) {
        d = d2;
        t = t2;
        side = 2;
        r = r2;
    }
    w[0] = w[1] = w[2] = 0.f;
    const int i0 = side, i1 = (side + 1) % 3;
    if (r == 0) {
        w[i0] = 1.f - t;
        w[i1] = t;
        region = 1 + side;
    } else {
        const int corner = r == 1 ? i0 : i1;
        w[corner] = 1.f;
        region = 4 + corner;
    }
    return d;
}

struct Answer {
    int32_t prim;            // type << 30 | id
    float cx, cy, cz, dist;
    float w[3];
    int32_t pv[3];
};

P2M_HD int32_t make_prim(int kind, int32_t id) { return (int32_t)(((uint32_t)kind << 30) | (uint32_t)id); }

struct ScanCounters {
    uint64_t nodes = 0, edges = 0, faces = 0;
};

// The whole query for one point.
P2M_HD Answer p2m_query_point(const MeshView& m, float qx, float qy, float qz, uint8_t& status, ScanCounters& cnt) {
    Answer a;
    status = 0;
    if (!finite3(qx, qy, qz)) {
        status = 2;
        a.prim = make_prim(KIND_NONE, 0);
        a.cx = a.cy = a.cz = a.dist = NAN;
        a.w[0] = a.w[1] = a.w[2] = 0.f;
        a.pv[0] = a.pv[1] = a.pv[2] = -1;
        return a;
    }
    if (qx < m.dlo[0] || qy < m.dlo[1] || qz < m.dlo[2] || qx > m.dhi[0] || qy > m.dhi[1] || qz > m.dhi[2])
        status = 1;
    const Nearest nv = kdt_nearest(m.node, m.nv, qx, qy, qz, cnt.nodes);
    // running minimum over v and v's list; kind/id/code of the best
    float best = nv.d2;
    int best_kind = KIND_VERTEX;
    int32_t best_id = nv.vid;
    const uint32_t e0 = m.off[2 * nv.vid], f0 = m.off[2 * nv.vid + 1], f1 = m.off[2 * nv.vid + 2];
    for (uint32_t k = e0; k < f0; ++k) {
        const int32_t e = m.ent[k];
        const float4 A = m.seg[2 * e], B = m.seg[2 * e + 1];
        float t;
        int r;
        const float d = seg_d2(qx, qy, qz, A, B, t, r);
        if (d < best) {
            best = d;
            best_kind = KIND_EDGE;
            best_id = e;
        }
    }
    for (uint32_t k = f0; k < f1; ++k) {
        const int32_t f = m.ent[k];
        const float4 A = m.tri[3 * f], B = m.tri[3 * f + 1], C = m.tri[3 * f + 2];
        float w[3];
        int r;
        const float d = tri_d2(qx, qy, qz, A, B, C, w, r);
        if (d < best) {
            best = d;
            best_kind = KIND_FACE;
            best_id = f;
        }
    }
    cnt.edges += f0 - e0;
    cnt.faces += f1 - f0;
    // resolve the winner: closest point, weights, reported primitive
    a.dist = sqrtf(best);
    a.w[0] = 1.f;
    a.w[1] = a.w[2] = 0.f;
    a.pv[1] = a.pv[2] = -1;
    if (best_kind == KIND_VERTEX) {
        a.prim = make_prim(KIND_VERTEX, nv.vid);
        a.cx = nv.px;
        a.cy = nv.py;
        a.cz = nv.pz;
        a.pv[0] = nv.vid;
    } else if (best_kind == KIND_EDGE) {
        const float4 A = m.seg[2 * best_id], B = m.seg[2 * best_id + 1];
        float t;
        int r;
        seg_d2(qx, qy, qz, A, B, t, r);
        a.cx = A.x + t * (B.x - A.x);
        a.cy = A.y + t * (B.y - A.y);
        a.cz = A.z + t * (B.z - A.z);
        if (r == 0) {
            a.prim = make_prim(KIND_EDGE, best_id);
            a.w[0] = 1.f - t;
            a.w[1] = t;
            a.pv[0] = as_int(A.w);
            a.pv[1] = as_int(B.w);
        } else {
            const float4& P = r == 1 ? A : B;
            a.prim = make_prim(KIND_VERTEX, as_int(P.w));
            a.cx = P.x;
            a.cy = P.y;
            a.cz = P.z;
            a.pv[0] = as_int(P.w);
        }
    } else {
        const float4 C3[3] = {m.tri[3 * best_id], m.tri[3 * best_id + 1], m.tri[3 * best_id + 2]};
        float w[3];
        int r;
        tri_d2(qx, qy, qz, C3[0], C3[1], C3[2], w, r);
        a.cx = w[0] * C3[0].x + w[1] * C3[1].x + w[2] * C3[2].x;
        a.cy = w[0] * C3[0].y + w[1] * C3[1].y + w[2] * C3[2].y;
        a.cz = w[0] * C3[0].z + w[1] * C3[1].z + w[2] * C3[2].z;
        if (r == 0) {
            a.prim = make_prim(KIND_FACE, best_id);
            for (int i = 0; i < 3; ++i) {
                a.w[i] = w[i];
                a.pv[i] = as_int(C3[i].w);
            }
        } else if (r <= 3) {
            const int s = r - 1, i0 = s, i1 = (s + 1) % 3;
            a.prim = make_prim(KIND_EDGE, m.fedge[4 * best_id + s]);
            a.w[0] = w[i0];
            a.w[1] = w[i1];
            a.pv[0] = as_int(C3[i0].w);
            a.pv[1] = as_int(C3[i1].w);
        } else {
            const int c = r - 4;
            a.prim = make_prim(KIND_VERTEX, as_int(C3[c].w));
            a.cx = C3[c].x;
            a.cy = C3[c].y;
            a.cz = C3[c].z;
            a.pv[0] = as_int(C3[c].w);
        }
    }
    return a;
}

}  // namespace p2m
