// Per-query arithmetic of the P2M query (Appendix, Algorithm A.2), shared by
// the device kernels and the host CPU baseline (compiled by hipcc only).
//
//  1. nearest vertex v (float32 distances; candidates whose squared
//     distances agree to within 2^-20 relative are decided in float64, then
//     by vertex id): a greedy walk over the Voronoi neighbour graph, or a
//     KD-tree search (subtrees pruned only when their lower bound exceeds
//     the best squared distance by more than 2^-20 relative);
//  2. d_min <- d(q, v);
//  3. scan of v's interception list with the paper's tests: an edge counts
//     only if the foot of q on its line lies on the edge (q in Space-perp(e))
//     and then gives the distance to the line; a face counts only if the
//     foot on its plane lies in the face (q in Space-perp(f)) and gives the
//     plane distance.  Each gate is evaluated from precomputed affine forms
//     (plane, barycentric rows, edge direction) with every boundary moved
//     outward by mu (a 2^-20 fraction of the domain diagonal, several times
//     the float32 error of the forms), so rounding cannot drop the true
//     answer and a primitive passes only if q's foot is within mu of it;
//  4. the winner alone is re-evaluated with the exact closed segment /
//     triangle distance, whose clamp region (inside, on a side, at a corner)
//     names the primitive returned, its closest point and weights.
//     A gated value is the distance to the primitive's plane (a face), or
//     to its line plus the foot's overshoot beyond the nearer end (an edge),
//     never more than the exact distance to the closed primitive and equal
//     to it when q's foot lies on the primitive (always, for an edge).  So
//     when the winner's exact distance does not exceed its own gated value,
//     no other candidate can be closer; otherwise (a face that passed its
//     gate within the margin, its foot just off it) the list is scanned
//     again and every candidate whose gated value is below the best exact
//     distance so far is evaluated exactly.  The answer is then the exact
//     minimum over the candidates, whatever the margin, up to float32
//     rounding and a slack of 2^-20 relative plus eta absolute (eta: 2^-21
//     of the mesh's size).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace p2m {

#define P2M_HD __host__ __device__ __forceinline__

constexpr float kTieLo = 0.99999904632568359375f;  // 1 - 2^-20
constexpr float kTieHi = 1.00000095367431640625f;  // 1 + 2^-20
constexpr int kMaxDepth = 32;
constexpr int kWalkGroup = 8;   // neighbour records loaded per walk group

enum : int { KIND_VERTEX = 0, KIND_EDGE = 1, KIND_FACE = 2, KIND_NONE = 3 };

struct MeshView {
    const struct KdNode* node;  // [nv] KD-tree nodes (point + child boxes)
    int32_t nv;
    // list head of vertex v: vhead[2v] = (first edge entry, first face entry,
    // end, 0); vhead[2v+1] = list box (union of the entry boxes) in D's
    // 16-bit frame: (lo.x | lo.y << 16, lo.z | hi.x << 16, hi.y | hi.z << 16, 0)
    const uint4* vhead;     // [2nv]
    // list entries, two per element: (id, box) with the box in 5 bits per
    // coordinate relative to the list box (lo.x, lo.y, lo.z, hi.x, hi.y,
    // hi.z from bit 0 up); each vertex's edge and face runs start at an even
    // entry and are padded to an even length with empty-box entries
    const uint4* lent;      // [padded nnz / 2]
    const float4* seg;      // [2ne]
    const float4* tri;      // [3nf]
    const int32_t* fedge;   // [4nf]
    // list-scan forms, in coordinates relative to ctr (see step 3 above):
    // face f: frec[3f] = (unit normal, offset), frec[3f+1..3f+2] = forms of
    // two barycentric weights (scaled, offsets moved by mu; the third weight
    // is tested as 1 minus their sum);
    // edge e: erec[2e] = (a - ctr, length), erec[2e+1] = (unit direction, 0)
    const float4* frec;     // [3nf]
    const float4* erec;     // [2ne]
    float ctr[3];           // centre of the domain box, rounded to float
    float mu;               // gate margin
    float eta;              // absolute slack of the winner check (step 4)
    float qlo[3], qs[3];    // 16-bit frame of D for the entry boxes
    float dlo[3], dhi[3];   // query domain rounded outward to float
    // Voronoi-neighbour walk (optional; null when absent)
    const uint32_t* nboff;  // [nv+1] Voronoi neighbours of each vertex, CSR
    const float4* nbrec;    // [nnz] neighbour position, id bits in .w
    const float4* seed;     // [grid^3] nearest vertex of each grid-cell centre (position, id bits)
    int32_t grid;
    float glo[3], gscale[3];  // cell = floor((q - glo) * gscale), clamped
    // finer seed grid over the mesh's box, grown (grid2 = 0: none), for the
    // queries inside it when D is much larger than the mesh
    const float4* seed2;
    int32_t grid2;
    float glo2[3], gscale2[3], ghi2[3];
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
    if (b.vid < 0) {
        take = true;  // first candidate
    } else if (d2 < b.d2 * kTieLo) {
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

// consider() when b already holds a candidate (b.vid >= 0); an infinite d2
// is never taken.
P2M_HD void consider_known(Nearest& b, float qx, float qy, float qz, float d2, const float4& p) {
    bool take;
    if (d2 < b.d2 * kTieLo) {
        take = true;
    } else if (d2 <= b.d2 * kTieHi) {
        const int32_t vid = as_int(p.w);
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
        b.vid = as_int(p.w);
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

// fetch(i) returns node i (from memory, or from a copy of the top levels).
template <class Fetch>
P2M_HD Nearest kdt_nearest_f(Fetch fetch, int32_t n, float qx, float qy, float qz, uint64_t& visits) {
    Nearest b;
    b.d2 = INFINITY;
    b.px = b.py = b.pz = 0.f;
    b.vid = -1;
    int32_t st_node[kMaxDepth];
    float st_d[kMaxDepth];
    int sp = 0;
    int32_t cur = 0;
    while (cur >= 0) {
        while (cur >= 0) {
            const KdNode nd = fetch(cur);
            ++visits;
            const float dx = qx - nd.p.x, dy = qy - nd.p.y, dz = qz - nd.p.z;
            consider(b, qx, qy, qz, dx * dx + dy * dy + dz * dz, nd.p);
            const float dl = box_d2(qx, qy, qz, nd.b0.x, nd.b0.y, nd.b0.z, nd.b0.w, nd.b1.x, nd.b1.y);
            const float dr = box_d2(qx, qy, qz, nd.b1.z, nd.b1.w, nd.b2.x, nd.b2.y, nd.b2.z, nd.b2.w);
            const bool left_first = dl <= dr;
            const int32_t c0 = 2 * cur + (left_first ? 1 : 2), c1 = 2 * cur + (left_first ? 2 : 1);
            const float d0 = left_first ? dl : dr, d1 = left_first ? dr : dl;
            const float lim = b.d2 * kTieHi;
            if (c1 < n && d1 <= lim && sp < kMaxDepth) {
                st_node[sp] = c1;
                st_d[sp] = d1;
                ++sp;
            }
            cur = (c0 < n && d0 <= lim) ? c0 : -1;
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

P2M_HD Nearest kdt_nearest(const KdNode* __restrict__ node, int32_t n, float qx, float qy, float qz,
                           uint64_t& visits) {
    return kdt_nearest_f([node](int32_t i) { return node[i]; }, n, qx, qy, qz, visits);
}

// Nearest vertex by a greedy walk over the Voronoi (Delaunay) neighbour
// graph of the vertices -- the graph the flooding inspection walks
// (Algorithm 1).  Start at the nearest vertex of q's grid cell centre and
// move to the best of the current vertex's neighbours while one is better
// (same float32 + float64-tie comparison as the tree search).  For q inside
// the query domain the walk stops only at the nearest vertex: if q is
// outside Cell(v), it violates the bisector half-space of some Voronoi
// neighbour of v, which is then closer.  The order is strict, so the walk
// cannot cycle; `cap` bounds it regardless.
P2M_HD Nearest voronoi_walk(const MeshView& m, float qx, float qy, float qz, uint64_t& visits, uint64_t& steps) {
    // the finer grid when q is inside its box (the walk is exact from any seed)
    const bool fine = m.grid2 > 0 && qx >= m.glo2[0] && qx < m.ghi2[0] && qy >= m.glo2[1] && qy < m.ghi2[1] &&
                      qz >= m.glo2[2] && qz < m.ghi2[2];
    const int32_t G = fine ? m.grid2 : m.grid;
    auto cell = [&](float x, float lo, float s) {
        const float t = (x - lo) * s;
        return t >= 0.f ? (t < (float)G ? (int32_t)t : G - 1) : 0;
    };
    const int32_t c = (cell(qz, fine ? m.glo2[2] : m.glo[2], fine ? m.gscale2[2] : m.gscale[2]) * G +
                       cell(qy, fine ? m.glo2[1] : m.glo[1], fine ? m.gscale2[1] : m.gscale[1])) * G +
                      cell(qx, fine ? m.glo2[0] : m.glo[0], fine ? m.gscale2[0] : m.gscale[0]);
    Nearest b;
    b.d2 = INFINITY;
    b.px = b.py = b.pz = 0.f;
    b.vid = -1;
    float4 p = (fine ? m.seed2 : m.seed)[c];
    {
        const float dx = qx - p.x, dy = qy - p.y, dz = qz - p.z;
        consider(b, qx, qy, qz, dx * dx + dy * dy + dz * dz, p);
    }
    const int cap = 1 << 16;
    for (int it = 0; it < cap; ++it) {
        const int32_t v = b.vid;
        ++steps;
        const uint32_t k0 = m.nboff[v], k1 = m.nboff[v + 1];
        // kWalkGroup consecutive neighbour records loaded before any is
        // compared (the record array is padded at its end, so the loads stay
        // in bounds); slots past the list's end do not count
        for (uint32_t k = k0; k < k1; k += kWalkGroup) {
            float4 r[kWalkGroup];
            const float4* g = m.nbrec + k;
#pragma unroll
            for (int u = 0; u < kWalkGroup; ++u) r[u] = g[u];
#pragma unroll
            for (int u = 0; u < kWalkGroup; ++u) {
                const float dx = qx - r[u].x, dy = qy - r[u].y, dz = qz - r[u].z;
                const float d2 = k + u < k1 ? dx * dx + dy * dy + dz * dz : INFINITY;
                consider_known(b, qx, qy, qz, d2, r[u]);
            }
            visits += k1 - k < (uint32_t)kWalkGroup ? k1 - k : (uint32_t)kWalkGroup;
        }
        if (b.vid == v) break;
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

struct SegHit {
    float d2, t;
    int region;
};

P2M_HD SegHit seg_hit(float qx, float qy, float qz, const float4& a, const float4& b) {
    SegHit h;
    h.d2 = seg_d2(qx, qy, qz, a, b, h.t, h.region);
    return h;
}

// Closest point on the closed triangle (a,b,c).
// region: 0 inside; 1,2,3 on side ab, bc, ca; 4,5,6 at corner a, b, c.
// w: barycentric weights of the closest point; (cx,cy,cz): the point.
// The foot of q on the plane is formed first and the inside test and weights
// use short vectors from the foot to the corners: the same signs as with q
// (the difference is along the normal) without the cancellation of long,
// nearly parallel vectors from a far query.
P2M_HD float tri_d2(float qx, float qy, float qz, const float4& a, const float4& b, const float4& c, float& w0,
                    float& w1, float& w2, int& region, float& cx, float& cy, float& cz) {
    const float abx = b.x - a.x, aby = b.y - a.y, abz = b.z - a.z;
    const float acx = c.x - a.x, acy = c.y - a.y, acz = c.z - a.z;
    const float nx = aby * acz - abz * acy, ny = abz * acx - abx * acz, nz = abx * acy - aby * acx;
    const float nn = nx * nx + ny * ny + nz * nz;
    const float inv = 1.f / nn;
    const float h = (qx - a.x) * nx + (qy - a.y) * ny + (qz - a.z) * nz;
    const float s = h * inv;
    const float px = qx - s * nx, py = qy - s * ny, pz = qz - s * nz;  // foot on the plane
    const float pax = a.x - px, pay = a.y - py, paz = a.z - pz;
    const float pbx = b.x - px, pby = b.y - py, pbz = b.z - pz;
    const float pcx = c.x - px, pcy = c.y - py, pcz = c.z - pz;
    // signed areas of the sub-triangles seen along the normal (scaled by nn)
    const float ua = (pby * pcz - pbz * pcy) * nx + (pbz * pcx - pbx * pcz) * ny + (pbx * pcy - pby * pcx) * nz;
    const float ub = (pcy * paz - pcz * pay) * nx + (pcz * pax - pcx * paz) * ny + (pcx * pay - pcy * pax) * nz;
    const float uc = (pay * pbz - paz * pby) * nx + (paz * pbx - pax * pbz) * ny + (pax * pby - pay * pbx) * nz;
    if (ua >= 0.f && ub >= 0.f && uc >= 0.f) {
        w0 = ua * inv;
        w1 = ub * inv;
        w2 = uc * inv;
        region = 0;
        cx = px;
        cy = py;
        cz = pz;
        return h * s;
    }
    const SegHit h0 = seg_hit(qx, qy, qz, a, b);
    const SegHit h1 = seg_hit(qx, qy, qz, b, c);
    const SegHit h2 = seg_hit(qx, qy, qz, c, a);
    const bool s1 = h1.d2 < h0.d2;
    const float d01 = s1 ? h1.d2 : h0.d2;
    const bool s2 = h2.d2 < d01;
    const float d = s2 ? h2.d2 : d01;
    const float t = s2 ? h2.t : (s1 ? h1.t : h0.t);
    const int r = s2 ? h2.region : (s1 ? h1.region : h0.region);
    const int side = s2 ? 2 : (s1 ? 1 : 0);
    // side s runs from corner s to corner s+1 (mod 3); no run-time array
    // indexing here, so everything stays in registers
    const float Ax = side == 0 ? a.x : (side == 1 ? b.x : c.x), Bx = side == 0 ? b.x : (side == 1 ? c.x : a.x);
    const float Ay = side == 0 ? a.y : (side == 1 ? b.y : c.y), By = side == 0 ? b.y : (side == 1 ? c.y : a.y);
    const float Az = side == 0 ? a.z : (side == 1 ? b.z : c.z), Bz = side == 0 ? b.z : (side == 1 ? c.z : a.z);
    cx = Ax + t * (Bx - Ax);
    cy = Ay + t * (By - Ay);
    cz = Az + t * (Bz - Az);
    float wa = 1.f - t, wb = t;  // weights of A and B
    if (r == 1) {
        wa = 1.f;
        wb = 0.f;
    } else if (r == 2) {
        wa = 0.f;
        wb = 1.f;
    }
    w0 = side == 0 ? wa : (side == 2 ? wb : 0.f);
    w1 = side == 1 ? wa : (side == 0 ? wb : 0.f);
    w2 = side == 2 ? wa : (side == 1 ? wb : 0.f);
    const int corner = r == 1 ? side : (side == 2 ? 0 : side + 1);
    region = r == 0 ? 1 + side : 4 + corner;
    return d;
}

// Whether the foot of q on the plane of (a,b,c) lies in the closed triangle:
// each side's edge-normal test signed against the face normal (the foot
// itself is not formed: q - foot is along the normal).
// tri_dist2: squared distance from q to the closed triangle alone, with few
// registers (for the rare margin cases): the plane distance when the foot
// lies in the triangle, else the nearest side's segment distance.  Near a
// side both give nearly the same value, so a rounding slip of the inside
// test costs only rounding.
P2M_HD bool foot_in_triangle(float qx, float qy, float qz, const float4& a, const float4& b, const float4& c) {
    const float abx = b.x - a.x, aby = b.y - a.y, abz = b.z - a.z;
    const float acx = c.x - a.x, acy = c.y - a.y, acz = c.z - a.z;
    const float nx = aby * acz - abz * acy, ny = abz * acx - abx * acz, nz = abx * acy - aby * acx;
    auto side = [&](const float4& u, const float4& w) {
        const float ex = w.x - u.x, ey = w.y - u.y, ez = w.z - u.z;
        const float px = qx - u.x, py = qy - u.y, pz = qz - u.z;
        return (ey * pz - ez * py) * nx + (ez * px - ex * pz) * ny + (ex * py - ey * px) * nz >= 0.f;
    };
    return side(a, b) && side(b, c) && side(c, a);
}

P2M_HD float tri_dist2(float qx, float qy, float qz, const float4& a, const float4& b, const float4& c) {
    if (foot_in_triangle(qx, qy, qz, a, b, c)) {
        const float abx = b.x - a.x, aby = b.y - a.y, abz = b.z - a.z;
        const float acx = c.x - a.x, acy = c.y - a.y, acz = c.z - a.z;
        const float nx = aby * acz - abz * acy, ny = abz * acx - abx * acz, nz = abx * acy - aby * acx;
        const float h = (qx - a.x) * nx + (qy - a.y) * ny + (qz - a.z) * nz;
        return h * (h / (nx * nx + ny * ny + nz * nz));
    }
    float t;
    int r;
    return fminf(fminf(seg_d2(qx, qy, qz, a, b, t, r), seg_d2(qx, qy, qz, b, c, t, r)), seg_d2(qx, qy, qz, c, a, t, r));
}

struct Answer {
    int32_t prim;            // type << 30 | id
    float cx, cy, cz, dist;
    // the closest point as staged (staged_point): the point itself for a
    // vertex (or no primitive), else the vector from q to the point
    float sx, sy, sz;
    float w[3];
    int32_t pv[3];
};

P2M_HD int32_t make_prim(int kind, int32_t id) { return (int32_t)(((uint32_t)kind << 30) | (uint32_t)id); }

struct ScanCounters {
    uint64_t nodes = 0, edges = 0, faces = 0, steps = 0;  // nodes: nearest-vertex candidates
    uint64_t edge_forms = 0, face_forms = 0;              // entries whose box held q
    uint64_t rescans = 0, rescan_exact = 0;               // second scans; exact evaluations in them
};

// |q - c|, each operation rounded on its own (no fused multiply-add), so
// that every kernel that forms a reported distance -- the query kernels and
// the write-outs that rebuild it from a staged answer (staged_point) --
// gives the same bits.
P2M_HD float point_dist(float qx, float qy, float qz, float cx, float cy, float cz) {
#if defined(__clang__)
#pragma clang fp contract(off)
#endif
    const float dx = qx - cx, dy = qy - cy, dz = qz - cz;
    const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    return sqrtf((xx + yy) + zz);
}

// The reported closest point c and distance d of an answer from its staged
// form s.  A vertex is reported exactly (c = s) and d = |q - c|.  An edge's
// or face's point is formed relative to the domain centre, where the
// coordinates are small even for a mesh far from the origin, and staged as
// the vector s from q to it: c = q + s (rounded once, as float32 output must
// be) and d = |s|, which keeps the distance to the accuracy of the
// arithmetic instead of the rounding of c's absolute coordinates.  The query
// kernels and the write-outs that rebuild c and d from a staged (prim, s)
// call this one function, so all give the same bits.
P2M_HD void staged_point(int32_t prim, float sx, float sy, float sz, float qx, float qy, float qz, float& cx,
                         float& cy, float& cz, float& dist) {
#if defined(__clang__)
#pragma clang fp contract(off)
#endif
    const uint32_t kind = (uint32_t)prim >> 30;
    if (kind == (uint32_t)KIND_EDGE || kind == (uint32_t)KIND_FACE) {
        cx = qx + sx;
        cy = qy + sy;
        cz = qz + sz;
        dist = point_dist(sx, sy, sz, 0.f, 0.f, 0.f);
    } else {
        cx = sx;
        cy = sy;
        cz = sz;
        dist = point_dist(qx, qy, qz, sx, sy, sz);
    }
}

P2M_HD Answer nonfinite_answer() {
    Answer a;
    a.prim = make_prim(KIND_NONE, 0);
    a.cx = a.cy = a.cz = a.dist = NAN;
    a.sx = a.sy = a.sz = NAN;
    a.w[0] = a.w[1] = a.w[2] = 0.f;
    a.pv[0] = a.pv[1] = a.pv[2] = -1;
    return a;
}

P2M_HD uint8_t domain_status(const MeshView& m, float qx, float qy, float qz) {
    return (qx < m.dlo[0] || qy < m.dlo[1] || qz < m.dlo[2] || qx > m.dhi[0] || qy > m.dhi[1] || qz > m.dhi[2]) ? 1 : 0;
}

// Steps 2-3 given the nearest vertex: list scan and the resolved answer.
// Gated squared distance to edge e (infinite when q's foot is more than mu
// beyond an end): the squared distance to its line plus the square of the
// foot's overshoot beyond the nearer end, i.e. the squared distance to the
// closed segment for a foot within the margin; r* = q - ctr.
P2M_HD float edge_gate_d2(const MeshView& m, int32_t e, float rx, float ry, float rz) {
    const float4 A = m.erec[2 * e], U = m.erec[2 * e + 1];
    const float wx = rx - A.x, wy = ry - A.y, wz = rz - A.z;
    const float t = wx * U.x + wy * U.y + wz * U.z;
    const float cx = wx - t * U.x, cy = wy - t * U.y, cz = wz - t * U.z;
    const float o = fmaxf(fmaxf(-t, t - A.w), 0.f);
    const float d = cx * cx + cy * cy + cz * cz + o * o;
    const bool in = (t >= -m.mu) & (t <= A.w + m.mu);  // no short-circuit: branch-free
    return in ? d : INFINITY;
}

// Gated squared distance to the plane of face f (infinite when q's foot is
// more than mu outside the face).
P2M_HD float face_gate_d2(const MeshView& m, int32_t f, float rx, float ry, float rz) {
    const float4 N = m.frec[3 * f], L1 = m.frec[3 * f + 1], L2 = m.frec[3 * f + 2];
    const float h = N.x * rx + N.y * ry + N.z * rz - N.w;
    const float l1 = L1.x * rx + L1.y * ry + L1.z * rz - L1.w;
    const float l2 = L2.x * rx + L2.y * ry + L2.z * rz - L2.w;
    const bool in = (l1 >= 0.f) & (l2 >= 0.f) & (l1 + l2 <= 1.f);
    return in ? h * h : INFINITY;
}

// Integer bounds of q in the list box's 5-bit frame: for integer box
// bounds, lo <= s exactly when lo <= floor(s), and s <= hi exactly when
// ceil(s) <= hi, so the integer test equals the real one.  Kept packed as
// an entry box is: f = the floors at bits 0, 5, 10; c = the ceilings at
// bits 15, 20, 25.
struct Cell5 {
    uint32_t f, c;
};

P2M_HD Cell5 cell5(float sx, float sy, float sz) {
    Cell5 c;
    c.f = (uint32_t)floorf(sx) | (uint32_t)floorf(sy) << 5 | (uint32_t)floorf(sz) << 10;
    c.c = ((uint32_t)ceilf(sx) | (uint32_t)ceilf(sy) << 5 | (uint32_t)ceilf(sz) << 10) << 15;
    return c;
}

// lo <= floor and hi >= ceil on all three axes, the six 5-bit fields
// compared at once: X = (floors, box highs) and Y = (box lows, ceilings)
// field by field; a field's low four bits are compared by a subtraction
// that cannot borrow across fields (X's top bit set, Y's cleared), and the
// top bits decide where they differ.
P2M_HD bool in_box5(uint32_t b, const Cell5& q) {
    constexpr uint32_t kHigh = 0x3FFF8000u;  // bits 15..29: the box's upper corner
    constexpr uint32_t kTop = 0x21084210u;   // the top bit of each 5-bit field
    const uint32_t X = (b & kHigh) | q.f, Y = (b & ~kHigh) | q.c;
    const uint32_t d = (X | kTop) - (Y & ~kTop);
    const uint32_t diff = X ^ Y;
    const uint32_t ge = (diff & X) | (~diff & d);
    return (ge & kTop) == kTop;
}

// Coordinate of q in the 5-bit frame of a list box side [lo, hi] (16-bit
// units of D), clamped to [0, 31].  Inside the list box the entry boxes
// keep a 16-bit unit of margin beyond their polytopes, far above the
// rounding of this rescale, except where both the box and q were clamped
// to D's edge; the clamp here keeps that case exact.  A q outside the list
// box is moved onto it, which can only let more entries through.
P2M_HD float frame5(float u, uint32_t lo, uint32_t hi) {
    const float span = (float)(hi > lo ? hi - lo : 1u);
    return fminf(fmaxf((u - (float)lo) * (31.f / span), 0.f), 31.f);
}

// Exact evaluation of candidate (kind, id) of the scan: fills a (reported
// primitive from the clamp region, closest point, weights and vertex ids)
// and returns the exact squared distance to the closed segment / triangle
// (a vertex candidate is the nearest vertex nv).
P2M_HD float resolve(const MeshView& m, float qx, float qy, float qz, const Nearest& nv, int kind, int32_t id,
                     Answer& a) {
    float exact = nv.d2;
    a.w[0] = 1.f;
    a.w[1] = a.w[2] = 0.f;
    a.pv[1] = a.pv[2] = -1;
    // edges and faces are evaluated relative to the domain centre (see
    // staged_point); a vertex is staged as itself
    const float ox = m.ctr[0], oy = m.ctr[1], oz = m.ctr[2];
    auto rel = [&](const float4& p) { return make_float4(p.x - ox, p.y - oy, p.z - oz, p.w); };
    const float rx = qx - ox, ry = qy - oy, rz = qz - oz;
    if (kind == KIND_VERTEX) {
        a.prim = make_prim(KIND_VERTEX, nv.vid);
        a.sx = nv.px;
        a.sy = nv.py;
        a.sz = nv.pz;
        a.pv[0] = nv.vid;
    } else if (kind == KIND_EDGE) {
        const float4 Ar = rel(m.seg[2 * id]), Br = rel(m.seg[2 * id + 1]);
        float t;
        int r;
        exact = seg_d2(rx, ry, rz, Ar, Br, t, r);
        if (r == 0) {
            a.prim = make_prim(KIND_EDGE, id);
            a.sx = (Ar.x + t * (Br.x - Ar.x)) - rx;
            a.sy = (Ar.y + t * (Br.y - Ar.y)) - ry;
            a.sz = (Ar.z + t * (Br.z - Ar.z)) - rz;
            a.w[0] = 1.f - t;
            a.w[1] = t;
            a.pv[0] = as_int(Ar.w);
            a.pv[1] = as_int(Br.w);
        } else {
            // an end point: reported exactly, read again
            const float4 P = m.seg[2 * id + (r == 1 ? 0 : 1)];
            a.prim = make_prim(KIND_VERTEX, as_int(P.w));
            a.sx = P.x;
            a.sy = P.y;
            a.sz = P.z;
            a.pv[0] = as_int(P.w);
        }
    } else {
        const float4 Ar = rel(m.tri[3 * id]), Br = rel(m.tri[3 * id + 1]), Cr = rel(m.tri[3 * id + 2]);
        float w0, w1, w2;
        int r;
        exact = tri_d2(rx, ry, rz, Ar, Br, Cr, w0, w1, w2, r, a.sx, a.sy, a.sz);
        a.sx -= rx;
        a.sy -= ry;
        a.sz -= rz;
        const int32_t ia = as_int(Ar.w), ib = as_int(Br.w), ic = as_int(Cr.w);
        if (r == 0) {
            a.prim = make_prim(KIND_FACE, id);
            a.w[0] = w0;
            a.w[1] = w1;
            a.w[2] = w2;
            a.pv[0] = ia;
            a.pv[1] = ib;
            a.pv[2] = ic;
        } else if (r <= 3) {
            const int side = r - 1;  // from corner side to corner side+1
            a.prim = make_prim(KIND_EDGE, m.fedge[4 * id + side]);
            a.w[0] = side == 0 ? w0 : (side == 1 ? w1 : w2);
            a.w[1] = side == 0 ? w1 : (side == 1 ? w2 : w0);
            a.pv[0] = side == 0 ? ia : (side == 1 ? ib : ic);
            a.pv[1] = side == 0 ? ib : (side == 1 ? ic : ia);
        } else {
            // a corner: reported exactly, read again
            const float4 P = m.tri[3 * id + (r - 4)];
            a.prim = make_prim(KIND_VERTEX, as_int(P.w));
            a.sx = P.x;
            a.sy = P.y;
            a.sz = P.z;
            a.pv[0] = as_int(P.w);
        }
    }
    return exact;
}

// q in the 5-bit frame of v's list box (h1 = vhead[2v+1]): q in the 16-bit
// frame of D, clamped to it (a query outside D is answered as an upper
// bound), then rescaled to the list box.
P2M_HD Cell5 list_cell(const MeshView& m, float qx, float qy, float qz, const uint4& h1) {
    const float ux = fminf(fmaxf((qx - m.qlo[0]) * m.qs[0], 0.f), 65535.f);
    const float uy = fminf(fmaxf((qy - m.qlo[1]) * m.qs[1], 0.f), 65535.f);
    const float uz = fminf(fmaxf((qz - m.qlo[2]) * m.qs[2], 0.f), 65535.f);
    return cell5(frame5(ux, h1.x & 0xffffu, h1.y >> 16), frame5(uy, h1.x >> 16, h1.z & 0xffffu),
                 frame5(uz, h1.y & 0xffffu, h1.z >> 16));
}

// Second scan of list(v), taken only when the winner of the gated ranking
// is not provably the closest (step 4): every candidate (box holds q, gate
// passes) whose gated value is below the best exact squared distance so far
// is evaluated exactly; (cur, kind, id) hold that best on entry and on exit.
// The list head and q's frame are read again here rather than kept live
// through the scan (fewer registers for the common path).
P2M_HD void rescan(const MeshView& m, float qx, float qy, float qz, int32_t v, float& cur, int& kind, int32_t& id,
                   ScanCounters& cnt) {
    const uint4 h0 = m.vhead[2 * v], h1 = m.vhead[2 * v + 1];
    const Cell5 qc = list_cell(m, qx, qy, qz, h1);
    const float rx = qx - m.ctr[0], ry = qy - m.ctr[1], rz = qz - m.ctr[2];
#pragma unroll 1
    for (uint32_t k = h0.x; k < h0.y; ++k) {
        const uint4 A = m.lent[k >> 1];
        const uint32_t pid = (k & 1u) ? A.z : A.x, box = (k & 1u) ? A.w : A.y;
        if (!in_box5(box, qc) || !(edge_gate_d2(m, (int32_t)pid, rx, ry, rz) < cur)) continue;
        ++cnt.rescan_exact;
        float t;
        int r;
        const float ex = seg_d2(qx, qy, qz, m.seg[2 * pid], m.seg[2 * pid + 1], t, r);
        if (ex < cur) {
            cur = ex;
            kind = KIND_EDGE;
            id = (int32_t)pid;
        }
    }
#pragma unroll 1
    for (uint32_t k = h0.y; k < h0.z; ++k) {
        const uint4 A = m.lent[k >> 1];
        const uint32_t pid = (k & 1u) ? A.z : A.x, box = (k & 1u) ? A.w : A.y;
        if (!in_box5(box, qc) || !(face_gate_d2(m, (int32_t)pid, rx, ry, rz) < cur)) continue;
        ++cnt.rescan_exact;
        const float ex = tri_dist2(qx, qy, qz, m.tri[3 * pid], m.tri[3 * pid + 1], m.tri[3 * pid + 2]);
        if (ex < cur) {
            cur = ex;
            kind = KIND_FACE;
            id = (int32_t)pid;
        }
    }
}

constexpr float kAcceptRel = 1.00000095367431640625f;  // 1 + 2^-20

// Step 3, one query at a time: the running minimum of the gated values
// over v and v's list, in list order (edges, then faces, ids ascending
// within each run), a later candidate replacing the best only when
// strictly smaller -- so the winner is the least (value, kind, id), vertex
// before edge before face, as the wavefront scan of the kernels finds it.
P2M_HD void scan_list(const MeshView& m, float qx, float qy, float qz, const Nearest& nv, float& best,
                      int& best_kind, int32_t& best_id, ScanCounters& cnt) {
    best = nv.d2;
    best_kind = KIND_VERTEX;
    best_id = nv.vid;
    const float rx = qx - m.ctr[0], ry = qy - m.ctr[1], rz = qz - m.ctr[2];
    const uint4 h0 = m.vhead[2 * nv.vid], h1 = m.vhead[2 * nv.vid + 1];
    const uint32_t e0 = h0.x, f0 = h0.y, f1 = h0.z;
    // Entry boxes first (Sec. 4.6): an entry whose box does not hold q is
    // skipped without reading its forms.
    const Cell5 qc = list_cell(m, qx, qy, qz, h1);
    // Four entries (two 16-byte loads) per step: all their boxes, then the
    // forms of those whose box holds q, are loaded before any is evaluated,
    // so a lane keeps several independent loads in flight.  Runs have even
    // length; a second load past the run's end re-reads the first and its
    // slots are discarded.
    for (uint32_t k = e0; k < f0; k += 4) {
        const uint4 A = m.lent[k >> 1], B = m.lent[(k + 2 < f0 ? k + 2 : k) >> 1];
        const uint32_t id[4] = {A.x, A.z, B.x, B.z}, bx[4] = {A.y, A.w, B.y, B.w};
        float d[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool hit = k + u < f0 && in_box5(bx[u], qc);
            cnt.edge_forms += hit;
            d[u] = hit ? edge_gate_d2(m, (int32_t)id[u], rx, ry, rz) : INFINITY;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (d[u] < best) {
                best = d[u];
                best_kind = KIND_EDGE;
                best_id = (int32_t)id[u];
            }
        }
    }
    for (uint32_t k = f0; k < f1; k += 4) {
        const uint4 A = m.lent[k >> 1], B = m.lent[(k + 2 < f1 ? k + 2 : k) >> 1];
        const uint32_t id[4] = {A.x, A.z, B.x, B.z}, bx[4] = {A.y, A.w, B.y, B.w};
        float d[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool hit = k + u < f1 && in_box5(bx[u], qc);
            cnt.face_forms += hit;
            d[u] = hit ? face_gate_d2(m, (int32_t)id[u], rx, ry, rz) : INFINITY;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (d[u] < best) {
                best = d[u];
                best_kind = KIND_FACE;
                best_id = (int32_t)id[u];
            }
        }
    }
    cnt.edges += f0 - e0;
    cnt.faces += f1 - f0;
}

// Step 4 given the scan's winner (value best, kind, id): the winner checked
// against its own gated value (second scan if needed) and resolved.
P2M_HD Answer finish_answer(const MeshView& m, float qx, float qy, float qz, const Nearest& nv, float best,
                            int best_kind, int32_t best_id, ScanCounters& cnt) {
    Answer a;
    // The winner of the gated ranking is the closest when its exact distance
    // is within the slack of its own gated value: that value is at most
    // every other candidate's gated value, itself at most that candidate's
    // exact distance.  An edge's gated value is its exact distance (the
    // overshoot term), and so is a face's when q's foot lies in the face.
    // Only a face that passed its gate with its foot just off it (within the
    // margin) can fail the test; then a second scan decides.  Then the
    // winner is resolved exactly: distance, closest point, weights and the
    // reported primitive from the closed segment / triangle.
    if (best_kind == KIND_FACE) {
        const float4 A = m.tri[3 * best_id], B = m.tri[3 * best_id + 1], C = m.tri[3 * best_id + 2];
        if (!foot_in_triangle(qx, qy, qz, A, B, C)) {
            const float ex = tri_dist2(qx, qy, qz, A, B, C);
            const float lim = sqrtf(best) * kAcceptRel + m.eta;
            if (!(ex <= lim * lim)) {
                ++cnt.rescans;
                float cur = ex;
                if (nv.d2 < cur) {
                    cur = nv.d2;
                    best_kind = KIND_VERTEX;
                    best_id = nv.vid;
                }
                rescan(m, qx, qy, qz, nv.vid, cur, best_kind, best_id, cnt);
            }
        }
    }
    const float exact = resolve(m, qx, qy, qz, nv, best_kind, best_id, a);
    // a primitive whose exact distance exceeds d(q, v) gives way to v
    if (best_kind != KIND_VERTEX && !(exact <= nv.d2)) {
        a.prim = make_prim(KIND_VERTEX, nv.vid);
        a.sx = nv.px;
        a.sy = nv.py;
        a.sz = nv.pz;
        a.w[0] = 1.f;
        a.w[1] = a.w[2] = 0.f;
        a.pv[0] = nv.vid;
        a.pv[1] = a.pv[2] = -1;
    }
    // the exact squared distance decided the answer; the reported point and
    // distance come from its staged form (report_answer)
    return a;
}


// The reported closest point and distance of an answer from finish_answer
// (staged_point on its staged form).
P2M_HD void report_answer(const MeshView& m, float qx, float qy, float qz, Answer& a) {
    staged_point(a.prim, a.sx, a.sy, a.sz, qx, qy, qz, a.cx, a.cy, a.cz, a.dist);
}

P2M_HD Answer p2m_answer(const MeshView& m, float qx, float qy, float qz, const Nearest& nv, ScanCounters& cnt) {
    float best;
    int best_kind;
    int32_t best_id;
    scan_list(m, qx, qy, qz, nv, best, best_kind, best_id, cnt);
    Answer a = finish_answer(m, qx, qy, qz, nv, best, best_kind, best_id, cnt);
    report_answer(m, qx, qy, qz, a);
    return a;
}

// The whole query for one point (per-lane KD-tree search).
P2M_HD Answer p2m_query_point(const MeshView& m, float qx, float qy, float qz, uint8_t& status, ScanCounters& cnt) {
    if (!finite3(qx, qy, qz)) {
        status = 2;
        return nonfinite_answer();
    }
    status = domain_status(m, qx, qy, qz);
    const Nearest nv = status == 0 && m.seed ? voronoi_walk(m, qx, qy, qz, cnt.nodes, cnt.steps)
                                             : kdt_nearest(m.node, m.nv, qx, qy, qz, cnt.nodes);
    return p2m_answer(m, qx, qy, qz, nv, cnt);
}

}  // namespace p2m
