// Device preprocessing: the Voronoi cell of every vertex (from its Delaunay
// neighbours), then the convexity filter (Theorems 5 and 6) and flooding
// (Algorithm 1) of every primitive, one vertex or primitive per wavefront.
//
// The arithmetic is the host builder's, operation for operation, in FP64,
// and this file is compiled without contraction (no fused multiply-adds), so
// every plane test, corner and box comes out bit for bit as on the host and
// the table is the host's.  The polytope is kept in the same dual form (a
// corner is a triangle of plane ids, counter-clockwise from outside); a cut
// removes the corners outside the plane and closes the hole with one new
// corner per boundary edge.  What a cut does depends only on the set of
// corners, not on their order, so the corners can be stored in any order:
// here corner t sits in lane t of the wavefront (at most 64), with the
// corners across its three edges kept explicitly, so a cut is a few
// wave-wide steps -- one plane test per lane, a ballot, the boundary read off
// the adjacency -- and the flood's queue and visited set live in LDS.  A
// primitive whose polytope outgrows 64 corners or whose flood outgrows the
// queue is handed back to the host, which floods it itself.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>

#include "flood_device.hpp"

namespace p2m {

namespace {

constexpr int kPlaneCap = 128; // planes of a polytope (ids fit in 8 bits)
constexpr int kWaveCorners = 64;  // corners of a polytope: one per lane
constexpr int kQueueCap = 512; // vertices one flood may visit
constexpr int kHashCap = 1024; // open-addressing set over them (power of two)
// A cell built on the device sits in its vertex's fixed slot: at most
// kSlotPlanes planes (n, off; the 6 box planes and one per neighbour) and
// kSlotCorners corners.  Cells built on the host, of any size, sit in a
// second allocation; a vertex's plane and corner offsets (in planes and in
// corners) are negative there: -(offset + 1).
constexpr int kSlotPlanes = 72;
constexpr int kSlotCorners = 64;

enum { UNCHANGED = 0, CLIPPED = 1, EMPTY = 2, SKIPPED = 3, OVERFLOW = 4 };

__device__ __forceinline__ double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
__device__ __forceinline__ void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// Plane ids 0..5 are the faces of D grown by tau: 2k keeps x_k >= blo_k,
// 2k+1 keeps x_k <= bhi_k.  Higher ids name their source in `src`: below 8
// a half-space of Space-perp(p), else plane (src - 8) of the current cell.
struct PlaneSrc {
    const double* blo;
    const double* bhi;
    const double* perp;   // 4 doubles per half-space of p
    const double* cellp;  // 4 doubles per plane of the current cell
    bool lds = false;     // the cell's planes are in LDS instead (cell construction)
};

__device__ __forceinline__ void plane_get(const PlaneSrc& S, const uint8_t* src, int id, double n[3], double& off) {
    if (id < 6) {
        const int k = id >> 1;
        const bool up = id & 1;
        const double sgn = up ? 1.0 : -1.0;
        n[0] = k == 0 ? sgn : 0.0;
        n[1] = k == 1 ? sgn : 0.0;
        n[2] = k == 2 ? sgn : 0.0;
        off = up ? S.bhi[k] : -S.blo[k];
        return;
    }
    const uint8_t s = src[id - 6];
    const double* h = s < 8 ? S.perp + 4 * s : S.cellp + 4 * (s - 8);
    n[0] = h[0];
    n[1] = h[1];
    n[2] = h[2];
    off = h[3];
}

struct Ctx {
    const double* perp;
    const double* blo;
    const double* bhi;
    const double* qlo;
    const double* qscale;
    double slack;
};

__device__ __forceinline__ double dist2(const FloodPrim& p, const double* x) {
    double d[3] = {x[0] - p.a[0], x[1] - p.a[1], x[2] - p.a[2]};
    if (p.face) {
        const double h = dot3(d, p.dir);
        return h * h;
    }
    double c[3];
    cross3(d, p.dir, c);
    return dot3(c, c);
}

__device__ void quantize_box(const Ctx& c, const double lo[3], const double hi[3], uint16_t out[6]) {
    for (int k = 0; k < 3; ++k) {
        const double a = floor((lo[k] - c.qlo[k]) * c.qscale[k]) - 1.0;
        const double b = ceil((hi[k] - c.qlo[k]) * c.qscale[k]) + 1.0;
        const double a1 = a < 0.0 ? 0.0 : a;  // max(0, a)
        const double b1 = b < 0.0 ? 0.0 : b;
        out[k] = (uint16_t)(65535.0 < a1 ? 65535.0 : a1);  // min(65535, .)
        out[3 + k] = (uint16_t)(65535.0 < b1 ? 65535.0 : b1);
    }
}

// A point x keeps w out of p's list when |x-w|^2 + slack <= Dist(x,p)^2
// (Theorems 5 and 6 with the margin).
__device__ __forceinline__ bool far_enough(const FloodPrim& p, const double* Wv, const double* x, double slack) {
    double d[3] = {x[0] - Wv[0], x[1] - Wv[1], x[2] - Wv[2]};
    return dot3(d, d) + slack <= dist2(p, x);
}

struct Counters {
    unsigned long long recs, redo, tests, hits, quick, skipped, next;
};

struct WPoly {
    double x, y, z;  // this lane's corner (lanes below nt)
    uint32_t tri;    // its planes a | b << 8 | c << 16, counter-clockwise from outside
    uint32_t adj;    // lanes of the corners across edges (a,b), (b,c), (c,a), 8 bits each
    int nt, np;      // wave-uniform
    bool empty;
};

struct WaveLds {
    int32_t queue[kQueueCap];
    int32_t hset[kHashCap];
    int32_t nxt[kPlaneCap];      // boundary cycle: next plane after a, or -1
    uint8_t newidx[kPlaneCap];   // new corner of the boundary edge starting at plane a
    uint8_t endidx[kPlaneCap];   // new corner of the boundary edge ending at plane b
    uint8_t o2n[kWaveCorners];   // kept corner: old lane -> new lane
    uint8_t srcB[kPlaneCap - 6]; // plane sources of the base and working polytopes
    uint8_t srcW[kPlaneCap - 6];
    double sx[kWaveCorners], sy[kWaveCorners], sz[kWaveCorners];  // staging of a cut's result
    uint32_t stri[kWaveCorners], sadj[kWaveCorners];
    double cpl[kWaveCorners][4];  // cell construction: the bisector planes so far
};

__device__ __forceinline__ int wlane() { return (int)__lane_id(); }
__device__ __forceinline__ uint64_t below(int l) { return l == 0 ? 0ull : (~0ull >> (64 - l)); }
__device__ __forceinline__ int tri_at(uint32_t tri, int e) { return (int)((tri >> (8 * e)) & 255u); }

struct WCorner {
    double x[3];
    bool ok;
};

// Corner of planes a, b and the new plane h (the host's formula), from the
// planes themselves.
__device__ __forceinline__ WCorner wcorner_of(double an0, double an1, double an2, double aoff, double bn0, double bn1,
                                           double bn2, double boff, double hn0, double hn1, double hn2, double hoff) {
    const double an[3] = {an0, an1, an2}, bn[3] = {bn0, bn1, bn2}, hn[3] = {hn0, hn1, hn2};
    WCorner r;
    double bc[3], ca[3], ab[3];
    cross3(bn, hn, bc);
    cross3(hn, an, ca);
    cross3(an, bn, ab);
    const double det = dot3(an, bc);
    const double scale = sqrt(dot3(an, an) * dot3(bn, bn) * dot3(hn, hn));
    r.ok = false;
    r.x[0] = r.x[1] = r.x[2] = 0.0;
    if (!(det > 1e-13 * scale)) return r;
    const double inv = 1.0 / det;
    for (int d = 0; d < 3; ++d) r.x[d] = (aoff * bc[d] + boff * ca[d] + hoff * ab[d]) * inv;
    r.ok = isfinite(r.x[0]) && isfinite(r.x[1]) && isfinite(r.x[2]);
    return r;
}

__device__ __forceinline__ void wplane_get(const PlaneSrc& S, const WaveLds& L, const uint8_t* src, int id,
                                           double n[3], double& off) {
    if (S.lds && id >= 6) {
        const int r = src[id - 6] - 8;
        n[0] = L.cpl[r][0];
        n[1] = L.cpl[r][1];
        n[2] = L.cpl[r][2];
        off = L.cpl[r][3];
        return;
    }
    plane_get(S, src, id, n, off);
}

__device__ __forceinline__ WCorner wcorner(const PlaneSrc& S, const WaveLds& L, const uint8_t* src, int i, int j,
                                           const double hn[3], double hoff) {
    double an[3], bn[3], aoff, boff;
    wplane_get(S, L, src, i, an, aoff);
    wplane_get(S, L, src, j, bn, boff);
    return wcorner_of(an[0], an[1], an[2], aoff, bn[0], bn[1], bn[2], boff, hn[0], hn[1], hn[2], hoff);
}

// The box D grown by tau, with the corners' adjacency found by search.
__device__ void winit_box(WPoly& P, const double* lo, const double* hi) {
    const int l = wlane();
    P.nt = 8;
    P.np = 6;
    P.empty = false;
    const int c = l & 7;
    const int sx = c & 1, sy = (c >> 1) & 1, sz = (c >> 2) & 1;
    uint32_t t0 = (uint32_t)(0 + sx), t1 = (uint32_t)(2 + sy), t2 = (uint32_t)(4 + sz);
    if ((sx ? 1 : -1) * (sy ? 1 : -1) * (sz ? 1 : -1) < 0) {
        const uint32_t t = t0;
        t0 = t1;
        t1 = t;
    }
    P.tri = t0 | (t1 << 8) | (t2 << 16);
    P.x = sx ? hi[0] : lo[0];
    P.y = sy ? hi[1] : lo[1];
    P.z = sz ? hi[2] : lo[2];
    uint32_t adj = 0;
    for (int e = 0; e < 3; ++e) {
        const int a = tri_at(P.tri, e), b = tri_at(P.tri, e == 2 ? 0 : e + 1);
        uint32_t found = 0;
        for (int j = 0; j < 8; ++j) {
            const uint32_t U = (uint32_t)__shfl((int)P.tri, j);
            const int u0 = tri_at(U, 0), u1 = tri_at(U, 1), u2 = tri_at(U, 2);
            if ((u0 == b && u1 == a) || (u1 == b && u2 == a) || (u2 == b && u0 == a)) found = (uint32_t)j;
        }
        adj |= found << (8 * e);
    }
    P.adj = adj;
}

// Corners strictly outside (hn, hoff): a wave-uniform mask.
__device__ __forceinline__ uint64_t woutside(const WPoly& P, const double hn[3], double hoff) {
    const bool valid = wlane() < P.nt;
    const double pos[3] = {P.x, P.y, P.z};
    const double v = valid ? dot3(hn, pos) - hoff : 0.0;
    return __ballot(valid && v > 0.0);
}

// Cut P (sources in src) by (hn, hoff) with source s, given the nonempty
// mask of corners outside.  Same outcome as the host's cut.
__device__ int wcut(WPoly& P, uint8_t* src, WaveLds& L, const PlaneSrc& S, const double hn[3], double hoff,
                    uint8_t s, uint64_t outmask) {
    const int l = wlane();
    const int nout = __popcll(outmask);
    if (nout == P.nt) {
        P.empty = true;
        P.nt = 0;
        return EMPTY;
    }
    const bool valid = l < P.nt;
    const bool out = (outmask >> l) & 1ull;
    const int a0 = tri_at(P.tri, 0), a1 = tri_at(P.tri, 1), a2 = tri_at(P.tri, 2);
    const int n0 = tri_at(P.adj, 0), n1 = tri_at(P.adj, 1), n2 = tri_at(P.adj, 2);
    // boundary edges: edges of removed corners whose neighbour is kept
    const bool be0 = out && !((outmask >> n0) & 1ull);
    const bool be1 = out && !((outmask >> n1) & 1ull);
    const bool be2 = out && !((outmask >> n2) & 1ull);
    const uint64_t m0 = __ballot(be0), m1 = __ballot(be1), m2 = __ballot(be2);
    const int nb = __popcll(m0) + __popcll(m1) + __popcll(m2);
    if (nb < 3) return SKIPPED;
    const int np = P.np;
    if (np + 1 > kPlaneCap) return OVERFLOW;
    // the boundary must be one cycle: one edge leaving each plane ...
    for (int i = l; i < np; i += 64) L.nxt[i] = -1;
    __syncthreads();
    bool dup = false;
    if (be0) dup |= atomicCAS(&L.nxt[a0], -1, a1) != -1;
    if (be1) dup |= atomicCAS(&L.nxt[a1], -1, a2) != -1;
    if (be2) dup |= atomicCAS(&L.nxt[a2], -1, a0) != -1;
    __syncthreads();
    if (__ballot(dup)) return SKIPPED;
    // ... and following them from one start visits all nb
    {
        const int f = __ffsll((long long)(m0 | m1 | m2)) - 1;
        const int mine = be0 ? a0 : (be1 ? a1 : a2);
        const int start = __shfl(mine, f);
        int a = start, steps = 0;
        bool ok = true;
        do {
            a = L.nxt[a];
            if (a < 0) {
                ok = false;
                break;
            }
            ++steps;
        } while (a != start && steps <= nb);
        if (!ok || steps != nb) return SKIPPED;
    }
    const int nk = P.nt - nout;
    const int ntn = nk + nb;
    if (ntn > kWaveCorners) return OVERFLOW;
    // new places: kept corners first, in lane order, then the new ones
    const bool kept = valid && !out;
    const uint64_t keptmask = __ballot(kept);
    const int dk = __popcll(keptmask & below(l));
    const int dn = nk + __popcll(m0 & below(l)) + __popcll(m1 & below(l)) + __popcll(m2 & below(l));
    const int d0 = dn, d1 = dn + (be0 ? 1 : 0), d2 = d1 + (be1 ? 1 : 0);
    // the new corners, one per boundary edge (a -> b): planes a, b, np,
    // staged at their new places (dropped if the cut is skipped)
    // a lane owns up to three boundary edges: the corners are computed in
    // passes, one edge of every owning lane per pass
    bool fail = false;
    const int kmine = (be0 ? 1 : 0) + (be1 ? 1 : 0) + (be2 ? 1 : 0);
    const int passes = __ballot(kmine >= 3) ? 3 : (__ballot(kmine >= 2) ? 2 : 1);
    for (int it = 0; it < passes; ++it) {
        // this lane's it-th boundary edge
        int e = -1, seen = 0;
        if (be0 && seen++ == it) e = 0;
        if (be1 && seen++ == it && e < 0) e = 1;
        if (be2 && seen++ == it && e < 0) e = 2;
        if (e >= 0) {
            const int a = e == 0 ? a0 : (e == 1 ? a1 : a2);
            const int b = e == 0 ? a1 : (e == 1 ? a2 : a0);
            const int d = e == 0 ? d0 : (e == 1 ? d1 : d2);
            const WCorner r = wcorner(S, L, src, a, b, hn, hoff);
            fail |= !r.ok;
            L.sx[d] = r.x[0];
            L.sy[d] = r.x[1];
            L.sz[d] = r.x[2];
        }
    }
    if (__ballot(fail)) return SKIPPED;
    if (kept) L.o2n[l] = (uint8_t)dk;
    if (be0) {
        L.newidx[a0] = (uint8_t)d0;
        L.endidx[a1] = (uint8_t)d0;
    }
    if (be1) {
        L.newidx[a1] = (uint8_t)d1;
        L.endidx[a2] = (uint8_t)d1;
    }
    if (be2) {
        L.newidx[a2] = (uint8_t)d2;
        L.endidx[a0] = (uint8_t)d2;
    }
    if (l == 0) src[np - 6] = s;
    __syncthreads();
    const uint32_t pid = (uint32_t)np;
    if (kept) {
        // an edge (c -> d) facing a removed corner now faces the new corner
        // of the boundary edge (d -> c)
        const int ends[3] = {a1, a2, a0};
        const int nbr[3] = {n0, n1, n2};
        uint32_t adj = 0;
        for (int e = 0; e < 3; ++e) {
            const int n = nbr[e];
            const uint32_t t = ((outmask >> n) & 1ull) ? L.newidx[ends[e]] : L.o2n[n];
            adj |= t << (8 * e);
        }
        L.sx[dk] = P.x;
        L.sy[dk] = P.y;
        L.sz[dk] = P.z;
        L.stri[dk] = P.tri;
        L.sadj[dk] = adj;
    }
    // new corner (a, b, np): across (a,b) the kept corner, across (b,np)
    // the new corner starting at b, across (np,a) the one ending at a
    if (be0) {
        L.stri[d0] = (uint32_t)a0 | ((uint32_t)a1 << 8) | (pid << 16);
        L.sadj[d0] = (uint32_t)L.o2n[n0] | ((uint32_t)L.newidx[a1] << 8) | ((uint32_t)L.endidx[a0] << 16);
    }
    if (be1) {
        L.stri[d1] = (uint32_t)a1 | ((uint32_t)a2 << 8) | (pid << 16);
        L.sadj[d1] = (uint32_t)L.o2n[n1] | ((uint32_t)L.newidx[a2] << 8) | ((uint32_t)L.endidx[a1] << 16);
    }
    if (be2) {
        L.stri[d2] = (uint32_t)a2 | ((uint32_t)a0 << 8) | (pid << 16);
        L.sadj[d2] = (uint32_t)L.o2n[n2] | ((uint32_t)L.newidx[a0] << 8) | ((uint32_t)L.endidx[a2] << 16);
    }
    __syncthreads();
    if (l < ntn) {
        P.x = L.sx[l];
        P.y = L.sy[l];
        P.z = L.sz[l];
        P.tri = L.stri[l];
        P.adj = L.sadj[l];
    }
    P.nt = ntn;
    P.np = np + 1;
    __syncthreads();
    return CLIPPED;
}

__device__ __forceinline__ int wclip(WPoly& P, uint8_t* src, WaveLds& L, const PlaneSrc& S, const double hn[3],
                                     double hoff, uint8_t s) {
    if (P.empty) return UNCHANGED;
    const uint64_t om = woutside(P, hn, hoff);
    if (om == 0ull) return UNCHANGED;
    return wcut(P, src, L, S, hn, hoff, s, om);
}

// ConvexPoly(w,p) into W: the base cut by Cell(w)'s planes (those on D's
// boundary skipped, as on the host).  False when empty; OVERFLOW via ovf.
__device__ bool wclip_to_cell(const Ctx& c, const WPoly& B, WPoly& W, WaveLds& L, const double* cellp, int np,
                              int64_t& skipped, bool& ovf) {
    W = B;
    for (int i = wlane(); i < B.np - 6; i += 64) L.srcW[i] = L.srcB[i];
    __syncthreads();
    if (W.empty) return true;
    const PlaneSrc S{c.blo, c.bhi, c.perp, cellp};
    for (int i = 0; i < np; ++i) {
        const double hn[3] = {cellp[4 * i], cellp[4 * i + 1], cellp[4 * i + 2]};
        const double hoff = cellp[4 * i + 3];
        const int axes = (hn[0] != 0.0) + (hn[1] != 0.0) + (hn[2] != 0.0);
        if (axes == 1 && (fabs(hn[0]) == 1.0 || fabs(hn[1]) == 1.0 || fabs(hn[2]) == 1.0)) {
            const int k = hn[0] != 0.0 ? 0 : (hn[1] != 0.0 ? 1 : 2);
            if ((hn[k] > 0 && hoff == c.bhi[k]) || (hn[k] < 0 && hoff == -c.blo[k])) continue;
        }
        const uint64_t om = woutside(W, hn, hoff);
        if (om == 0ull) continue;
        const int r = wcut(W, L.srcW, L, S, hn, hoff, (uint8_t)(8 + i), om);
        if (r == EMPTY) return false;
        if (r == SKIPPED) ++skipped;
        if (r == OVERFLOW) {
            ovf = true;
            return false;
        }
    }
    return true;
}

__device__ __forceinline__ double wmin(double v) {
    for (int d = 32; d >= 1; d >>= 1) {
        const double o = __shfl_xor(v, d);
        v = o < v ? o : v;
    }
    return v;
}
__device__ __forceinline__ double wmax(double v) {
    for (int d = 32; d >= 1; d >>= 1) {
        const double o = __shfl_xor(v, d);
        v = v < o ? o : v;
    }
    return v;
}

__device__ void wpoly_box(const Ctx& c, const WPoly& P, uint16_t out[6]) {
    if (P.empty || P.nt == 0) {
        for (int k = 0; k < 3; ++k) {
            out[k] = 65535;
            out[3 + k] = 0;
        }
        return;
    }
    const bool valid = wlane() < P.nt;
    double lo[3], hi[3];
    lo[0] = wmin(valid ? P.x : INFINITY);
    lo[1] = wmin(valid ? P.y : INFINITY);
    lo[2] = wmin(valid ? P.z : INFINITY);
    hi[0] = wmax(valid ? P.x : -INFINITY);
    hi[1] = wmax(valid ? P.y : -INFINITY);
    hi[2] = wmax(valid ? P.z : -INFINITY);
    quantize_box(c, lo, hi, out);
}

// LDS visited set: true when u is new.
__device__ __forceinline__ bool whash_visit(int32_t* hset, int32_t u) {
    uint32_t h = ((uint32_t)u * 2654435761u) & (kHashCap - 1);
    for (;;) {
        const int32_t old = atomicCAS(&hset[h], -1, u);
        if (old == -1) return true;
        if (old == u) return false;
        h = (h + 1) & (kHashCap - 1);
    }
}

struct CellCounters {
    unsigned long long next, back, skipped;
};

// The Voronoi cell of every vertex, one vertex per wavefront, as on the
// host: the box D grown by tau cut by the bisector of v and each Voronoi
// (Delaunay) neighbour w, nearest first (ties by id), each moved outward by
// tau; then the planes that bound a corner, in the order they were added,
// and the corners go to the vertex's slot.  A vertex with more than 64
// neighbours or a cell of more than 64 corners is handed back to the host.
__global__ __launch_bounds__(64) void k_cells(int64_t nv, const double* __restrict__ Vd,
                                              const int64_t* __restrict__ nb_off, const int32_t* __restrict__ nb,
                                              const double* __restrict__ dom, double* __restrict__ slot_planes,
                                              double* __restrict__ slot_pos, int32_t* __restrict__ cnp_of,
                                              int32_t* __restrict__ cnt_of, int64_t* __restrict__ pl_at,
                                              int64_t* __restrict__ co_at, int64_t* __restrict__ back,
                                              CellCounters* __restrict__ cc) {
    __shared__ WaveLds L;
    const int l = wlane();
    const double* blo = dom;
    const double* bhi = dom + 3;
    const double tau = dom[12];
    unsigned long long skipped_all = 0;
    WPoly W;
    for (;;) {
        unsigned long long tv = 0;
        if (l == 0) tv = atomicAdd(&cc->next, 1ull);
        tv = __shfl(tv, 0);
        if (tv >= (unsigned long long)nv) break;
        const int64_t v = __builtin_amdgcn_readfirstlane((int)tv);
        const int64_t k0 = nb_off[v];
        const int deg = (int)(nb_off[v + 1] - k0);
        if (deg > 64) {
            if (l == 0) back[atomicAdd(&cc->back, 1ull)] = v;
            continue;
        }
        const double pv[3] = {Vd[3 * v], Vd[3 * v + 1], Vd[3 * v + 2]};
        // neighbour l and its squared distance; its rank in (distance, id) order
        const bool have = l < deg;
        const int32_t wl = have ? nb[k0 + l] : 0x7fffffff;
        double pw[3] = {0.0, 0.0, 0.0};
        double d2 = INFINITY;
        if (have) {
            pw[0] = Vd[3 * (int64_t)wl];
            pw[1] = Vd[3 * (int64_t)wl + 1];
            pw[2] = Vd[3 * (int64_t)wl + 2];
            const double d[3] = {pw[0] - pv[0], pw[1] - pv[1], pw[2] - pv[2]};
            d2 = dot3(d, d);
        }
        int rank = 0;
        for (int i = 0; i < deg; ++i) {
            const double di = __shfl(d2, i);
            const int32_t wi = __shfl(wl, i);
            rank += (di < d2 || (di == d2 && wi < wl)) ? 1 : 0;
        }
        winit_box(W, blo, bhi);
        const PlaneSrc S{blo, bhi, blo, blo, true};
        int64_t skipped = 0;
        bool ovf = false;
        for (int r = 0; r < deg && !ovf; ++r) {
            const int o = __ffsll((long long)__ballot(have && rank == r)) - 1;
            // bisector of v and w, on v's side, moved outward by tau
            double n[3] = {pw[0] - pv[0], pw[1] - pv[1], pw[2] - pv[2]};
            const double nl = sqrt(dot3(n, n));
            const double off = 0.5 * (dot3(pw, pw) - dot3(pv, pv)) + tau * nl;
            const double hn[3] = {__shfl(n[0], o), __shfl(n[1], o), __shfl(n[2], o)};
            const double hoff = __shfl(off, o);
            if (l == 0) {
                L.cpl[r][0] = hn[0];
                L.cpl[r][1] = hn[1];
                L.cpl[r][2] = hn[2];
                L.cpl[r][3] = hoff;
            }
            __syncthreads();
            const int res = wclip(W, L.srcW, L, S, hn, hoff, (uint8_t)(8 + r));
            if (res == SKIPPED) ++skipped;
            if (res == OVERFLOW) ovf = true;
        }
        if (ovf) {
            if (l == 0) back[atomicAdd(&cc->back, 1ull)] = v;
            __syncthreads();
            continue;
        }
        // the planes that bound a corner, renumbered in their order
        const bool valid = l < W.nt;
        uint64_t u0 = 0, u1 = 0;
        if (valid)
            for (int e = 0; e < 3; ++e) {
                const int id = tri_at(W.tri, e);
                if (id < 64) u0 |= 1ull << id;
                else u1 |= 1ull << (id - 64);
            }
        for (int d = 32; d >= 1; d >>= 1) {
            u0 |= __shfl_xor(u0, d);
            u1 |= __shfl_xor(u1, d);
        }
        u0 = __shfl(u0, 0);
        u1 = __shfl(u1, 0);
        double* sp = slot_planes + v * (4 * kSlotPlanes);
        for (int id = l; id < W.np; id += 64) {
            const bool used = id < 64 ? ((u0 >> id) & 1ull) : ((u1 >> (id - 64)) & 1ull);
            if (!used) continue;
            const int k = id < 64 ? __popcll(u0 & below(id)) : __popcll(u0) + __popcll(u1 & below(id - 64));
            double hn[3], hoff;
            wplane_get(S, L, L.srcW, id, hn, hoff);
            sp[4 * k] = hn[0];
            sp[4 * k + 1] = hn[1];
            sp[4 * k + 2] = hn[2];
            sp[4 * k + 3] = hoff;
        }
        if (valid) {
            double* xp = slot_pos + (v * kSlotCorners + l) * 3;
            xp[0] = W.x;
            xp[1] = W.y;
            xp[2] = W.z;
        }
        if (l == 0) {
            cnp_of[v] = W.empty ? 0 : __popcll(u0) + __popcll(u1);
            cnt_of[v] = W.empty ? 0 : W.nt;
            pl_at[v] = v * kSlotPlanes;
            co_at[v] = v * kSlotCorners;
        }
        skipped_all += (unsigned long long)skipped;
        __syncthreads();
    }
    if (l == 0) atomicAdd(&cc->skipped, skipped_all);
}

// Places of the cells built on the host: vertex, plane and corner offsets
// (already negative) and counts.
__global__ __launch_bounds__(256) void k_set_cells(int64_t n, const int64_t* __restrict__ meta,
                                                   int64_t* __restrict__ pl_at, int64_t* __restrict__ co_at,
                                                   int32_t* __restrict__ cnp_of, int32_t* __restrict__ cnt_of) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t v = meta[5 * i];
    pl_at[v] = meta[5 * i + 1];
    co_at[v] = meta[5 * i + 2];
    cnp_of[v] = (int32_t)meta[5 * i + 3];
    cnt_of[v] = (int32_t)meta[5 * i + 4];
}

// Each wavefront (a block of 64 lanes) takes primitives from a shared counter
// until none are left and floods each one: base polytope, then for every
// queued vertex the quick whole-cell test, the cut by the cell's planes, the
// corner test and the entry box, and on a hit the vertex's Voronoi
// neighbours are queued.
__global__ __launch_bounds__(64) void k_flood(int64_t nprim, const FloodPrim* __restrict__ prims,
                                                   const double* __restrict__ perp, const double* __restrict__ Vd,
                                                   const int64_t* __restrict__ nb_off, const int32_t* __restrict__ nb,
                                                   const int32_t* __restrict__ cnp_of,
                                                   const double* __restrict__ cplanes,
                                                   const int32_t* __restrict__ cnt_of, const double* __restrict__ cpos,
                                                   const int64_t* __restrict__ pl_at, const int64_t* __restrict__ co_at,
                                                   const double* __restrict__ xplanes,
                                                   const double* __restrict__ xpos,
                                                   const double* __restrict__ dom, FloodRec* __restrict__ recs,
                                                   uint64_t rec_cap, int64_t* __restrict__ redo,
                                                   Counters* __restrict__ cnt, int visit_cap) {
    __shared__ WaveLds L;
    const int l = wlane();
    Ctx c;
    c.blo = dom;
    c.bhi = dom + 3;
    c.qlo = dom + 6;
    c.qscale = dom + 9;
    c.slack = 2.0 * dom[12] * dom[13];
    unsigned long long t_tests = 0, t_hits = 0, t_quick = 0, t_skipped = 0;
    WPoly B, W;
    for (;;) {
        // wave-uniform values are moved to scalar registers, so the
        // primitive, the cell and its planes are read with scalar loads
        unsigned long long ti = 0;
        if (l == 0) ti = atomicAdd(&cnt->next, 1ull);
        ti = __shfl(ti, 0);
        if (ti >= (unsigned long long)nprim) break;
        const int64_t i = __builtin_amdgcn_readfirstlane((int)ti);
        const FloodPrim p = prims[i];
        c.perp = perp + 4 * p.perp_off;
        const uint32_t code = (p.face ? 0x80000000u : 0u) | (uint32_t)p.id;
        int64_t tests = 0, hits = 0, quick = 0, skipped = 0;
        bool ovf = false;
        // base polytope Space-perp(p) n D
        winit_box(B, c.blo, c.bhi);
        bool base_empty = false;
        {
            const PlaneSrc S{c.blo, c.bhi, c.perp, c.perp};  // the base has no cell planes
            for (int j = 0; j < p.nperp && !base_empty && !ovf; ++j) {
                const double hn[3] = {c.perp[4 * j], c.perp[4 * j + 1], c.perp[4 * j + 2]};
                const int r = wclip(B, L.srcB, L, S, hn, c.perp[4 * j + 3], (uint8_t)j);
                if (r == EMPTY) base_empty = true;
                if (r == SKIPPED) ++skipped;
                if (r == OVERFLOW) ovf = true;
            }
        }
        for (int k = l; k < kHashCap; k += 64) L.hset[k] = -1;
        __syncthreads();
        int qn = 0;
        if (l == 0)
            for (int k = 0; k < p.nverts; ++k) {
                whash_visit(L.hset, p.verts[k]);
                L.queue[k] = p.verts[k];
            }
        qn = p.nverts;
        __syncthreads();
        for (int head = 0; head < qn && !ovf; ++head) {
            const int32_t w = __builtin_amdgcn_readfirstlane(L.queue[head]);
            bool own = false;
            for (int k = 0; k < p.nverts; ++k) own |= (p.verts[k] == w);
            const int64_t pa = pl_at[w];
            const double* cellp = pa >= 0 ? cplanes + 4 * pa : xplanes + 4 * (-pa - 1);
            const int cnp = cnp_of[w];
            if (cnp > kPlaneCap - 8 - 8) {
                ovf = true;
                break;
            }
            uint16_t box[6];
            bool hit;
            if (own) {  // Theorem 2
                if (base_empty || !wclip_to_cell(c, B, W, L, cellp, cnp, skipped, ovf)) W.empty = true;
                if (ovf) break;
                wpoly_box(c, W, box);
                hit = true;
            } else {
                ++tests;
                const double* X = Vd + 3 * (int64_t)w;
                const double Wv[3] = {X[0], X[1], X[2]};
                // |x-w| - Dist(x,p) is convex: the whole cell keeping w out settles it
                const int64_t ca = co_at[w];
                const double* cposw = ca >= 0 ? cpos + 3 * ca : xpos + 3 * (-ca - 1);
                const int64_t t0 = 0, t1 = cnt_of[w];
                bool all_far = true;
                for (int64_t t = t0; t < t1 && all_far; t += 64) {
                    const bool far = t + l >= t1 || far_enough(p, Wv, cposw + 3 * (t + l), c.slack);
                    all_far = __ballot(!far) == 0ull;
                }
                hit = false;
                if (all_far) {
                    ++quick;
                } else if (!base_empty && wclip_to_cell(c, B, W, L, cellp, cnp, skipped, ovf)) {
                    const double pos[3] = {W.x, W.y, W.z};
                    const bool near = l < W.nt && !far_enough(p, Wv, pos, c.slack);
                    if (__ballot(near)) {
                        wpoly_box(c, W, box);
                        hit = true;
                    }
                }
                if (ovf) break;
            }
            if (!hit) continue;
            ++hits;
            if (l == 0) {
                const unsigned long long slot = atomicAdd(&cnt->recs, 1ull);
                if (slot < rec_cap) {
                    FloodRec r;
                    r.v = (uint32_t)w;
                    r.code = code;
                    for (int k = 0; k < 6; ++k) r.box[k] = box[k];
                    recs[slot] = r;
                }
            }
            const int64_t k0 = nb_off[w], deg = nb_off[w + 1] - k0;
            for (int64_t k = 0; k < deg; k += 64) {
                const bool have = k + l < deg;
                const int32_t u = have ? nb[k0 + k + l] : -1;
                const bool isnew = have && whash_visit(L.hset, u);
                const uint64_t m = __ballot(isnew);
                const int cntn = __popcll(m);
                if (qn + cntn > visit_cap) {
                    ovf = true;
                    break;
                }
                if (isnew) L.queue[qn + __popcll(m & below(l))] = u;
                qn += cntn;
            }
            __syncthreads();
        }
        if (ovf) {
            if (l == 0) {
                const unsigned long long slot = atomicAdd(&cnt->redo, 1ull);
                redo[slot] = i;
            }
        } else {
            t_tests += (unsigned long long)tests;
            t_hits += (unsigned long long)hits;
            t_quick += (unsigned long long)quick;
            t_skipped += (unsigned long long)skipped;
        }
        __syncthreads();
    }
    if (l == 0) {
        atomicAdd(&cnt->tests, t_tests);
        atomicAdd(&cnt->hits, t_hits);
        atomicAdd(&cnt->quick, t_quick);
        atomicAdd(&cnt->skipped, t_skipped);
    }
}

using Clock = std::chrono::steady_clock;
double since(Clock::time_point t0) { return std::chrono::duration<double>(Clock::now() - t0).count(); }

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

bool device_flood(const FloodInput& in, FloodResult& out, std::string& err) {
    auto hip_ok = [&](hipError_t e, const char* what) {
        if (e == hipSuccess) return true;
        err = std::string("device inspection: ") + what + ": " + hipGetErrorString(e);
        return false;
    };
    out = FloodResult();
    if (in.nprim == 0) return true;
    auto t0 = Clock::now();
    const size_t nv = (size_t)in.nv;
    const uint64_t rec_cap = std::max<uint64_t>(1u << 20, 64ull * nv + 16ull * (uint64_t)in.nprim);
    struct Part {
        const void* src;
        size_t bytes;
    };
    double dom[14];
    for (int k = 0; k < 3; ++k) {
        dom[k] = in.blo[k];
        dom[3 + k] = in.bhi[k];
        dom[6 + k] = in.qlo[k];
        dom[9 + k] = in.qscale[k];
    }
    dom[12] = in.tau;
    dom[13] = in.dmax;
    // uploaded parts, then the parts the device fills
    const Part parts[] = {
        {in.prims, sizeof(FloodPrim) * (size_t)in.nprim},
        {in.perp, sizeof(double) * 4 * (size_t)std::max<int64_t>(1, in.nperp_total)},
        {in.Vd, sizeof(double) * 3 * nv},
        {in.nb_off, sizeof(int64_t) * (nv + 1)},
        {in.nb, sizeof(int32_t) * std::max<size_t>(1, (size_t)in.nb_off[nv])},
        {dom, sizeof(dom)},
        {nullptr, sizeof(double) * 4 * kSlotPlanes * nv},   // 6: cell planes
        {nullptr, sizeof(double) * 3 * kSlotCorners * nv},  // 7: cell corners
        {nullptr, sizeof(int32_t) * nv},                    // 8: planes per cell
        {nullptr, sizeof(int32_t) * nv},                    // 9: corners per cell
        {nullptr, sizeof(int64_t) * nv},                    // 10: cells handed back
        {nullptr, sizeof(FloodRec) * rec_cap},              // 11: table entries
        {nullptr, sizeof(int64_t) * (size_t)in.nprim},      // 12: primitives handed back
        {nullptr, 256},                                     // 13: counters
        {nullptr, sizeof(int64_t) * nv},                    // 14: plane offset of each cell
        {nullptr, sizeof(int64_t) * nv},                    // 15: corner offset of each cell
    };
    constexpr int kParts = sizeof(parts) / sizeof(parts[0]);
    size_t off[kParts];
    size_t total = 0;
    for (int k = 0; k < kParts; ++k) {
        off[k] = total;
        total += (parts[k].bytes + 255) / 256 * 256;
    }
    DevBuf buf;
    if (!hip_ok(hipMalloc(&buf.p, total), "hipMalloc")) return false;
    char* d = (char*)buf.p;
    for (int k = 0; k < kParts; ++k)
        if (parts[k].src && parts[k].bytes &&
            !hip_ok(hipMemcpy(d + off[k], parts[k].src, parts[k].bytes, hipMemcpyHostToDevice), "upload"))
            return false;
    if (!hip_ok(hipMemset(d + off[13], 0, 256), "hipMemset")) return false;
    if (!hip_ok(hipDeviceSynchronize(), "upload")) return false;
    out.t_upload = since(t0);
    const double* dVd = (const double*)(d + off[2]);
    const int64_t* dnb_off = (const int64_t*)(d + off[3]);
    const int32_t* dnb = (const int32_t*)(d + off[4]);
    const double* ddom = (const double*)(d + off[5]);
    double* cplanes = (double*)(d + off[6]);
    double* cpos = (double*)(d + off[7]);
    int32_t* cnp = (int32_t*)(d + off[8]);
    int32_t* cnt = (int32_t*)(d + off[9]);
    int64_t* cback = (int64_t*)(d + off[10]);
    int64_t* pl_at = (int64_t*)(d + off[14]);
    int64_t* co_at = (int64_t*)(d + off[15]);
    DevBuf xbuf;  // cells built on the host
    const double* xplanes = cplanes;
    const double* xpos = cpos;
    Counters* counters = (Counters*)(d + off[13]);
    CellCounters* ccount = (CellCounters*)(d + off[13] + 128);
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int block = 64;

    // 1. cells: on the device, those it hands back on the host
    t0 = Clock::now();
    {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cells, block, 0) != hipSuccess || per_cu < 1)
            per_cu = 8;
        const int64_t grid = std::min<int64_t>(in.nv, (int64_t)cus * per_cu);
        k_cells<<<(unsigned)grid, block, 0, 0>>>(in.nv, dVd, dnb_off, dnb, ddom, cplanes, cpos, cnp, cnt, pl_at,
                                                 co_at, cback, ccount);
        if (!hip_ok(hipGetLastError(), "launch")) return false;
        if (!hip_ok(hipDeviceSynchronize(), "cell kernel")) return false;
        CellCounters cc;
        if (!hip_ok(hipMemcpy(&cc, ccount, sizeof(cc), hipMemcpyDeviceToHost), "download")) return false;
        out.cells_skipped = (int64_t)cc.skipped;
        out.cells_back = (int64_t)cc.back;
        std::vector<int64_t> back((size_t)cc.back);
        if (cc.back && !hip_ok(hipMemcpy(back.data(), cback, sizeof(int64_t) * cc.back, hipMemcpyDeviceToHost),
                               "download"))
            return false;
        if (!back.empty()) {
            // the cells handed back, built on the host, packed into a second
            // allocation; their places and counts scattered by k_set_cells
            std::vector<double> XP, XX;
            std::vector<std::vector<double>> PS, XS;
            out.cells_skipped += in.host_cell(back, PS, XS);
            std::vector<int64_t> meta;
            meta.reserve(5 * back.size());
            for (size_t k = 0; k < back.size(); ++k) {
                const int64_t v = back[k];
                const std::vector<double>& P = PS[k];
                const std::vector<double>& X = XS[k];
                meta.push_back(v);
                meta.push_back(-(int64_t)(XP.size() / 4) - 1);
                meta.push_back(-(int64_t)(XX.size() / 3) - 1);
                meta.push_back((int64_t)(P.size() / 4));
                meta.push_back((int64_t)(X.size() / 3));
                XP.insert(XP.end(), P.begin(), P.end());
                XX.insert(XX.end(), X.begin(), X.end());
            }
            const size_t bp = (sizeof(double) * std::max<size_t>(4, XP.size()) + 255) / 256 * 256;
            const size_t bx = (sizeof(double) * std::max<size_t>(3, XX.size()) + 255) / 256 * 256;
            const size_t bm = sizeof(int64_t) * meta.size();
            if (!hip_ok(hipMalloc(&xbuf.p, bp + bx + bm), "hipMalloc")) return false;
            char* x = (char*)xbuf.p;
            if ((!XP.empty() && !hip_ok(hipMemcpy(x, XP.data(), sizeof(double) * XP.size(), hipMemcpyHostToDevice),
                                        "upload")) ||
                (!XX.empty() && !hip_ok(hipMemcpy(x + bp, XX.data(), sizeof(double) * XX.size(),
                                                  hipMemcpyHostToDevice), "upload")) ||
                !hip_ok(hipMemcpy(x + bp + bx, meta.data(), bm, hipMemcpyHostToDevice), "upload"))
                return false;
            xplanes = (const double*)x;
            xpos = (const double*)(x + bp);
            const int64_t nb_back = (int64_t)back.size();
            k_set_cells<<<(unsigned)((nb_back + 255) / 256), 256, 0, 0>>>(nb_back, (const int64_t*)(x + bp + bx),
                                                                        pl_at, co_at, cnp, cnt);
            if (!hip_ok(hipGetLastError(), "launch")) return false;
            if (!hip_ok(hipDeviceSynchronize(), "cell placement")) return false;
        }
    }
    out.t_cells = since(t0);

    // 2. filter + flooding of every primitive
    t0 = Clock::now();
    {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_flood, block, 0) != hipSuccess || per_cu < 1)
            per_cu = 8;
        const int64_t grid = std::min<int64_t>(in.nprim, (int64_t)cus * per_cu);
        k_flood<<<(unsigned)grid, block, 0, 0>>>(
            in.nprim, (const FloodPrim*)(d + off[0]), (const double*)(d + off[1]), dVd, dnb_off, dnb, cnp, cplanes,
            cnt, cpos, pl_at, co_at, xplanes, xpos, ddom, (FloodRec*)(d + off[11]), rec_cap,
            (int64_t*)(d + off[12]), counters,
            in.visit_cap > 0 && in.visit_cap < kQueueCap ? in.visit_cap : kQueueCap);
        if (!hip_ok(hipGetLastError(), "launch")) return false;
        if (!hip_ok(hipDeviceSynchronize(), "kernel")) return false;
    }
    out.t_kernel = since(t0);
    t0 = Clock::now();
    Counters c;
    if (!hip_ok(hipMemcpy(&c, counters, sizeof(c), hipMemcpyDeviceToHost), "download")) return false;
    if (c.recs > rec_cap) {
        err = "device inspection: more table entries than the record buffer holds";
        return false;
    }
    out.recs.resize((size_t)c.recs);
    out.redo.resize((size_t)c.redo);
    if (c.recs && !hip_ok(hipMemcpy(out.recs.data(), d + off[11], sizeof(FloodRec) * c.recs,
                                    hipMemcpyDeviceToHost), "download"))
        return false;
    if (c.redo && !hip_ok(hipMemcpy(out.redo.data(), d + off[12], sizeof(int64_t) * c.redo,
                                    hipMemcpyDeviceToHost), "download"))
        return false;
    out.tests = (int64_t)c.tests;
    out.hits = (int64_t)c.hits;
    out.quick = (int64_t)c.quick;
    out.skipped = (int64_t)c.skipped;
    out.t_download = since(t0);
    return true;
}

}  // namespace p2m
