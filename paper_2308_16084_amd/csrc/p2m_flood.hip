// Device inspection: the convexity filter (Theorems 5 and 6) and flooding
// (Algorithm 1) of every primitive, one primitive per lane.
//
// The arithmetic is the host builder's, operation for operation, in FP64,
// and this file is compiled without contraction (no fused multiply-adds), so
// every plane test, corner and box comes out bit for bit as on the host and
// the table is the host's.  The polytope is kept in the same dual form (a
// corner is a triangle of plane ids, counter-clockwise from outside); a cut
// removes the corners outside the plane and closes the hole with one new
// corner per boundary edge.  What a cut does depends only on the set of
// corners, not on their order, so the corners can be stored in any order.
//
// Each lane holds its primitive's base polytope Space-perp(p) n D, a working
// polytope ConvexPoly(w,p) = base n Cell(w), the flood queue and a hash set
// of visited vertices, all of fixed capacity.  A primitive that outgrows any
// of them is handed back to the host, which floods it itself.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>

#include "flood_device.hpp"

namespace p2m {

namespace {

constexpr int kTriCap = 96;    // corners of the working polytope, new ones included during a cut
constexpr int kBaseCap = 32;   // corners of the base polytope
constexpr int kPlaneCap = 128; // planes of a polytope (ids fit in 8 bits)
constexpr int kQueueCap = 512; // vertices one flood may visit
constexpr int kHashCap = 1024; // open-addressing set over them (power of two)

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
};

template <int Cap>
struct Poly {
    int nt, np;
    bool empty;
    uint8_t src[kPlaneCap - 6];
    uint8_t tri[Cap][3];
    double pos[Cap][3];
};

__device__ __forceinline__ void plane_get(const PlaneSrc& S, const uint8_t* src, int id, double n[3], double& off) {
    if (id < 6) {
        const int k = id >> 1;
        n[0] = 0.0;
        n[1] = 0.0;
        n[2] = 0.0;
        if (id & 1) {
            n[k] = 1.0;
            off = S.bhi[k];
        } else {
            n[k] = -1.0;
            off = -S.blo[k];
        }
        return;
    }
    const uint8_t s = src[id - 6];
    const double* h = s < 8 ? S.perp + 4 * s : S.cellp + 4 * (s - 8);
    n[0] = h[0];
    n[1] = h[1];
    n[2] = h[2];
    off = h[3];
}

template <int Cap>
__device__ void init_box(Poly<Cap>& P, const double* lo, const double* hi) {
    P.nt = 8;
    P.np = 6;
    P.empty = false;
    for (int c = 0; c < 8; ++c) {
        const int sx = c & 1, sy = (c >> 1) & 1, sz = (c >> 2) & 1;
        uint8_t t0 = (uint8_t)(0 + sx), t1 = (uint8_t)(2 + sy), t2 = (uint8_t)(4 + sz);
        const int sgn = (sx ? 1 : -1) * (sy ? 1 : -1) * (sz ? 1 : -1);
        if (sgn < 0) {
            const uint8_t t = t0;
            t0 = t1;
            t1 = t;
        }
        P.tri[c][0] = t0;
        P.tri[c][1] = t1;
        P.tri[c][2] = t2;
        P.pos[c][0] = sx ? hi[0] : lo[0];
        P.pos[c][1] = sy ? hi[1] : lo[1];
        P.pos[c][2] = sz ? hi[2] : lo[2];
    }
}

// Corner where planes i, j (existing ids) and the new plane h meet.
template <int Cap>
__device__ bool corner_of(const Poly<Cap>& P, const PlaneSrc& S, int i, int j, const double hn[3], double hoff,
                          double x[3]) {
    double an[3], bn[3], aoff, boff;
    plane_get(S, P.src, i, an, aoff);
    plane_get(S, P.src, j, bn, boff);
    double bc[3], ca[3], ab[3];
    cross3(bn, hn, bc);
    cross3(hn, an, ca);
    cross3(an, bn, ab);
    const double det = dot3(an, bc);
    const double scale = sqrt(dot3(an, an) * dot3(bn, bn) * dot3(hn, hn));
    if (!(det > 1e-13 * scale)) return false;
    const double inv = 1.0 / det;
    for (int d = 0; d < 3; ++d) x[d] = (aoff * bc[d] + boff * ca[d] + hoff * ab[d]) * inv;
    return isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]);
}

// Corners of P strictly outside the half-space (hn, hoff): bit t of out.
template <int Cap>
__device__ __forceinline__ int outside(const Poly<Cap>& P, const double hn[3], double hoff, uint64_t out[2]) {
    out[0] = 0ull;
    out[1] = 0ull;
    int nout = 0;
    for (int t = 0; t < P.nt; ++t) {
        const double v = dot3(hn, P.pos[t]) - hoff;
        if (v > 0.0) {
            out[t >> 6] |= 1ull << (t & 63);
            ++nout;
        }
    }
    return nout;
}

// Cut P by the half-space (hn, hoff), recorded as plane source `s`, given
// the nout > 0 corners outside it (bits of out).
template <int Cap>
__device__ __noinline__ int cut(Poly<Cap>& P, const PlaneSrc& S, const double hn[3], double hoff, uint8_t s,
                                const uint64_t out[2], int nout) {
    const int nt = P.nt;
    if (nout == nt) {
        P.empty = true;
        P.nt = 0;
        return EMPTY;
    }
    // Boundary of the removed region, searched inside the smaller side.
    const bool from_removed = 2 * nout <= nt;
    uint8_t side[Cap];
    int ns = 0;
    for (int t = 0; t < nt; ++t)
        if ((((out[t >> 6] >> (t & 63)) & 1ull) != 0) == from_removed) side[ns++] = (uint8_t)t;
    uint8_t ba[Cap], bb[Cap];
    int nb = 0;
    for (int i = 0; i < ns; ++i) {
        const uint8_t* T = P.tri[side[i]];
        for (int e = 0; e < 3; ++e) {
            const uint8_t a = T[e], b = T[e == 2 ? 0 : e + 1];
            int twins = 0;
            for (int k = 0; k < ns; ++k) {
                const uint8_t* U = P.tri[side[k]];
                twins += (U[0] == b && U[1] == a) + (U[1] == b && U[2] == a) + (U[2] == b && U[0] == a);
            }
            if (twins == 0) {
                if (nb >= Cap) return OVERFLOW;
                ba[nb] = from_removed ? a : b;
                bb[nb] = from_removed ? b : a;
                ++nb;
            } else if (twins != 1) {
                return SKIPPED;
            }
        }
    }
    if (nb < 3) return SKIPPED;
    const int np = P.np;
    if (np + 1 > kPlaneCap) return OVERFLOW;
    // the boundary must be one cycle
    int16_t nxt[kPlaneCap];
    for (int i = 0; i < np; ++i) nxt[i] = -1;
    for (int i = 0; i < nb; ++i) {
        if (nxt[ba[i]] != -1) return SKIPPED;
        nxt[ba[i]] = bb[i];
    }
    {
        int a = ba[0];
        int steps = 0;
        do {
            a = nxt[a];
            if (a < 0) return SKIPPED;
            ++steps;
        } while (a != (int)ba[0] && steps <= nb);
        if (steps != nb) return SKIPPED;
    }
    if (nt + nb > Cap) return OVERFLOW;
    // new corners go after the current ones until every one is known
    const uint8_t pid = (uint8_t)np;
    for (int i = 0; i < nb; ++i) {
        double x[3];
        if (!corner_of(P, S, ba[i], bb[i], hn, hoff, x)) return SKIPPED;
        P.tri[nt + i][0] = ba[i];
        P.tri[nt + i][1] = bb[i];
        P.tri[nt + i][2] = pid;
        P.pos[nt + i][0] = x[0];
        P.pos[nt + i][1] = x[1];
        P.pos[nt + i][2] = x[2];
    }
    P.src[np - 6] = s;
    P.np = np + 1;
    int w = 0;
    for (int t = 0; t < nt + nb; ++t) {
        if (t < nt && ((out[t >> 6] >> (t & 63)) & 1ull)) continue;
        if (w != t) {
            P.tri[w][0] = P.tri[t][0];
            P.tri[w][1] = P.tri[t][1];
            P.tri[w][2] = P.tri[t][2];
            P.pos[w][0] = P.pos[t][0];
            P.pos[w][1] = P.pos[t][1];
            P.pos[w][2] = P.pos[t][2];
        }
        ++w;
    }
    P.nt = w;
    return CLIPPED;
}

template <int Cap>
__device__ int clip(Poly<Cap>& P, const PlaneSrc& S, const double hn[3], double hoff, uint8_t s) {
    if (P.empty) return UNCHANGED;
    uint64_t out[2];
    const int nout = outside(P, hn, hoff, out);
    if (nout == 0) return UNCHANGED;
    return cut(P, S, hn, hoff, s, out, nout);
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

template <int Cap>
__device__ void poly_box(const Ctx& c, const Poly<Cap>& P, uint16_t out[6]) {
    if (P.empty || P.nt == 0) {
        for (int k = 0; k < 3; ++k) {
            out[k] = 65535;
            out[3 + k] = 0;
        }
        return;
    }
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int t = 0; t < P.nt; ++t)
        for (int k = 0; k < 3; ++k) {
            const double x = P.pos[t][k];
            lo[k] = x < lo[k] ? x : lo[k];
            hi[k] = hi[k] < x ? x : hi[k];
        }
    quantize_box(c, lo, hi, out);
}

// ConvexPoly(w,p) into W: the base polytope cut by the planes of Cell(w)
// (its faces on D's boundary are already faces of the base).  Returns
// false when it is empty; OVERFLOW through `ovf`.
__device__ __noinline__ bool clip_to_cell(const Ctx& c, const Poly<kBaseCap>& B, Poly<kTriCap>& W, const double* cellp, int np,
                             int64_t& skipped, bool& ovf) {
    W.nt = B.nt;
    W.np = B.np;
    W.empty = B.empty;
    for (int i = 0; i < B.np - 6; ++i) W.src[i] = B.src[i];
    for (int t = 0; t < B.nt; ++t) {
        W.tri[t][0] = B.tri[t][0];
        W.tri[t][1] = B.tri[t][1];
        W.tri[t][2] = B.tri[t][2];
        W.pos[t][0] = B.pos[t][0];
        W.pos[t][1] = B.pos[t][1];
        W.pos[t][2] = B.pos[t][2];
    }
    if (W.empty) return true;
    const PlaneSrc S{c.blo, c.bhi, c.perp, cellp};
    // Planes that leave W unchanged are passed over in a tight loop of their
    // own, so the lanes of a wavefront reach their next real cut together.
    int i = 0;
    for (;;) {
        uint64_t out[2] = {0ull, 0ull};
        int nout = 0;
        double hn[3], hoff = 0.0;
        for (; i < np; ++i) {
            hn[0] = cellp[4 * i];
            hn[1] = cellp[4 * i + 1];
            hn[2] = cellp[4 * i + 2];
            hoff = cellp[4 * i + 3];
            const int axes = (hn[0] != 0.0) + (hn[1] != 0.0) + (hn[2] != 0.0);
            if (axes == 1 && (fabs(hn[0]) == 1.0 || fabs(hn[1]) == 1.0 || fabs(hn[2]) == 1.0)) {
                const int k = hn[0] != 0.0 ? 0 : (hn[1] != 0.0 ? 1 : 2);
                if ((hn[k] > 0 && hoff == c.bhi[k]) || (hn[k] < 0 && hoff == -c.blo[k])) continue;
            }
            nout = outside(W, hn, hoff, out);
            if (nout > 0) break;
        }
        if (i >= np) return true;
        const int r = cut(W, S, hn, hoff, (uint8_t)(8 + i), out, nout);
        if (r == EMPTY) return false;
        if (r == SKIPPED) ++skipped;
        if (r == OVERFLOW) {
            ovf = true;
            return false;
        }
        ++i;
    }
}

// Open-addressing set of visited vertices: true when u is new.  Never full:
// it has twice the slots of the most vertices a flood may visit.
__device__ __forceinline__ bool hash_visit(int32_t* hset, int32_t u) {
    uint32_t h = ((uint32_t)u * 2654435761u) & (kHashCap - 1);
    for (;;) {
        if (hset[h] == u) return false;
        if (hset[h] < 0) {
            hset[h] = u;
            return true;
        }
        h = (h + 1) & (kHashCap - 1);
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

// Each lane takes primitives from a shared counter and runs one flood step
// (one visited vertex) per trip of a single loop; a lane whose flood has
// ended takes the next primitive at once instead of waiting for the longest
// flood of its wavefront.
__global__ __launch_bounds__(64) void k_flood(int64_t nprim, const FloodPrim* __restrict__ prims,
                                              const double* __restrict__ perp, const double* __restrict__ Vd,
                                              const int64_t* __restrict__ nb_off, const int32_t* __restrict__ nb,
                                              const uint64_t* __restrict__ cpoff, const double* __restrict__ cplanes,
                                              const uint64_t* __restrict__ ctoff, const double* __restrict__ cpos,
                                              const double* __restrict__ dom,  // blo, bhi, qlo, qscale, tau, dmax
                                              FloodRec* __restrict__ recs, uint64_t rec_cap,
                                              int64_t* __restrict__ redo, Counters* __restrict__ cnt,
                                              int visit_cap) {
    Ctx c;
    c.blo = dom;
    c.bhi = dom + 3;
    c.qlo = dom + 6;
    c.qscale = dom + 9;
    c.slack = 2.0 * dom[12] * dom[13];
    // lane totals over the primitives it finished
    unsigned long long t_tests = 0, t_hits = 0, t_quick = 0, t_skipped = 0;
    // the current primitive
    int64_t i = -1;
    FloodPrim p;
    uint32_t code = 0;
    int64_t tests = 0, hits = 0, quick = 0, skipped = 0;
    bool ovf = false, base_empty = false;
    int head = 0, qn = 0;
    Poly<kBaseCap> B;
    Poly<kTriCap> W;
    int32_t queue[kQueueCap];
    int32_t hset[kHashCap];
    for (;;) {
        if (ovf || head >= qn) {
            // the current primitive is done: account for it, take the next
            if (i >= 0) {
                if (ovf) {
                    const unsigned long long slot = atomicAdd(&cnt->redo, 1ull);
                    redo[slot] = i;
                } else {
                    t_tests += (unsigned long long)tests;
                    t_hits += (unsigned long long)hits;
                    t_quick += (unsigned long long)quick;
                    t_skipped += (unsigned long long)skipped;
                }
            }
            i = (int64_t)atomicAdd(&cnt->next, 1ull);
            if (i >= nprim) break;
            p = prims[i];
            c.perp = perp + 4 * p.perp_off;
            code = (p.face ? 0x80000000u : 0u) | (uint32_t)p.id;
            tests = hits = quick = skipped = 0;
            ovf = false;
            // base polytope Space-perp(p) n D
            init_box(B, c.blo, c.bhi);
            base_empty = false;
            {
                const PlaneSrc S{c.blo, c.bhi, c.perp, nullptr};
                for (int j = 0; j < p.nperp && !base_empty && !ovf; ++j) {
                    const double hn[3] = {c.perp[4 * j], c.perp[4 * j + 1], c.perp[4 * j + 2]};
                    const int r = clip(B, S, hn, c.perp[4 * j + 3], (uint8_t)j);
                    if (r == EMPTY) base_empty = true;
                    if (r == SKIPPED) ++skipped;
                    if (r == OVERFLOW) ovf = true;
                }
            }
            for (int k = 0; k < kHashCap; ++k) hset[k] = -1;
            qn = 0;
            head = 0;
            for (int k = 0; k < p.nverts; ++k) {
                hash_visit(hset, p.verts[k]);
                queue[qn++] = p.verts[k];
            }
            continue;
        }
        // one flood step: the next queued vertex w
        const int32_t w = queue[head++];
        bool own = false;
        for (int k = 0; k < p.nverts; ++k) own |= (p.verts[k] == w);
        const double* cellp = cplanes + 4 * cpoff[w];
        const int cnp = (int)(cpoff[w + 1] - cpoff[w]);
        if (cnp > kPlaneCap - 8 - 8) {
            ovf = true;
            continue;
        }
        uint16_t box[6];
        bool hit;
        if (own) {  // Theorem 2
            if (base_empty || !clip_to_cell(c, B, W, cellp, cnp, skipped, ovf)) W.empty = true;
            if (ovf) continue;
            poly_box(c, W, box);
            hit = true;
        } else {
            ++tests;
            const double* X = Vd + 3 * (int64_t)w;
            const double Wv[3] = {X[0], X[1], X[2]};
            // |x-w| - Dist(x,p) is convex: the whole cell keeping w out settles it
            const int64_t t0 = (int64_t)ctoff[w], t1 = (int64_t)ctoff[w + 1];
            bool all_far = true;
            for (int64_t t = t0; t < t1 && all_far; ++t) all_far = far_enough(p, Wv, cpos + 3 * t, c.slack);
            hit = false;
            if (all_far) {
                ++quick;
            } else if (!base_empty && clip_to_cell(c, B, W, cellp, cnp, skipped, ovf)) {
                for (int t = 0; t < W.nt; ++t)
                    if (!far_enough(p, Wv, W.pos[t], c.slack)) {
                        poly_box(c, W, box);
                        hit = true;
                        break;
                    }
            }
            if (ovf) continue;
        }
        if (!hit) continue;
        ++hits;
        const unsigned long long slot = atomicAdd(&cnt->recs, 1ull);
        if (slot < rec_cap) {
            FloodRec r;
            r.v = (uint32_t)w;
            r.code = code;
            for (int k = 0; k < 6; ++k) r.box[k] = box[k];
            recs[slot] = r;
        }
        for (int64_t k = nb_off[w]; k < nb_off[w + 1]; ++k) {
            const int32_t u = nb[k];
            if (!hash_visit(hset, u)) continue;
            if (qn >= visit_cap) {
                ovf = true;
                break;
            }
            queue[qn++] = u;
        }
    }
    atomicAdd(&cnt->tests, t_tests);
    atomicAdd(&cnt->hits, t_hits);
    atomicAdd(&cnt->quick, t_quick);
    atomicAdd(&cnt->skipped, t_skipped);
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
    const FlatCells& cs = *in.cells;
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
    const Part parts[] = {
        {in.prims, sizeof(FloodPrim) * (size_t)in.nprim},
        {in.perp, sizeof(double) * 4 * (size_t)std::max<int64_t>(1, in.nperp_total)},
        {in.Vd, sizeof(double) * 3 * nv},
        {in.nb_off, sizeof(int64_t) * (nv + 1)},
        {in.nb, sizeof(int32_t) * std::max<size_t>(1, (size_t)in.nb_off[nv])},
        {cs.poff.data(), sizeof(uint64_t) * (nv + 1)},
        {cs.planes.data(), sizeof(double) * std::max<size_t>(4, cs.planes.size())},
        {cs.toff.data(), sizeof(uint64_t) * (nv + 1)},
        {cs.pos.data(), sizeof(double) * std::max<size_t>(3, cs.pos.size())},
        {dom, sizeof(dom)},
    };
    constexpr int kParts = sizeof(parts) / sizeof(parts[0]);
    size_t off[kParts + 3];
    size_t total = 0;
    for (int k = 0; k < kParts; ++k) {
        off[k] = total;
        total += (parts[k].bytes + 255) / 256 * 256;
    }
    off[kParts] = total;  // records
    total += (sizeof(FloodRec) * rec_cap + 255) / 256 * 256;
    off[kParts + 1] = total;  // redo list
    total += (sizeof(int64_t) * (size_t)in.nprim + 255) / 256 * 256;
    off[kParts + 2] = total;  // counters
    total += 256;
    DevBuf buf;
    if (!hip_ok(hipMalloc(&buf.p, total), "hipMalloc")) return false;
    char* d = (char*)buf.p;
    for (int k = 0; k < kParts; ++k)
        if (parts[k].src && parts[k].bytes &&
            !hip_ok(hipMemcpy(d + off[k], parts[k].src, parts[k].bytes, hipMemcpyHostToDevice), "upload"))
            return false;
    if (!hip_ok(hipMemset(d + off[kParts + 2], 0, sizeof(Counters)), "hipMemset")) return false;
    if (!hip_ok(hipDeviceSynchronize(), "upload")) return false;
    out.t_upload = since(t0);
    t0 = Clock::now();
    // enough wavefronts to fill the chip; each lane loops over primitives
    const int block = 64;
    int dev = 0, cus = 256, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_flood, block, 0) != hipSuccess || per_cu < 1) per_cu = 8;
    const int64_t grid = std::min<int64_t>((in.nprim + block - 1) / block, (int64_t)cus * per_cu);
    k_flood<<<(unsigned)grid, block, 0, 0>>>(
        in.nprim, (const FloodPrim*)(d + off[0]), (const double*)(d + off[1]), (const double*)(d + off[2]),
        (const int64_t*)(d + off[3]), (const int32_t*)(d + off[4]), (const uint64_t*)(d + off[5]),
        (const double*)(d + off[6]), (const uint64_t*)(d + off[7]), (const double*)(d + off[8]),
        (const double*)(d + off[9]), (FloodRec*)(d + off[kParts]), rec_cap, (int64_t*)(d + off[kParts + 1]),
        (Counters*)(d + off[kParts + 2]), in.visit_cap > 0 && in.visit_cap < kQueueCap ? in.visit_cap : kQueueCap);
    if (!hip_ok(hipGetLastError(), "launch")) return false;
    if (!hip_ok(hipDeviceSynchronize(), "kernel")) return false;
    out.t_kernel = since(t0);
    t0 = Clock::now();
    Counters c;
    if (!hip_ok(hipMemcpy(&c, d + off[kParts + 2], sizeof(c), hipMemcpyDeviceToHost), "download")) return false;
    if (c.recs > rec_cap) {
        err = "device inspection: more table entries than the record buffer holds";
        return false;
    }
    out.recs.resize((size_t)c.recs);
    out.redo.resize((size_t)c.redo);
    if (c.recs && !hip_ok(hipMemcpy(out.recs.data(), d + off[kParts], sizeof(FloodRec) * c.recs,
                                    hipMemcpyDeviceToHost), "download"))
        return false;
    if (c.redo && !hip_ok(hipMemcpy(out.redo.data(), d + off[kParts + 1], sizeof(int64_t) * c.redo,
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
