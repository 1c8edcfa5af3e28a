#include "interception.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

#include "convex_cell.hpp"
#include "delaunay.hpp"

#ifdef _OPENMP
#include <omp.h>
#include <parallel/algorithm>
#endif

namespace p2m {

namespace {

using Clock = std::chrono::steady_clock;
double since(Clock::time_point t0) { return std::chrono::duration<double>(Clock::now() - t0).count(); }

inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
inline void normalize3(double* a) {
    double l = std::sqrt(dot3(a, a));
    a[0] /= l;
    a[1] /= l;
    a[2] /= l;
}
inline double dist3(const double* a, const double* b) {
    double d[3] = {a[0] - b[0], a[1] - b[1], a[2] - b[2]};
    return std::sqrt(dot3(d, d));
}

int num_threads(int requested) {
#ifdef _OPENMP
    return requested > 0 ? requested : omp_get_max_threads();
#else
    (void)requested;
    return 1;
#endif
}

// Voronoi cells of all vertices, clipped to D, in per-thread flat buffers.
struct CellStore {
    struct Ref {
        int32_t thread;
        uint32_t np, nt;
        uint64_t poff, toff;
    };
    std::vector<Ref> ref;
    std::vector<std::vector<double>> planes, pos;
    std::vector<std::vector<uint16_t>> tris;

    void load(int64_t v, ConvexCell& c) const {
        const Ref& r = ref[(size_t)v];
        c.load(planes[(size_t)r.thread].data() + 4 * r.poff, r.np, tris[(size_t)r.thread].data() + 3 * r.toff,
               pos[(size_t)r.thread].data() + 3 * r.toff, r.nt);
    }
};

// Space-perp(p) as half-spaces, the vertices of p, and the distance from a
// point to the line (edge) or plane (face) of p.
struct Primitive {
    bool face;
    int nverts;
    int32_t verts[3];
    double a[3];  // a point of p
    double dir[3];  // unit edge direction, or unit face normal
    HalfSpace perp[8];
    int nperp;

    double dist(const double* x) const {
        double d[3] = {x[0] - a[0], x[1] - a[1], x[2] - a[2]};
        if (face) return std::fabs(dot3(d, dir));
        double c[3];
        cross3(d, dir, c);
        return std::sqrt(dot3(c, c));
    }
};

void make_face(const MeshData& m, int64_t f, double tau, Primitive& p) {
    p.face = true;
    p.nverts = 3;
    const double* P[3];
    for (int s = 0; s < 3; ++s) {
        p.verts[s] = m.F[(size_t)(3 * f + s)];
        P[s] = &m.Vd[3 * (size_t)p.verts[s]];
    }
    std::memcpy(p.a, P[0], sizeof(p.a));
    double u[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
    double w[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
    cross3(u, w, p.dir);
    normalize3(p.dir);
    p.nperp = 0;
    for (int s = 0; s < 3; ++s) {
        const double* A = P[s];
        const double* B = P[(s + 1) % 3];
        const double* C = P[(s + 2) % 3];
        double e[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
        double mm[3];
        cross3(e, p.dir, mm);
        normalize3(mm);
        double ac[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
        if (dot3(mm, ac) < 0) {
            mm[0] = -mm[0];
            mm[1] = -mm[1];
            mm[2] = -mm[2];
        }
        // Space-perp(f) keeps the side of the vertical plane through (A,B) holding C.
        HalfSpace h{{-mm[0], -mm[1], -mm[2]}, -dot3(mm, A) + tau};
        p.perp[p.nperp++] = h;
    }
}

void make_edge(const MeshData& m, int64_t e, double tau, Primitive& p) {
    p.face = false;
    p.nverts = 2;
    p.verts[0] = m.E[(size_t)(2 * e)];
    p.verts[1] = m.E[(size_t)(2 * e + 1)];
    const double* A = &m.Vd[3 * (size_t)p.verts[0]];
    const double* B = &m.Vd[3 * (size_t)p.verts[1]];
    std::memcpy(p.a, A, sizeof(p.a));
    double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    std::memcpy(p.dir, u, sizeof(u));
    normalize3(p.dir);
    p.nperp = 0;
    // the two end planes
    p.perp[p.nperp++] = HalfSpace{{-p.dir[0], -p.dir[1], -p.dir[2]}, -dot3(p.dir, A) + tau};
    p.perp[p.nperp++] = HalfSpace{{p.dir[0], p.dir[1], p.dir[2]}, dot3(p.dir, B) + tau};
    // for every incident face, the side of its vertical plane away from the face
    for (int64_t k = m.ef_off[(size_t)e]; k < m.ef_off[(size_t)e + 1] && p.nperp < 8; ++k) {
        int64_t f = m.ef_face[(size_t)k];
        int32_t c = -1;
        for (int s = 0; s < 3; ++s) {
            int32_t x = m.F[(size_t)(3 * f + s)];
            if (x != p.verts[0] && x != p.verts[1]) c = x;
        }
        const double* C = &m.Vd[3 * (size_t)c];
        double w[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
        double nf[3];
        cross3(u, w, nf);
        normalize3(nf);
        double mm[3];
        cross3(u, nf, mm);
        normalize3(mm);
        if (dot3(mm, w) < 0) {
            mm[0] = -mm[0];
            mm[1] = -mm[1];
            mm[2] = -mm[2];
        }
        p.perp[p.nperp++] = HalfSpace{{mm[0], mm[1], mm[2]}, dot3(mm, A) + tau};
    }
}

struct ThreadCtx {
    ConvexCell cell;
    std::vector<uint32_t> stamp;
    uint32_t cur = 0;
    std::vector<int32_t> queue;
    std::vector<uint64_t> pairs;
    int64_t tests = 0, hits = 0, quick = 0, skipped = 0;
};

// Convexity filter (Theorems 5/6) on ConvexPoly(w,p) = Cell(w) n Space-perp(p).
bool intercepts(const MeshData& m, const CellStore& cs, int64_t w, const Primitive& p, double tau, ThreadCtx& c) {
    ++c.tests;
    cs.load(w, c.cell);
    const double* W = &m.Vd[3 * (size_t)w];
    // The filtered quantity |x-w| - Dist(x, p) is convex, so if it is below
    // -tau on every corner of the whole cell it is below on any sub-polytope.
    bool all_far = true;
    for (size_t t = 0; t < c.cell.num_corners() && all_far; ++t) {
        const double* x = c.cell.corner(t);
        all_far = dist3(x, W) <= p.dist(x) - tau;
    }
    if (all_far) {
        ++c.quick;
        return false;
    }
    for (int i = 0; i < p.nperp; ++i) {
        ConvexCell::ClipResult r = c.cell.clip(p.perp[i]);
        if (r == ConvexCell::EMPTY) return false;
        if (r == ConvexCell::SKIPPED) ++c.skipped;
    }
    for (size_t t = 0; t < c.cell.num_corners(); ++t) {
        const double* x = c.cell.corner(t);
        if (dist3(x, W) > p.dist(x) - tau) return true;
    }
    return false;
}

inline uint64_t pair_key(int64_t v, bool face, int64_t id) {
    return ((uint64_t)v << 32) | (face ? 0x80000000ull : 0ull) | (uint64_t)id;
}

void flood(const MeshData& m, const CellStore& cs, const Table& t, const Primitive& p, int64_t pid, double tau,
           ThreadCtx& c) {
    if (++c.cur == 0) {
        std::fill(c.stamp.begin(), c.stamp.end(), 0u);
        c.cur = 1;
    }
    c.queue.clear();
    for (int i = 0; i < p.nverts; ++i) {
        c.queue.push_back(p.verts[i]);
        c.stamp[(size_t)p.verts[i]] = c.cur;
    }
    for (size_t head = 0; head < c.queue.size(); ++head) {
        int32_t w = c.queue[head];
        bool own = false;
        for (int i = 0; i < p.nverts; ++i) own |= (p.verts[i] == w);
        bool hit = own || intercepts(m, cs, w, p, tau, c);  // Theorem 2 for the primitive's own vertices
        if (!hit) continue;
        ++c.hits;
        c.pairs.push_back(pair_key(w, p.face, pid));
        for (int64_t k = t.nb_off[(size_t)w]; k < t.nb_off[(size_t)w + 1]; ++k) {
            int32_t u = t.nb[(size_t)k];
            if (c.stamp[(size_t)u] == c.cur) continue;
            c.stamp[(size_t)u] = c.cur;
            c.queue.push_back(u);
        }
    }
}

}  // namespace

bool build_table(const MeshData& m, const TableOptions& o, Table& t, TableStats& st, std::string& err) {
    const int64_t nv = m.nv;
    const int nth = num_threads(o.threads);
    // 1. Voronoi neighbours
    auto t0 = Clock::now();
    {
        DelaunayStats ds;
        if (!delaunay_neighbors(m.Vd.data(), nv, o.lo, o.hi, t.nb_off, t.nb, &ds)) {
            err = "duplicate vertices";
            return false;
        }
        st.delaunay_edges = ds.edges;
        st.tets = ds.tets;
        st.exact_predicates = ds.exact_predicates;
    }
    st.t_delaunay = since(t0);

    // 2. Voronoi cells clipped to D (box moved outward by tau)
    t0 = Clock::now();
    CellStore cs;
    cs.ref.resize((size_t)nv);
    cs.planes.resize((size_t)nth);
    cs.pos.resize((size_t)nth);
    cs.tris.resize((size_t)nth);
    int64_t skipped_cells = 0;
    double blo[3], bhi[3];
    for (int k = 0; k < 3; ++k) {
        blo[k] = o.lo[k] - o.tau;
        bhi[k] = o.hi[k] + o.tau;
    }
#pragma omp parallel num_threads(nth) reduction(+ : skipped_cells)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        ConvexCell cell;
        std::vector<std::pair<double, int32_t>> order;
        auto& P = cs.planes[(size_t)tid];
        auto& X = cs.pos[(size_t)tid];
        auto& T = cs.tris[(size_t)tid];
#pragma omp for schedule(dynamic, 256)
        for (int64_t v = 0; v < nv; ++v) {
            const double* pv = &m.Vd[3 * (size_t)v];
            cell.init_box(blo, bhi);
            order.clear();
            for (int64_t k = t.nb_off[(size_t)v]; k < t.nb_off[(size_t)v + 1]; ++k) {
                int32_t w = t.nb[(size_t)k];
                const double* pw = &m.Vd[3 * (size_t)w];
                double d[3] = {pw[0] - pv[0], pw[1] - pv[1], pw[2] - pv[2]};
                order.push_back({dot3(d, d), w});
            }
            std::sort(order.begin(), order.end());
            for (const auto& e : order) {
                const double* pw = &m.Vd[3 * (size_t)e.second];
                HalfSpace h;
                for (int k = 0; k < 3; ++k) h.n[k] = pw[k] - pv[k];
                double nl = std::sqrt(dot3(h.n, h.n));
                // bisector of v and w, on v's side, moved outward by tau
                h.off = 0.5 * (dot3(pw, pw) - dot3(pv, pv)) + o.tau * nl;
                if (cell.clip(h) == ConvexCell::SKIPPED) ++skipped_cells;
            }
            cell.compact();
            CellStore::Ref r;
            r.thread = tid;
            r.poff = P.size() / 4;
            r.toff = T.size() / 3;
            cell.save(P, T, X);
            r.np = (uint32_t)(P.size() / 4 - r.poff);
            r.nt = (uint32_t)(T.size() / 3 - r.toff);
            cs.ref[(size_t)v] = r;
        }
    }
    st.skipped_clips += skipped_cells;
    st.t_cells = since(t0);

    // 3. inspection
    t0 = Clock::now();
    std::vector<ThreadCtx> ctx((size_t)nth);
    const int64_t nprim = m.ne + m.nf;
#pragma omp parallel num_threads(nth)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        ThreadCtx& c = ctx[(size_t)tid];
        c.stamp.assign((size_t)nv, 0u);
        Primitive p;
#pragma omp for schedule(dynamic, 64)
        for (int64_t q = 0; q < nprim; ++q) {
            bool face = q >= m.ne;
            int64_t id = face ? q - m.ne : q;
            if (face) make_face(m, id, o.tau, p);
            else make_edge(m, id, o.tau, p);
            if (o.mode == TABLE_FLOODING) {
                flood(m, cs, t, p, id, o.tau, c);
            } else {
                for (int64_t w = 0; w < nv; ++w) {
                    bool own = false;
                    for (int i = 0; i < p.nverts; ++i) own |= (p.verts[i] == w);
                    if (o.mode == TABLE_EVERYTHING || own || intercepts(m, cs, w, p, o.tau, c))
                        c.pairs.push_back(pair_key(w, face, id));
                }
            }
        }
    }
    std::vector<uint64_t> pairs;
    {
        size_t tot = 0;
        for (auto& c : ctx) tot += c.pairs.size();
        pairs.reserve(tot);
        for (auto& c : ctx) {
            pairs.insert(pairs.end(), c.pairs.begin(), c.pairs.end());
            std::vector<uint64_t>().swap(c.pairs);
            st.flood_tests += c.tests;
            st.flood_hits += c.hits;
            st.quick_rejects += c.quick;
            st.skipped_clips += c.skipped;
        }
    }
    st.t_flood = since(t0);

    // 4. CSR: per vertex, edge ids then face ids, each ascending
    t0 = Clock::now();
#ifdef _OPENMP
    __gnu_parallel::sort(pairs.begin(), pairs.end());
#else
    std::sort(pairs.begin(), pairs.end());
#endif
    if (pairs.size() >= (size_t)UINT32_MAX) {
        err = "interception table exceeds 2^32 entries";
        return false;
    }
    t.off.assign((size_t)(2 * nv + 1), 0u);
    t.ent.resize(pairs.size());
    std::vector<uint32_t> ecount((size_t)nv, 0), fcount((size_t)nv, 0);
    for (size_t i = 0; i < pairs.size(); ++i) {
        uint64_t k = pairs[i];
        int64_t v = (int64_t)(k >> 32);
        uint32_t code = (uint32_t)(k & 0xffffffffu);
        t.ent[i] = (int32_t)(code & 0x7fffffffu);
        if (code & 0x80000000u) fcount[(size_t)v]++;
        else ecount[(size_t)v]++;
    }
    uint32_t acc = 0;
    for (int64_t v = 0; v < nv; ++v) {
        t.off[(size_t)(2 * v)] = acc;
        acc += ecount[(size_t)v];
        t.off[(size_t)(2 * v + 1)] = acc;
        acc += fcount[(size_t)v];
        st.nnz_edges += ecount[(size_t)v];
        st.nnz_faces += fcount[(size_t)v];
        st.max_list = std::max<int64_t>(st.max_list, (int64_t)ecount[(size_t)v] + fcount[(size_t)v]);
    }
    t.off[(size_t)(2 * nv)] = acc;
    st.t_pack = since(t0);
    return true;
}

}  // namespace p2m
