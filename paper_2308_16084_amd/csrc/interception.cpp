#include "interception.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <unordered_map>

#include "convex_cell.hpp"
#include "delaunay.hpp"
#include "flood_device.hpp"

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

int num_threads(int requested) {
#ifdef _OPENMP
    return requested > 0 ? requested : omp_get_max_threads();
#else
    (void)requested;
    return 1;
#endif
}

// Voronoi cell of vertex v clipped to the box blo..bhi (D grown by tau): the
// box cut by the bisector of v and each Voronoi (Delaunay) neighbour, nearest
// first (ties by id), each moved outward by tau; planes that bound no corner
// dropped.  Returns the number of cuts skipped.
int64_t build_cell(const MeshData& m, const Table& t, int64_t v, const double blo[3], const double bhi[3],
                   double tau, ConvexCell& cell, std::vector<std::pair<double, int32_t>>& order) {
    int64_t skipped = 0;
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
        h.off = 0.5 * (dot3(pw, pw) - dot3(pv, pv)) + tau * nl;
        if (cell.clip(h) == ConvexCell::SKIPPED) ++skipped;
    }
    cell.compact();
    return skipped;
}

// Voronoi cells of all vertices, clipped to D, in per-thread flat buffers;
// or, when `lazy`, each built on first use (the inspection on the device
// builds its own and the host needs only those of the primitives it takes
// back).  The inspection reads a cell's planes and corners.
struct CellStore {
    bool lazy = false;
    const MeshData* m = nullptr;
    const Table* t = nullptr;
    double blo[3], bhi[3], tau = 0;
    struct Built {
        std::vector<double> planes, pos;
    };
    mutable std::mutex mu;
    mutable std::unordered_map<int64_t, Built> built;

    const Built& get(int64_t v) const {
        std::lock_guard<std::mutex> g(mu);
        auto it = built.find(v);
        if (it != built.end()) return it->second;
        ConvexCell cell;
        std::vector<std::pair<double, int32_t>> order;
        build_cell(*m, *t, v, blo, bhi, tau, cell, order);
        Built b;
        std::vector<uint16_t> tris;
        cell.save(b.planes, tris, b.pos);
        return built.emplace(v, std::move(b)).first->second;
    }

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
    const double* corners(int64_t v, uint32_t& n) const {
        if (lazy) {
            const Built& b = get(v);
            n = (uint32_t)(b.pos.size() / 3);
            return b.pos.data();
        }
        const Ref& r = ref[(size_t)v];
        n = r.nt;
        return pos[(size_t)r.thread].data() + 3 * r.toff;
    }
    const double* plane_data(int64_t v, uint32_t& n) const {
        if (lazy) {
            const Built& b = get(v);
            n = (uint32_t)(b.planes.size() / 4);
            return b.planes.data();
        }
        const Ref& r = ref[(size_t)v];
        n = r.np;
        return planes[(size_t)r.thread].data() + 4 * r.poff;
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

    // squared distance to the line (edge) or plane (face)
    double dist2(const double* x) const {
        double d[3] = {x[0] - a[0], x[1] - a[1], x[2] - a[2]};
        if (face) {
            double h = dot3(d, dir);
            return h * h;
        }
        double c[3];
        cross3(d, dir, c);
        return dot3(c, c);
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

// A table entry before packing: key (vertex, kind, id) and the entry's box.
struct PairRec {
    uint64_t key;
    uint16_t box[6];
};

struct ThreadCtx {
    ConvexCell cell, base;
    double blo_[3], bhi_[3];
    double qlo_[3], qscale_[3];  // 16-bit frame of D for the entry boxes
    std::vector<uint32_t> stamp;
    uint32_t cur = 0;
    std::vector<int32_t> queue;
    std::vector<PairRec> pairs;
    int64_t tests = 0, hits = 0, quick = 0, skipped = 0;
};

// Entry box (Sec. 4.6: the bounding box of Region(w,p), here of the larger
// ConvexPoly(w,p) = Cell(w) n Space-perp(p) n D with every half-space moved
// out by tau) in the 16-bit frame of D, rounded outward by one more unit.
// Lower corner 65535 and upper 0 on every axis: an empty polytope.
void quantize_box(const ThreadCtx& c, const double lo[3], const double hi[3], uint16_t out[6]) {
    for (int k = 0; k < 3; ++k) {
        const double a = std::floor((lo[k] - c.qlo_[k]) * c.qscale_[k]) - 1.0;
        const double b = std::ceil((hi[k] - c.qlo_[k]) * c.qscale_[k]) + 1.0;
        out[k] = (uint16_t)std::min(65535.0, std::max(0.0, a));
        out[3 + k] = (uint16_t)std::min(65535.0, std::max(0.0, b));
    }
}

void cell_box(const ThreadCtx& c, const ConvexCell& cell, uint16_t out[6]) {
    if (cell.empty() || cell.num_corners() == 0) {
        for (int k = 0; k < 3; ++k) {
            out[k] = 65535;
            out[3 + k] = 0;
        }
        return;
    }
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (size_t t = 0; t < cell.num_corners(); ++t) {
        const double* x = cell.corner(t);
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], x[k]);
            hi[k] = std::max(hi[k], x[k]);
        }
    }
    quantize_box(c, lo, hi, out);
}

void full_box(uint16_t out[6]) {
    for (int k = 0; k < 3; ++k) {
        out[k] = 0;
        out[3 + k] = 65535;
    }
}

// Space-perp(p) n D (all half-spaces moved outward by tau), built once per
// primitive; ConvexPoly(w,p) is then this polytope cut by w's cell planes.
// base_empty: the primitive's Space-perp misses D altogether.
void make_base(const Primitive& p, const double blo[3], const double bhi[3], ThreadCtx& c, bool& base_empty) {
    c.base.init_box(blo, bhi);
    base_empty = false;
    for (int i = 0; i < p.nperp && !base_empty; ++i) {
        ConvexCell::ClipResult r = c.base.clip(p.perp[i]);
        if (r == ConvexCell::EMPTY) base_empty = true;
        if (r == ConvexCell::SKIPPED) ++c.skipped;
    }
}

// ConvexPoly(w,p) into c.cell: the base polytope cut by w's cell planes.
// False when it is empty.
bool clip_to_cell(const CellStore& cs, int64_t w, ThreadCtx& c) {
    c.cell = c.base;
    uint32_t np = 0;
    const double* H = cs.plane_data(w, np);
    for (uint32_t i = 0; i < np; ++i) {
        HalfSpace h{{H[4 * i], H[4 * i + 1], H[4 * i + 2]}, H[4 * i + 3]};
        // the cell's domain-box faces are already faces of the base polytope
        const int axes = (h.n[0] != 0.0) + (h.n[1] != 0.0) + (h.n[2] != 0.0);
        if (axes == 1 && (std::fabs(h.n[0]) == 1.0 || std::fabs(h.n[1]) == 1.0 || std::fabs(h.n[2]) == 1.0)) {
            const int k = h.n[0] != 0.0 ? 0 : (h.n[1] != 0.0 ? 1 : 2);
            if ((h.n[k] > 0 && h.off == c.bhi_[k]) || (h.n[k] < 0 && h.off == -c.blo_[k])) continue;
        }
        ConvexCell::ClipResult r = c.cell.clip(h);
        if (r == ConvexCell::EMPTY) return false;
        if (r == ConvexCell::SKIPPED) ++c.skipped;
    }
    return true;
}

// Box of ConvexPoly(w,p) for a vertex of p itself (Theorem 2 keeps it in
// the list without the filter).
void own_box(const CellStore& cs, int64_t w, bool base_empty, ThreadCtx& c, uint16_t out[6]) {
    if (base_empty || !clip_to_cell(cs, w, c)) {
        c.cell = ConvexCell();
        cell_box(c, c.cell, out);
        return;
    }
    cell_box(c, c.cell, out);
}

// Convexity filter (Theorems 5/6) on ConvexPoly(w,p) = Cell(w) n Space-perp(p).
// A corner x keeps w out when |x-w| <= Dist(x,p) - tau; with Dist <= dmax this
// follows from the squared test |x-w|^2 + 2 tau dmax <= Dist^2, used here.
// On a hit, box receives the entry box of (w,p).
bool intercepts(const MeshData& m, const CellStore& cs, int64_t w, const Primitive& p, double tau, double dmax,
                bool base_empty, ThreadCtx& c, uint16_t box[6]) {
    ++c.tests;
    const double* W = &m.Vd[3 * (size_t)w];
    const double slack = 2.0 * tau * dmax;
    auto far_enough = [&](const double* x) {
        double d[3] = {x[0] - W[0], x[1] - W[1], x[2] - W[2]};
        return dot3(d, d) + slack <= p.dist2(x);
    };
    // |x-w| - Dist(x, p) is convex, so if every corner of the whole cell keeps
    // w out, every corner of any sub-polytope does too.
    uint32_t nc = 0;
    const double* X = cs.corners(w, nc);
    bool all_far = true;
    for (uint32_t t = 0; t < nc && all_far; ++t) all_far = far_enough(X + 3 * t);
    if (all_far) {
        ++c.quick;
        return false;
    }
    if (base_empty) return false;
    if (!clip_to_cell(cs, w, c)) return false;
    for (size_t t = 0; t < c.cell.num_corners(); ++t)
        if (!far_enough(c.cell.corner(t))) {
            cell_box(c, c.cell, box);
            return true;
        }
    return false;
}

inline uint64_t pair_key(int64_t v, bool face, int64_t id) {
    return ((uint64_t)v << 32) | (face ? 0x80000000ull : 0ull) | (uint64_t)id;
}

void flood(const MeshData& m, const CellStore& cs, const Table& t, const Primitive& p, int64_t pid, double tau,
           double dmax, bool base_empty, ThreadCtx& c) {
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
        PairRec rec;
        rec.key = pair_key(w, p.face, pid);
        bool hit;
        if (own) {  // Theorem 2
            own_box(cs, w, base_empty, c, rec.box);
            hit = true;
        } else {
            hit = intercepts(m, cs, w, p, tau, dmax, base_empty, c, rec.box);
        }
        if (!hit) continue;
        ++c.hits;
        c.pairs.push_back(rec);
        for (int64_t k = t.nb_off[(size_t)w]; k < t.nb_off[(size_t)w + 1]; ++k) {
            int32_t u = t.nb[(size_t)k];
            if (c.stamp[(size_t)u] == c.cur) continue;
            c.stamp[(size_t)u] = c.cur;
            c.queue.push_back(u);
        }
    }
}

// The device inspection: the cells and then the filter and flooding of
// every primitive on the device, from the primitives' Space-perp
// half-spaces; it returns every entry of the primitives it finished and the
// list of those it hands back (their entries, if any, are dropped here; the
// host floods them afterwards, with cells it builds on demand).
bool inspect_on_device(const MeshData& m, const CellStore& cs, const Table& t, const TableOptions& o,
                       const double blo[3], const double bhi[3], double dmax, int nth, std::vector<PairRec>& pairs,
                       std::vector<int64_t>& redo, TableStats& st, std::string& err) {
    const int64_t nv = m.nv, nprim = m.ne + m.nf;
    // half-spaces per primitive: a face has 3, an edge its 2 end planes and
    // one per incident face, 8 at most (as make_edge keeps them)
    std::vector<FloodPrim> prims((size_t)nprim);
    std::vector<int64_t> poff((size_t)nprim + 1, 0);
    for (int64_t q = 0; q < nprim; ++q) {
        const int64_t np = q >= m.ne ? 3 : std::min<int64_t>(8, 2 + (m.ef_off[(size_t)q + 1] - m.ef_off[(size_t)q]));
        poff[(size_t)q + 1] = poff[(size_t)q] + np;
    }
    std::vector<double> perp(4 * (size_t)std::max<int64_t>(1, poff[(size_t)nprim]));
#pragma omp parallel num_threads(nth)
    {
        Primitive p;
#pragma omp for schedule(static, 1024)
        for (int64_t q = 0; q < nprim; ++q) {
            const bool face = q >= m.ne;
            const int64_t id = face ? q - m.ne : q;
            if (face) make_face(m, id, o.tau, p);
            else make_edge(m, id, o.tau, p);
            FloodPrim& f = prims[(size_t)q];
            std::memcpy(f.a, p.a, sizeof(f.a));
            std::memcpy(f.dir, p.dir, sizeof(f.dir));
            for (int k = 0; k < 3; ++k) f.verts[k] = k < p.nverts ? p.verts[k] : -1;
            f.nverts = p.nverts;
            f.face = face ? 1 : 0;
            f.nperp = p.nperp;
            f.perp_off = poff[(size_t)q];
            f.id = id;
            for (int k = 0; k < p.nperp; ++k) {
                double* h = &perp[4 * (size_t)(poff[(size_t)q] + k)];
                h[0] = p.perp[k].n[0];
                h[1] = p.perp[k].n[1];
                h[2] = p.perp[k].n[2];
                h[3] = p.perp[k].off;
            }
        }
    }
    FloodInput in;
    in.nv = nv;
    in.nprim = nprim;
    in.Vd = m.Vd.data();
    in.nb_off = t.nb_off.data();
    in.nb = t.nb.data();
    in.host_cell = [&](const std::vector<int64_t>& vs, std::vector<std::vector<double>>& P,
                       std::vector<std::vector<double>>& X) -> int64_t {
        const int64_t n = (int64_t)vs.size();
        P.assign((size_t)n, {});
        X.assign((size_t)n, {});
        int64_t sk = 0;
#pragma omp parallel num_threads(nth) reduction(+ : sk)
        {
            ConvexCell cell;
            std::vector<std::pair<double, int32_t>> order;
            std::vector<uint16_t> tris;
#pragma omp for schedule(dynamic, 16)
            for (int64_t k = 0; k < n; ++k) {
                sk += build_cell(m, t, vs[(size_t)k], blo, bhi, o.tau, cell, order);
                tris.clear();
                cell.save(P[(size_t)k], tris, X[(size_t)k]);
            }
        }
        return sk;
    };
    in.prims = prims.data();
    in.perp = perp.data();
    in.nperp_total = poff[(size_t)nprim];
    for (int k = 0; k < 3; ++k) {
        in.blo[k] = blo[k];
        in.bhi[k] = bhi[k];
        in.qlo[k] = o.lo[k];
        in.qscale[k] = 65535.0 / (o.hi[k] - o.lo[k]);
    }
    in.tau = o.tau;
    in.dmax = dmax;
    in.visit_cap = o.visit_cap;
    FloodResult r;
    if (!device_flood(in, r, err)) return false;
    pairs.resize(r.recs.size());
    const int64_t nrec = (int64_t)r.recs.size();
#pragma omp parallel for num_threads(nth) schedule(static, 65536)
    for (int64_t k = 0; k < nrec; ++k) {
        const FloodRec& f = r.recs[(size_t)k];
        PairRec& rec = pairs[(size_t)k];
        rec.key = ((uint64_t)f.v << 32) | (uint64_t)f.code;
        std::memcpy(rec.box, f.box, sizeof(rec.box));
    }
    if (!r.redo.empty()) {
        std::vector<uint8_t> back((size_t)nprim, 0);
        for (int64_t q : r.redo) back[(size_t)q] = 1;
        auto handed_back = [&](const PairRec& rec) {
            const uint32_t code = (uint32_t)(rec.key & 0xffffffffu);
            const int64_t q = (code & 0x80000000u) ? m.ne + (int64_t)(code & 0x7fffffffu) : (int64_t)code;
            return back[(size_t)q] != 0;
        };
        pairs.erase(std::remove_if(pairs.begin(), pairs.end(), handed_back), pairs.end());
    }
    redo = std::move(r.redo);
    std::sort(redo.begin(), redo.end());
    st.flood_tests += r.tests;
    st.flood_hits += r.hits;
    st.quick_rejects += r.quick;
    st.skipped_clips += r.skipped + r.cells_skipped;
    st.t_cells = r.t_cells;
    st.device_cells_back = r.cells_back;
    st.t_dev_upload = r.t_upload;
    st.t_dev_kernel = r.t_kernel;
    st.t_dev_download = r.t_download;
    st.device_redo = (int64_t)redo.size();
    return true;
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
    if (o.mode == TABLE_FLOODING_DEVICE) {
        // the device builds the cells; the host builds on demand those it needs
        cs.lazy = true;
        cs.m = &m;
        cs.t = &t;
        cs.tau = o.tau;
        for (int k = 0; k < 3; ++k) {
            cs.blo[k] = blo[k];
            cs.bhi[k] = bhi[k];
        }
    }
#pragma omp parallel num_threads(nth) reduction(+ : skipped_cells) if (!cs.lazy)
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
        const int64_t ncell = cs.lazy ? 0 : nv;
#pragma omp for schedule(dynamic, 256)
        for (int64_t v = 0; v < ncell; ++v) {
            skipped_cells += build_cell(m, t, v, blo, bhi, o.tau, cell, order);
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
    // every distance inside the (tau-grown) domain is below its diagonal
    double dmax = 0.0;
    for (int k = 0; k < 3; ++k) dmax += (bhi[k] - blo[k]) * (bhi[k] - blo[k]);
    dmax = std::sqrt(dmax);
    std::vector<ThreadCtx> ctx((size_t)nth);
    const int64_t nprim = m.ne + m.nf;
    std::vector<PairRec> dev_pairs;
    std::vector<int64_t> redo;
    if (o.mode == TABLE_FLOODING_DEVICE) {
        if (!inspect_on_device(m, cs, t, o, blo, bhi, dmax, nth, dev_pairs, redo, st, err)) return false;
    }
#pragma omp parallel num_threads(nth)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        ThreadCtx& c = ctx[(size_t)tid];
        c.stamp.assign((size_t)nv, 0u);
        for (int k = 0; k < 3; ++k) {
            c.blo_[k] = blo[k];
            c.bhi_[k] = bhi[k];
            c.qlo_[k] = o.lo[k];
            c.qscale_[k] = 65535.0 / (o.hi[k] - o.lo[k]);
        }
        Primitive p;
        const bool dev = o.mode == TABLE_FLOODING_DEVICE;
        const int64_t nwork = dev ? (int64_t)redo.size() : nprim;
#pragma omp for schedule(dynamic, 64)
        for (int64_t qi = 0; qi < nwork; ++qi) {
            const int64_t q = dev ? redo[(size_t)qi] : qi;
            bool face = q >= m.ne;
            int64_t id = face ? q - m.ne : q;
            if (face) make_face(m, id, o.tau, p);
            else make_edge(m, id, o.tau, p);
            bool base_empty = false;
            make_base(p, blo, bhi, c, base_empty);
            if (o.mode == TABLE_FLOODING || dev) {
                flood(m, cs, t, p, id, o.tau, dmax, base_empty, c);
            } else {
                for (int64_t w = 0; w < nv; ++w) {
                    bool own = false;
                    for (int i = 0; i < p.nverts; ++i) own |= (p.verts[i] == w);
                    PairRec rec;
                    rec.key = pair_key(w, face, id);
                    bool hit = true;
                    if (o.mode == TABLE_EVERYTHING) full_box(rec.box);
                    else if (own) own_box(cs, w, base_empty, c, rec.box);
                    else hit = intercepts(m, cs, w, p, o.tau, dmax, base_empty, c, rec.box);
                    if (hit) c.pairs.push_back(rec);
                }
            }
        }
    }
    std::vector<PairRec> pairs;
    pairs.swap(dev_pairs);
    {
        size_t tot = pairs.size();
        for (auto& c : ctx) tot += c.pairs.size();
        pairs.reserve(tot);
        for (auto& c : ctx) {
            pairs.insert(pairs.end(), c.pairs.begin(), c.pairs.end());
            std::vector<PairRec>().swap(c.pairs);
            st.flood_tests += c.tests;
            st.flood_hits += c.hits;
            st.quick_rejects += c.quick;
            st.skipped_clips += c.skipped;
        }
    }
    st.t_flood = since(t0);

    // 4. CSR: per vertex, edge ids then face ids, each ascending
    t0 = Clock::now();
    auto by_key = [](const PairRec& a, const PairRec& b) { return a.key < b.key; };
#ifdef _OPENMP
    __gnu_parallel::sort(pairs.begin(), pairs.end(), by_key);
#else
    std::sort(pairs.begin(), pairs.end(), by_key);
#endif
    if (pairs.size() >= (size_t)UINT32_MAX) {
        err = "interception table exceeds 2^32 entries";
        return false;
    }
    t.off.assign((size_t)(2 * nv + 1), 0u);
    t.ent.resize(pairs.size());
    t.box.resize(6 * pairs.size());
    std::vector<uint32_t> ecount((size_t)nv, 0), fcount((size_t)nv, 0);
    for (size_t i = 0; i < pairs.size(); ++i) {
        std::memcpy(&t.box[6 * i], pairs[i].box, sizeof(pairs[i].box));
        uint64_t k = pairs[i].key;
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
