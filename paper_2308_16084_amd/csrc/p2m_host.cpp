// Host side of the C interface: mesh creation, precompute, inspection,
// save/load and error reporting.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "p2m_internal.hpp"

namespace p2m {

namespace {
thread_local std::string g_last_error;
using Clock = std::chrono::steady_clock;
double since(Clock::time_point t0) { return std::chrono::duration<double>(Clock::now() - t0).count(); }
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

p2m_status fail(p2m_status s, const std::string& msg) {
    set_error(msg);
    return s;
}

namespace {

// Nearest vertex of q by a greedy walk over the Voronoi (Delaunay) neighbour
// graph from vertex v: exact for q in D (a vertex whose cell does not hold
// q has a closer Voronoi neighbour), float64, ties to the smaller id.
int32_t walk_nearest(const MeshData& m, const Table& t, const double q[3], int32_t v) {
    auto d2 = [&](int32_t w) {
        const double* p = &m.Vd[3 * (size_t)w];
        return (q[0] - p[0]) * (q[0] - p[0]) + (q[1] - p[1]) * (q[1] - p[1]) + (q[2] - p[2]) * (q[2] - p[2]);
    };
    double best = d2(v);
    for (int it = 0; it < (1 << 20); ++it) {
        int32_t nb = v;
        for (int64_t k = t.nb_off[(size_t)v]; k < t.nb_off[(size_t)v + 1]; ++k) {
            const int32_t w = t.nb[(size_t)k];
            const double d = d2(w);
            if (d < best || (d == best && w < nb)) {
                best = d;
                nb = w;
            }
        }
        if (nb == v) break;
        v = nb;
    }
    return v;
}

uint64_t mix64(uint64_t x) {  // splitmix64 finaliser
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// The list statistics of Table 1: per vertex the edges and faces of its
// interception list; Avg^1 the mean over vertices, Avg^2 the mean weighted
// by the volume of the vertex's Voronoi cell (in D here: the expected list
// of a query uniform in D), estimated from one sample in each cell of a
// 128^3 grid on D (jittered by a hash of the cell, so the estimate is
// deterministic) and the sample's nearest vertex (a walk from the previous
// sample's); the maxima over vertices.
void list_stats(const MeshState& s, int threads, p2m_build_stats& st) {
    const int64_t nv = s.m.nv;
    const std::vector<uint32_t>& off = s.t.off;
    double se = 0, sf = 0;
    int64_t me = 0, mf = 0;
    for (int64_t v = 0; v < nv; ++v) {
        const int64_t e = off[(size_t)(2 * v + 1)] - off[(size_t)(2 * v)];
        const int64_t f = off[(size_t)(2 * v + 2)] - off[(size_t)(2 * v + 1)];
        se += (double)e;
        sf += (double)f;
        me = std::max(me, e);
        mf = std::max(mf, f);
    }
    st.avg_edges = se / (double)nv;
    st.avg_faces = sf / (double)nv;
    st.max_edges = me;
    st.max_faces = mf;
    constexpr int G = 128;
    int nt = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
    nt = std::min(nt, G);
    std::vector<double> ae((size_t)nt, 0.0), af((size_t)nt, 0.0);
    auto work = [&](int w) {
        int32_t v = 0;
        for (int i = w; i < G; i += nt)
            for (int j = 0; j < G; ++j)
                for (int k = 0; k < G; ++k) {
                    const uint64_t h = mix64(((uint64_t)i * G + (uint64_t)j) * G + (uint64_t)k);
                    const double u[3] = {(double)(h & 0x1FFFFF) / 2097152.0, (double)((h >> 21) & 0x1FFFFF) / 2097152.0,
                                         (double)((h >> 42) & 0x1FFFFF) / 2097152.0};
                    const int c[3] = {i, j, k};
                    double q[3];
                    for (int a = 0; a < 3; ++a) q[a] = s.dlo[a] + (c[a] + u[a]) / G * (s.dhi[a] - s.dlo[a]);
                    v = walk_nearest(s.m, s.t, q, v);
                    ae[(size_t)w] += (double)(off[(size_t)(2 * v + 1)] - off[(size_t)(2 * v)]);
                    af[(size_t)w] += (double)(off[(size_t)(2 * v + 2)] - off[(size_t)(2 * v + 1)]);
                }
    };
    std::vector<std::thread> th;
    for (int w = 1; w < nt; ++w) th.emplace_back(work, w);
    work(0);
    for (auto& x : th) x.join();
    double te = 0, tf = 0;
    for (int w = 0; w < nt; ++w) {
        te += ae[(size_t)w];
        tf += af[(size_t)w];
    }
    const double ns = (double)G * G * G;
    st.avg_edges_volw = te / ns;
    st.avg_faces_volw = tf / ns;
    st.avg_list_volw = (te + tf) / ns;
}

}  // namespace

}  // namespace p2m

using namespace p2m;

extern "C" {

const char* p2m_last_error(void) { return g_last_error.c_str(); }

p2m_status p2m_mesh_create(const float* V, int64_t nv, const int32_t* F, int64_t nf, p2m_mesh** out) {
    if (!out) return fail(P2M_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!V || !F) return fail(P2M_ERR_ARG, "V or F is NULL");
    if (nv < 0 || nf < 0) return fail(P2M_ERR_ARG, "negative count");
    if (nv < 1 || nf < 1) return fail(P2M_ERR_MESH, "mesh needs at least one vertex and one face");
    return p2m_mesh_create_mixed(V, nv, F, nf, nullptr, 0, out);
}

p2m_status p2m_mesh_create_mixed(const float* V, int64_t nv, const int32_t* F, int64_t nf, const int32_t* S,
                                 int64_t ns, p2m_mesh** out) {
    if (!out) return fail(P2M_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!V || (nf > 0 && !F) || (ns > 0 && !S)) return fail(P2M_ERR_ARG, "V, F or S is NULL");
    if (nv < 0 || nf < 0 || ns < 0) return fail(P2M_ERR_ARG, "negative count");
    try {
        auto t0 = Clock::now();
        p2m_mesh* m = new p2m_mesh();
        std::string err = build_mesh(V, nv, F, nf, S, ns, m->s.m);
        if (!err.empty()) {
            delete m;
            return fail(P2M_ERR_MESH, err);
        }
        m->s.t_validate = since(t0);
        *out = m;
        return P2M_OK;
    } catch (const std::bad_alloc&) {
        return fail(P2M_ERR_OOM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(P2M_ERR_INTERNAL, e.what());
    }
}

void p2m_mesh_destroy(p2m_mesh* m) {
    if (!m) return;
    device_release(m->s);
    delete m;
}

p2m_status p2m_mesh_counts(const p2m_mesh* m, int64_t* nv, int64_t* ne, int64_t* nf) {
    if (!m) return fail(P2M_ERR_ARG, "mesh is NULL");
    if (nv) *nv = m->s.m.nv;
    if (ne) *ne = m->s.m.ne;
    if (nf) *nf = m->s.m.nf;
    return P2M_OK;
}

p2m_status p2m_mesh_edges(const p2m_mesh* m, int64_t* ne, int32_t* pairs) {
    if (!m || !ne) return fail(P2M_ERR_ARG, "NULL argument");
    *ne = m->s.m.ne;
    if (pairs && m->s.m.ne > 0) std::memcpy(pairs, m->s.m.E.data(), sizeof(int32_t) * (size_t)(2 * m->s.m.ne));
    return P2M_OK;
}

p2m_status p2m_precompute(p2m_mesh* m, const p2m_build_opts* opts, p2m_build_stats* stats) {
    if (!m) return fail(P2M_ERR_ARG, "mesh is NULL");
    MeshState& s = m->s;
    p2m_build_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    else o.use_default_domain = 1;
    if (o.table_mode < 0 || o.table_mode > 3) return fail(P2M_ERR_ARG, "bad table_mode");
    if (o.device_visit_cap < 0 || o.device_visit_cap > 512) return fail(P2M_ERR_ARG, "device_visit_cap outside 0..512");
    if (o.num_threads < 0) return fail(P2M_ERR_ARG, "negative num_threads");
    if (o.margin_rel < 0 || !std::isfinite(o.margin_rel)) return fail(P2M_ERR_ARG, "bad margin_rel");
    double lo[3], hi[3];
    if (o.use_default_domain) {
        for (int k = 0; k < 3; ++k) {
            double c = 0.5 * (s.m.lo[k] + s.m.hi[k]);
            double h = 0.5 * (s.m.hi[k] - s.m.lo[k]) * 10.0;
            if (!(h > 0)) h = 1.0;
            lo[k] = c - h;
            hi[k] = c + h;
        }
    } else {
        for (int k = 0; k < 3; ++k) {
            lo[k] = o.domain_lo[k];
            hi[k] = o.domain_hi[k];
            if (!std::isfinite(lo[k]) || !std::isfinite(hi[k]) || !(hi[k] > lo[k]))
                return fail(P2M_ERR_ARG, "domain box must be finite with lo < hi");
        }
    }
    double diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                            (hi[2] - lo[2]) * (hi[2] - lo[2]));
    double margin = o.margin_rel > 0 ? o.margin_rel : 1e-9;
    try {
        auto t0 = Clock::now();
        build_kdtree(s.m.V.data(), s.m.nv, s.kd);
        s.t_kdt = since(t0);
        TableOptions to;
        for (int k = 0; k < 3; ++k) {
            to.lo[k] = lo[k];
            to.hi[k] = hi[k];
        }
        to.tau = margin * diag;
        to.threads = o.num_threads;
        to.mode = o.table_mode;
        to.visit_cap = o.device_visit_cap;
        s.ts = TableStats();
        std::string err;
        if (!build_table(s.m, to, s.t, s.ts, err))
            return fail(err.rfind("device inspection", 0) == 0 ? P2M_ERR_HIP : P2M_ERR_MESH, err);
        for (int k = 0; k < 3; ++k) {
            s.dlo[k] = lo[k];
            s.dhi[k] = hi[k];
        }
        s.tau = to.tau;
        s.precomputed = true;
        s.packed = false;
    } catch (const std::bad_alloc&) {
        return fail(P2M_ERR_OOM, "host allocation failed during precompute");
    } catch (const std::exception& e) {
        return fail(P2M_ERR_INTERNAL, e.what());
    }
    if (stats) {
        p2m_build_stats& st = *stats;
        std::memset(&st, 0, sizeof(st));
        st.t_validate = s.t_validate;
        st.t_kdt = s.t_kdt;
        st.t_delaunay = s.ts.t_delaunay;
        st.t_cells = s.ts.t_cells;
        st.t_flood = s.ts.t_flood;
        st.t_pack = s.ts.t_pack;
        st.nv = s.m.nv;
        st.ne = s.m.ne;
        st.nf = s.m.nf;
        st.delaunay_edges = s.ts.delaunay_edges;
        st.tets = s.ts.tets;
        st.exact_predicates = s.ts.exact_predicates;
        st.flood_tests = s.ts.flood_tests;
        st.flood_hits = s.ts.flood_hits;
        st.quick_rejects = s.ts.quick_rejects;
        st.skipped_clips = s.ts.skipped_clips;
        st.nnz_edges = s.ts.nnz_edges;
        st.nnz_faces = s.ts.nnz_faces;
        st.max_list = s.ts.max_list;
        st.avg_list = (double)(s.ts.nnz_edges + s.ts.nnz_faces) / (double)s.m.nv;
        st.t_dev_upload = s.ts.t_dev_upload;
        st.t_dev_kernel = s.ts.t_dev_kernel;
        st.t_dev_download = s.ts.t_dev_download;
        st.device_redo = s.ts.device_redo;
        st.device_cells_back = s.ts.device_cells_back;
        // the flood (Algorithm 1) takes each primitive's own vertices, then
        // every vertex it filter-tests, from its queue
        const bool flooded = o.table_mode == P2M_TABLE_FLOODING || o.table_mode == P2M_TABLE_FLOODING_DEVICE;
        st.flood_visits = flooded ? s.ts.flood_tests + 2 * s.m.ne + 3 * s.m.nf : 0;
        list_stats(s, o.num_threads, st);
    }
    return P2M_OK;
}

p2m_status p2m_mesh_table(const p2m_mesh* m, int64_t* nnz, uint32_t* off, int32_t* ent) {
    if (!m || !nnz) return fail(P2M_ERR_ARG, "NULL argument");
    if (!m->s.precomputed) return fail(P2M_ERR_STATE, "mesh not precomputed");
    *nnz = (int64_t)m->s.t.ent.size();
    if (off) std::memcpy(off, m->s.t.off.data(), sizeof(uint32_t) * m->s.t.off.size());
    if (ent && !m->s.t.ent.empty()) std::memcpy(ent, m->s.t.ent.data(), sizeof(int32_t) * m->s.t.ent.size());
    return P2M_OK;
}

p2m_status p2m_mesh_table_boxes(const p2m_mesh* m, uint16_t* boxes) {
    if (!m || !boxes) return fail(P2M_ERR_ARG, "NULL argument");
    if (!m->s.precomputed) return fail(P2M_ERR_STATE, "mesh not precomputed");
    if (!m->s.t.box.empty()) std::memcpy(boxes, m->s.t.box.data(), sizeof(uint16_t) * m->s.t.box.size());
    return P2M_OK;
}

p2m_status p2m_mesh_neighbors(const p2m_mesh* m, int64_t* nnz, int64_t* nb_off, int32_t* nb) {
    if (!m || !nnz) return fail(P2M_ERR_ARG, "NULL argument");
    if (!m->s.precomputed) return fail(P2M_ERR_STATE, "mesh not precomputed");
    *nnz = (int64_t)m->s.t.nb.size();
    if (nb_off) std::memcpy(nb_off, m->s.t.nb_off.data(), sizeof(int64_t) * m->s.t.nb_off.size());
    if (nb && !m->s.t.nb.empty()) std::memcpy(nb, m->s.t.nb.data(), sizeof(int32_t) * m->s.t.nb.size());
    return P2M_OK;
}

p2m_status p2m_mesh_kdtree(const p2m_mesh* m, float* xyz, int32_t* vid) {
    if (!m) return fail(P2M_ERR_ARG, "NULL argument");
    if (!m->s.precomputed) return fail(P2M_ERR_STATE, "mesh not precomputed");
    const KdTree& t = m->s.kd;
    for (int64_t i = 0; i < t.n; ++i) {
        if (xyz) {
            xyz[3 * i] = t.x[(size_t)i];
            xyz[3 * i + 1] = t.y[(size_t)i];
            xyz[3 * i + 2] = t.z[(size_t)i];
        }
        if (vid) vid[i] = t.vid[(size_t)i];
    }
    return P2M_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- save/load
//
// File: magic, version, payload length, payload, FNV-1a of the payload.
// Payload: domain (6 doubles), tau, then length-prefixed arrays V, F, S, KD-tree
// x, y, z, vid, table off, ent, entry boxes, neighbour off, nb.

namespace {
const char kMagic[8] = {'P', '2', 'M', 'M', 'E', 'S', 'H', '1'};
const uint32_t kVersion = 4;

uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char* p = (const unsigned char*)data;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

struct Writer {
    std::vector<char> b;
    void raw(const void* p, size_t n) { b.insert(b.end(), (const char*)p, (const char*)p + n); }
    template <class T>
    void vec(const std::vector<T>& v) {
        uint64_t n = v.size();
        raw(&n, sizeof(n));
        raw(v.data(), n * sizeof(T));
    }
};

struct Reader {
    const std::vector<char>& b;
    size_t pos = 0;
    bool ok = true;
    void raw(void* p, size_t n) {
        if (!ok || b.size() - pos < n) {
            ok = false;
            return;
        }
        if (n == 0) return;  // (p may be the data() of an empty vector)
        std::memcpy(p, b.data() + pos, n);
        pos += n;
    }
    template <class T>
    void vec(std::vector<T>& v) {
        uint64_t n = 0;
        raw(&n, sizeof(n));
        if (!ok || n > (b.size() - pos) / sizeof(T)) {
            ok = false;
            return;
        }
        v.resize(n);
        raw(v.data(), n * sizeof(T));
    }
};
}  // namespace

extern "C" {

p2m_status p2m_save(const p2m_mesh* m, const char* path) {
    if (!m || !path) return fail(P2M_ERR_ARG, "NULL argument");
    const MeshState& s = m->s;
    if (!s.precomputed) return fail(P2M_ERR_STATE, "mesh not precomputed");
    Writer w;
    w.raw(s.dlo, sizeof(s.dlo));
    w.raw(s.dhi, sizeof(s.dhi));
    w.raw(&s.tau, sizeof(s.tau));
    w.vec(s.m.V);
    w.vec(s.m.F);
    w.vec(s.m.S);
    w.vec(s.kd.x);
    w.vec(s.kd.y);
    w.vec(s.kd.z);
    w.vec(s.kd.vid);
    w.vec(s.t.off);
    w.vec(s.t.ent);
    w.vec(s.t.box);
    w.vec(s.t.nb_off);
    w.vec(s.t.nb);
    uint64_t len = w.b.size(), h = fnv1a(w.b.data(), w.b.size());
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(P2M_ERR_IO, std::string("cannot open ") + path);
    bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(&kVersion, sizeof(kVersion), 1, f) == 1 &&
              fwrite(&len, sizeof(len), 1, f) == 1 && fwrite(w.b.data(), 1, len, f) == len &&
              fwrite(&h, sizeof(h), 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(P2M_ERR_IO, std::string("write failed: ") + path);
    return P2M_OK;
}

p2m_status p2m_load(const char* path, p2m_mesh** out) {
    if (!path || !out) return fail(P2M_ERR_ARG, "NULL argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(P2M_ERR_IO, std::string("cannot open ") + path);
    char magic[8];
    uint32_t ver = 0;
    uint64_t len = 0, h = 0;
    std::vector<char> buf;
    bool ok = fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 &&
              fread(&ver, sizeof(ver), 1, f) == 1 && ver == kVersion && fread(&len, sizeof(len), 1, f) == 1 &&
              len < (uint64_t(1) << 40);
    if (ok) {
        try {
            buf.resize(len);
        } catch (const std::bad_alloc&) {
            std::fclose(f);
            return fail(P2M_ERR_OOM, "cannot allocate the file buffer");
        }
        ok = fread(buf.data(), 1, len, f) == len && fread(&h, sizeof(h), 1, f) == 1;
    }
    std::fclose(f);
    if (!ok) return fail(P2M_ERR_IO, std::string("not a p2m mesh file (or wrong version): ") + path);
    if (fnv1a(buf.data(), buf.size()) != h) return fail(P2M_ERR_IO, std::string("checksum mismatch: ") + path);
    Reader r{buf};
    double dlo[3], dhi[3], tau;
    std::vector<float> V;
    std::vector<int32_t> F;
    r.raw(dlo, sizeof(dlo));
    r.raw(dhi, sizeof(dhi));
    r.raw(&tau, sizeof(tau));
    r.vec(V);
    r.vec(F);
    std::vector<int32_t> S;
    r.vec(S);
    if (!r.ok || V.size() % 3 || F.size() % 3 || S.size() % 2)
        return fail(P2M_ERR_IO, std::string("corrupt p2m mesh file: ") + path);
    p2m_mesh* m = nullptr;
    p2m_status st = p2m_mesh_create_mixed(V.data(), (int64_t)V.size() / 3, F.data(), (int64_t)F.size() / 3, S.data(),
                                          (int64_t)S.size() / 2, &m);
    if (st != P2M_OK) return st;
    MeshState& s = m->s;
    r.vec(s.kd.x);
    r.vec(s.kd.y);
    r.vec(s.kd.z);
    r.vec(s.kd.vid);
    r.vec(s.t.off);
    r.vec(s.t.ent);
    r.vec(s.t.box);
    r.vec(s.t.nb_off);
    r.vec(s.t.nb);
    const size_t nv = (size_t)s.m.nv;
    ok = r.ok && r.pos == buf.size() && s.kd.x.size() == nv && s.kd.y.size() == nv && s.kd.z.size() == nv &&
         s.kd.vid.size() == nv && s.t.off.size() == 2 * nv + 1 && s.t.off.back() == s.t.ent.size() &&
         s.t.box.size() == 6 * s.t.ent.size() && s.t.nb_off.size() == nv + 1;
    for (size_t v = 0; ok && v < nv; ++v) {
        ok = s.kd.vid[v] >= 0 && (size_t)s.kd.vid[v] < nv && s.t.off[2 * v] <= s.t.off[2 * v + 1] &&
             s.t.off[2 * v + 1] <= s.t.off[2 * v + 2];
        for (uint32_t k = s.t.off[2 * v]; ok && k < s.t.off[2 * v + 1]; ++k) ok = s.t.ent[k] >= 0 && s.t.ent[k] < s.m.ne;
        for (uint32_t k = s.t.off[2 * v + 1]; ok && k < s.t.off[2 * v + 2]; ++k)
            ok = s.t.ent[k] >= 0 && s.t.ent[k] < s.m.nf;
    }
    if (!ok) {
        p2m_mesh_destroy(m);
        return fail(P2M_ERR_IO, std::string("corrupt p2m mesh file: ") + path);
    }
    s.kd.n = (int64_t)nv;
    for (int k = 0; k < 3; ++k) {
        s.dlo[k] = dlo[k];
        s.dhi[k] = dhi[k];
    }
    s.tau = tau;
    s.precomputed = true;
    *out = m;
    return P2M_OK;
}

}  // extern "C"
