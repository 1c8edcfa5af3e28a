// Incremental Delaunay tetrahedralisation (Bowyer-Watson) with exact
// predicates; see delaunay.hpp.
//
// Invariants: every live tetrahedron (v0,v1,v2,v3) has orient3d > 0; n[i]
// is the tetrahedron across the face opposite v[i].  A point is inserted by
// (1) a visibility walk to a tetrahedron containing it, (2) collecting the
// connected set of tetrahedra whose circumsphere strictly contains it, and
// (3) joining it to every boundary face of that cavity.  With exact
// predicates and strict conflicts the cavity is star-shaped from the new
// point, so every new tetrahedron is positively oriented.
#include "delaunay.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <stdexcept>

#include "predicates.hpp"

#ifdef _OPENMP
#include <omp.h>
#include <parallel/algorithm>
#endif

namespace p2m {
namespace {

struct Tet {
    int32_t v[4];
    int32_t n[4];
};

struct Rng {
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed * 0x9E3779B97F4A7C15ull + 1) {}
    uint32_t next() {
        s ^= s << 13;
        s ^= s >> 7;
        s ^= s << 17;
        return (uint32_t)(s >> 11);
    }
};

inline uint64_t spread3(uint64_t x) {
    x &= 0x1fffff;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

class Builder {
   public:
    Builder(const double* pts, int64_t n, const double lo[3], const double hi[3]) : n_(n) {
        P_.resize(3 * (size_t)(n + 4));
        std::memcpy(P_.data(), pts, sizeof(double) * 3 * (size_t)n);
        double c[3], ext = 0.0;
        for (int k = 0; k < 3; ++k) {
            c[k] = 0.5 * (lo[k] + hi[k]);
            ext = std::max(ext, hi[k] - lo[k]);
        }
        if (!(ext > 0.0)) ext = 1.0;
        const double s = 40.0 * ext;
        const double corner[4][3] = {{1, 1, 1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};
        for (int i = 0; i < 4; ++i)
            for (int k = 0; k < 3; ++k) P_[3 * (n + i) + k] = c[k] + s * corner[i][k];
        Tet t;
        for (int i = 0; i < 4; ++i) {
            t.v[i] = (int32_t)(n + i);
            t.n[i] = -1;
        }
        if (orient3d(pt(t.v[0]), pt(t.v[1]), pt(t.v[2]), pt(t.v[3])) < 0) std::swap(t.v[0], t.v[1]);
        tets_.push_back(t);
        alive_.push_back(1);
        stamp_.push_back(0);
        conflict_.push_back(0);
    }

    const double* pt(int32_t i) const { return &P_[3 * (size_t)i]; }

    bool run(DelaunayStats* st) {
        std::vector<int32_t> order = insertion_order();
        int32_t hint = 0;
        for (int32_t p : order) {
            if (!insert(p, hint)) return false;
        }
        if (st) {
            int64_t live = 0;
            for (size_t t = 0; t < tets_.size(); ++t) live += alive_[t];
            st->tets = live;
            st->walk_steps = walk_steps_;
        }
        return true;
    }

    void edges(std::vector<int64_t>& off, std::vector<int32_t>& nbr, DelaunayStats* st) const {
        std::vector<uint64_t> keys;
        keys.reserve(tets_.size() * 6);
        for (size_t t = 0; t < tets_.size(); ++t) {
            if (!alive_[t]) continue;
            const Tet& T = tets_[t];
            for (int a = 0; a < 4; ++a)
                for (int b = a + 1; b < 4; ++b) {
                    int64_t x = T.v[a], y = T.v[b];
                    if (x >= n_ || y >= n_) continue;
                    if (x > y) std::swap(x, y);
                    keys.push_back(((uint64_t)x << 32) | (uint64_t)y);
                }
        }
#ifdef _OPENMP
        __gnu_parallel::sort(keys.begin(), keys.end());
#else
        std::sort(keys.begin(), keys.end());
#endif
        keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
        off.assign((size_t)n_ + 1, 0);
        for (uint64_t k : keys) {
            off[(k >> 32) + 1]++;
            off[(k & 0xffffffffull) + 1]++;
        }
        for (int64_t i = 0; i < n_; ++i) off[i + 1] += off[i];
        nbr.resize((size_t)off[n_]);
        std::vector<int64_t> pos(off.begin(), off.end() - 1);
        for (uint64_t k : keys) {
            int32_t a = (int32_t)(k >> 32), b = (int32_t)(k & 0xffffffffull);
            nbr[(size_t)pos[a]++] = b;
            nbr[(size_t)pos[b]++] = a;
        }
        for (int64_t i = 0; i < n_; ++i) std::sort(nbr.begin() + off[i], nbr.begin() + off[i + 1]);
        if (st) st->edges = (int64_t)keys.size();
    }

   private:
    // Biased randomised insertion order: random rounds of doubling size,
    // each round sorted along a Morton curve.
    std::vector<int32_t> insertion_order() const {
        std::vector<int32_t> idx((size_t)n_);
        std::iota(idx.begin(), idx.end(), 0);
        Rng r(12345);
        for (int64_t i = n_ - 1; i > 0; --i) std::swap(idx[(size_t)i], idx[r.next() % (uint32_t)(i + 1)]);
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t i = 0; i < n_; ++i)
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], P_[3 * i + k]);
                hi[k] = std::max(hi[k], P_[3 * i + k]);
            }
        std::vector<uint64_t> key((size_t)n_);
        for (int64_t i = 0; i < n_; ++i) {
            uint64_t m = 0;
            for (int k = 0; k < 3; ++k) {
                double e = hi[k] - lo[k];
                double t = e > 0 ? (P_[3 * i + k] - lo[k]) / e : 0.0;
                uint64_t c = (uint64_t)std::min(2097151.0, std::max(0.0, t * 2097152.0));
                m |= spread3(c) << (2 - k);
            }
            key[(size_t)i] = m;
        }
        int64_t start = 0, len = std::min<int64_t>(n_, 1000);
        while (start < n_) {
            int64_t end = std::min(n_, start + len);
            std::sort(idx.begin() + start, idx.begin() + end,
                      [&](int32_t a, int32_t b) { return key[(size_t)a] < key[(size_t)b]; });
            start = end;
            len *= 2;
        }
        return idx;
    }

    int32_t alloc_tet() {
        if (!free_.empty()) {
            int32_t t = free_.back();
            free_.pop_back();
            alive_[(size_t)t] = 1;
            return t;
        }
        tets_.push_back(Tet{});
        alive_.push_back(1);
        stamp_.push_back(0);
        conflict_.push_back(0);
        return (int32_t)(tets_.size() - 1);
    }

    // Orientation of tet t with vertex i replaced by point p.
    int orient_replaced(const Tet& T, int i, int32_t p) const {
        const double* q[4] = {pt(T.v[0]), pt(T.v[1]), pt(T.v[2]), pt(T.v[3])};
        q[i] = pt(p);
        return orient3d(q[0], q[1], q[2], q[3]);
    }

    int32_t locate(int32_t p, int32_t start) {
        int32_t t = start;
        int64_t steps = 0;
        const int64_t limit = 64 + 8 * (int64_t)tets_.size();
        while (true) {
            const Tet& T = tets_[(size_t)t];
            int r = (int)(rng_.next() & 3);
            int moved = -1;
            for (int k = 0; k < 4; ++k) {
                int i = (r + k) & 3;
                if (orient_replaced(T, i, p) < 0) {
                    moved = i;
                    break;
                }
            }
            if (moved < 0) return t;
            t = T.n[moved];
            if (t < 0) throw std::runtime_error("delaunay: walked outside the bounding simplex");
            if (++steps > limit) return locate_brute(p);
            ++walk_steps_;
        }
    }

    int32_t locate_brute(int32_t p) {
        for (size_t t = 0; t < tets_.size(); ++t) {
            if (!alive_[t]) continue;
            bool in = true;
            for (int i = 0; i < 4 && in; ++i) in = orient_replaced(tets_[t], i, p) >= 0;
            if (in) return (int32_t)t;
        }
        throw std::runtime_error("delaunay: point location failed");
    }

    bool in_conflict(int32_t t, int32_t p) {
        if (stamp_[(size_t)t] == epoch_) return conflict_[(size_t)t] != 0;
        const Tet& T = tets_[(size_t)t];
        bool c = insphere(pt(T.v[0]), pt(T.v[1]), pt(T.v[2]), pt(T.v[3]), pt(p)) > 0;
        stamp_[(size_t)t] = epoch_;
        conflict_[(size_t)t] = c ? 1 : 0;
        return c;
    }

    bool insert(int32_t p, int32_t& hint) {
        ++epoch_;
        int32_t t0 = locate(p, hint);
        {
            const Tet& T = tets_[(size_t)t0];
            for (int i = 0; i < 4; ++i) {
                const double* a = pt(T.v[i]);
                const double* b = pt(p);
                if (a[0] == b[0] && a[1] == b[1] && a[2] == b[2]) return false;  // duplicate point
            }
        }
        if (!in_conflict(t0, p)) throw std::runtime_error("delaunay: containing tetrahedron not in conflict");
        cavity_.clear();
        boundary_.clear();
        stack_.clear();
        stack_.push_back(t0);
        cavity_.push_back(t0);
        while (!stack_.empty()) {
            int32_t t = stack_.back();
            stack_.pop_back();
            for (int i = 0; i < 4; ++i) {
                int32_t nb = tets_[(size_t)t].n[i];
                if (nb >= 0) {
                    bool seen = stamp_[(size_t)nb] == epoch_;
                    if (in_conflict(nb, p)) {
                        if (!seen) {
                            stack_.push_back(nb);
                            cavity_.push_back(nb);
                        }
                        continue;
                    }
                }
                boundary_.push_back({t, i, nb});
            }
        }
        // Join p to every boundary face.
        const size_t nb = boundary_.size();
        size_t cap = 16;
        while (cap < 4 * 3 * nb) cap <<= 1;
        if (hkey_.size() < cap) {
            hkey_.assign(cap, UINT64_MAX);
            hval_.assign(cap, 0);
        }
        const uint64_t mask = cap - 1;
        used_.clear();
        newt_.clear();
        for (const Face& f : boundary_) {
            Tet T = tets_[(size_t)f.t];
            T.v[f.i] = p;
            T.n[f.i] = f.out;
            int32_t nt = alloc_tet();
            for (int j = 0; j < 4; ++j)
                if (j != f.i) T.n[j] = -1;
            tets_[(size_t)nt] = T;
            newt_.push_back(nt);
            if (f.out >= 0) {
                Tet& O = tets_[(size_t)f.out];
                for (int j = 0; j < 4; ++j)
                    if (O.n[j] == f.t) {
                        O.n[j] = nt;
                        break;
                    }
            }
            for (int j = 0; j < 4; ++j) {
                if (j == f.i) continue;
                int32_t e0 = -1, e1 = -1;
                for (int k = 0; k < 4; ++k) {
                    if (k == j || k == f.i) continue;
                    if (e0 < 0) e0 = T.v[k];
                    else e1 = T.v[k];
                }
                if (e0 > e1) std::swap(e0, e1);
                uint64_t key = ((uint64_t)(uint32_t)e0 << 32) | (uint32_t)e1;
                uint64_t h = (key * 0x9E3779B97F4A7C15ull) >> 20;
                for (;;) {
                    uint64_t slot = h & mask;
                    if (hkey_[slot] == UINT64_MAX) {
                        hkey_[slot] = key;
                        hval_[slot] = ((uint64_t)(uint32_t)nt << 2) | (uint64_t)j;
                        used_.push_back(slot);
                        break;
                    }
                    if (hkey_[slot] == key) {
                        int32_t ot = (int32_t)(hval_[slot] >> 2);
                        int oj = (int)(hval_[slot] & 3);
                        tets_[(size_t)nt].n[j] = ot;
                        tets_[(size_t)ot].n[oj] = nt;
                        hkey_[slot] = UINT64_MAX - 1;  // consumed: keep probing chains intact
                        break;
                    }
                    ++h;
                }
            }
        }
        for (uint64_t s : used_) hkey_[s] = UINT64_MAX;
        for (int32_t t : cavity_) {
            alive_[(size_t)t] = 0;
            free_.push_back(t);
        }
        hint = newt_.back();
        return true;
    }

    struct Face {
        int32_t t;
        int i;
        int32_t out;
    };

    int64_t n_;
    std::vector<double> P_;
    std::vector<Tet> tets_;
    std::vector<uint8_t> alive_;
    std::vector<uint32_t> stamp_;
    std::vector<uint8_t> conflict_;
    std::vector<int32_t> free_, cavity_, stack_, newt_;
    std::vector<Face> boundary_;
    std::vector<uint64_t> hkey_, hval_, used_;
    uint32_t epoch_ = 0;
    int64_t walk_steps_ = 0;
    Rng rng_{777};
};

}  // namespace

bool delaunay_neighbors(const double* pts, int64_t n, const double cover_lo[3], const double cover_hi[3],
                        std::vector<int64_t>& off, std::vector<int32_t>& nbr, DelaunayStats* stats) {
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = cover_lo[k];
        hi[k] = cover_hi[k];
    }
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], pts[3 * i + k]);
            hi[k] = std::max(hi[k], pts[3 * i + k]);
        }
    long long ex0 = predicate_exact_calls();
    Builder b(pts, n, lo, hi);
    if (!b.run(stats)) return false;
    b.edges(off, nbr, stats);
    if (stats) stats->exact_predicates = predicate_exact_calls() - ex0;
    return true;
}

}  // namespace p2m
