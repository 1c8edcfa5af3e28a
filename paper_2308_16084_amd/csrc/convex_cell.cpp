#include "convex_cell.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace p2m {

namespace {
inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
}  // namespace

void ConvexCell::init_box(const double lo[3], const double hi[3]) {
    planes_.clear();
    tris_.clear();
    pos_.clear();
    empty_ = false;
    // planes 0..5: -x <= -lo.x, x <= hi.x, -y <= -lo.y, y <= hi.y, -z <= -lo.z, z <= hi.z
    for (int k = 0; k < 3; ++k) {
        HalfSpace a{{0, 0, 0}, -lo[k]};
        a.n[k] = -1.0;
        HalfSpace b{{0, 0, 0}, hi[k]};
        b.n[k] = 1.0;
        planes_.push_back(a);
        planes_.push_back(b);
    }
    for (int c = 0; c < 8; ++c) {
        int sx = c & 1, sy = (c >> 1) & 1, sz = (c >> 2) & 1;
        std::array<uint16_t, 3> t = {(uint16_t)(0 + sx), (uint16_t)(2 + sy), (uint16_t)(4 + sz)};
        // det(n_i,n_j,n_k) = (+-1)(+-1)(+-1): make it positive
        int sgn = (sx ? 1 : -1) * (sy ? 1 : -1) * (sz ? 1 : -1);
        if (sgn < 0) std::swap(t[0], t[1]);
        tris_.push_back(t);
        pos_.push_back({sx ? hi[0] : lo[0], sy ? hi[1] : lo[1], sz ? hi[2] : lo[2]});
    }
}

bool ConvexCell::corner_of(int i, int j, int k, std::array<double, 3>& x) const {
    const HalfSpace& a = planes_[(size_t)i];
    const HalfSpace& b = planes_[(size_t)j];
    const HalfSpace& c = planes_[(size_t)k];
    double bc[3], ca[3], ab[3];
    cross3(b.n, c.n, bc);
    cross3(c.n, a.n, ca);
    cross3(a.n, b.n, ab);
    double det = dot3(a.n, bc);
    double scale = std::sqrt(dot3(a.n, a.n) * dot3(b.n, b.n) * dot3(c.n, c.n));
    if (!(det > 1e-13 * scale)) return false;
    double inv = 1.0 / det;
    for (int d = 0; d < 3; ++d) x[(size_t)d] = (a.off * bc[d] + b.off * ca[d] + c.off * ab[d]) * inv;
    return std::isfinite(x[0]) && std::isfinite(x[1]) && std::isfinite(x[2]);
}

ConvexCell::ClipResult ConvexCell::clip(const HalfSpace& h) {
    if (empty_) return UNCHANGED;
    const size_t nt = tris_.size();
    out_.resize(nt);
    size_t nout = 0;
    for (size_t t = 0; t < nt; ++t) {
        double s = dot3(h.n, pos_[t].data()) - h.off;
        out_[t] = s > 0.0;
        nout += out_[t];
    }
    if (nout == 0) return UNCHANGED;
    if (nout == nt) {
        empty_ = true;
        tris_.clear();
        pos_.clear();
        return EMPTY;
    }
    // Boundary of the removed region: directed edges (a -> b) of removed
    // triangles whose reverse (b -> a) belongs to a kept triangle.  Found by
    // a direct search inside the smaller of the two sets: from the removed
    // side an edge is on the boundary when its reverse is not among removed
    // edges; from the kept side, a kept edge (b -> a) whose reverse is not
    // among kept edges gives the boundary edge (a -> b).
    const bool from_removed = 2 * nout <= nt;
    removed_.clear();
    for (size_t t = 0; t < nt; ++t)
        if ((out_[t] != 0) == from_removed) removed_.push_back((uint32_t)t);
    std::vector<std::array<uint16_t, 2>>& boundary = boundary_;
    boundary.clear();
    for (uint32_t ti : removed_) {
        const auto& T = tris_[ti];
        for (int e = 0; e < 3; ++e) {
            const uint16_t a = T[(size_t)e], b = T[(size_t)((e + 1) % 3)];
            int twins = 0;
            for (uint32_t tj : removed_) {
                const auto& U = tris_[tj];
                twins += (U[0] == b && U[1] == a) + (U[1] == b && U[2] == a) + (U[2] == b && U[0] == a);
            }
            if (twins == 0) {
                if (from_removed) boundary.push_back({a, b});
                else boundary.push_back({b, a});
            } else if (twins != 1) {
                return SKIPPED;  // inconsistent topology
            }
        }
    }
    if (boundary.size() < 3) return SKIPPED;
    // boundary must be one cycle
    const size_t np = planes_.size();
    if (np + 1 > 65535) return SKIPPED;
    next_.assign(np, -1);
    for (const auto& e : boundary) {
        if (next_[e[0]] != -1) return SKIPPED;
        next_[e[0]] = e[1];
    }
    {
        int32_t a = boundary[0][0];
        size_t steps = 0;
        do {
            a = next_[(size_t)a];
            if (a < 0) return SKIPPED;
            ++steps;
        } while (a != (int32_t)boundary[0][0] && steps <= boundary.size());
        if (steps != boundary.size()) return SKIPPED;
    }
    const uint16_t pid = (uint16_t)np;
    planes_.push_back(h);
    std::vector<std::array<uint16_t, 3>>& newt = newt_;
    std::vector<std::array<double, 3>>& newp = newp_;
    newt.clear();
    newp.clear();
    for (const auto& e : boundary) {
        std::array<double, 3> x;
        if (!corner_of(e[0], e[1], pid, x)) {
            planes_.pop_back();
            return SKIPPED;
        }
        newt.push_back({e[0], e[1], pid});
        newp.push_back(x);
    }
    size_t w = 0;
    for (size_t t = 0; t < nt; ++t) {
        if (out_[t]) continue;
        tris_[w] = tris_[t];
        pos_[w] = pos_[t];
        ++w;
    }
    tris_.resize(w);
    pos_.resize(w);
    tris_.insert(tris_.end(), newt.begin(), newt.end());
    pos_.insert(pos_.end(), newp.begin(), newp.end());
    return CLIPPED;
}

void ConvexCell::compact() {
    std::vector<int32_t> remap(planes_.size(), -1);
    for (const auto& t : tris_)
        for (uint16_t i : t) remap[i] = 0;
    std::vector<HalfSpace> np;
    for (size_t i = 0; i < planes_.size(); ++i) {
        if (remap[i] < 0) continue;
        remap[i] = (int32_t)np.size();
        np.push_back(planes_[i]);
    }
    for (auto& t : tris_)
        for (auto& i : t) i = (uint16_t)remap[i];
    planes_.swap(np);
}

void ConvexCell::save(std::vector<double>& planes, std::vector<uint16_t>& tris, std::vector<double>& pos) const {
    for (const auto& p : planes_) {
        planes.push_back(p.n[0]);
        planes.push_back(p.n[1]);
        planes.push_back(p.n[2]);
        planes.push_back(p.off);
    }
    for (const auto& t : tris_) tris.insert(tris.end(), t.begin(), t.end());
    for (const auto& x : pos_) pos.insert(pos.end(), x.begin(), x.end());
}

void ConvexCell::load(const double* planes, size_t np, const uint16_t* tris, const double* pos, size_t nt) {
    planes_.resize(np);
    for (size_t i = 0; i < np; ++i) {
        planes_[i].n[0] = planes[4 * i];
        planes_[i].n[1] = planes[4 * i + 1];
        planes_[i].n[2] = planes[4 * i + 2];
        planes_[i].off = planes[4 * i + 3];
    }
    tris_.resize(nt);
    pos_.resize(nt);
    for (size_t t = 0; t < nt; ++t) {
        tris_[t] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
        pos_[t] = {pos[3 * t], pos[3 * t + 1], pos[3 * t + 2]};
    }
    empty_ = (nt == 0);
}

}  // namespace p2m
