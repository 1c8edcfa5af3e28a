#include "mesh.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#ifdef _OPENMP
#include <parallel/algorithm>
#endif

namespace p2m {

namespace {
template <class It, class Cmp>
void psort(It b, It e, Cmp c) {
#ifdef _OPENMP
    __gnu_parallel::sort(b, e, c);
#else
    std::sort(b, e, c);
#endif
}
}  // namespace

std::string build_mesh(const float* V, int64_t nv, const int32_t* F, int64_t nf, const int32_t* S, int64_t ns,
                       MeshData& m) {
    if (nf < 0 || ns < 0) return "negative face or segment count";
    if (!V || (nf > 0 && !F) || (ns > 0 && !S)) return "null vertex, face or segment array";
    if (nv < 1 || nf + ns < 1) return "mesh needs at least one vertex and one face or segment";
    if (nv > kMaxPrimitives || nf > kMaxPrimitives || ns > kMaxPrimitives) return "more than 2^30-1 vertices, faces or segments";
    m.nv = nv;
    m.nf = nf;
    m.ns = ns;
    m.V.assign(V, V + 3 * nv);
    m.Vd.resize((size_t)(3 * nv));
    for (int k = 0; k < 3; ++k) {
        m.lo[k] = INFINITY;
        m.hi[k] = -INFINITY;
    }
    for (int64_t i = 0; i < 3 * nv; ++i) {
        if (!std::isfinite(V[i])) return "non-finite vertex coordinate at vertex " + std::to_string(i / 3);
        m.Vd[(size_t)i] = (double)V[i];
        m.lo[i % 3] = std::min(m.lo[i % 3], m.Vd[(size_t)i]);
        m.hi[i % 3] = std::max(m.hi[i % 3], m.Vd[(size_t)i]);
    }
    m.F.assign(F, F + 3 * nf);
    m.S.assign(S, S + 2 * ns);
    for (int64_t k = 0; k < ns; ++k) {
        const int32_t a = S[2 * k], b = S[2 * k + 1];
        if (a < 0 || b < 0 || a >= nv || b >= nv)
            return "segment " + std::to_string(k) + " has a vertex index out of range";
        if (a == b) return "segment " + std::to_string(k) + " repeats a vertex";
    }
    for (int64_t f = 0; f < nf; ++f) {
        int32_t a = F[3 * f], b = F[3 * f + 1], c = F[3 * f + 2];
        if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv)
            return "face " + std::to_string(f) + " has a vertex index out of range";
        if (a == b || b == c || a == c) return "face " + std::to_string(f) + " repeats a vertex";
        const double* pa = &m.Vd[3 * (size_t)a];
        const double* pb = &m.Vd[3 * (size_t)b];
        const double* pc = &m.Vd[3 * (size_t)c];
        double u[3] = {pb[0] - pa[0], pb[1] - pa[1], pb[2] - pa[2]};
        double w[3] = {pc[0] - pa[0], pc[1] - pa[1], pc[2] - pa[2]};
        double n[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
        if (n[0] == 0.0 && n[1] == 0.0 && n[2] == 0.0) return "face " + std::to_string(f) + " has zero area";
    }
    // duplicate vertices (exactly equal coordinates)
    {
        std::vector<int32_t> idx((size_t)nv);
        std::iota(idx.begin(), idx.end(), 0);
        psort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) {
            const float* p = &V[3 * (size_t)a];
            const float* q = &V[3 * (size_t)b];
            if (p[0] != q[0]) return p[0] < q[0];
            if (p[1] != q[1]) return p[1] < q[1];
            return p[2] < q[2];
        });
        for (int64_t i = 1; i < nv; ++i) {
            const float* p = &V[3 * (size_t)idx[(size_t)i - 1]];
            const float* q = &V[3 * (size_t)idx[(size_t)i]];
            if (p[0] == q[0] && p[1] == q[1] && p[2] == q[2])
                return "vertices " + std::to_string(std::min(idx[(size_t)i - 1], idx[(size_t)i])) + " and " +
                       std::to_string(std::max(idx[(size_t)i - 1], idx[(size_t)i])) + " coincide";
        }
    }
    // canonical edges: sort (min,max) keys of all face sides and segments
    std::vector<uint64_t> keys((size_t)(3 * nf));
    for (int64_t f = 0; f < nf; ++f)
        for (int s = 0; s < 3; ++s) {
            uint64_t a = (uint32_t)F[3 * f + s], b = (uint32_t)F[3 * f + (s + 1) % 3];
            if (a > b) std::swap(a, b);
            keys[(size_t)(3 * f + s)] = (a << 32) | b;
        }
    std::vector<uint64_t> uk = keys;
    for (int64_t k = 0; k < ns; ++k) {
        uint64_t a = (uint32_t)S[2 * k], b = (uint32_t)S[2 * k + 1];
        if (a > b) std::swap(a, b);
        uk.push_back((a << 32) | b);
    }
    psort(uk.begin(), uk.end(), std::less<uint64_t>());
    uk.erase(std::unique(uk.begin(), uk.end()), uk.end());
    m.ne = (int64_t)uk.size();
    if (m.ne > kMaxPrimitives) return "more than 2^30-1 edges";
    m.E.resize((size_t)(2 * m.ne));
    for (int64_t e = 0; e < m.ne; ++e) {
        m.E[(size_t)(2 * e)] = (int32_t)(uk[(size_t)e] >> 32);
        m.E[(size_t)(2 * e + 1)] = (int32_t)(uk[(size_t)e] & 0xffffffffu);
    }
    m.FE.resize((size_t)(3 * nf));
    for (int64_t i = 0; i < 3 * nf; ++i)
        m.FE[(size_t)i] = (int32_t)(std::lower_bound(uk.begin(), uk.end(), keys[(size_t)i]) - uk.begin());
    m.ef_off.assign((size_t)m.ne + 1, 0);
    for (int64_t i = 0; i < 3 * nf; ++i) m.ef_off[(size_t)m.FE[(size_t)i] + 1]++;
    for (int64_t e = 0; e < m.ne; ++e) m.ef_off[(size_t)e + 1] += m.ef_off[(size_t)e];
    m.ef_face.resize((size_t)m.ef_off[(size_t)m.ne]);
    std::vector<int64_t> pos(m.ef_off.begin(), m.ef_off.end() - 1);
    for (int64_t i = 0; i < 3 * nf; ++i) m.ef_face[(size_t)pos[(size_t)m.FE[(size_t)i]]++] = (int32_t)(i / 3);
    return "";
}

}  // namespace p2m
