// Exact-sign orientation and in-sphere predicates (see predicates.hpp).
//
// Floating-point expansions: a value is held as a sum of doubles of
// increasing magnitude that do not overlap, so its sign is the sign of the
// largest component.  Sums use error-free two-sum, products error-free
// two-product (fma); an expansion grows one component at a time (Shewchuk
// 1997, Grow-Expansion and Scale-Expansion with zero elimination).
// This file must be compiled without fast-math or FP contraction.
#include "predicates.hpp"

#include <atomic>
#include <cmath>
#include <vector>

namespace p2m {
namespace {

std::atomic<long long> g_exact_calls{0};

using Exp = std::vector<double>;

inline void two_sum(double a, double b, double& x, double& y) {
    x = a + b;
    double bv = x - a;
    double av = x - bv;
    y = (a - av) + (b - bv);
}

inline void two_prod(double a, double b, double& x, double& y) {
    x = a * b;
    y = std::fma(a, b, -x);
}

Exp from_diff(double a, double b) {
    double x, y;
    two_sum(a, -b, x, y);
    Exp e;
    if (y != 0.0) e.push_back(y);
    if (x != 0.0) e.push_back(x);
    return e;
}

// e + b
Exp grow(const Exp& e, double b) {
    Exp h;
    h.reserve(e.size() + 1);
    double q = b;
    for (double ei : e) {
        double s, err;
        two_sum(q, ei, s, err);
        if (err != 0.0) h.push_back(err);
        q = s;
    }
    if (q != 0.0) h.push_back(q);
    return h;
}

// Renormalise to few components (Shewchuk's Compress): a top-down pass that
// merges components into the running sum, then a bottom-up pass.
Exp compress(const Exp& e) {
    if (e.size() < 3) return e;
    const size_t m = e.size();
    std::vector<double> g(m);
    double q = e[m - 1];
    size_t bottom = m - 1;
    for (size_t i = m - 1; i-- > 0;) {
        double qn, r;
        two_sum(q, e[i], qn, r);
        if (r != 0.0) {
            g[bottom--] = qn;
            q = r;
        } else {
            q = qn;
        }
    }
    g[bottom] = q;
    Exp h;
    h.reserve(m - bottom);
    q = g[bottom];
    for (size_t i = bottom + 1; i < m; ++i) {
        double qn, r;
        two_sum(g[i], q, qn, r);
        if (r != 0.0) h.push_back(r);
        q = qn;
    }
    if (q != 0.0 || h.empty()) h.push_back(q);
    if (h.size() == 1 && h[0] == 0.0) h.clear();
    return h;
}

Exp add(const Exp& e, const Exp& f) {
    Exp h = e;
    for (double fi : f) h = grow(h, fi);
    return compress(h);
}

Exp neg(Exp e) {
    for (double& x : e) x = -x;
    return e;
}

Exp sub(const Exp& e, const Exp& f) { return add(e, neg(f)); }

// e * b
Exp scale(const Exp& e, double b) {
    Exp h;
    if (e.empty() || b == 0.0) return h;
    h.reserve(2 * e.size());
    double q, err;
    two_prod(e[0], b, q, err);
    if (err != 0.0) h.push_back(err);
    for (size_t i = 1; i < e.size(); ++i) {
        double p1, p0, s;
        two_prod(e[i], b, p1, p0);
        two_sum(q, p0, s, err);
        if (err != 0.0) h.push_back(err);
        two_sum(p1, s, q, err);
        if (err != 0.0) h.push_back(err);
    }
    if (q != 0.0) h.push_back(q);
    return h;
}

Exp mul(const Exp& e, const Exp& f) {
    Exp h;
    for (double fi : f) h = add(h, scale(e, fi));
    return compress(h);
}

int sign_of(const Exp& e) {
    if (e.empty()) return 0;
    double top = e.back();
    return (top > 0.0) - (top < 0.0);
}

struct V3 {
    Exp x, y, z;
};

V3 diff3(const double* a, const double* b) { return {from_diff(a[0], b[0]), from_diff(a[1], b[1]), from_diff(a[2], b[2])}; }

// det[p; q; r] = p . (q x r)
Exp det3(const V3& p, const V3& q, const V3& r) {
    Exp m1 = sub(mul(q.y, r.z), mul(q.z, r.y));
    Exp m2 = sub(mul(q.x, r.z), mul(q.z, r.x));
    Exp m3 = sub(mul(q.x, r.y), mul(q.y, r.x));
    return add(sub(mul(p.x, m1), mul(p.y, m2)), mul(p.z, m3));
}

Exp lift(const V3& p) { return add(add(mul(p.x, p.x), mul(p.y, p.y)), mul(p.z, p.z)); }

inline double det3d(const double* p, const double* q, const double* r, double& perm) {
    double a1 = q[1] * r[2], a2 = q[2] * r[1];
    double b1 = q[0] * r[2], b2 = q[2] * r[0];
    double c1 = q[0] * r[1], c2 = q[1] * r[0];
    perm = std::fabs(p[0]) * (std::fabs(a1) + std::fabs(a2)) + std::fabs(p[1]) * (std::fabs(b1) + std::fabs(b2)) +
           std::fabs(p[2]) * (std::fabs(c1) + std::fabs(c2));
    return p[0] * (a1 - a2) - p[1] * (b1 - b2) + p[2] * (c1 - c2);
}

}  // namespace

long long predicate_exact_calls() { return g_exact_calls.load(); }

int orient3d(const double* a, const double* b, const double* c, const double* d) {
    double ba[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double ca[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double da[3] = {d[0] - a[0], d[1] - a[1], d[2] - a[2]};
    double perm;
    double det = det3d(ba, ca, da, perm);
    // Rounding error of this evaluation is below ~8 eps * perm; 1e-14 leaves a wide margin.
    double bound = 1e-14 * perm;
    if (det > bound) return 1;
    if (det < -bound) return -1;
    g_exact_calls.fetch_add(1, std::memory_order_relaxed);
    Exp e = det3(diff3(b, a), diff3(c, a), diff3(d, a));
    return sign_of(e);
}

// Lifted determinant with e as origin, expanded along the lifted column:
//   raw = -la*det(b',c',d') + lb*det(a',c',d') - lc*det(a',b',d') + ld*det(a',b',c')
// For a positively oriented (a,b,c,d), raw < 0 exactly when e is inside.
int insphere(const double* a, const double* b, const double* c, const double* d, const double* e) {
    double ae[3] = {a[0] - e[0], a[1] - e[1], a[2] - e[2]};
    double be[3] = {b[0] - e[0], b[1] - e[1], b[2] - e[2]};
    double ce[3] = {c[0] - e[0], c[1] - e[1], c[2] - e[2]};
    double de[3] = {d[0] - e[0], d[1] - e[1], d[2] - e[2]};
    double la = ae[0] * ae[0] + ae[1] * ae[1] + ae[2] * ae[2];
    double lb = be[0] * be[0] + be[1] * be[1] + be[2] * be[2];
    double lc = ce[0] * ce[0] + ce[1] * ce[1] + ce[2] * ce[2];
    double ld = de[0] * de[0] + de[1] * de[1] + de[2] * de[2];
    double pa, pb, pc, pd;
    double da = det3d(be, ce, de, pa);
    double db = det3d(ae, ce, de, pb);
    double dc = det3d(ae, be, de, pc);
    double dd = det3d(ae, be, ce, pd);
    double raw = -la * da + lb * db - lc * dc + ld * dd;
    double perm = la * pa + lb * pb + lc * pc + ld * pd;
    double bound = 2e-14 * perm;
    if (raw < -bound) return 1;
    if (raw > bound) return -1;
    g_exact_calls.fetch_add(1, std::memory_order_relaxed);
    V3 A = diff3(a, e), B = diff3(b, e), C = diff3(c, e), D = diff3(d, e);
    Exp r = add(sub(mul(lift(B), det3(A, C, D)), mul(lift(A), det3(B, C, D))),
                sub(mul(lift(D), det3(A, B, C)), mul(lift(C), det3(A, B, D))));
    return -sign_of(r);
}

}  // namespace p2m
