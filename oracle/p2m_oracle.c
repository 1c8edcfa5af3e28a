/*
 * TEST ORACLE -- test infrastructure only.  Nothing on the product path may
 * link, load or call this file; only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark do.
 *
 * Plain, slow FP64 brute force for the point-to-mesh query, written from the
 * problem statement (Sec. 4.1): vertices are points, edges are open segments,
 * faces are open triangles, and the answer is the generator of the
 * generalised Voronoi diagram of V, E, F whose cell holds the query point,
 * with its closest point and distance (Sec. 1).  With open primitives the
 * gated tests of the query procedure (Appendix, Algorithm A.2) give, for
 * every primitive, either its exact distance or "infinity":
 *
 *   d_V(i) = |q - v_i|
 *   d_E(j) = distance from q to the line of e_j   iff the foot parameter
 *            t = (q-a).(b-a)/|b-a|^2 lies in (0,1)  (the two end planes of
 *            Space-perp(e) in Algorithm A.2), else infinity
 *   d_F(k) = distance from q to the plane of f_k  iff the foot lies strictly
 *            inside the triangle (q in Space-perp(f), Eq. (4)), else infinity
 *
 * The minimum of these over ALL of V, E, F is the point-to-mesh distance;
 * the paper's KD tree + interception table only restricts which primitives
 * are examined (Theorems 1 and 7).  Ties are broken by (d, dim, id) with
 * dim vertex 0 < edge 1 < face 2.
 *
 * Edge ids: the undirected pairs (min,max) of all face sides, deduplicated
 * and sorted lexicographically; the id is the rank.  Face id = input row,
 * vertex id = input index.
 *
 * A second, independent closed-form distance -- the clamped point-triangle
 * distance from the Voronoi regions of a closed triangle (Ericson, Real-Time
 * Collision Detection, Sec. 5.1.5) -- is provided for self-checks.
 *
 * OpenMP parallelises over queries only; every query's arithmetic is the
 * plain definition above.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { O_VERTEX = 0, O_EDGE = 1, O_FACE = 2, O_NONE = 3 };

typedef struct { double x, y, z; } d3;

static d3 mk(double x, double y, double z) { d3 r = {x, y, z}; return r; }
static d3 at(const double* V, int64_t i) { return mk(V[3 * i], V[3 * i + 1], V[3 * i + 2]); }
static d3 sub(d3 a, d3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static d3 add(d3 a, d3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static d3 scl(d3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static d3 cross(d3 a, d3 b) { return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
static double norm(d3 a) { return sqrt(dot(a, a)); }

int p2mo_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void p2mo_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------- edges */

static int cmp_pair(const void* a, const void* b) {
    const int64_t* x = (const int64_t*)a;
    const int64_t* y = (const int64_t*)b;
    return (*x > *y) - (*x < *y);
}

/* Canonical edge list.  pairs_out (capacity 3*nf*2 int32) may be NULL to
 * query the count only.  Returns the number of edges. */
int64_t p2mo_edges(int64_t nv, const int32_t* F, int64_t nf, int32_t* pairs_out) {
    int64_t m = 3 * nf;
    int64_t* key = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    for (int64_t f = 0; f < nf; ++f) {
        for (int s = 0; s < 3; ++s) {
            int64_t a = F[3 * f + s], b = F[3 * f + (s + 1) % 3];
            int64_t lo = a < b ? a : b, hi = a < b ? b : a;
            key[3 * f + s] = lo * nv + hi;
        }
    }
    qsort(key, (size_t)m, sizeof(int64_t), cmp_pair);
    int64_t ne = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (i > 0 && key[i] == key[i - 1]) continue;
        if (pairs_out) {
            pairs_out[2 * ne] = (int32_t)(key[i] / nv);
            pairs_out[2 * ne + 1] = (int32_t)(key[i] % nv);
        }
        ++ne;
    }
    free(key);
    return ne;
}

/* ------------------------------------------------ gated primitive tests */

/* Vertex: always defined. */
static double vertex_dist(d3 q, d3 v, d3* foot) {
    *foot = v;
    return norm(sub(q, v));
}

/* Open edge: distance to the line if the foot parameter is in (lo_t, hi_t),
 * else +inf.  Strict gates use lo_t = 0, hi_t = 1. */
static double edge_dist(d3 q, d3 a, d3 b, double lo_t, double hi_t, d3* foot, double* t_out) {
    d3 ab = sub(b, a);
    double t = dot(sub(q, a), ab) / dot(ab, ab);
    *t_out = t;
    if (!(t > lo_t && t < hi_t)) return INFINITY;
    *foot = add(a, scl(ab, t));
    return norm(sub(q, *foot));
}

/* Foot of q on the plane of (a,b,c) and its barycentric coordinates from
 * signed sub-triangle areas measured against the face normal n. */
static d3 face_foot(d3 q, d3 a, d3 b, d3 c, double w[3]) {
    d3 n = cross(sub(b, a), sub(c, a));
    double nn = dot(n, n);
    d3 p = sub(q, scl(n, dot(sub(q, a), n) / nn));
    w[0] = dot(cross(sub(b, p), sub(c, p)), n) / nn;
    w[1] = dot(cross(sub(c, p), sub(a, p)), n) / nn;
    w[2] = dot(cross(sub(a, p), sub(b, p)), n) / nn;
    return p;
}

/* Open face: distance to the plane if the foot is strictly inside. */
static double face_dist(d3 q, d3 a, d3 b, d3 c, d3* foot, double w[3]) {
    d3 p = face_foot(q, a, b, c, w);
    if (!(w[0] > 0.0 && w[1] > 0.0 && w[2] > 0.0)) return INFINITY;
    *foot = p;
    return norm(sub(q, p));
}

static int better(double d, int dim, int64_t id, double bd, int bdim, int64_t bid) {
    if (d < bd) return 1;
    if (d > bd) return 0;
    if (dim != bdim) return dim < bdim;
    return id < bid;
}

/* Brute force over all of V, E, F for every query.
 * Outputs: type [nq] (0 vertex, 1 edge, 2 face), id [nq], closest [nq*3],
 * dist [nq]; runner_up [nq] (the smallest gated distance of any other
 * primitive) may be NULL. */
void p2mo_query(const double* V, int64_t nv, const int32_t* F, int64_t nf,
                const int32_t* E, int64_t ne, const double* Q, int64_t nq,
                int32_t* type, int64_t* id, double* closest, double* dist,
                double* runner_up) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nq; ++i) {
        d3 q = at(Q, i);
        double bd = INFINITY, rd = INFINITY;
        int bdim = O_NONE;
        int64_t bid = -1;
        d3 bc = mk(NAN, NAN, NAN), foot;
        double t, w[3];
        for (int64_t k = 0; k < nv; ++k) {
            double d = vertex_dist(q, at(V, k), &foot);
            if (better(d, O_VERTEX, k, bd, bdim, bid)) {
                rd = bd < rd ? bd : rd;
                bd = d; bdim = O_VERTEX; bid = k; bc = foot;
            } else if (d < rd) {
                rd = d;
            }
        }
        for (int64_t k = 0; k < ne; ++k) {
            double d = edge_dist(q, at(V, E[2 * k]), at(V, E[2 * k + 1]), 0.0, 1.0, &foot, &t);
            if (better(d, O_EDGE, k, bd, bdim, bid)) {
                rd = bd < rd ? bd : rd;
                bd = d; bdim = O_EDGE; bid = k; bc = foot;
            } else if (d < rd) {
                rd = d;
            }
        }
        for (int64_t k = 0; k < nf; ++k) {
            double d = face_dist(q, at(V, F[3 * k]), at(V, F[3 * k + 1]), at(V, F[3 * k + 2]), &foot, w);
            if (better(d, O_FACE, k, bd, bdim, bid)) {
                rd = bd < rd ? bd : rd;
                bd = d; bdim = O_FACE; bid = k; bc = foot;
            } else if (d < rd) {
                rd = d;
            }
        }
        type[i] = bdim;
        id[i] = bid;
        closest[3 * i] = bc.x; closest[3 * i + 1] = bc.y; closest[3 * i + 2] = bc.z;
        dist[i] = bd;
        if (runner_up) runner_up[i] = rd;
    }
}

/* In-plane distance from a foot point p (on the plane of a,b,c) to the
 * closed triangle: 0 when all barycentrics are >= 0, else the distance to
 * the nearest closed side. */
static double seg_dist(d3 p, d3 a, d3 b) {
    d3 ab = sub(b, a);
    double t = dot(sub(p, a), ab) / dot(ab, ab);
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    return norm(sub(p, add(a, scl(ab, t))));
}

/* Near-optimal set of one query: every primitive whose distance under
 * tolerance-relaxed gates is <= dstar + tol.  Relaxed gates: edge foot
 * parameter in [-tol/|e|, 1 + tol/|e|]; face foot within tol of the closed
 * triangle (in its plane).  Writes up to cap (type, id) pairs and returns
 * the total count. */
int64_t p2mo_near_set(const double* V, int64_t nv, const int32_t* F, int64_t nf,
                      const int32_t* E, int64_t ne, const double* q3, double dstar,
                      double tol, int32_t* types, int64_t* ids, int64_t cap) {
    d3 q = mk(q3[0], q3[1], q3[2]);
    int64_t cnt = 0;
    d3 foot;
    double t, w[3];
    for (int64_t k = 0; k < nv; ++k) {
        if (vertex_dist(q, at(V, k), &foot) <= dstar + tol) {
            if (cnt < cap) { types[cnt] = O_VERTEX; ids[cnt] = k; }
            ++cnt;
        }
    }
    for (int64_t k = 0; k < ne; ++k) {
        d3 a = at(V, E[2 * k]), b = at(V, E[2 * k + 1]);
        d3 ab = sub(b, a);
        double r = tol / norm(ab);
        t = dot(sub(q, a), ab) / dot(ab, ab);
        if (!(t >= -r && t <= 1.0 + r)) continue;
        if (norm(sub(q, add(a, scl(ab, t)))) <= dstar + tol) {
            if (cnt < cap) { types[cnt] = O_EDGE; ids[cnt] = k; }
            ++cnt;
        }
    }
    for (int64_t k = 0; k < nf; ++k) {
        d3 a = at(V, F[3 * k]), b = at(V, F[3 * k + 1]), c = at(V, F[3 * k + 2]);
        d3 p = face_foot(q, a, b, c, w);
        double off = 0.0;
        if (!(w[0] >= 0.0 && w[1] >= 0.0 && w[2] >= 0.0)) {
            double d0 = seg_dist(p, a, b), d1 = seg_dist(p, b, c), d2 = seg_dist(p, c, a);
            off = d0 < d1 ? d0 : d1;
            off = off < d2 ? off : d2;
        }
        if (off <= tol && norm(sub(q, p)) <= dstar + tol) {
            if (cnt < cap) { types[cnt] = O_FACE; ids[cnt] = k; }
            ++cnt;
        }
    }
    return cnt;
}

/* ------------------------------------- independent clamped formulation */

/* Closest point on the closed triangle (a,b,c) to p, by the triangle's
 * Voronoi regions (vertex, edge, face), Ericson RTCD Sec. 5.1.5. */
static d3 closest_on_triangle(d3 p, d3 a, d3 b, d3 c) {
    d3 ab = sub(b, a), ac = sub(c, a), ap = sub(p, a);
    double d1 = dot(ab, ap), d2 = dot(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) return a;
    d3 bp = sub(p, b);
    double d3_ = dot(ab, bp), d4 = dot(ac, bp);
    if (d3_ >= 0.0 && d4 <= d3_) return b;
    double vc = d1 * d4 - d3_ * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3_ <= 0.0) return add(a, scl(ab, d1 / (d1 - d3_)));
    d3 cp = sub(p, c);
    double d5 = dot(ab, cp), d6 = dot(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) return c;
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) return add(a, scl(ac, d2 / (d2 - d6)));
    double va = d3_ * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3_) >= 0.0 && (d5 - d6) >= 0.0)
        return add(b, scl(sub(c, b), (d4 - d3_) / ((d4 - d3_) + (d5 - d6))));
    double den = 1.0 / (va + vb + vc);
    return add(a, add(scl(ab, vb * den), scl(ac, vc * den)));
}

/* min over all closed triangles of the clamped distance. */
void p2mo_dist_clamped(const double* V, int64_t nv, const int32_t* F, int64_t nf,
                       const double* Q, int64_t nq, double* dist) {
    (void)nv;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nq; ++i) {
        d3 q = at(Q, i);
        double best = INFINITY;
        for (int64_t k = 0; k < nf; ++k) {
            d3 c = closest_on_triangle(q, at(V, F[3 * k]), at(V, F[3 * k + 1]), at(V, F[3 * k + 2]));
            double d = norm(sub(q, c));
            if (d < best) best = d;
        }
        dist[i] = best;
    }
}

/* Distance from q to one closed primitive given by (type, id): used by the
 * tests to check that a reported closest point lies on the reported
 * primitive.  Returns the distance from point x to that closed primitive. */
double p2mo_point_to_primitive(const double* V, const int32_t* F, const int32_t* E,
                               int32_t type, int64_t id, const double* x3) {
    d3 x = mk(x3[0], x3[1], x3[2]);
    if (type == O_VERTEX) return norm(sub(x, at(V, id)));
    if (type == O_EDGE) return seg_dist(x, at(V, E[2 * id]), at(V, E[2 * id + 1]));
    if (type == O_FACE) {
        d3 c = closest_on_triangle(x, at(V, F[3 * id]), at(V, F[3 * id + 1]), at(V, F[3 * id + 2]));
        return norm(sub(x, c));
    }
    return INFINITY;
}
