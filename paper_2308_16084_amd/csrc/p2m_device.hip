// Device side of the P2M query for gfx950: arena upload, query ordering
// (Morton keys + stable LSD radix sort), the query kernel (Algorithm A.2),
// the nearest-vertex kernel, the backward kernel, and the host CPU baseline
// that runs the same per-query code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "device_common.hpp"
#include "p2m_internal.hpp"
#include "nearest.hpp"
#include "query_core.hpp"
#include "regroup.hpp"
#include "wave_scan.hpp"

namespace p2m {

// ------------------------------------------------------------- packing

float float_down(double d) {
    float f = (float)d;
    if ((double)f > d) f = std::nextafter(f, -INFINITY);
    return f;
}
float float_up(double d) {
    float f = (float)d;
    if ((double)f < d) f = std::nextafter(f, INFINITY);
    return f;
}

static float bits_as_float(int32_t i) {
    float f;
    std::memcpy(&f, &i, 4);
    return f;
}

// List-scan forms (see query_core.hpp, step 3), built in float64 in
// coordinates relative to the domain centre rounded to float, then rounded.
// mu = 2^-20 of the domain diagonal: the float32 error of a form evaluated
// at a query in D is a few 2^-24 of the domain size, well inside mu.
static void pack_scan_forms(MeshState& s) {
    const MeshData& m = s.m;
    double c[3], diag2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        s.ctr[k] = (float)(0.5 * (s.dlo[k] + s.dhi[k]));
        c[k] = (double)s.ctr[k];
        diag2 += (s.dhi[k] - s.dlo[k]) * (s.dhi[k] - s.dlo[k]);
    }
    const double mu = std::ldexp(std::sqrt(diag2), -20);
    s.mu = (float)mu;
    auto P = [&](int32_t v, double o[3]) {
        for (int k = 0; k < 3; ++k) o[k] = (double)m.V[3 * (size_t)v + k] - c[k];
    };
    auto cross = [](const double a[3], const double b[3], double o[3]) {
        o[0] = a[1] * b[2] - a[2] * b[1];
        o[1] = a[2] * b[0] - a[0] * b[2];
        o[2] = a[0] * b[1] - a[1] * b[0];
    };
    auto dot = [](const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
    s.pk_erec.assign((size_t)(8 * m.ne), 0.f);
    for (int64_t e = 0; e < m.ne; ++e) {
        double a[3], b[3], u[3];
        P(m.E[(size_t)(2 * e)], a);
        P(m.E[(size_t)(2 * e + 1)], b);
        for (int k = 0; k < 3; ++k) u[k] = b[k] - a[k];
        const double L = std::sqrt(dot(u, u));
        float* d = &s.pk_erec[(size_t)(8 * e)];
        for (int k = 0; k < 3; ++k) {
            d[k] = (float)a[k];
            d[4 + k] = (float)(u[k] / L);
        }
        d[3] = (float)L;
    }
    s.pk_frec.assign((size_t)(12 * m.nf), 0.f);
    for (int64_t f = 0; f < m.nf; ++f) {
        double p[3][3];
        for (int k = 0; k < 3; ++k) P(m.F[(size_t)(3 * f + k)], p[k]);
        double e1[3], e2[3], n[3];
        for (int k = 0; k < 3; ++k) {
            e1[k] = p[1][k] - p[0][k];
            e2[k] = p[2][k] - p[0][k];
        }
        cross(e1, e2, n);
        const double twice_area = std::sqrt(dot(n, n));
        for (int k = 0; k < 3; ++k) n[k] /= twice_area;
        float* d = &s.pk_frec[(size_t)(12 * f)];
        for (int k = 0; k < 3; ++k) d[k] = (float)n[k];
        d[3] = (float)dot(n, p[0]);
        // Barycentric weight of corner i as an affine form r.x - o (the
        // signed area of x and the opposite side over the face's): r =
        // n x (p[i+2] - p[i+1]) / 2A, |r| = 1 / height_i.  The corner opposite
        // the longest side (smallest height) is not stored: its weight is 1
        // minus the other two, whose rounding, in distance units, is then at
        // most twice that of a stored form.  Each weight may go down to
        // -mu / height_i (the foot within mu outside that side).
        double len[3];
        for (int i = 0; i < 3; ++i) {
            double ed[3];
            for (int k = 0; k < 3; ++k) ed[k] = p[(i + 2) % 3][k] - p[(i + 1) % 3][k];
            len[i] = std::sqrt(dot(ed, ed));
        }
        const int skip = len[0] >= len[1] ? (len[0] >= len[2] ? 0 : 2) : (len[1] >= len[2] ? 1 : 2);
        // The stored forms give w_i + mu / h_i; the third weight may go down to
        // -mu / h_skip when their sum is at most 1 + mu (len_0 + len_1 + len_2)
        // / 2A (this lets it go a further mu (1/h_1 + 1/h_2) <= 2 mu / h_skip,
        // so its side's margin is at most 3 mu); both forms are divided by that
        // bound so the test reads <= 1.
        const double scale = 1.0 / (1.0 + mu * (len[0] + len[1] + len[2]) / twice_area);
        for (int j = 0; j < 2; ++j) {
            const int i = (skip + 1 + j) % 3;
            const double* b = p[(i + 1) % 3];
            const double* cc = p[(i + 2) % 3];
            double ed[3], r[3], bc[3];
            for (int k = 0; k < 3; ++k) ed[k] = cc[k] - b[k];
            cross(n, ed, r);
            cross(b, cc, bc);
            float* o = d + 4 * (j + 1);
            for (int k = 0; k < 3; ++k) o[k] = (float)(r[k] / twice_area * scale);
            o[3] = (float)((-dot(n, bc) - mu * len[i]) / twice_area * scale);
        }
    }
}

// List heads and 8-byte list entries (see MeshView::vhead, ::lent): each
// entry box re-quantised to 5 bits per coordinate inside the list box (the
// union of the list's entry boxes), rounded outward; runs padded to even
// length with empty-box entries.
static void pack_lists(MeshState& s) {
    const Table& t = s.t;
    const int64_t nv = s.m.nv;
    const uint32_t kEmpty = 31u | 31u << 5 | 31u << 10;  // lower corner 31, upper 0
    s.pk_vhead.assign((size_t)(8 * nv), 0u);
    s.pk_lent.clear();
    s.pk_lent.reserve(2 * t.ent.size() + 4 * (size_t)nv);
    for (int64_t v = 0; v < nv; ++v) {
        const uint32_t a = t.off[(size_t)(2 * v)], b = t.off[(size_t)(2 * v + 1)], c = t.off[(size_t)(2 * v + 2)];
        uint32_t lo[3] = {65535u, 65535u, 65535u}, hi[3] = {0u, 0u, 0u};
        for (uint32_t k = a; k < c; ++k) {
            const uint16_t* bx = &t.box[6 * (size_t)k];
            if (bx[0] > bx[3] || bx[1] > bx[4] || bx[2] > bx[5]) continue;  // empty
            for (int i = 0; i < 3; ++i) {
                lo[i] = std::min<uint32_t>(lo[i], bx[i]);
                hi[i] = std::max<uint32_t>(hi[i], bx[3 + i]);
            }
        }
        if (lo[0] > hi[0]) lo[0] = lo[1] = lo[2] = hi[0] = hi[1] = hi[2] = 0u;  // no entry holds any point
        uint32_t* h = &s.pk_vhead[(size_t)(8 * v)];
        h[4] = lo[0] | lo[1] << 16;
        h[5] = lo[2] | hi[0] << 16;
        h[6] = hi[1] | hi[2] << 16;
        auto run = [&](uint32_t k0, uint32_t k1) {
            for (uint32_t k = k0; k < k1; ++k) {
                const uint16_t* bx = &t.box[6 * (size_t)k];
                uint32_t code = kEmpty;
                if (!(bx[0] > bx[3] || bx[1] > bx[4] || bx[2] > bx[5])) {
                    code = 0u;
                    for (int i = 0; i < 3; ++i) {
                        const double span = (double)std::max<uint32_t>(hi[i] - lo[i], 1u);
                        const double l = std::floor(((double)bx[i] - lo[i]) * 31.0 / span);
                        const double u = std::ceil(((double)bx[3 + i] - lo[i]) * 31.0 / span);
                        code |= (uint32_t)std::min(31.0, std::max(0.0, l)) << (5 * i);
                        code |= (uint32_t)std::min(31.0, std::max(0.0, u)) << (15 + 5 * i);
                    }
                }
                s.pk_lent.push_back((uint32_t)t.ent[k]);
                s.pk_lent.push_back(code);
            }
            if ((k1 - k0) & 1u) {
                s.pk_lent.push_back(0u);
                s.pk_lent.push_back(kEmpty);
            }
        };
        h[0] = (uint32_t)(s.pk_lent.size() / 2);
        run(a, b);
        h[1] = (uint32_t)(s.pk_lent.size() / 2);
        run(b, c);
        h[2] = (uint32_t)(s.pk_lent.size() / 2);
    }
}

void pack_mesh(MeshState& s) {
    if (s.packed) return;
    const MeshData& m = s.m;
    // KD-tree nodes: point + vertex id, then left / right subtree boxes
    const int64_t n = m.nv;
    std::vector<float> box((size_t)(6 * n));  // subtree box of node i: lo.xyz, hi.xyz
    for (int64_t i = n - 1; i >= 0; --i) {
        float* bx = &box[(size_t)(6 * i)];
        const float p[3] = {s.kd.x[(size_t)i], s.kd.y[(size_t)i], s.kd.z[(size_t)i]};
        for (int k = 0; k < 3; ++k) bx[k] = bx[3 + k] = p[k];
        for (int64_t c = 2 * i + 1; c <= 2 * i + 2 && c < n; ++c)
            for (int k = 0; k < 3; ++k) {
                bx[k] = std::min(bx[k], box[(size_t)(6 * c + k)]);
                bx[3 + k] = std::max(bx[3 + k], box[(size_t)(6 * c + 3 + k)]);
            }
    }
    s.pk_node.assign((size_t)(16 * n), 0.f);
    for (int64_t i = 0; i < n; ++i) {
        float* d = &s.pk_node[(size_t)(16 * i)];
        d[0] = s.kd.x[(size_t)i];
        d[1] = s.kd.y[(size_t)i];
        d[2] = s.kd.z[(size_t)i];
        d[3] = bits_as_float(s.kd.vid[(size_t)i]);
        for (int side = 0; side < 2; ++side) {
            const int64_t c = 2 * i + 1 + side;
            float* o = d + 4 + 6 * side;
            for (int k = 0; k < 3; ++k) {
                o[k] = c < n ? box[(size_t)(6 * c + k)] : INFINITY;
                o[3 + k] = c < n ? box[(size_t)(6 * c + 3 + k)] : -INFINITY;
            }
        }
    }
    s.pk_seg.resize((size_t)(8 * m.ne));
    for (int64_t e = 0; e < m.ne; ++e)
        for (int k = 0; k < 2; ++k) {
            int32_t v = m.E[(size_t)(2 * e + k)];
            float* d = &s.pk_seg[(size_t)(8 * e + 4 * k)];
            d[0] = m.V[3 * (size_t)v];
            d[1] = m.V[3 * (size_t)v + 1];
            d[2] = m.V[3 * (size_t)v + 2];
            d[3] = bits_as_float(v);
        }
    s.pk_tri.resize((size_t)(12 * m.nf));
    s.pk_fedge.resize((size_t)(4 * m.nf));
    for (int64_t f = 0; f < m.nf; ++f) {
        for (int k = 0; k < 3; ++k) {
            int32_t v = m.F[(size_t)(3 * f + k)];
            float* d = &s.pk_tri[(size_t)(12 * f + 4 * k)];
            d[0] = m.V[3 * (size_t)v];
            d[1] = m.V[3 * (size_t)v + 1];
            d[2] = m.V[3 * (size_t)v + 2];
            d[3] = bits_as_float(v);
            s.pk_fedge[(size_t)(4 * f + k)] = m.FE[(size_t)(3 * f + k)];
        }
        s.pk_fedge[(size_t)(4 * f + 3)] = -1;
    }
    pack_scan_forms(s);
    pack_lists(s);
    // Voronoi walk: 32-bit neighbour offsets, and each neighbour's position
    // with its id stored in the neighbour list itself (one 16-byte record per
    // entry: a walk step reads one contiguous run, no id -> position gather)
    s.pk_nboff.resize(s.t.nb_off.size());
    for (size_t k = 0; k < s.t.nb_off.size(); ++k) s.pk_nboff[k] = (uint32_t)s.t.nb_off[k];
    // kWalkGroup - 1 records of padding at the end (copies of the last): a
    // walk group loads kWalkGroup consecutive records from any list start
    s.pk_nbrec.resize(4 * (s.t.nb.size() + kWalkGroup - 1));
    for (size_t k = 0; k < s.t.nb.size() + kWalkGroup - 1; ++k) {
        const int32_t w = s.t.nb[std::min(k, s.t.nb.size() - 1)];
        float* d = &s.pk_nbrec[4 * k];
        for (int c = 0; c < 3; ++c) d[c] = m.V[3 * (size_t)w + c];
        d[3] = bits_as_float(w);
    }
    s.pk_seed.clear();
    s.pk_seed2.clear();
    s.packed = true;
}

// Absolute slack of the winner check (query_core.hpp, step 4): 2^-21 of the
// mesh's diagonal plus its largest coordinate magnitude, a few times the
// float32 rounding of a distance computed near the mesh.
float winner_slack(const MeshState& s) {
    double diag2 = 0.0, amax = 0.0;
    for (int k = 0; k < 3; ++k) {
        diag2 += (s.m.hi[k] - s.m.lo[k]) * (s.m.hi[k] - s.m.lo[k]);
        amax = std::max(amax, std::max(std::fabs(s.m.lo[k]), std::fabs(s.m.hi[k])));
    }
    return (float)std::ldexp(std::sqrt(diag2) + amax, -21);
}

MeshView host_view(const MeshState& s) {
    MeshView v;
    v.node = (const KdNode*)s.pk_node.data();
    v.nv = (int32_t)s.m.nv;
    v.vhead = (const uint4*)s.pk_vhead.data();
    v.lent = (const uint4*)s.pk_lent.data();
    v.seg = (const float4*)s.pk_seg.data();
    v.tri = (const float4*)s.pk_tri.data();
    v.fedge = s.pk_fedge.data();
    v.frec = (const float4*)s.pk_frec.data();
    v.erec = (const float4*)s.pk_erec.data();
    for (int k = 0; k < 3; ++k) v.ctr[k] = s.ctr[k];
    v.mu = s.mu;
    v.eta = winner_slack(s);
    for (int k = 0; k < 3; ++k) {
        v.qlo[k] = (float)s.dlo[k];
        v.qs[k] = (float)(65535.0 / (s.dhi[k] - s.dlo[k]));
    }
    for (int k = 0; k < 3; ++k) {
        v.dlo[k] = float_down(s.dlo[k]);
        v.dhi[k] = float_up(s.dhi[k]);
    }
    v.nboff = nullptr;
    v.nbrec = nullptr;
    v.seed = s.pk_seed.empty() ? nullptr : (const float4*)s.pk_seed.data();
    v.grid = walk_grid_side(s.m.nv);
    for (int k = 0; k < 3; ++k) {
        v.glo[k] = v.dlo[k];
        v.gscale[k] = (float)((double)v.grid / ((double)v.dhi[k] - (double)v.dlo[k]));
    }
    // the finer grid: the mesh's box grown by 5 % of its diagonal, when D
    // is more than twice as long on some axis (for a D just around the mesh
    // the second grid costs more in cache than it saves in walk steps)
    v.seed2 = s.pk_seed2.empty() ? nullptr : (const float4*)s.pk_seed2.data();
    v.grid2 = 0;
    {
        double diag = 0.0;
        for (int k = 0; k < 3; ++k) diag += (s.m.hi[k] - s.m.lo[k]) * (s.m.hi[k] - s.m.lo[k]);
        const double grow = 0.05 * std::sqrt(diag);
        bool wide = false;
        double flo[3], fhi[3];
        for (int k = 0; k < 3; ++k) {
            flo[k] = s.m.lo[k] - grow;
            fhi[k] = s.m.hi[k] + grow;
            if (!(fhi[k] > flo[k])) fhi[k] = flo[k] + 1.0;
            wide |= (s.dhi[k] - s.dlo[k]) > 2.0 * (fhi[k] - flo[k]);
        }
        if (wide) {
            v.grid2 = walk_grid_side(s.m.nv);
            for (int k = 0; k < 3; ++k) {
                v.glo2[k] = (float)flo[k];
                v.gscale2[k] = (float)((double)v.grid2 / (fhi[k] - flo[k]));
                v.ghi2[k] = (float)fhi[k];
            }
        } else {
            for (int k = 0; k < 3; ++k) v.glo2[k] = v.gscale2[k] = v.ghi2[k] = 0.f;
        }
    }
    v.nboff = s.pk_nboff.data();
    v.nbrec = (const float4*)s.pk_nbrec.data();
    return v;
}

int32_t walk_grid_side(int64_t nv) {
    const double g = std::ceil(3.0 * std::cbrt((double)std::max<int64_t>(nv, 1)));
    return (int32_t)std::min(256.0, std::max(8.0, g));
}

MeshView device_view(const MeshState& s) {
    MeshView v = host_view(s);
    v.node = (const KdNode*)s.dev.node;
    v.vhead = (const uint4*)s.dev.vhead;
    v.lent = (const uint4*)s.dev.lent;
    v.seg = (const float4*)s.dev.seg;
    v.tri = (const float4*)s.dev.tri;
    v.fedge = (const int32_t*)s.dev.fedge;
    v.frec = (const float4*)s.dev.frec;
    v.erec = (const float4*)s.dev.erec;
    v.nboff = (const uint32_t*)s.dev.nboff;
    v.nbrec = (const float4*)s.dev.nbrec;
    v.seed = (const float4*)s.dev.seed;
    v.seed2 = (const float4*)s.dev.seed2;
    return v;
}

void device_release(MeshState& s) {
    if (s.dev.device < 0) return;
    int old = -1;
    (void)hipGetDevice(&old);
    (void)hipSetDevice(s.dev.device);
    if (s.dev.base) (void)hipFree(s.dev.base);
    if (s.dev.scratch) (void)hipFree(s.dev.scratch);
    for (void*& e : s.dev.ev)
        if (e) (void)hipEventDestroy((hipEvent_t)e);
    if (old >= 0) (void)hipSetDevice(old);
    s.dev = DeviceMesh();
}

// ------------------------------------------------------------- kernels

// XCD-aware tile order: consecutive hardware blocks go round-robin to the 8
// XCDs, each with its own L2.  Tiles are dealt to the XCDs in runs of G
// consecutive (Morton-ordered, so spatially adjacent) tiles: blocks b of
// one super-group of 8G hold tiles sg*8G + x*G + k, XCD x = b mod 8 taking
// the run x*G .. x*G+G-1.  A run shares its L2, and the blocks resident at
// one time cover a compact stretch of the batch, which the shared Infinity
// Cache holds.  Measured on 10^7 and 10^6 queries of one mesh: one
// contiguous eighth of the batch per XCD was 4 % slower on the larger batch,
// G = 1 8 % slower on the smaller.  The grid is a multiple of 8G; tiles >=
// ntiles are skipped.
constexpr int64_t kXcdRun = 16;
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t G) {
    const int64_t sg = b / (kXcds * G), r = b % (kXcds * G);
    return sg * kXcds * G + (r % kXcds) * G + r / kXcds;
}

__global__ void k_morton(const float* __restrict__ q, int64_t n, float lox, float loy, float loz, float sx, float sy,
                         float sz, uint32_t* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = morton30(q[3 * i], q[3 * i + 1], q[3 * i + 2], lox, loy, loz, sx, sy, sz);
}

// Morton keys of one sort tile (kRadixTile queries) and the tile's counts of
// the sort's first digit, key bits [shift, shift + 8), written to the tile's
// column of the digit-major count matrix: the sort's first pass then needs
// no histogram kernel of its own.  kRadixHistThreads threads a tile, four
// consecutive queries each; with kVec (q 16-byte aligned) a thread reads its
// four queries as three float4 and writes their keys as one uint4.
template <bool kVec>
__global__ __launch_bounds__(kRadixHistThreads) void k_morton_hist(const float* __restrict__ q, int64_t n, float lox,
                                                                   float loy, float loz, float sx, float sy, float sz,
                                                                   int shift, uint32_t* __restrict__ keys,
                                                                   uint32_t* __restrict__ counts, int64_t tiles) {
    constexpr int kHI = (int)(kRadixTile / kRadixHistThreads);
    static_assert(kHI == 4, "four queries a thread");
    __shared__ uint32_t h[256];
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * kRadixTile + 4 * t;
    uint32_t key[kHI] = {0u, 0u, 0u, 0u};
    if (kVec && i0 + 3 < n) {
        const float4* q4 = reinterpret_cast<const float4*>(q + 3 * i0);
        const float4 a = q4[0], b = q4[1], c = q4[2];
        key[0] = morton30(a.x, a.y, a.z, lox, loy, loz, sx, sy, sz);
        key[1] = morton30(a.w, b.x, b.y, lox, loy, loz, sx, sy, sz);
        key[2] = morton30(b.z, b.w, c.x, lox, loy, loz, sx, sy, sz);
        key[3] = morton30(c.y, c.z, c.w, lox, loy, loz, sx, sy, sz);
        *reinterpret_cast<uint4*>(keys + i0) = make_uint4(key[0], key[1], key[2], key[3]);
    } else {
#pragma unroll
        for (int k = 0; k < kHI; ++k) {
            const int64_t i = i0 + k;
            if (i < n) {
                key[k] = morton30(q[3 * i], q[3 * i + 1], q[3 * i + 2], lox, loy, loz, sx, sy, sz);
                keys[i] = key[k];
            }
        }
    }
    if (t < 256) h[t] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kHI; ++k) radix_hist_add(h, (key[k] >> shift) & 255u, i0 + k < n);
    __syncthreads();
    if (t < 256) counts[(int64_t)t * tiles + blockIdx.x] = h[t];
}

// Dynamic LDS of k_query: the regroup bins, then per slot 7 floats (q, the
// nearest vertex's d2 and position) and 2 ints (query index, vertex); after
// the regroup, the slots of each wavefront hold its scan keys and owners;
// then the scan rings' candidate ids, per wavefront.
constexpr size_t regroup_slot_bytes(int block) { return sizeof(uint32_t) * (kRegroupBins + 9 * (size_t)block); }
constexpr size_t regroup_lds_bytes(int block) {
    return regroup_slot_bytes(block) + sizeof(WaveScanIds) * (size_t)(block / 64);
}
static_assert(sizeof(WaveScanKeys) <= 9 * 64 * sizeof(uint32_t), "scan keys exceed a wavefront's regroup slots");
// then, for the per-lane tree search, the staged top of the tree (16-byte aligned)
constexpr size_t top_lds_offset(int block) { return (regroup_lds_bytes(block) + 15) / 16 * 16; }

// stage (ordered batches): query i's answer goes to one aligned record at
// its input position instead of several partial cache lines in the output
// arrays, and a write-out kernel then fills those arrays with coalesced
// stores.  Without the backward extras the record is 16 bytes, (prim,
// staged point): the write-out forms the closest point and distance
// (staged_point) and the status from q itself.  Each record is a write to a random place of the batch,
// and these writes cost about a sixth of the kernel on 10^7 queries; 16
// bytes cost less than the 32 of (prim, closest), (dist, status).  With
// the extras: 48 bytes, (prim, closest), (dist, status, w0, w1), (w2, pv0,
// pv1, pv2).  Without stage the answer goes to the output arrays directly.
template <bool kWriteExtras, int kWalk>
__global__ __launch_bounds__(kQueryMaxBlock) void k_query(MeshView m, const float* __restrict__ q,
                                                const int32_t* __restrict__ perm, int64_t n, int64_t run,
                                                int32_t* __restrict__ prim, float* __restrict__ closest,
                                                float* __restrict__ dist, uint8_t* __restrict__ status,
                                                float* __restrict__ bary, int32_t* __restrict__ pvid,
                                                float4* __restrict__ stage, int32_t ntop) {
    extern __shared__ uint32_t lds[];
    const int64_t tile = xcd_tile(blockIdx.x, run);
    const int t = threadIdx.x, B = blockDim.x;
    const int64_t j = tile * B + t;
    int64_t i = j < n ? (perm ? (int64_t)perm[j] : j) : -1;
    if (i >= n) i = -1;
    float qx = 0.f, qy = 0.f, qz = 0.f;
    if (i >= 0) {
        qx = q[3 * i];
        qy = q[3 * i + 1];
        qz = q[3 * i + 2];
    }
    bool fin = finite3(qx, qy, qz);
    ScanCounters c;
    // the per-lane tree search may read the tree's top levels from a copy in
    // LDS, after the regroup slots and the scan ids
    const KdNode* top = nullptr;
    if (kWalk == WALK_LANE && ntop > 0) {
        KdNode* staged = reinterpret_cast<KdNode*>((char*)lds + top_lds_offset(B));
        stage_top(m.node, ntop, staged);
        __syncthreads();
        top = staged;
    }
    // with WALK_WAVE every lane of the wavefront takes part in the shared walk
    Nearest nv = nearest_vertex<kWalk>(m, qx, qy, qz, i >= 0 && fin, c.nodes, c.steps, top, ntop);

    // regroup the block's queries by list length (regroup.hpp)
    uint32_t* hist = lds;
    float* col = (float*)(lds + kRegroupBins);  // qx qy qz d2 px py pz, B each
    int32_t* icol = (int32_t*)(col + 7 * B);    // query index, vertex
    const int bin = (i >= 0 && fin) ? regroup_bin(m, nv.vid) : 0;
    if (t < kRegroupBins) hist[t] = 0;
    __syncthreads();
    const uint32_t rank = atomicAdd(&hist[bin], 1u);
    __syncthreads();
    regroup_scan(hist);
    __syncthreads();
    const uint32_t pos = (bin ? hist[bin - 1] : 0u) + rank;
    col[pos] = qx;
    col[B + pos] = qy;
    col[2 * B + pos] = qz;
    col[3 * B + pos] = nv.d2;
    col[4 * B + pos] = nv.px;
    col[5 * B + pos] = nv.py;
    col[6 * B + pos] = nv.pz;
    icol[pos] = (int32_t)i;
    icol[B + pos] = nv.vid;
    __syncthreads();
    i = icol[t];
    qx = col[t];
    qy = col[B + t];
    qz = col[2 * B + t];
    nv.d2 = col[3 * B + t];
    nv.px = col[4 * B + t];
    nv.py = col[5 * B + t];
    nv.pz = col[6 * B + t];
    nv.vid = icol[B + t];
    fin = finite3(qx, qy, qz);
    // the regroup slots are free again: each wavefront's scan rings go there
    __syncthreads();
    WaveScanLds ring;
    ring.k = reinterpret_cast<WaveScanKeys*>(lds + kRegroupBins) + (t >> 6);
    ring.i = reinterpret_cast<WaveScanIds*>((char*)lds + regroup_slot_bytes(B)) + (t >> 6);
    float best;
    int best_kind;
    int32_t best_id;
    wave_scan(m, ring, i >= 0 && fin, qx, qy, qz, nv, best, best_kind, best_id, c);
    if (i < 0) return;
    uint8_t st = fin ? domain_status(m, qx, qy, qz) : (uint8_t)2;
    Answer a = fin ? finish_answer(m, qx, qy, qz, nv, best, best_kind, best_id, c) : nonfinite_answer();
    if (stage && !kWriteExtras) {
        stage[i] = make_float4(__int_as_float(a.prim), a.sx, a.sy, a.sz);
        return;
    }
    if (fin) report_answer(m, qx, qy, qz, a);
    if (stage) {
        if (kWriteExtras) {
            stage[3 * i] = make_float4(__int_as_float(a.prim), a.cx, a.cy, a.cz);
            stage[3 * i + 1] = make_float4(a.dist, __int_as_float((int)st), a.w[0], a.w[1]);
            stage[3 * i + 2] = make_float4(a.w[2], __int_as_float(a.pv[0]), __int_as_float(a.pv[1]),
                                           __int_as_float(a.pv[2]));
        }
        return;
    }
    prim[i] = a.prim;
    closest[3 * i] = a.cx;
    closest[3 * i + 1] = a.cy;
    closest[3 * i + 2] = a.cz;
    dist[i] = a.dist;
    if (status) status[i] = st;
    if (kWriteExtras) {
        for (int k = 0; k < 3; ++k) {
            bary[3 * i + k] = a.w[k];
            pvid[3 * i + k] = a.pv[k];
        }
    }
}

template <bool kExtras>
__global__ __launch_bounds__(256) void k_split(const float4* __restrict__ stage, int64_t n, int32_t* __restrict__ prim,
                                               float* __restrict__ closest, float* __restrict__ dist,
                                               uint8_t* __restrict__ status, float* __restrict__ bary,
                                               int32_t* __restrict__ pvid) {
    constexpr int S = kExtras ? 3 : 2;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 a = stage[S * i], b = stage[S * i + 1];
    prim[i] = __float_as_int(a.x);
    closest[3 * i] = a.y;
    closest[3 * i + 1] = a.z;
    closest[3 * i + 2] = a.w;
    dist[i] = b.x;
    if (status) status[i] = (uint8_t)__float_as_int(b.y);
    if (kExtras) {
        const float4 c = stage[S * i + 2];
        bary[3 * i] = b.z;
        bary[3 * i + 1] = b.w;
        bary[3 * i + 2] = c.x;
        pvid[3 * i] = __float_as_int(c.y);
        pvid[3 * i + 1] = __float_as_int(c.z);
        pvid[3 * i + 2] = __float_as_int(c.w);
    }
}

// Write-out of 16-byte records (prim, staged point) of one mesh's ordered
// query: the closest point and distance (staged_point, as the query kernel
// forms them) and the status (outside the domain box, non-finite) are
// rebuilt from q, read here in input order.
__global__ __launch_bounds__(256) void k_split_compact(const float4* __restrict__ stage, const float* __restrict__ q,
                                                       int64_t n, float lox, float loy, float loz, float hix,
                                                       float hiy, float hiz, int32_t* __restrict__ prim,
                                                       float* __restrict__ closest, float* __restrict__ dist,
                                                       uint8_t* __restrict__ status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 a = stage[i];
    const float qx = q[3 * i], qy = q[3 * i + 1], qz = q[3 * i + 2];
    const int32_t pr = __float_as_int(a.x);
    float cx, cy, cz, d;
    staged_point(pr, a.y, a.z, a.w, qx, qy, qz, cx, cy, cz, d);
    prim[i] = pr;
    closest[3 * i] = cx;
    closest[3 * i + 1] = cy;
    closest[3 * i + 2] = cz;
    dist[i] = d;
    if (status) {
        const bool out = qx < lox || qy < loy || qz < loz || qx > hix || qy > hiy || qz > hiz;
        status[i] = finite3(qx, qy, qz) ? (out ? 1 : 0) : 2;
    }
}

hipError_t launch_split(const float4* stage, int64_t n, int32_t* prim, float* closest, float* dist, uint8_t* status,
                        float* bary, int32_t* pvid, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (bary) k_split<true><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(stage, n, prim, closest, dist, status, bary, pvid);
    else k_split<false><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(stage, n, prim, closest, dist, status, bary, pvid);
    return hipGetLastError();
}

template <int kWalk>
__global__ __launch_bounds__(256) void k_nearest(MeshView m, const float* __restrict__ q, int64_t n,
                                                  int32_t* __restrict__ vid, float* __restrict__ d2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float qx = 0.f, qy = 0.f, qz = 0.f;
    if (i < n) {
        qx = q[3 * i];
        qy = q[3 * i + 1];
        qz = q[3 * i + 2];
    }
    const bool fin = finite3(qx, qy, qz);
    uint64_t visits = 0, steps = 0;
    const Nearest b = nearest_vertex<kWalk>(m, qx, qy, qz, i < n && fin, visits, steps);
    if (i >= n) return;
    vid[i] = fin ? b.vid : -1;
    if (d2) d2[i] = fin ? b.d2 : NAN;
}

// Seed grid of the Voronoi walk: nearest vertex of every cell centre.
__global__ __launch_bounds__(256) void k_seed_grid(MeshView m, float4* __restrict__ seed) {
    const int64_t G = m.grid;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= G * G * G) return;
    const int64_t ix = i % G, iy = (i / G) % G, iz = i / (G * G);
    const float cx = m.glo[0] + ((float)ix + 0.5f) / m.gscale[0];
    const float cy = m.glo[1] + ((float)iy + 0.5f) / m.gscale[1];
    const float cz = m.glo[2] + ((float)iz + 0.5f) / m.gscale[2];
    uint64_t visits = 0;
    const Nearest b = kdt_nearest(m.node, m.nv, cx, cy, cz, visits);
    seed[i] = make_float4(b.px, b.py, b.pz, __int_as_float(b.vid));
}

// Host copy of the seed grid for the host query, same definition as the
// device kernel above.
static void host_seed_grid_one(MeshState& s, int nt, const MeshView& v, std::vector<float>& out);

static void host_seed_grid(MeshState& s, int nt) {
    MeshView v = host_view(s);
    host_seed_grid_one(s, nt, v, s.pk_seed);
    if (v.grid2 > 0) {
        v.grid = v.grid2;
        for (int k = 0; k < 3; ++k) {
            v.glo[k] = v.glo2[k];
            v.gscale[k] = v.gscale2[k];
        }
        host_seed_grid_one(s, nt, v, s.pk_seed2);
    }
}

static void host_seed_grid_one(MeshState& s, int nt, const MeshView& v, std::vector<float>& out) {
    (void)s;
    const int64_t G = v.grid, cells = G * G * G;
    out.assign((size_t)(4 * cells), 0.f);
    std::atomic<int64_t> cursor{0};
    auto work = [&]() {
        for (;;) {
            const int64_t b = cursor.fetch_add(4096);
            if (b >= cells) break;
            for (int64_t i = b; i < std::min(cells, b + 4096); ++i) {
                const int64_t ix = i % G, iy = (i / G) % G, iz = i / (G * G);
                const float cx = v.glo[0] + ((float)ix + 0.5f) / v.gscale[0];
                const float cy = v.glo[1] + ((float)iy + 0.5f) / v.gscale[1];
                const float cz = v.glo[2] + ((float)iz + 0.5f) / v.gscale[2];
                uint64_t visits = 0;
                const Nearest b = kdt_nearest(v.node, v.nv, cx, cy, cz, visits);
                float* d = &out[(size_t)(4 * i)];
                d[0] = b.px;
                d[1] = b.py;
                d[2] = b.pz;
                d[3] = bits_as_float(b.vid);
            }
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(work);
    work();
    for (auto& x : th) x.join();
}

hipError_t launch_seed_grid(const MeshView& m, float4* seed, hipStream_t st) {
    const int64_t cells = (int64_t)m.grid * m.grid * m.grid;
    k_seed_grid<<<(unsigned)((cells + 255) / 256), 256, 0, st>>>(m, seed);
    return hipGetLastError();
}

// Bucketed reduction of the vertex gradient for large meshes: every valid
// (query, corner) contribution goes, as a 16-byte record (its three
// components and the vertex), into the run of its bucket of 2^kBucketShift
// consecutive vertices; each bucket is then summed in LDS by one workgroup
// (several, merged with float atomics, when there are too few buckets to
// fill the chip) and added to grad_V -- no scattered global atomics and no
// sort.
constexpr int kBucketShift = 10;
constexpr int kMaxBuckets = 4096;                // per-block LDS counters; beyond, direct atomics
constexpr int64_t kAtomicMaxVertices = 65536;    // below this the direct atomics stay in L2
constexpr int kBwdQueriesPerThread = 4;

// Unit direction (q - c) / d of query i, zero when d is 0 or not finite.
__device__ __forceinline__ void bwd_dir(const float* __restrict__ q, const float* __restrict__ closest, float d,
                                        int64_t i, float& ux, float& uy, float& uz) {
    ux = uy = uz = 0.f;
    if (d > 0.f && isfinite(d)) {
        const float inv = 1.f / d;
        ux = (q[3 * i] - closest[3 * i]) * inv;
        uy = (q[3 * i + 1] - closest[3 * i + 1]) * inv;
        uz = (q[3 * i + 2] - closest[3 * i + 2]) * inv;
    }
}

// Counts of each block's contributions per bucket (in LDS), written to a
// bucket-major matrix mat[b * blocks + block] whose exclusive scan gives
// every (bucket, block) its first place; and grad_q.
__global__ __launch_bounds__(256) void k_bwd_count(const float* __restrict__ q, int64_t n,
                                                   const float* __restrict__ closest, const float* __restrict__ dist,
                                                   const float* __restrict__ bary, const int32_t* __restrict__ pvid,
                                                   const float* __restrict__ gd, float* __restrict__ gq, int32_t nv,
                                                   int nbk, uint32_t* __restrict__ mat) {
    __shared__ uint32_t h[kMaxBuckets];
    for (int b = threadIdx.x; b < nbk; b += blockDim.x) h[b] = 0u;
    __syncthreads();
    // a block takes kBwdQueriesPerThread * 256 consecutive queries, lanes
    // adjacent in each round (coalesced)
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x * kBwdQueriesPerThread + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kBwdQueriesPerThread; ++u) {
        const int64_t i = i0 + (int64_t)u * blockDim.x;
        float ux = 0.f, uy = 0.f, uz = 0.f, g = 0.f;
        if (i < n) {
            g = gd[i];
            bwd_dir(q, closest, dist[i], i, ux, uy, uz);
            if (gq) {
                gq[3 * i] = g * ux;
                gq[3 * i + 1] = g * uy;
                gq[3 * i + 2] = g * uz;
            }
        }
        const bool any = i < n && (ux != 0.f || uy != 0.f || uz != 0.f) && g != 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int32_t v = any ? pvid[3 * i + k] : -1;
            const float w = any ? bary[3 * i + k] : 0.f;
            if (v >= 0 && v < nv && w != 0.f) atomicAdd(&h[(uint32_t)v >> kBucketShift], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbk; b += blockDim.x) mat[(int64_t)b * gridDim.x + blockIdx.x] = h[b];
    if (blockIdx.x == 0 && threadIdx.x == 0) mat[(int64_t)nbk * gridDim.x] = 0u;  // becomes the total
}

// Writes every valid contribution as (x, y, z, vertex) into its bucket's
// run: a block ranks its contributions per bucket in LDS and places them
// after the scanned offset of (bucket, block).
__global__ __launch_bounds__(256) void k_bwd_scatter(const float* __restrict__ q, int64_t n,
                                                     const float* __restrict__ closest, const float* __restrict__ dist,
                                                     const float* __restrict__ bary, const int32_t* __restrict__ pvid,
                                                     const float* __restrict__ gd, int32_t nv, int nbk,
                                                     const uint32_t* __restrict__ mat, float4* __restrict__ recs) {
    __shared__ uint32_t h[kMaxBuckets];
    for (int b = threadIdx.x; b < nbk; b += blockDim.x) h[b] = 0u;
    __syncthreads();
    constexpr int kC = 3 * kBwdQueriesPerThread;
    uint32_t vb[kC], rank[kC];
    float cx[kC], cy[kC], cz[kC];
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x * kBwdQueriesPerThread + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kBwdQueriesPerThread; ++u) {
        const int64_t i = i0 + (int64_t)u * blockDim.x;
        float ux = 0.f, uy = 0.f, uz = 0.f, g = 0.f;
        if (i < n) {
            g = gd[i];
            bwd_dir(q, closest, dist[i], i, ux, uy, uz);
        }
        const bool any = i < n && (ux != 0.f || uy != 0.f || uz != 0.f) && g != 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int c = 3 * u + k;
            const int32_t v = any ? pvid[3 * i + k] : -1;
            const float w = any ? bary[3 * i + k] : 0.f;
            const bool ok = v >= 0 && v < nv && w != 0.f;
            const float s = -g * w;
            vb[c] = ok ? (uint32_t)v : 0xffffffffu;
            cx[c] = s * ux;
            cy[c] = s * uy;
            cz[c] = s * uz;
            rank[c] = ok ? atomicAdd(&h[(uint32_t)v >> kBucketShift], 1u) : 0u;
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbk; b += blockDim.x)
        if (h[b]) h[b] = mat[(int64_t)b * gridDim.x + blockIdx.x];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kC; ++c)
        if (vb[c] != 0xffffffffu)
            recs[h[vb[c] >> kBucketShift] + rank[c]] = make_float4(cx[c], cy[c], cz[c], __uint_as_float(vb[c]));
}

// Sum of one slice of a bucket's run in LDS, added to grad_V (with float
// atomics when the bucket's run is split over several blocks).
__global__ __launch_bounds__(512) void k_bwd_accum(const float4* __restrict__ recs,
                                                   const uint32_t* __restrict__ mat, int64_t stride,
                                                   float* __restrict__ gV, int32_t nv, int splits) {
    __shared__ __align__(16) float acc[3 << kBucketShift];
    const uint32_t b = blockIdx.x / (uint32_t)splits;
    const uint32_t part = blockIdx.x % (uint32_t)splits;
    // bucket b's run: from its first block's offset to the next bucket's
    const uint32_t s0 = mat[(int64_t)b * stride], s1 = mat[(int64_t)(b + 1) * stride];
    if (s1 <= s0) return;  // uniform: empty bucket
    const uint64_t len = s1 - s0;
    const uint32_t a0 = s0 + (uint32_t)(len * part / (uint32_t)splits);
    const uint32_t a1 = s0 + (uint32_t)(len * (part + 1) / (uint32_t)splits);
    if (a1 <= a0) return;  // uniform
    for (int t = threadIdx.x; t < (3 << kBucketShift) / 4; t += blockDim.x)
        reinterpret_cast<float4*>(acc)[t] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    const int64_t v0 = (int64_t)b << kBucketShift;
    const uint32_t bs = blockDim.x;
    for (uint32_t j = a0 + threadIdx.x; j < a1; j += 4 * bs) {
        float4 r[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t jj = j + (uint32_t)u * bs;
            r[u] = jj < a1 ? recs[jj] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (j + (uint32_t)u * bs >= a1) break;
            const int l = (int)(__float_as_uint(r[u].w) - (uint32_t)v0);
            atomicAdd(&acc[3 * l], r[u].x);
            atomicAdd(&acc[3 * l + 1], r[u].y);
            atomicAdd(&acc[3 * l + 2], r[u].z);
        }
    }
    __syncthreads();
    const int64_t lim = std::min<int64_t>((int64_t)3 << kBucketShift, 3 * ((int64_t)nv - v0));
    if (splits == 1) {  // the block alone holds these vertices: float4 read-modify-write
        float4* g4 = reinterpret_cast<float4*>(gV + 3 * v0);  // 3 * v0 floats: a multiple of 4
        const float4* a4 = reinterpret_cast<const float4*>(acc);
        for (int t = threadIdx.x; t < lim / 4; t += blockDim.x) {
            float4 x = g4[t];
            const float4 y = a4[t];
            x.x += y.x;
            x.y += y.y;
            x.z += y.z;
            x.w += y.w;
            g4[t] = x;
        }
        for (int64_t t = (lim / 4) * 4 + threadIdx.x; t < lim; t += blockDim.x) gV[3 * v0 + t] += acc[t];
    } else {
        for (int t = threadIdx.x; t < lim; t += blockDim.x)
            if (acc[t] != 0.f) unsafeAtomicAdd(&gV[3 * v0 + t], acc[t]);
    }
}

__global__ __launch_bounds__(256) void k_backward(const float* __restrict__ q, int64_t n,
                                                   const float* __restrict__ closest, const float* __restrict__ dist,
                                                   const float* __restrict__ bary, const int32_t* __restrict__ pvid,
                                                   const float* __restrict__ gd, float* __restrict__ gq,
                                                   float* __restrict__ gV, int32_t nv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float d = dist[i];
    const float g = gd[i];
    float ux = 0.f, uy = 0.f, uz = 0.f;
    if (d > 0.f && isfinite(d)) {
        const float inv = 1.f / d;
        ux = (q[3 * i] - closest[3 * i]) * inv;
        uy = (q[3 * i + 1] - closest[3 * i + 1]) * inv;
        uz = (q[3 * i + 2] - closest[3 * i + 2]) * inv;
    }
    if (gq) {
        gq[3 * i] = g * ux;
        gq[3 * i + 1] = g * uy;
        gq[3 * i + 2] = g * uz;
    }
    if (gV && (ux != 0.f || uy != 0.f || uz != 0.f) && g != 0.f) {
        for (int k = 0; k < 3; ++k) {
            const int32_t v = pvid[3 * i + k];
            const float w = bary[3 * i + k];
            if (v < 0 || v >= nv || w == 0.f) continue;
            const float s = -g * w;
            unsafeAtomicAdd(&gV[3 * (int64_t)v], s * ux);
            unsafeAtomicAdd(&gV[3 * (int64_t)v + 1], s * uy);
            unsafeAtomicAdd(&gV[3 * (int64_t)v + 2], s * uz);
        }
    }
}

// ------------------------------------------------------------ launches

// The query orders its batch by the top 24 bits of the Morton key (a 256^3
// grid over D): three sort passes instead of four; within a grid cell the
// input order is kept.
constexpr int kQuerySortLoBit = 6;
// The default orders a batch of at least this many queries.  Smaller
// batches put too few queries in each Voronoi cell for the ordering to make
// neighbouring lanes share cells and lists, and its launches cost more than
// the coherence saves (on the sphere, heightfield and near-surface
// workloads the unordered query is faster up to 2^18 queries and slower
// from 2^19).
constexpr int64_t kOrderMinQueries = int64_t(1) << 19;
// Tree levels the per-lane search may read from LDS (511 nodes, 32 KB).
constexpr int kMaxLdsLevels = 9;

// traversal option (0 default, 1 per-lane tree, 2 wavefront tree, 3 Voronoi
// walk) -> Walk.  The Voronoi walk reads a few dozen vertices per query
// where the tree searches read hundreds of nodes, on ordered and unordered
// batches alike, so it is the default.
static int pick_walk(int traversal) {
    switch (traversal) {
        case 1: return WALK_LANE;
        case 2: return WALK_WAVE;
        default: return WALK_VORONOI;
    }
}

struct DeviceGuard {
    int old = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&old) != hipSuccess) old = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (old >= 0) (void)hipSetDevice(old);
    }
};

static p2m_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(P2M_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return P2M_OK;
}

static p2m_status ensure_scratch(MeshState& s, int64_t bytes) {
    if (s.dev.scratch_bytes >= bytes) return P2M_OK;
    if (s.dev.scratch) {
        (void)hipFree(s.dev.scratch);
        s.dev.scratch = nullptr;
        s.dev.scratch_bytes = 0;
    }
    hipError_t e = hipMalloc(&s.dev.scratch, (size_t)bytes);
    if (e != hipSuccess) {
        s.dev.scratch = nullptr;
        return fail(e == hipErrorOutOfMemory ? P2M_ERR_OOM : P2M_ERR_HIP,
                    std::string("scratch allocation: ") + hipGetErrorString(e));
    }
    s.dev.scratch_bytes = bytes;
    return P2M_OK;
}

// Morton keys + stable sort by key bits [lo_bit, 30) into scratch; returns
// the permutation pointer, and the sorted keys when keys_out is not NULL.  `extra` bytes of scratch after the sort's own
// (256-byte aligned) are returned in *extra_out (order_into_scratch below).
static int64_t order_scratch_bytes(int64_t n) { return (radix_plan(n).bytes + 255) / 256 * 256; }

// The same into a given device buffer of at least order_scratch_bytes(n) +
// extra bytes (256-byte aligned).
static p2m_status order_into(MeshState& s, void* base, const float* q, int64_t n, int lo_bit, hipStream_t st,
                             uint32_t** keys_out, int32_t** perm_out, void** extra_out) {
    RadixPlan plan = radix_plan(n);
    const int64_t sort_bytes = order_scratch_bytes(n);
    RadixBuffers b = radix_buffers(plan, base);
    float lo[3], sc[3];
    morton_params(s.dlo, s.dhi, lo, sc);
    // with a sort to run, the key kernel also counts the first pass's digits
    const bool passes = n > 1 && lo_bit < 30;
    if (passes) {
        // the keys start the 256-byte aligned scratch, so a uint4 of keys is aligned
        if (((uintptr_t)q & 15u) == 0u)
            k_morton_hist<true><<<(unsigned)plan.tiles, kRadixHistThreads, 0, st>>>(
                q, n, lo[0], lo[1], lo[2], sc[0], sc[1], sc[2], lo_bit, b.keys[0], b.counts, plan.tiles);
        else
            k_morton_hist<false><<<(unsigned)plan.tiles, kRadixHistThreads, 0, st>>>(
                q, n, lo[0], lo[1], lo[2], sc[0], sc[1], sc[2], lo_bit, b.keys[0], b.counts, plan.tiles);
    } else {
        const int64_t blocks = (n + 255) / 256;
        k_morton<<<(unsigned)blocks, 256, 0, st>>>(q, n, lo[0], lo[1], lo[2], sc[0], sc[1], sc[2], b.keys[0]);
    }
    p2m_status r = check_launch("morton keys");
    if (r != P2M_OK) return r;
    int cur = radix_sort_pairs(plan, b, lo_bit, 30, keys_out != nullptr, st, nullptr, passes);
    r = check_launch("radix sort");
    if (r != P2M_OK) return r;
    if (keys_out) *keys_out = b.keys[cur];
    *perm_out = b.vals[cur];
    if (extra_out) *extra_out = (char*)base + sort_bytes;
    return P2M_OK;
}

static p2m_status order_into_scratch(MeshState& s, const float* q, int64_t n, int lo_bit, hipStream_t st,
                                     uint32_t** keys_out, int32_t** perm_out, int64_t extra = 0,
                                     void** extra_out = nullptr) {
    p2m_status r = ensure_scratch(s, order_scratch_bytes(n) + extra);
    if (r != P2M_OK) return r;
    return order_into(s, s.dev.scratch, q, n, lo_bit, st, keys_out, perm_out, extra_out);
}

}  // namespace p2m

using namespace p2m;

extern "C" {

p2m_status p2m_upload(p2m_mesh* mh, int device, void* stream, int64_t* bytes) {
    if (!mh) return fail(P2M_ERR_ARG, "mesh is NULL");
    MeshState& s = mh->s;
    if (!s.precomputed) return fail(P2M_ERR_STATE, "p2m_upload before p2m_precompute");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(P2M_ERR_HIP, "no HIP device");
    if (device < 0 || device >= ndev) return fail(P2M_ERR_ARG, "device index out of range");
    DeviceGuard g(device);
    if (!g.ok) return fail(P2M_ERR_HIP, "hipSetDevice failed");
    device_release(s);
    pack_mesh(s);
    const size_t a = 256;
    auto up = [&](size_t x) { return (x + a - 1) / a * a; };
    const size_t b_node = sizeof(float) * s.pk_node.size();
    const size_t b_off = sizeof(uint32_t) * s.pk_vhead.size();
    const size_t b_ent = sizeof(uint32_t) * std::max<size_t>(4, s.pk_lent.size());
    const size_t b_seg = sizeof(float) * s.pk_seg.size();
    const size_t b_tri = sizeof(float) * s.pk_tri.size();
    const size_t b_fe = sizeof(int32_t) * s.pk_fedge.size();
    // Voronoi walk: vertex positions, neighbour CSR (32-bit offsets), seed grid
    if (s.t.nb.size() >= (size_t)UINT32_MAX || s.t.nb_off.size() != (size_t)s.m.nv + 1)
        return fail(P2M_ERR_INTERNAL, "Voronoi neighbour graph missing or too large");
    const int32_t G = walk_grid_side(s.m.nv);
    const size_t b_nboff = sizeof(uint32_t) * s.pk_nboff.size();
    const size_t b_nb = sizeof(float) * std::max<size_t>(4, s.pk_nbrec.size());
    const size_t b_seed = sizeof(float4) * (size_t)G * (size_t)G * (size_t)G;
    const MeshView hv = host_view(s);
    const size_t b_seed2 = sizeof(float4) * (size_t)hv.grid2 * (size_t)hv.grid2 * (size_t)hv.grid2;
    const size_t b_frec = sizeof(float) * s.pk_frec.size();
    const size_t b_erec = sizeof(float) * std::max<size_t>(1, s.pk_erec.size());
    const size_t total = up(b_node) + up(b_off) + up(b_ent) + up(b_seg) + up(b_tri) + up(b_fe) + up(b_nboff) +
                         up(b_nb) + up(b_seed) + up(b_seed2) + up(b_frec) + up(b_erec);
    void* base = nullptr;
    hipError_t e = hipMalloc(&base, total);
    if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? P2M_ERR_OOM : P2M_ERR_HIP, "device arena allocation");
    s.dev.device = device;
    s.dev.base = base;
    s.dev.bytes = (int64_t)total;
    char* p = (char*)base;
    s.dev.node = p;
    p += up(b_node);
    s.dev.vhead = p;
    p += up(b_off);
    s.dev.lent = p;
    p += up(b_ent);
    s.dev.seg = p;
    p += up(b_seg);
    s.dev.tri = p;
    p += up(b_tri);
    s.dev.fedge = p;
    p += up(b_fe);
    s.dev.nboff = p;
    p += up(b_nboff);
    s.dev.nbrec = p;
    p += up(b_nb);
    s.dev.seed = p;
    p += up(b_seed);
    s.dev.seed2 = b_seed2 ? p : nullptr;
    p += up(b_seed2);
    s.dev.frec = p;
    p += up(b_frec);
    s.dev.erec = p;
    hipStream_t st = (hipStream_t)stream;
    struct Cp {
        void* dst;
        const void* src;
        size_t n;
    } cps[] = {{s.dev.node, s.pk_node.data(), b_node}, {s.dev.vhead, s.pk_vhead.data(), b_off},
               {s.dev.lent, s.pk_lent.data(), s.pk_lent.size() * sizeof(uint32_t)}, {s.dev.seg, s.pk_seg.data(), b_seg},
               {s.dev.tri, s.pk_tri.data(), b_tri}, {s.dev.fedge, s.pk_fedge.data(), b_fe},
               {s.dev.nboff, s.pk_nboff.data(), b_nboff},
               {s.dev.nbrec, s.pk_nbrec.data(), s.pk_nbrec.size() * sizeof(float)},
               {s.dev.frec, s.pk_frec.data(), b_frec},
               {s.dev.erec, s.pk_erec.data(), s.pk_erec.size() * sizeof(float)}};
    for (const Cp& c : cps) {
        if (c.n == 0) continue;
        e = hipMemcpyAsync(c.dst, c.src, c.n, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            device_release(s);
            return fail(P2M_ERR_HIP, std::string("upload copy: ") + hipGetErrorString(e));
        }
    }
    e = launch_seed_grid(device_view(s), (float4*)s.dev.seed, st);
    if (e == hipSuccess && hv.grid2 > 0) {
        // the finer grid: the same kernel on a view with that grid's frame
        MeshView fv = device_view(s);
        fv.grid = fv.grid2;
        for (int k = 0; k < 3; ++k) {
            fv.glo[k] = fv.glo2[k];
            fv.gscale[k] = fv.gscale2[k];
        }
        e = launch_seed_grid(fv, (float4*)s.dev.seed2, st);
    }
    if (e != hipSuccess) {
        device_release(s);
        return fail(P2M_ERR_HIP, std::string("seed grid kernel: ") + hipGetErrorString(e));
    }
    if (bytes) *bytes = (int64_t)total;
    return P2M_OK;
}

}  // extern "C"

namespace p2m {

// The query of p2m_query.  fixed != nullptr: the ordering and the staged
// answers go to that device buffer (p2m_query_noalloc) instead of the
// mesh's scratch, which may be grown; nothing is allocated then.
static p2m_status run_query(p2m_mesh* mh, const float* q, int64_t n, int32_t* prim, float* closest, float* dist,
                            uint8_t* status, float* bary, int32_t* pvid, const p2m_query_opts* opts, void* stream,
                            void* (*fixed)(int device)) {
    if (!mh) return fail(P2M_ERR_ARG, "mesh is NULL");
    MeshState& s = mh->s;
    if (n < 0) return fail(P2M_ERR_ARG, "negative query count");
    if (s.dev.device < 0) return fail(P2M_ERR_STATE, "p2m_query before p2m_upload");
    if (n == 0) return P2M_OK;
    if (!q || !prim || !closest || !dist) return fail(P2M_ERR_ARG, "NULL query or output pointer");
    if ((bary == nullptr) != (pvid == nullptr)) return fail(P2M_ERR_ARG, "bary and pvid must both be set or both NULL");
    if (n > (int64_t)INT32_MAX) return fail(P2M_ERR_ARG, "more than 2^31-1 queries in one call");
    int sort = n >= kOrderMinQueries ? 1 : 0, block = 256, profile = 0, traversal = 0, lds_levels = 0;
    if (opts) {
        profile = opts->profile;
        traversal = opts->traversal;
        lds_levels = opts->lds_levels;
        if (traversal < 0 || traversal > 3) return fail(P2M_ERR_ARG, "traversal must be 0, 1, 2 or 3");
        if (lds_levels < 0 || lds_levels > kMaxLdsLevels) return fail(P2M_ERR_ARG, "lds_levels must be in [0, 9]");
        if (opts->sort_queries >= 0) sort = opts->sort_queries ? 1 : 0;
        if (opts->block_size != 0) {
            if (opts->block_size < 64 || opts->block_size > kQueryMaxBlock || opts->block_size % 64)
                return fail(P2M_ERR_ARG, "block_size must be a multiple of 64 in [64, 256]");
            block = opts->block_size;
        }
    }
    if (fixed && profile) return fail(P2M_ERR_ARG, "profile is not available without allocation (p2m_query_noalloc)");
    DeviceGuard g(s.dev.device);
    if (!g.ok) return fail(P2M_ERR_HIP, "hipSetDevice failed");
    hipStream_t st = (hipStream_t)stream;
    void* fixed_buf = nullptr;
    if (fixed && sort) {
        fixed_buf = fixed(s.dev.device);
        if (!fixed_buf) return P2M_ERR_HIP;  // message set by the provider
    }
    if (profile) {
        for (void*& e : s.dev.ev)
            if (!e && hipEventCreate((hipEvent_t*)&e) != hipSuccess) return fail(P2M_ERR_HIP, "hipEventCreate");
        (void)hipEventRecord((hipEvent_t)s.dev.ev[0], st);
    }
    int32_t* perm = nullptr;
    float4* stage = nullptr;
    if (sort) {
        void* x = nullptr;
        p2m_status r = fixed_buf ? order_into(s, fixed_buf, q, n, kQuerySortLoBit, st, nullptr, &perm, &x)
                                 : order_into_scratch(s, q, n, kQuerySortLoBit, st, nullptr, &perm,
                                                      (bary ? 48 : 16) * n, &x);
        if (r != P2M_OK) return r;
        stage = (float4*)x;
    }
    if (profile) (void)hipEventRecord((hipEvent_t)s.dev.ev[1], st);
    const MeshView v = device_view(s);
    const int64_t tiles = (n + block - 1) / block;
    const int64_t run = std::min<int64_t>(kXcdRun, (tiles + kXcds - 1) / kXcds);
    const unsigned grid = (unsigned)((tiles + kXcds * run - 1) / (kXcds * run) * (kXcds * run));
    const int walk = pick_walk(traversal);
    // the top levels of the tree in LDS: the per-lane tree search only
    const int32_t ntop = walk == WALK_LANE ? top_nodes(lds_levels, v.nv) : 0;
    const size_t lds_bytes = top_lds_offset(block) + sizeof(KdNode) * (size_t)ntop;
#define P2M_LAUNCH_QUERY(X, W) \
    k_query<X, W><<<grid, block, lds_bytes, st>>>(v, q, perm, n, run, prim, closest, dist, status, bary, pvid, stage, ntop)
    if (bary) {
        if (walk == WALK_WAVE) P2M_LAUNCH_QUERY(true, WALK_WAVE);
        else if (walk == WALK_VORONOI) P2M_LAUNCH_QUERY(true, WALK_VORONOI);
        else P2M_LAUNCH_QUERY(true, WALK_LANE);
    } else {
        if (walk == WALK_WAVE) P2M_LAUNCH_QUERY(false, WALK_WAVE);
        else if (walk == WALK_VORONOI) P2M_LAUNCH_QUERY(false, WALK_VORONOI);
        else P2M_LAUNCH_QUERY(false, WALK_LANE);
    }
#undef P2M_LAUNCH_QUERY
    p2m_status r = check_launch("query kernel");
    if (profile) (void)hipEventRecord((hipEvent_t)s.dev.ev[2], st);
    if (r == P2M_OK && stage) {
        hipError_t e = hipSuccess;
        if (bary) {
            e = launch_split(stage, n, prim, closest, dist, status, bary, pvid, st);
        } else {
            k_split_compact<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(stage, q, n, v.dlo[0], v.dlo[1], v.dlo[2],
                                                                          v.dhi[0], v.dhi[1], v.dhi[2], prim, closest,
                                                                          dist, status);
            e = hipGetLastError();
        }
        if (e != hipSuccess) r = fail(P2M_ERR_HIP, std::string("answer write-out: ") + hipGetErrorString(e));
    }
    if (r == P2M_OK && profile) {
        (void)hipEventRecord((hipEvent_t)s.dev.ev[3], st);
        s.dev.ev_recorded = true;
        s.dev.ev_sorted = sort != 0;
    }
    return r;
}

// ------------------------------------------------ allocation-free query

// Fixed device scratch of p2m_query_noalloc: the ordering buffers and the
// staged answers (48 bytes per query with bary/pvid) of at most
// kNoAllocMaxQueries queries.  Each device the library runs on holds its
// own copy until the process ends.
constexpr int64_t kNoAllocMaxQueries = int64_t(1) << 20;
constexpr int64_t noalloc_up256(int64_t x) { return (x + 255) / 256 * 256; }
constexpr int64_t noalloc_sort_bytes(int64_t n) {
    // radix_plan(n).bytes rounded up: keys and values, double-buffered; the
    // count matrix (256 per tile of kRadixTile keys); the digit totals or
    // scan sums
    return noalloc_up256(4 * noalloc_up256(4 * n) + noalloc_up256(4 * 256 * ((n + kRadixTile - 1) / kRadixTile)) +
                         noalloc_up256(4 * std::max<int64_t>(256, (256 * ((n + kRadixTile - 1) / kRadixTile) +
                                                                   kRadixTile - 1) / kRadixTile)));
}
constexpr int64_t kNoAllocScratchBytes = noalloc_sort_bytes(kNoAllocMaxQueries) + 48 * kNoAllocMaxQueries;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// Device address of `scratch` on each device, looked up once per device
// (with that device current) on its first p2m_query_noalloc call; host code
// uses only these addresses, never the symbol itself.
constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_noalloc_mu;
static void* g_noalloc_ptr[kNoAllocMaxDevices] = {};

static void* noalloc_scratch(int device) {
    if (device < 0 || device >= kNoAllocMaxDevices) {
        fail(P2M_ERR_HIP, "device index beyond the allocation-free scratch table");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            fail(P2M_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return nullptr;
        }
        g_noalloc_ptr[device] = ptr;
    }
    return g_noalloc_ptr[device];
}

}  // namespace p2m

extern "C" {

p2m_status p2m_query(p2m_mesh* mh, const float* q, int64_t n, int32_t* prim, float* closest, float* dist,
                     uint8_t* status, float* bary, int32_t* pvid, const p2m_query_opts* opts, void* stream) {
    return run_query(mh, q, n, prim, closest, dist, status, bary, pvid, opts, stream, nullptr);
}

p2m_status p2m_query_noalloc(p2m_mesh* mh, const float* q, int64_t n, int32_t* prim, float* closest, float* dist,
                             uint8_t* status, float* bary, int32_t* pvid, const p2m_query_opts* opts, void* stream) {
    if (n > kNoAllocMaxQueries)
        return fail(P2M_ERR_ARG, "p2m_query_noalloc: more than " + std::to_string(kNoAllocMaxQueries) +
                                     " queries (the fixed scratch's limit)");
    if (n > 0 && order_scratch_bytes(n) + 48 * n > kNoAllocScratchBytes)
        return fail(P2M_ERR_INTERNAL, "p2m_query_noalloc: fixed scratch smaller than the ordering needs");
    return run_query(mh, q, n, prim, closest, dist, status, bary, pvid, opts, stream, noalloc_scratch);
}

p2m_status p2m_query_profile(p2m_mesh* mh, float* order_ms, float* query_ms, float* finish_ms) {
    if (!mh) return fail(P2M_ERR_ARG, "mesh is NULL");
    MeshState& s = mh->s;
    if (!s.dev.ev_recorded) return fail(P2M_ERR_STATE, "no profiled p2m_query on this mesh");
    DeviceGuard g(s.dev.device);
    float a = 0.f, b = 0.f, c = 0.f;
    hipError_t e = hipEventSynchronize((hipEvent_t)s.dev.ev[3]);
    if (e == hipSuccess) e = hipEventElapsedTime(&a, (hipEvent_t)s.dev.ev[0], (hipEvent_t)s.dev.ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&b, (hipEvent_t)s.dev.ev[1], (hipEvent_t)s.dev.ev[2]);
    if (e == hipSuccess) e = hipEventElapsedTime(&c, (hipEvent_t)s.dev.ev[2], (hipEvent_t)s.dev.ev[3]);
    if (e != hipSuccess) return fail(P2M_ERR_HIP, std::string("profile events: ") + hipGetErrorString(e));
    if (order_ms) *order_ms = s.dev.ev_sorted ? a : 0.f;
    if (query_ms) *query_ms = b;
    if (finish_ms) *finish_ms = s.dev.ev_sorted ? c : 0.f;
    return P2M_OK;
}

p2m_status p2m_nearest_vertex(p2m_mesh* mh, const float* q, int64_t n, int32_t* vid, float* d2, int traversal,
                              void* stream) {
    if (!mh) return fail(P2M_ERR_ARG, "mesh is NULL");
    MeshState& s = mh->s;
    if (n < 0) return fail(P2M_ERR_ARG, "negative query count");
    if (s.dev.device < 0) return fail(P2M_ERR_STATE, "p2m_nearest_vertex before p2m_upload");
    if (n == 0) return P2M_OK;
    if (!q || !vid) return fail(P2M_ERR_ARG, "NULL pointer");
    if (traversal < 0 || traversal > 3) return fail(P2M_ERR_ARG, "traversal must be 0, 1, 2 or 3");
    DeviceGuard g(s.dev.device);
    const MeshView v = device_view(s);
    const unsigned grid = (unsigned)((n + 255) / 256);
    const int walk = pick_walk(traversal);
    hipStream_t st = (hipStream_t)stream;
    if (walk == WALK_WAVE) k_nearest<WALK_WAVE><<<grid, 256, 0, st>>>(v, q, n, vid, d2);
    else if (walk == WALK_VORONOI) k_nearest<WALK_VORONOI><<<grid, 256, 0, st>>>(v, q, n, vid, d2);
    else k_nearest<WALK_LANE><<<grid, 256, 0, st>>>(v, q, n, vid, d2);
    return check_launch("nearest-vertex kernel");
}

p2m_status p2m_order_queries(p2m_mesh* mh, const float* q, int64_t n, uint32_t* keys_out, int32_t* perm_out,
                             void* stream) {
    if (!mh) return fail(P2M_ERR_ARG, "mesh is NULL");
    MeshState& s = mh->s;
    if (n < 0) return fail(P2M_ERR_ARG, "negative query count");
    if (s.dev.device < 0) return fail(P2M_ERR_STATE, "p2m_order_queries before p2m_upload");
    if (n == 0) return P2M_OK;
    if (!q || !keys_out || !perm_out) return fail(P2M_ERR_ARG, "NULL pointer");
    if (n > (int64_t)INT32_MAX) return fail(P2M_ERR_ARG, "more than 2^31-1 queries in one call");
    DeviceGuard g(s.dev.device);
    hipStream_t st = (hipStream_t)stream;
    uint32_t* keys = nullptr;
    int32_t* perm = nullptr;
    p2m_status r = order_into_scratch(s, q, n, 0, st, &keys, &perm);
    if (r != P2M_OK) return r;
    hipError_t e = hipMemcpyAsync(keys_out, keys, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(perm_out, perm, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return fail(P2M_ERR_HIP, std::string("order copy: ") + hipGetErrorString(e));
    return P2M_OK;
}

p2m_status p2m_query_backward(p2m_mesh* mh, const float* q, int64_t n, const float* closest, const float* dist,
                              const float* bary, const int32_t* pvid, const float* gd, float* gq, float* gV,
                              void* stream) {
    if (!mh) return fail(P2M_ERR_ARG, "mesh is NULL");
    MeshState& s = mh->s;
    if (n < 0) return fail(P2M_ERR_ARG, "negative query count");
    if (s.dev.device < 0) return fail(P2M_ERR_STATE, "p2m_query_backward before p2m_upload");
    if (n == 0) return P2M_OK;
    if (!q || !closest || !dist || !gd) return fail(P2M_ERR_ARG, "NULL pointer");
    if (gV && (!bary || !pvid)) return fail(P2M_ERR_ARG, "grad_V needs bary and pvid from the forward");
    if (gV && ((uintptr_t)gV & 15u)) return fail(P2M_ERR_ARG, "grad_V must be 16-byte aligned");
    DeviceGuard g(s.dev.device);
    hipStream_t st = (hipStream_t)stream;
    const int64_t nv = s.m.nv;
    if (!gV || nv <= kAtomicMaxVertices || ((nv - 1) >> kBucketShift) + 1 > kMaxBuckets ||
        3 * n > (int64_t)INT32_MAX) {
        k_backward<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(q, n, closest, dist, bary, pvid, gd, gq, gV,
                                                                (int32_t)nv);
        return check_launch("backward kernel");
    }
    // bucketed reduction: per-block counts per bucket, their scan, the
    // records, the sums
    const int nbk = (int)((nv - 1) >> kBucketShift) + 1;
    const int64_t m = 3 * n;
    const int64_t threads = (n + kBwdQueriesPerThread - 1) / kBwdQueriesPerThread;
    const int64_t blocks = (threads + 255) / 256;
    const int64_t cells = (int64_t)nbk * blocks + 1;
    const int64_t b_mat = (4 * cells + 255) / 256 * 256;
    const int64_t b_sums = (4 * scan_sums_size(cells) + 255) / 256 * 256;
    p2m_status r = ensure_scratch(s, b_mat + b_sums + 16 * m);
    if (r != P2M_OK) return r;
    uint32_t* mat = (uint32_t*)s.dev.scratch;
    uint32_t* sums = (uint32_t*)((char*)s.dev.scratch + b_mat);
    float4* recs = (float4*)((char*)s.dev.scratch + b_mat + b_sums);
    k_bwd_count<<<(unsigned)blocks, 256, 0, st>>>(q, n, closest, dist, bary, pvid, gd, gq, (int32_t)nv, nbk, mat);
    scan_exclusive_u32(mat, cells, sums, st);
    k_bwd_scatter<<<(unsigned)blocks, 256, 0, st>>>(q, n, closest, dist, bary, pvid, gd, (int32_t)nv, nbk, mat, recs);
    // each bucket split over enough blocks to give the chip about 4 per CU
    const int splits = (4 * 256 + nbk - 1) / nbk;
    k_bwd_accum<<<(unsigned)(nbk * splits), 512, 0, st>>>(recs, mat, blocks, gV, (int32_t)nv, splits);
    return check_launch("backward kernels");
}

p2m_status p2m_query_host(const p2m_mesh* mh, const float* q, int64_t n, int32_t* prim, float* closest, float* dist,
                          uint8_t* status, int num_threads, int64_t counters[8]) {
    if (!mh) return fail(P2M_ERR_ARG, "mesh is NULL");
    MeshState& s = const_cast<MeshState&>(mh->s);
    if (!s.precomputed) return fail(P2M_ERR_STATE, "p2m_query_host before p2m_precompute");
    if (n < 0) return fail(P2M_ERR_ARG, "negative query count");
    if (n > 0 && (!q || !prim || !closest || !dist)) return fail(P2M_ERR_ARG, "NULL pointer");
    pack_mesh(s);
    int nt = num_threads > 0 ? num_threads : (int)std::max(1u, std::thread::hardware_concurrency());
    if (s.pk_seed.empty()) host_seed_grid(s, nt);
    const MeshView v = host_view(s);
    nt = (int)std::min<int64_t>(nt, std::max<int64_t>(1, n / 1024));
    std::vector<ScanCounters> cnt((size_t)nt);
    std::atomic<int64_t> cursor{0};
    auto work = [&](int t) {
        ScanCounters& c = cnt[(size_t)t];
        for (;;) {
            int64_t b = cursor.fetch_add(1024);
            if (b >= n) break;
            int64_t e = std::min(n, b + 1024);
            for (int64_t i = b; i < e; ++i) {
                uint8_t stt;
                Answer a = p2m_query_point(v, q[3 * i], q[3 * i + 1], q[3 * i + 2], stt, c);
                prim[i] = a.prim;
                closest[3 * i] = a.cx;
                closest[3 * i + 1] = a.cy;
                closest[3 * i + 2] = a.cz;
                dist[i] = a.dist;
                if (status) status[i] = stt;
            }
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(work, t);
    work(0);
    for (auto& x : th) x.join();
    if (counters) {
        for (int k = 0; k < 8; ++k) counters[k] = 0;
        for (auto& c : cnt) {
            counters[0] += c.nodes;
            counters[1] += c.edges;
            counters[2] += c.faces;
            counters[3] += c.steps;
            counters[4] += c.edge_forms;
            counters[5] += c.face_forms;
            counters[6] += c.rescans;
            counters[7] += c.rescan_exact;
        }
    }
    return P2M_OK;
}

}  // extern "C"
