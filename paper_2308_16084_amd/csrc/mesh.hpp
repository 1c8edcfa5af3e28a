// Triangle mesh with one copy of each vertex (problem statement, Sec. 4.1),
// optionally with free segments (a mixed set of segments and triangles,
// Sec. 5.5): validation, canonical edges and the face/edge incidence the
// precompute needs.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace p2m {

constexpr int64_t kMaxPrimitives = (int64_t(1) << 30) - 1;

struct MeshData {
    int64_t nv = 0, nf = 0, ne = 0;
    std::vector<float> V;          // [nv*3] as given
    std::vector<double> Vd;        // [nv*3] exact widening
    std::vector<int32_t> F;        // [nf*3]
    std::vector<int32_t> S;        // [ns*2] free segments as given
    int64_t ns = 0;
    std::vector<int32_t> E;        // [ne*2] canonical: (min,max), lexicographic order; sides of faces and segments
    std::vector<int32_t> FE;       // [nf*3] edge id of side s = (F[s], F[s+1 mod 3])
    std::vector<int64_t> ef_off;   // [ne+1] edge -> incident faces
    std::vector<int32_t> ef_face;
    double lo[3], hi[3];           // AABB of V
};

// Returns an empty string on success, else the reason the mesh is rejected:
// counts out of range (at least one vertex and one face or segment), index
// out of range, a face or segment repeating a vertex, a face of zero area,
// non-finite coordinates, or two vertices with equal coordinates.  F may be
// NULL when nf = 0 and S when ns = 0.
std::string build_mesh(const float* V, int64_t nv, const int32_t* F, int64_t nf, const int32_t* S, int64_t ns,
                       MeshData& m);

}  // namespace p2m
