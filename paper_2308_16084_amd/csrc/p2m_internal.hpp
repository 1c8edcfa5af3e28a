// Internal state behind the opaque p2m_mesh / p2m_batch handles, shared by
// the host translation units (g++) and the device one (hipcc).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "p2m.h"
#include "interception.hpp"
#include "kdtree.hpp"
#include "mesh.hpp"

namespace p2m {

// Device copy of one mesh's query structures (all in one allocation).
// Layouts (device):
//   node  float4[4nv]    KD-tree node: x, y, z, vertex id (int bits), then the
//                        bounding boxes of the left and right subtrees
//   off   uint32[2nv+1]  interception-table offsets (edges, then faces, per vertex)
//   ent   int32[nnz]     edge / face ids
//   seg   float4[2ne]    edge end points: a.xyz|id_a, b.xyz|id_b
//   tri   float4[3nf]    face corners:    a.xyz|id_a, b.xyz|id_b, c.xyz|id_c
//   fedge int32[4nf]     edge ids of the sides (a,b), (b,c), (c,a), pad
struct DeviceMesh {
    int device = -1;
    void* base = nullptr;
    int64_t bytes = 0;
    void* node = nullptr;
    void* vhead = nullptr;  // list heads, uint4 [2nv]
    void* lent = nullptr;  // list entries with boxes, uint4 [nnz]
    void* seg = nullptr;
    void* tri = nullptr;
    void* fedge = nullptr;
    // Voronoi-neighbour walk: nboff uint32[nv+1], nbrec float4[nnz] (neighbour
    // position + id), seed float4[grid^3] (nearest vertex of each cell centre)
    void* nboff = nullptr;
    void* nbrec = nullptr;
    void* seed = nullptr;
    void* seed2 = nullptr;  // finer grid over the mesh's box (may be absent)
    // list-scan forms: frec float4[3nf], erec float4[2ne]
    void* frec = nullptr;
    void* erec = nullptr;
    // ordering scratch (keys/values, double-buffered), grown on demand
    void* scratch = nullptr;
    int64_t scratch_bytes = 0;
    // profiling events (hipEvent_t): start, after ordering, after query
    void* ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool ev_recorded = false;
    bool ev_sorted = false;
};

struct MeshState {
    MeshData m;
    KdTree kd;
    Table t;
    TableStats ts;
    bool precomputed = false;
    double dlo[3] = {0, 0, 0}, dhi[3] = {0, 0, 0};
    double tau = 0.0;
    double t_validate = 0.0, t_kdt = 0.0;
    // Packed query structures (host staging of the device layouts above;
    // also read directly by the host CPU query).
    bool packed = false;
    std::vector<float> pk_node;                  // 16 floats per KD-tree node
    std::vector<float> pk_seg, pk_tri;           // 4 floats per entry
    std::vector<int32_t> pk_fedge;               // 4 ints per face
    std::vector<uint32_t> pk_nboff;              // 32-bit neighbour offsets
    std::vector<float> pk_nbrec;                 // 4 floats per neighbour entry (position, id)
    std::vector<float> pk_seed;                  // host copy of the seed grid, 4 floats per cell (host query only)
    std::vector<float> pk_seed2;                 // and of the finer grid
    std::vector<float> pk_frec, pk_erec;         // list-scan forms: 12 floats per face, 8 per edge
    std::vector<uint32_t> pk_vhead;              // list heads: 8 words per vertex
    std::vector<uint32_t> pk_lent;               // list entries: id + 5-bit box, 2 words each, runs padded
    float ctr[3] = {0.f, 0.f, 0.f};              // origin of the forms
    float mu = 0.f;                              // gate margin
    DeviceMesh dev;
};

void set_error(const std::string& msg);
p2m_status fail(p2m_status s, const std::string& msg);

// Device-side teardown (defined in the device translation unit).
void device_release(MeshState& s);

}  // namespace p2m

struct p2m_mesh {
    p2m::MeshState s;
};
