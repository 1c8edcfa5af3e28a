// Interception table (Sec. 4): for each vertex v, the edges and faces whose
// generalised-Voronoi cell meets v's Voronoi cell (Eqs. (2)-(3)).
//
// Built as in the paper's preprocess (Appendix, Algorithm A.1):
//   * Voronoi cell of every vertex, clipped to the query domain box D (the
//     paper bounds cells with 8 far virtual points instead; for queries in D
//     both give the same cells -- Remark in Sec. 4.3);
//   * Space-perp of every edge and face (Sec. 4.2, Eqs. (4)-(5));
//   * convexity filter (Theorems 5 and 6): v cannot intercept p when every
//     corner of ConvexPoly(v,p) = Cell(v) n Space-perp(p) is at least as close
//     to v as to the line/plane of p;
//   * flooding from the primitive's own vertices over Voronoi neighbours
//     (Algorithm 1), complete by Theorem 7;
//   * the vertices of a primitive always intercept it (Theorem 2).
// All geometry is FP64.  Every half-space is moved outward by a margin tau
// and the filter excludes a vertex only with a margin tau, so rounding can
// only add entries, never drop one.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "mesh.hpp"

namespace p2m {

// TABLE_FLOODING_DEVICE runs the filter and flooding on the current HIP
// device with the host's arithmetic; the table is the TABLE_FLOODING one.
enum TableMode { TABLE_FLOODING = 0, TABLE_ALL_PAIRS = 1, TABLE_EVERYTHING = 2, TABLE_FLOODING_DEVICE = 3 };

struct TableOptions {
    double lo[3], hi[3];  // query domain D
    double tau;           // absolute margin
    int threads;          // 0: all
    int mode;             // TableMode
    int visit_cap = 0;    // TABLE_FLOODING_DEVICE: flood size the device keeps (0: its most)
};

struct TableStats {
    double t_delaunay = 0, t_cells = 0, t_flood = 0, t_pack = 0;
    // device inspection: upload, kernel, download; primitives left to the host
    double t_dev_upload = 0, t_dev_kernel = 0, t_dev_download = 0;
    int64_t device_redo = 0, device_cells_back = 0;
    int64_t delaunay_edges = 0, tets = 0;
    long long exact_predicates = 0;
    int64_t flood_tests = 0, flood_hits = 0, quick_rejects = 0, skipped_clips = 0;
    int64_t nnz_edges = 0, nnz_faces = 0, max_list = 0;
};

struct Table {
    // Per vertex v: edge ids ent[off[2v] .. off[2v+1]), face ids
    // ent[off[2v+1] .. off[2v+2]), each ascending.
    std::vector<uint32_t> off;  // [2*nv+1]
    std::vector<int32_t> ent;
    // Entry boxes, 6 per entry (lower x,y,z then upper x,y,z) in the 16-bit
    // frame of D: u = (x - lo) * 65535 / (hi - lo), rounded outward by one
    // unit beyond the floor / ceiling and clamped to [0, 65535].  The box
    // holds ConvexPoly(v,p) = Cell(v) n Space-perp(p) n D (Sec. 4.6 bounds
    // Region(v,p), a subset, the same way); a query in D outside it is not in
    // Space-perp(p) and p is not its answer.
    std::vector<uint16_t> box;
    // Voronoi (Delaunay) neighbours, kept for inspection.
    std::vector<int64_t> nb_off;
    std::vector<int32_t> nb;
};

bool build_table(const MeshData& m, const TableOptions& o, Table& t, TableStats& st, std::string& err);

}  // namespace p2m
