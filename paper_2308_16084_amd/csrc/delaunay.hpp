// 3D Delaunay triangulation of the mesh vertices, used only for its edge
// graph: two vertices are Delaunay neighbours exactly when their Voronoi
// cells share a facet (or touch, in degenerate cospherical input), which is
// the neighbour relation of the vertex Voronoi diagram that flooding walks
// (Sec. 4.5, Algorithm 1).  The paper takes this diagram from TetGen; this
// is an incremental Bowyer-Watson construction with exact predicates.
#pragma once

#include <cstdint>
#include <vector>

namespace p2m {

struct DelaunayStats {
    int64_t tets = 0;
    int64_t edges = 0;
    long long exact_predicates = 0;
    int64_t walk_steps = 0;
};

// pts: n points (xyz, double).  cover_lo/cover_hi: a box that must be
// unaffected by the bounding simplex (the query domain); the simplex is
// placed far enough away that Voronoi cells inside the box are exactly those
// of the input points.  Fails (returns false) on duplicate points.
// Output: CSR adjacency (off[n+1], nbr) of Delaunay edges between input points.
bool delaunay_neighbors(const double* pts, int64_t n, const double cover_lo[3], const double cover_hi[3],
                        std::vector<int64_t>& off, std::vector<int32_t>& nbr, DelaunayStats* stats);

}  // namespace p2m
