// KD tree of the mesh vertices (Sec. 2.1): median split, splitting
// dimension alternating x, y, z with depth.  Stored as a left-balanced
// implicit tree: node i has children 2i+1 and 2i+2, every level but the last
// is full and the last is filled from the left, so no child pointers are
// stored; the split dimension of a node is its depth mod 3.
#pragma once

#include <cstdint>
#include <vector>

namespace p2m {

struct KdTree {
    int64_t n = 0;
    std::vector<float> x, y, z;   // node coordinates (tree order)
    std::vector<int32_t> vid;     // node -> vertex id
};

void build_kdtree(const float* V, int64_t n, KdTree& t);

}  // namespace p2m
