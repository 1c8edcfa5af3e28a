#include "kdtree.hpp"

#include <algorithm>
#include <numeric>

namespace p2m {

namespace {

// Size of the left subtree of a left-balanced tree with m nodes.
int64_t left_size(int64_t m) {
    if (m <= 1) return 0;
    int h = 63 - __builtin_clzll((unsigned long long)m);  // levels 0..h
    int64_t full_above = (int64_t(1) << h) - 1;            // nodes in levels 0..h-1
    int64_t last = m - full_above;                         // nodes in level h
    int64_t half = int64_t(1) << (h - 1);                  // level-h slots of the left subtree
    return (half - 1) + std::min(last, half);
}

struct Builder {
    const float* V;
    std::vector<int32_t>& perm;
    KdTree& t;
    void build(int64_t node, int64_t lo, int64_t hi, int depth) {
        // points perm[lo..hi) form the subtree rooted at `node`
        int64_t m = hi - lo;
        if (m <= 0) return;
        int dim = depth % 3;
        int64_t L = left_size(m);
        auto key = [&](int32_t i) { return V[3 * (size_t)i + dim]; };
        std::nth_element(perm.begin() + lo, perm.begin() + lo + L, perm.begin() + hi,
                         [&](int32_t a, int32_t b) { return key(a) < key(b) || (key(a) == key(b) && a < b); });
        int32_t p = perm[(size_t)(lo + L)];
        t.x[(size_t)node] = V[3 * (size_t)p];
        t.y[(size_t)node] = V[3 * (size_t)p + 1];
        t.z[(size_t)node] = V[3 * (size_t)p + 2];
        t.vid[(size_t)node] = p;
        build(2 * node + 1, lo, lo + L, depth + 1);
        build(2 * node + 2, lo + L + 1, hi, depth + 1);
    }
};

}  // namespace

void build_kdtree(const float* V, int64_t n, KdTree& t) {
    t.n = n;
    t.x.assign((size_t)n, 0.f);
    t.y.assign((size_t)n, 0.f);
    t.z.assign((size_t)n, 0.f);
    t.vid.assign((size_t)n, -1);
    std::vector<int32_t> perm((size_t)n);
    std::iota(perm.begin(), perm.end(), 0);
    Builder b{V, perm, t};
    b.build(0, 0, n, 0);
}

}  // namespace p2m
