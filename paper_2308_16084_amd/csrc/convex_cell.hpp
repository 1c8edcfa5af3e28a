// Bounded convex polytope cut by half-spaces (Sec. 4.4, "Implementation").
//
// The paper keeps every corner with its three defining planes and every
// polytope edge by its end corners; a new half-space removes the corners on
// its invisible side and adds a corner where it crosses each surviving edge.
// This implementation stores the same information in dual form: a corner is
// a triangle (i,j,k) of plane indices, ordered so that det(n_i,n_j,n_k) > 0
// (counter-clockwise seen from outside), and a polytope edge is a pair of
// triangles sharing two planes in opposite order.  Cutting by a plane P
// deletes the triangles whose corner lies strictly outside P, walks the
// boundary cycle (a -> b) of the deleted region and adds triangle (a, b, P)
// for each boundary edge.  Corners are kept in FP64.
#pragma once

#include <array>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace p2m {

struct HalfSpace {
    double n[3];  // keeps points x with n.x <= off
    double off;
};

class ConvexCell {
   public:
    enum ClipResult { UNCHANGED = 0, CLIPPED = 1, EMPTY = 2, SKIPPED = 3 };

    void init_box(const double lo[3], const double hi[3]);
    // Cut by h.  SKIPPED means the cut could not be applied consistently in
    // floating point and the polytope was left as it was (a superset).
    ClipResult clip(const HalfSpace& h);
    bool empty() const { return empty_; }
    size_t num_corners() const { return tris_.size(); }
    const double* corner(size_t t) const { return pos_[t].data(); }
    size_t num_planes() const { return planes_.size(); }
    const HalfSpace& plane(size_t i) const { return planes_[i]; }
    // Drop planes that support no corner and renumber.
    void compact();

    // Flat serialisation: planes (4 doubles), triangles (3 uint16), corners (3 doubles).
    void save(std::vector<double>& planes, std::vector<uint16_t>& tris, std::vector<double>& pos) const;
    void load(const double* planes, size_t np, const uint16_t* tris, const double* pos, size_t nt);

   private:
    bool corner_of(int i, int j, int k, std::array<double, 3>& x) const;

    std::vector<HalfSpace> planes_;
    std::vector<std::array<uint16_t, 3>> tris_;
    std::vector<std::array<double, 3>> pos_;
    bool empty_ = false;
    // scratch
    std::vector<uint8_t> out_;
    std::vector<uint32_t> removed_;
    std::vector<std::array<uint16_t, 2>> bedges_, boundary_;
    std::vector<std::array<uint16_t, 3>> newt_;
    std::vector<std::array<double, 3>> newp_;
    std::vector<int32_t> next_;
};

}  // namespace p2m
