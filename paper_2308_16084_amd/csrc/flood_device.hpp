// Interface between the host table builder and the device inspection
// (plane cutting + flooding, Sec. 4.4-4.5, Algorithm 1) in p2m_flood.hip.
// Plain types only: the host side is compiled without HIP.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace p2m {

// One primitive as the filter sees it: a point of it, the unit edge
// direction or face normal, its vertices, and its Space-perp half-spaces
// (n.x <= off, moved outward by tau) at perp[4*perp_off ...].
struct FloodPrim {
    double a[3];
    double dir[3];
    int32_t verts[3];
    int32_t nverts;  // 2 (edge) or 3 (face)
    int32_t face;    // 0 edge, 1 face
    int32_t nperp;   // at most 8
    int64_t perp_off;
    int64_t id;      // edge or face id
};

// Builds the Voronoi cells of vertices vs on the host (for each, the planes
// (n, off) that bound a corner, 4 doubles each, and the corners, 3 doubles
// each); returns the number of cuts it had to skip.
using HostCellFn = std::function<int64_t(const std::vector<int64_t>& vs, std::vector<std::vector<double>>& planes,
                                         std::vector<std::vector<double>>& pos)>;

struct FloodInput {
    int64_t nv = 0, nprim = 0;
    const double* Vd = nullptr;  // [3*nv]
    const int64_t* nb_off = nullptr;  // [nv+1] Voronoi neighbours
    const int32_t* nb = nullptr;
    HostCellFn host_cell;             // cells the device hands back
    const FloodPrim* prims = nullptr;  // [nprim]
    const double* perp = nullptr;      // [4 * total half-spaces]
    int64_t nperp_total = 0;
    double blo[3], bhi[3];     // D grown by tau (the cells' box)
    double qlo[3], qscale[3];  // 16-bit frame of D for the entry boxes
    double tau = 0, dmax = 0;
    int visit_cap = 0;  // vertices a flood may visit before the host takes it over (0: the most)
};

// A table entry found on the device: vertex, code (face bit 31 | id), box.
struct FloodRec {
    uint32_t v, code;
    uint16_t box[6];
};

struct FloodResult {
    std::vector<FloodRec> recs;      // entries of every primitive not in `redo`
    std::vector<int64_t> redo;       // primitive indices the device could not
                                     // finish (a working polytope or visited
                                     // set beyond its fixed capacity): the
                                     // host floods these itself
    int64_t tests = 0, hits = 0, quick = 0, skipped = 0;
    int64_t cells_skipped = 0, cells_back = 0;  // cell construction: skipped cuts, cells built on the host
    double t_upload = 0, t_cells = 0, t_kernel = 0, t_download = 0;
};

// Builds every vertex's Voronoi cell and then runs the inspection of every
// primitive on the current HIP device.  False (with err) on a HIP error.
bool device_flood(const FloodInput& in, FloodResult& out, std::string& err);

}  // namespace p2m
