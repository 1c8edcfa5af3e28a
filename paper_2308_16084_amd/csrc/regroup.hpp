// Regrouping of a block's queries by list length, between the
// nearest-vertex step and the list scan (device only).
//
// A wavefront runs each list loop as long as its longest lane, and lanes of
// one wavefront hold lists of quite different lengths.  After the walk, the
// queries of a block (or of several rounds of one) are sorted by the steps
// their vertex's lists take -- a counting sort over kRegroupBins bins in
// LDS -- and each lane then answers the query of its sorted place, so a
// wavefront scans lists of nearly one length.  Only which lane answers a
// query changes, never the answer.
#pragma once

#include <hip/hip_runtime.h>

#include "query_core.hpp"

namespace p2m {

constexpr int kRegroupBins = 64;

// Steps of vertex vid's two list loops (edge then face entries, four a
// step), capped to the last bin.
__device__ __forceinline__ int regroup_bin(const MeshView& m, int32_t vid) {
    const uint4 h = m.vhead[2 * vid];
    const int steps = (int)(((h.y - h.x + 3u) >> 2) + ((h.z - h.y + 3u) >> 2));
    return steps < kRegroupBins - 1 ? steps : kRegroupBins - 1;
}

// The bins' counts in hist[0..kRegroupBins) become inclusive prefix sums
// (the first wavefront scans; the caller puts barriers around the call).
// Place of a query of bin b and rank r within it: (b ? hist[b-1] : 0) + r.
__device__ __forceinline__ void regroup_scan(uint32_t* hist) {
    const int t = threadIdx.x;
    if (t < kRegroupBins) {
        uint32_t x = hist[t];
#pragma unroll
        for (int d = 1; d < kRegroupBins; d <<= 1) {
            const uint32_t y = __shfl_up(x, d);
            if (t >= d) x += y;
        }
        hist[t] = x;
    }
}

}  // namespace p2m
