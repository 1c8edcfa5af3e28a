// Device helpers shared by the query, batch and sort translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace p2m {

constexpr int kXcds = 8;  // MI355X: 8 XCDs, blocks dispatched round-robin
constexpr int kQueryMaxBlock = 256;  // launch bound of the query kernels

// Block b of a grid of G blocks -> the tile it takes, such that the blocks
// of each XCD (b = x mod 8) take one contiguous stretch of the tiles, in
// order: tiles processed side by side then share an L2.
__host__ __device__ __forceinline__ int64_t xcd_chunk(int64_t b, int64_t G) {
    const int64_t x = b % kXcds, k = b / kXcds, q = G / kXcds, r = G % kXcds;
    return x * q + (x < r ? x : r) + k;
}

// 30-bit Morton key: 10 bits per axis, cell = clamp(floor((q-lo)*s), 0, 1023)
// in float32 (one subtract, one multiply); x takes the top bit of each triple.
__host__ __device__ __forceinline__ uint32_t spread10(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__host__ __device__ __forceinline__ uint32_t quant10(float q, float lo, float s) {
    const float t = (q - lo) * s;
    if (!(t >= 0.f)) return 0u;
    if (t >= 1023.f) return 1023u;
    return (uint32_t)t;
}

__host__ __device__ __forceinline__ uint32_t morton30(float x, float y, float z, float lox, float loy, float loz,
                                                      float sx, float sy, float sz) {
    return (spread10(quant10(x, lox, sx)) << 2) | (spread10(quant10(y, loy, sy)) << 1) | spread10(quant10(z, loz, sz));
}

// lo rounded to float, s = float(1024 / (hi - lo)) computed in double.
inline void morton_params(const double dlo[3], const double dhi[3], float lo[3], float s[3]) {
    for (int k = 0; k < 3; ++k) {
        lo[k] = (float)dlo[k];
        s[k] = (float)(1024.0 / (dhi[k] - dlo[k]));
    }
}

// Writes staged answers to the output arrays with coalesced stores: per
// query (prim bits, closest), (dist, status bits, w0, w1) and, when bary
// is set, (w2, pv0, pv1, pv2); status may be NULL, bary and pvid both NULL
// or both set.  Enqueued on `st`.
hipError_t launch_split(const float4* stage, int64_t n, int32_t* prim, float* closest, float* dist, uint8_t* status,
                        float* bary, int32_t* pvid, hipStream_t st);

// ---------------------------------------------------------------- sort

// Stable LSD radix sort of (uint32 key, int32 value) pairs, 8-bit digits.
struct RadixPlan {
    int64_t n = 0;
    int64_t tiles = 0;       // blocks of at most kRadixTile keys
    int64_t counts = 0;      // 256 * tiles
    int64_t scan_blocks = 0; // blocks of the count scan
    int64_t totals = 256;    // digit totals: 256 per segment
    int64_t bytes = 0;       // scratch bytes
};

struct RadixBuffers {
    uint32_t* keys[2];
    int32_t* vals[2];
    uint32_t* counts;  // digit-major count matrix [256 * tiles]
    uint32_t* sums;    // the 256 digit totals of a pass
};

constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 16;
constexpr int64_t kRadixTile = kRadixThreads * kRadixItems;
constexpr int kRadixHistThreads = 1024;  // threads of a histogram block (4 keys each)

// Segmented sort: the keys form consecutive segments (the queries of one
// mesh of a batch) and each is sorted on its own, in place, so the segment
// index needs no digits of the key.  Tiles never straddle a segment; the
// count matrix holds, per segment, a digit-major block of 256 x (its tiles).
struct RadixSegTile {
    int64_t start;          // first key of the tile
    int32_t count, j, seg;  // keys in the tile, its index within its segment, the segment
    int32_t pad;
};
struct RadixSegInfo {
    int64_t start;  // first key of the segment
    int64_t base;   // its block of the count matrix: 256 * (tiles of earlier segments)
    int32_t cols;   // its tiles
    int32_t pad;
};
struct RadixSegments {
    const RadixSegTile* tiles = nullptr;  // device [ntiles]
    const RadixSegInfo* segs = nullptr;   // device [nseg]
    int64_t ntiles = 0;
    int32_t nseg = 0;
};

RadixPlan radix_plan(int64_t n);
// Plan of a segmented sort of n keys in ntiles tiles over nseg segments.
RadixPlan radix_plan_segmented(int64_t n, int64_t ntiles, int32_t nseg);
// The tiles and segment records of a segmented sort (host side); seg_start
// holds nseg+1 non-decreasing key offsets.
void radix_segment_tiles(const std::vector<int64_t>& seg_start, std::vector<RadixSegTile>& tiles,
                         std::vector<RadixSegInfo>& segs);
RadixBuffers radix_buffers(const RadixPlan& p, void* scratch);
// Stable sort of the positions 0..n-1 by bits [lo_bit, hi_bit) of keys[0]
// (8 bits per pass; the span is a multiple of 8): vals[r] receives the
// permutation (the input position of each sorted place) and, with
// keep_keys, keys[r] the sorted keys, where r (0/1) is returned; vals[0] is
// not read.  All work is enqueued on `st`.
// first_counts: the first pass's count matrix was already written by the
// kernel that made the keys (radix_hist_add), so that pass skips its
// histogram kernel.
int radix_sort_pairs(const RadixPlan& p, RadixBuffers& b, int lo_bit, int hi_bit, bool keep_keys, hipStream_t st,
                     const RadixSegments* seg = nullptr, bool first_counts = false);

// Adds digit d of one key per lane (when valid) to the 256 LDS counters h
// of a tile's histogram.  When every valid lane of the wavefront holds the
// same digit (runs of equal high digits in partly sorted keys), the first of
// them adds the wavefront's count with one atomic instead of 64 serialized
// ones on one counter.  Every lane of the wavefront calls it.
__device__ __forceinline__ void radix_hist_add(uint32_t* h, uint32_t d, bool valid) {
    const unsigned long long vm = __ballot(valid);
    if (vm == 0ull) return;
    const uint32_t d0 = (uint32_t)__shfl(d, __ffsll((long long)vm) - 1);
    if (__ballot(valid && d == d0) == vm) {
        if (valid && __popcll(vm & ((1ull << (threadIdx.x & 63)) - 1ull)) == 0) atomicAdd(&h[d], (uint32_t)__popcll(vm));
    } else if (valid) {
        atomicAdd(&h[d], 1u);
    }
}
// Exclusive prefix sum of a[0..n) in place; sums needs scan_sums_size(n)
// entries of scratch.
int64_t scan_sums_size(int64_t n);
void scan_exclusive_u32(uint32_t* a, int64_t n, uint32_t* sums, hipStream_t st);

}  // namespace p2m
