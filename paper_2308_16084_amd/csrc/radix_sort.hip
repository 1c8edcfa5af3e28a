// Stable LSD radix sort of (uint32 key, int32 value) pairs for gfx950.
//
// Per 8-bit digit pass: (1) every tile of 4096 keys counts its digits in
// LDS; (2) one block per digit scans that digit's column of the digit-major
// count matrix (the digit's offset within its run of the output) and keeps
// the column total; (3) every tile adds the exclusive scan of the 256 digit
// totals to its column offsets, re-reads its keys, ranks
// each key among equal digits with wave-wide ballots (stable within a
// wave), adds the counts of earlier waves and of earlier chunks of the
// tile, places the pair in LDS in digit order and finally writes each
// digit's run of the tile to its output offset with coalesced stores.
// A segmented sort (RadixSegments) runs the same passes over tiles that
// never straddle a segment, with one count block and one set of digit
// totals per segment, so each segment is sorted within its own range.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.hpp"

namespace p2m {

namespace {

constexpr int kT = kRadixThreads;
constexpr int kI = kRadixItems;
constexpr int kWaves = kT / 64;
constexpr int kColRegs = 16;  // column values a colscan thread keeps in registers
// Scatter blocks: 512 threads, 8 keys a thread, 8 wavefronts (at about 55
// registers, three blocks -- 24 wavefronts -- fit on a CU by LDS, where 256
// threads of 16 keys needed 100 registers and fitted 16).
constexpr int kST = 512;
constexpr int kSI = (int)(kRadixTile / kST);
constexpr int kSWaves = kST / 64;

// Where block b's tile lies: keys [start, start+count), column j of the
// `cols` columns of its count block at `base`, and its segment.
struct TileGeo {
    int64_t start, base;
    int32_t count, j, cols, seg;
};

// The blocks of each XCD take a contiguous stretch of tiles (xcd_chunk): in
// a scatter, the runs that neighbouring tiles write for one digit are
// adjacent, so they meet in one L2 and leave it as whole lines.
template <bool kSeg>
__device__ __forceinline__ TileGeo tile_geo(int64_t n, int64_t tiles, const RadixSegments& sg) {
    TileGeo g;
    const int64_t b = xcd_chunk(blockIdx.x, gridDim.x);
    if (kSeg) {
        const RadixSegTile st = sg.tiles[b];
        const RadixSegInfo si = sg.segs[st.seg];
        g.start = st.start;
        g.count = st.count;
        g.j = st.j;
        g.seg = st.seg;
        g.base = si.base;
        g.cols = si.cols;
    } else {
        g.start = b * kRadixTile;
        g.count = (int32_t)std::min<int64_t>(kRadixTile, n - g.start);
        g.j = (int32_t)b;
        g.seg = 0;
        g.base = 0;
        g.cols = (int32_t)tiles;
    }
    return g;
}

// Digit counts of one tile in LDS (radix_hist_add), written to the tile's
// column of the count matrix.  kRadixHistThreads threads a tile, four keys
// each, all loaded before any is counted: the grid has as many blocks as the
// sort has tiles, and short blocks keep the chip busy to the end.
template <bool kSeg>
__global__ __launch_bounds__(kRadixHistThreads) void k_radix_hist(const uint32_t* __restrict__ keys, int64_t n,
                                                                  int shift, uint32_t* __restrict__ counts,
                                                                  int64_t tiles, RadixSegments sg) {
    constexpr int kHT = kRadixHistThreads, kHI = (int)(kRadixTile / kRadixHistThreads);
    __shared__ uint32_t h[256];
    const int t = threadIdx.x;
    const TileGeo g = tile_geo<kSeg>(n, tiles, sg);
    uint32_t key[kHI];
#pragma unroll
    for (int it = 0; it < kHI; ++it) {
        const int i = it * kHT + t;
        key[it] = i < g.count ? keys[g.start + i] : 0u;
    }
    if (t < 256) h[t] = 0;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kHI; ++it) radix_hist_add(h, (key[it] >> shift) & 255u, it * kHT + t < g.count);
    __syncthreads();
    if (t < 256) counts[g.base + (int64_t)t * g.cols + g.j] = h[t];
}

// Exclusive scan of 4096-element blocks in place; block totals to sums.
__global__ __launch_bounds__(kT) void k_scan_local(uint32_t* __restrict__ a, int64_t n, uint32_t* __restrict__ sums) {
    __shared__ uint32_t part[kT];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kRadixTile + (int64_t)t * kI;
    uint32_t v[kI];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kI; ++k) {
        v[k] = (base + k < n) ? a[base + k] : 0u;
        s += v[k];
    }
    part[t] = s;
    __syncthreads();
    // inclusive Hillis-Steele scan of the per-thread sums
    for (int d = 1; d < kT; d <<= 1) {
        uint32_t x = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    uint32_t run = t > 0 ? part[t - 1] : 0u;
#pragma unroll
    for (int k = 0; k < kI; ++k) {
        if (base + k < n) a[base + k] = run;
        run += v[k];
    }
    if (t == kT - 1) sums[blockIdx.x] = part[kT - 1];
}

// Exclusive scan of `n` block sums by one block, in chunks with a carry.
__global__ __launch_bounds__(kT) void k_scan_sums(uint32_t* __restrict__ a, int64_t n) {
    __shared__ uint32_t part[kT];
    __shared__ uint32_t carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int64_t c = 0; c < n; c += kT) {
        const int64_t i = c + t;
        const uint32_t x0 = i < n ? a[i] : 0u;
        part[t] = x0;
        __syncthreads();
        for (int d = 1; d < kT; d <<= 1) {
            uint32_t x = t >= d ? part[t - d] : 0u;
            __syncthreads();
            part[t] += x;
            __syncthreads();
        }
        const uint32_t excl = part[t] - x0 + carry;
        __syncthreads();
        if (i < n) a[i] = excl;
        if (t == kT - 1) carry += part[kT - 1];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kT) void k_scan_add(uint32_t* __restrict__ a, int64_t n, const uint32_t* __restrict__ sums) {
    const uint32_t add = sums[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kRadixTile + (int64_t)threadIdx.x * kI;
#pragma unroll
    for (int k = 0; k < kI; ++k)
        if (base + k < n) a[base + k] += add;
}

// Exclusive scan of one value per thread over the kT threads of a block;
// *total receives the block's sum.  Every thread calls it (barriers inside).
template <int kW = kWaves>
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t x, uint32_t* wsum, uint32_t* total) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kW; ++k) {
        before += k < w ? wsum[k] : 0u;
        all += wsum[k];
    }
    __syncthreads();  // wsum may be reused by the caller's next scan
    *total = all;
    return before + incl - x;
}

// Column d of the digit-major count matrix of a plain sort (the tiles'
// counts of digit d; block d): exclusive scan in place -- each thread sums a
// contiguous stretch of the column, one block scan of the stretch sums, then
// each thread writes its stretch's running offsets; totals[d] = the
// column's sum.
__global__ __launch_bounds__(kT) void k_radix_colscan(uint32_t* __restrict__ counts, int64_t tiles,
                                                      uint32_t* __restrict__ totals) {
    __shared__ uint32_t wsum[kWaves];
    const int d = (int)blockIdx.x;
    uint32_t* col = counts + (int64_t)d * tiles;
    const int64_t per = (tiles + kT - 1) / kT;
    const int64_t a = std::min<int64_t>(tiles, (int64_t)threadIdx.x * per), e = std::min<int64_t>(tiles, a + per);
    uint32_t sum;
    if (per <= kColRegs) {
        // up to kColRegs values a thread: loaded together, kept in registers
        uint32_t x[kColRegs];
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < kColRegs; ++k) {
            x[k] = a + k < e ? col[a + k] : 0u;
            s += x[k];
        }
        uint32_t run = block_scan_excl(s, wsum, &sum);
#pragma unroll
        for (int k = 0; k < kColRegs; ++k) {
            if (a + k < e) col[a + k] = run;
            run += x[k];
        }
    } else {
        uint32_t s = 0;
        for (int64_t i = a; i < e; ++i) s += col[i];
        uint32_t run = block_scan_excl(s, wsum, &sum);
        for (int64_t i = a; i < e; ++i) {
            const uint32_t x = col[i];
            col[i] = run;
            run += x;
        }
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = sum;
}

// The columns of a segmented sort: one block per segment, thread d scans
// segment s's column d (its tiles' counts of digit d, a few to a few
// hundred), kColRegs values at a time loaded together; totals[256*s+d] =
// the column's sum.  (One block per column and segment, as in the plain
// sort, would launch 256 blocks per mesh, most with a handful of values.)
__global__ __launch_bounds__(kT) void k_radix_colscan_seg(uint32_t* __restrict__ counts,
                                                          uint32_t* __restrict__ totals, RadixSegments sg) {
    const RadixSegInfo si = sg.segs[blockIdx.x];
    const int d = threadIdx.x;
    uint32_t* col = counts + si.base + (int64_t)d * si.cols;
    uint32_t run = 0;
    for (int32_t j0 = 0; j0 < si.cols; j0 += kColRegs) {
        uint32_t x[kColRegs];
#pragma unroll
        for (int k = 0; k < kColRegs; ++k) x[k] = j0 + k < si.cols ? col[j0 + k] : 0u;
#pragma unroll
        for (int k = 0; k < kColRegs; ++k) {
            if (j0 + k < si.cols) col[j0 + k] = run;
            run += x[k];
        }
    }
    totals[256 * (int64_t)blockIdx.x + d] = run;
}

// Scatter of one tile (kPositions: the values are the keys' positions, as in
// the first pass, and vin is not read; !kKeysOut: the keys are not written,
// as in a last pass whose caller needs only the permutation): the tile's
// 4096 pairs are first placed in LDS in
// digit order (stable: by digit, then by position in the tile), then written
// out so that consecutive threads write consecutive places of each digit's
// run -- coalesced runs of ~16 keys instead of one cache line per key.
// Each wavefront ranks its own contiguous eighth of the tile, 64 keys per
// round, against a running per-digit count of its earlier rounds (ballots
// on the 8 digit bits find the lanes of equal digit), so the block meets at
// a barrier only a few times per tile.
template <bool kPositions, bool kKeysOut, bool kSeg>
__global__ __launch_bounds__(kST) void k_radix_scatter(const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin,
                                                      int64_t n, int shift, const uint32_t* __restrict__ offs,
                                                      const uint32_t* __restrict__ totals, int64_t tiles,
                                                      uint32_t* __restrict__ kout, int32_t* __restrict__ vout,
                                                      RadixSegments sg) {
    __shared__ uint32_t gbase[256];        // global start of each digit's run of this tile
    __shared__ uint32_t lstart[256];       // start of each digit in the tile's LDS order
    __shared__ uint32_t wc[kSWaves][256];   // per wave: running count, then its base per digit
    __shared__ uint32_t lk[kRadixTile];
    __shared__ int32_t lv[kRadixTile];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int w = t >> 6;
    const TileGeo g = tile_geo<kSeg>(n, tiles, sg);
    const int64_t tile0 = g.start;
    const int cnt = g.count;
    // the tile's pairs: loaded first, so that their latency overlaps the
    // digit offsets' loads and scan
    const int wbase = w * (kSI * 64);
    uint32_t key[kSI];
    int32_t val[kSI];
#pragma unroll
    for (int it = 0; it < kSI; ++it) {
        const int i = wbase + it * 64 + lane;
        const bool valid = i < cnt;
        key[it] = valid ? kin[tile0 + i] : 0u;
        val[it] = valid ? (kPositions ? (int32_t)(tile0 + i) : vin[tile0 + i]) : 0;
    }
    __shared__ uint32_t wsum[kSWaves];
    {
        // digit t's run starts after the runs of smaller digits (of the
        // tile's segment, which starts at its first key)
        uint32_t all;
        const uint32_t dpre = block_scan_excl<kSWaves>(t < 256 ? totals[256 * g.seg + t] : 0u, wsum, &all);
        const uint32_t seg0 = kSeg ? (uint32_t)sg.segs[g.seg].start : 0u;
        if (t < 256) gbase[t] = seg0 + dpre + offs[g.base + (int64_t)t * g.cols + g.j];
    }
    for (int i = t; i < kSWaves * 256; i += kST) (&wc[0][0])[i] = 0u;
    __syncthreads();
    // lanes below this one, as two 32-bit halves
    const uint32_t ltlo = lane >= 32 ? ~0u : (1u << lane) - 1u;
    const uint32_t lthi = lane <= 32 ? 0u : (1u << (lane - 32)) - 1u;
    uint32_t rank[kSI];
#pragma unroll
    for (int it = 0; it < kSI; ++it) {
        const bool valid = wbase + it * 64 + lane < cnt;
        const uint32_t d = (key[it] >> shift) & 255u;
        // the lanes holding the same digit: per bit, the ballot of the lanes
        // with the bit set, or its complement when this lane's bit is clear
        const unsigned long long vm = __ballot(valid);
        uint32_t mlo = (uint32_t)vm, mhi = (uint32_t)(vm >> 32);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint32_t nb = ((d >> b) & 1u) - 1u;  // 0 when set, all ones when clear
            const unsigned long long bm = __ballot(nb == 0u);
            mlo &= (uint32_t)bm ^ nb;
            mhi &= (uint32_t)(bm >> 32) ^ nb;
        }
        const uint32_t r = (uint32_t)(__popc(mlo & ltlo) + __popc(mhi & lthi));
        const uint32_t prior = valid ? wc[w][d] : 0u;
        rank[it] = prior + r;
        // the lowest lane of each digit advances the wave's count; this
        // wave's LDS accesses stay in program order
        if (valid && r == 0) wc[w][d] = prior + (uint32_t)(__popc(mlo) + __popc(mhi));
    }
    __syncthreads();
    // digit totals, their exclusive scan (the tile's LDS order), and each
    // wave's base within each digit
    uint32_t c[kSWaves], tot = 0;
#pragma unroll
    for (int k = 0; k < kSWaves; ++k) {
        c[k] = t < 256 ? wc[k][t] : 0u;
        tot += c[k];
    }
    if (t < 256) lstart[t] = tot;
    __syncthreads();
    if (w == 0) {
        uint32_t v[4], sum = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = lstart[4 * lane + k];
            sum += v[k];
        }
        uint32_t incl = sum;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const uint32_t x = __shfl_up(incl, dd);
            if (lane >= dd) incl += x;
        }
        uint32_t e = incl - sum;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            lstart[4 * lane + k] = e;
            e += v[k];
        }
    }
    __syncthreads();
    if (t < 256) {
        uint32_t base = lstart[t];
#pragma unroll
        for (int k = 0; k < kSWaves; ++k) {
            wc[k][t] = base;
            base += c[k];
        }
        // LDS place p of digit t goes to gbase[t] + p - lstart[t]
        gbase[t] -= lstart[t];
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSI; ++it) {
        if (wbase + it * 64 + lane < cnt) {
            const uint32_t d = (key[it] >> shift) & 255u;
            const uint32_t pos = wc[w][d] + rank[it];
            lk[pos] = key[it];
            lv[pos] = val[it];
        }
    }
    __syncthreads();
    // coalesced write-out: LDS place p of digit d goes to gbase[d] + p
    for (int p = t; p < cnt; p += kST) {
        const uint32_t k = lk[p];
        const uint32_t d = (k >> shift) & 255u;
        const uint32_t pos = gbase[d] + (uint32_t)p;
        if (pos < (uint64_t)n) {
            if (kKeysOut) kout[pos] = k;
            vout[pos] = lv[p];
        }
    }
}

int64_t up256(int64_t x) { return (x + 255) / 256 * 256; }

}  // namespace

RadixPlan radix_plan(int64_t n) {
    RadixPlan p;
    p.n = n;
    p.tiles = (n + kRadixTile - 1) / kRadixTile;
    p.counts = 256 * p.tiles;
    p.scan_blocks = (p.counts + kRadixTile - 1) / kRadixTile;
    p.totals = 256;
    p.bytes = 4 * up256(4 * n) + up256(4 * p.counts) + up256(4 * std::max(p.totals, p.scan_blocks));
    return p;
}

RadixPlan radix_plan_segmented(int64_t n, int64_t ntiles, int32_t nseg) {
    RadixPlan p;
    p.n = n;
    p.tiles = ntiles;
    p.counts = 256 * ntiles;
    p.scan_blocks = 0;
    p.totals = 256 * (int64_t)std::max(1, nseg);
    p.bytes = 4 * up256(4 * n) + up256(4 * std::max<int64_t>(1, p.counts)) + up256(4 * p.totals);
    return p;
}

void radix_segment_tiles(const std::vector<int64_t>& seg_start, std::vector<RadixSegTile>& tiles,
                         std::vector<RadixSegInfo>& segs) {
    tiles.clear();
    segs.clear();
    for (size_t k = 0; k + 1 < seg_start.size(); ++k) {
        const int64_t a = seg_start[k], len = seg_start[k + 1] - a;
        const int32_t cols = (int32_t)((len + kRadixTile - 1) / kRadixTile);
        segs.push_back(RadixSegInfo{a, 256 * (int64_t)tiles.size(), cols, 0});
        for (int32_t j = 0; j < cols; ++j)
            tiles.push_back(RadixSegTile{a + (int64_t)j * kRadixTile,
                                         (int32_t)std::min<int64_t>(kRadixTile, len - (int64_t)j * kRadixTile), j,
                                         (int32_t)k, 0});
    }
}

RadixBuffers radix_buffers(const RadixPlan& p, void* scratch) {
    RadixBuffers b;
    char* c = (char*)scratch;
    const int64_t s = up256(4 * p.n);
    b.keys[0] = (uint32_t*)c;
    b.keys[1] = (uint32_t*)(c + s);
    b.vals[0] = (int32_t*)(c + 2 * s);
    b.vals[1] = (int32_t*)(c + 3 * s);
    b.counts = (uint32_t*)(c + 4 * s);
    b.sums = (uint32_t*)(c + 4 * s + up256(4 * p.counts));
    return b;
}

int64_t scan_sums_size(int64_t n) { return std::max<int64_t>(1, (n + kRadixTile - 1) / kRadixTile); }

void scan_exclusive_u32(uint32_t* a, int64_t n, uint32_t* sums, hipStream_t st) {
    if (n <= 0) return;
    const int64_t blocks = scan_sums_size(n);
    k_scan_local<<<(unsigned)blocks, kT, 0, st>>>(a, n, sums);
    k_scan_sums<<<1, kT, 0, st>>>(sums, blocks);
    k_scan_add<<<(unsigned)blocks, kT, 0, st>>>(a, n, sums);
}

__global__ void k_iota(int32_t* __restrict__ v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = (int32_t)i;
}

int radix_sort_pairs(const RadixPlan& p, RadixBuffers& b, int lo_bit, int hi_bit, bool keep_keys, hipStream_t st,
                     const RadixSegments* seg, bool first_counts) {
    int cur = 0;
    if (p.n <= 0) return cur;
    if (p.n == 1 || lo_bit >= hi_bit) {  // nothing to sort: the identity permutation
        k_iota<<<(unsigned)((p.n + 255) / 256), 256, 0, st>>>(b.vals[0], p.n);
        return cur;
    }
    const RadixSegments sg = seg ? *seg : RadixSegments{};
    for (int shift = lo_bit; shift < hi_bit; shift += 8) {
        const bool first = shift == lo_bit, last = shift + 8 >= hi_bit;
        const bool keys_out = !last || keep_keys;
#define P2M_SCATTER(P, K, S)                                                                                       \
    k_radix_scatter<P, K, S><<<(unsigned)p.tiles, kST, 0, st>>>(b.keys[cur], b.vals[cur], p.n, shift, b.counts,      \
                                                               b.sums, p.tiles, b.keys[cur ^ 1], b.vals[cur ^ 1], sg)
#define P2M_PASS(S)                                                                                             \
    do {                                                                                                        \
        if (!(first && first_counts))                                                                           \
            k_radix_hist<S><<<(unsigned)p.tiles, kRadixHistThreads, 0, st>>>(b.keys[cur], p.n, shift, b.counts,  \
                                                                          p.tiles, sg);                       \
        if (S) k_radix_colscan_seg<<<(unsigned)seg->nseg, kT, 0, st>>>(b.counts, b.sums, sg);                    \
        else k_radix_colscan<<<256u, kT, 0, st>>>(b.counts, p.tiles, b.sums);                                    \
        if (first) {                                                                                            \
            if (keys_out) P2M_SCATTER(true, true, S);                                                           \
            else P2M_SCATTER(true, false, S);                                                                   \
        } else {                                                                                                \
            if (keys_out) P2M_SCATTER(false, true, S);                                                          \
            else P2M_SCATTER(false, false, S);                                                                  \
        }                                                                                                       \
    } while (0)
        if (seg) P2M_PASS(true);
        else P2M_PASS(false);
#undef P2M_PASS
#undef P2M_SCATTER
        cur ^= 1;
    }
    return cur;
}

}  // namespace p2m
