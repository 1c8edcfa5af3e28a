// Batched P2M queries: many meshes of uneven size with uneven query counts
// served by one persistent launch over a packed arena, captured in a HIP
// graph, with the launch shape chosen by a small autotuner.
//
// Ordering: key = the top 24 bits of the query's Morton code in its mesh's
// domain box; a segmented radix sort (one segment per mesh: each mesh's
// queries are contiguous in the batch) orders each mesh's queries
// spatially in place, in three 8-bit passes.
// Work list: tiles (mesh, first sorted position, count) of block x qpl
// queries, meshes with the most work first.  By default the launch has one
// workgroup per tile, in list order, and the hardware dispatcher hands the
// workgroups to CUs as they free up (largest-first balancing for free).
// The persistent schedule (p2m_batch_set_schedule) launches as many
// workgroups as fit on the chip, each taking the next tile from an atomic
// counter until the list is exhausted, so every workgroup reaches the exit;
// on a batch of many small tiles its single counter serialises.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "device_common.hpp"
#include "p2m_internal.hpp"
#include "nearest.hpp"
#include "query_core.hpp"
#include "regroup.hpp"
#include "wave_scan.hpp"

namespace p2m {

void pack_mesh(MeshState& s);
MeshView host_view(const MeshState& s);

struct BatchMesh {
    int64_t node, head, ent, seg, tri, fedge;  // element offsets into the typed arenas
    int64_t nboff, nbrec, seed;               // Voronoi walk arrays (local ids inside)
    int64_t frec, erec;                       // list-scan forms
    int32_t nv;
    int32_t grid;          // seed grid side
    float dlo[3], dhi[3];  // domain rounded outward (status flag)
    float mlo[3], msc[3];  // Morton quantisation of the domain
    float gscale[3];       // seed grid cells per unit length (grid origin = dlo)
    float ctr[3], mu;      // origin and gate margin of the list-scan forms
    float eta;             // absolute slack of the winner check
    float qlo[3], qs[3];   // 16-bit frame of D for the entry boxes
};

// View of mesh d inside the arena.
__host__ __device__ inline MeshView arena_view(const BatchMesh& d, const KdNode* node, const uint4* vhead,
                                               const uint4* lent, const float4* seg, const float4* tri,
                                               const int32_t* fedge, const uint32_t* nboff, const float4* nbrec,
                                               const float4* seed, const float4* frec,
                                               const float4* erec) {
    MeshView v;
    v.node = node + d.node;
    v.nv = d.nv;
    v.vhead = vhead + d.head;
    v.lent = lent + d.ent;
    v.seg = seg + d.seg;
    v.tri = tri + d.tri;
    v.fedge = fedge + d.fedge;
    v.nboff = nboff + d.nboff;
    v.nbrec = nbrec + d.nbrec;
    v.seed = seed + d.seed;
    v.seed2 = nullptr;  // one grid per mesh in the batch arena
    v.grid2 = 0;
    for (int k = 0; k < 3; ++k) v.glo2[k] = v.gscale2[k] = v.ghi2[k] = 0.f;
    v.frec = frec + d.frec;
    v.erec = erec + d.erec;
    v.mu = d.mu;
    v.eta = d.eta;
    v.grid = d.grid;
    for (int k = 0; k < 3; ++k) {
        v.dlo[k] = d.dlo[k];
        v.dhi[k] = d.dhi[k];
        v.glo[k] = d.dlo[k];
        v.gscale[k] = d.gscale[k];
        v.ctr[k] = d.ctr[k];
        v.qlo[k] = d.qlo[k];
        v.qs[k] = d.qs[k];
    }
    return v;
}

struct Tile {
    int32_t mesh, start, count, pad;
};

}  // namespace p2m

struct p2m_batch {
    int device = -1;
    int32_t count = 0;
    void* base = nullptr;
    int64_t bytes = 0;
    p2m::KdNode* node = nullptr;
    uint4* vhead = nullptr;
    uint4* lent = nullptr;
    float4* seg = nullptr;
    float4* tri = nullptr;
    int32_t* fedge = nullptr;
    uint32_t* nboff = nullptr;
    float4* nbrec = nullptr;
    float4* seed = nullptr;
    float4* frec = nullptr;
    float4* erec = nullptr;
    p2m::BatchMesh* desc = nullptr;
    std::vector<double> cost;  // per-mesh cost weight (log of vertex count)
    // per query layout
    std::vector<int64_t> layout;
    int64_t n = 0;
    void* work = nullptr;  // tiles, counter, sort tiles and segments, sort scratch, staged answers
    int64_t work_bytes = 0;
    p2m::Tile* tiles = nullptr;
    int64_t ntiles = 0;
    uint32_t* counter = nullptr;
    p2m::RadixSegments sort_seg;  // the segmented sort's tiles and segments (device)
    void* scratch = nullptr;
    float4* stage = nullptr;  // 16-byte answer record per query (prim, closest point)
    int tile_block = 0, tile_qpl = 0;
    // launch shape
    int block = 256, qpl = 1, traversal = 3;
    int persistent = 0;  // 0: one workgroup per tile; 1: persistent workgroups and a tile counter
    int lds_levels = 0;  // traversal 1: tree levels staged in LDS per tile
    int grid = 0;
    // captured graph
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* g_ptrs[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    int g_shape[4] = {0, 0, 0, 0};
};

namespace p2m {

namespace {

int64_t up256(int64_t x) { return (x + 255) / 256 * 256; }

// Keys of one radix tile of the batch (a tile lies in one mesh: the
// segmented sort's tiles) -- the top 24 bits of the query's Morton code in
// its mesh's domain box -- and the counts of their low digit, the first
// pass's column of the count matrix.
__global__ __launch_bounds__(kRadixHistThreads) void k_batch_keys(const float* __restrict__ q,
                                                                  const BatchMesh* __restrict__ desc, RadixSegments sg,
                                                                  uint32_t* __restrict__ keys,
                                                                  uint32_t* __restrict__ counts) {
    constexpr int kHI = (int)(kRadixTile / kRadixHistThreads);
    __shared__ uint32_t h[256];
    const int t = threadIdx.x;
    const RadixSegTile st = sg.tiles[blockIdx.x];
    const RadixSegInfo si = sg.segs[st.seg];
    const BatchMesh& d = desc[st.seg];
    uint32_t key[kHI];
#pragma unroll
    for (int it = 0; it < kHI; ++it) {
        const int j = it * kRadixHistThreads + t;
        key[it] = 0u;
        if (j < st.count) {
            const int64_t i = st.start + j;
            key[it] = morton30(q[3 * i], q[3 * i + 1], q[3 * i + 2], d.mlo[0], d.mlo[1], d.mlo[2], d.msc[0],
                               d.msc[1], d.msc[2]) >> 6;
            keys[i] = key[it];
        }
    }
    if (t < 256) h[t] = 0;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kHI; ++it) radix_hist_add(h, key[it] & 255u, it * kRadixHistThreads + t < st.count);
    __syncthreads();
    if (t < 256) counts[si.base + (int64_t)t * si.cols + st.j] = h[t];
}

// Write-out of the batch's 16-byte records (prim, staged point) in input
// order: the closest point and distance (staged_point, as the query kernel
// forms them) are rebuilt from q; for the status (outside the domain box,
// non-finite), row i belongs to the last mesh whose query range starts at
// or before it (empty ranges are skipped that way).
__global__ __launch_bounds__(256) void k_batch_split(const float4* __restrict__ stage, const float* __restrict__ q,
                                                     int64_t n, const RadixSegInfo* __restrict__ segs, int32_t nseg,
                                                     const BatchMesh* __restrict__ desc, int32_t* __restrict__ prim,
                                                     float* __restrict__ closest, float* __restrict__ dist,
                                                     uint8_t* __restrict__ status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 a = stage[i];
    const float qx = q[3 * i], qy = q[3 * i + 1], qz = q[3 * i + 2];
    const int32_t pr = __float_as_int(a.x);
    float cx, cy, cz, dd;
    staged_point(pr, a.y, a.z, a.w, qx, qy, qz, cx, cy, cz, dd);
    prim[i] = pr;
    closest[3 * i] = cx;
    closest[3 * i + 1] = cy;
    closest[3 * i + 2] = cz;
    dist[i] = dd;
    if (status) {
        int32_t lo = 0, hi = nseg - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (segs[mid].start <= i) lo = mid;
            else hi = mid - 1;
        }
        const BatchMesh& d = desc[lo];
        const bool out = qx < d.dlo[0] || qy < d.dlo[1] || qz < d.dlo[2] || qx > d.dhi[0] || qy > d.dhi[1] ||
                         qz > d.dhi[2];
        status[i] = finite3(qx, qy, qz) ? (out ? 1 : 0) : 2;
    }
}

__global__ void k_reset(uint32_t* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] = 0u;
}

// Arena arrays of a batch, passed by value to the kernel.
struct Arena {
    const KdNode* node;
    const uint4* vhead;
    const uint4* lent;
    const float4* seg;
    const float4* tri;
    const int32_t* fedge;
    const uint32_t* nboff;
    const float4* nbrec;
    const float4* seed;
    const float4* frec;
    const float4* erec;
    const BatchMesh* desc;
};

// Queries regrouped by list length together (regroup.hpp): `group` rounds
// of a tile, at most kRegroupSlots queries.
constexpr int kRegroupSlots = 256;
int regroup_rounds(int block, int qpl) { return std::max(1, std::min(qpl, kRegroupSlots / block)); }
// Dynamic LDS: the bins, then per slot 7 floats (q, the nearest vertex's d2
// and position) and 4 ints (query index, vertex, bin and rank, source slot).
size_t batch_slots_bytes(int block, int qpl) {
    return sizeof(uint32_t) * (kRegroupBins + 11 * (size_t)block * (size_t)regroup_rounds(block, qpl));
}
// the regroup slots, then each wavefront's scan rings (keys and owners, ids),
// then (traversal 1) the tile's mesh's top tree levels
size_t batch_lds_bytes(int block, int qpl, int32_t ntop_max) {
    return (batch_slots_bytes(block, qpl) + 15) / 16 * 16 +
           (sizeof(WaveScanKeys) + sizeof(WaveScanIds)) * (size_t)(block / 64) + sizeof(KdNode) * (size_t)ntop_max;
}

// One-workgroup-per-tile order: the tiles are dealt to the 8 XCDs
// (workgroups go to them round-robin) in runs of kTileRun consecutive tiles,
// so a run of one mesh's spatially adjacent tiles shares an L2; the grid is
// a multiple of 8 * kTileRun and workgroups past the list exit at once.
constexpr int64_t kTileRun = 16;
// Persistent schedule: tiles a workgroup claims with one counter increment.
constexpr int64_t kTileChunk = 16;
// Tree levels the per-lane search may stage in LDS (511 nodes, 32 KB).
constexpr int kBatchMaxLdsLevels = 9;
__device__ __forceinline__ int64_t run_tile(int64_t b) {
    const int64_t sg = b / (kXcds * kTileRun), r = b % (kXcds * kTileRun);
    return sg * kXcds * kTileRun + (r % kXcds) * kTileRun + r / kXcds;
}

template <int kWalk, bool kPersistent>
__device__ __forceinline__ void batch_query(Arena A, const Tile* __restrict__ tiles, int64_t ntiles,
                                            uint32_t* counter, int qpl, int group, const float* __restrict__ q,
                                            const int32_t* __restrict__ perm, int64_t n,
                                            float4* __restrict__ stage, int32_t ntop_max) {
    extern __shared__ uint32_t lds[];
    __shared__ int64_t s_tile;
    const int t = threadIdx.x, B = blockDim.x;
    const int S = B * group;
    uint32_t* hist = lds;
    float* col = (float*)(lds + kRegroupBins);  // qx qy qz d2 px py pz, S each
    int32_t* icol = (int32_t*)(col + 7 * S);    // query index, vertex, bin << 24 | rank, source slot
    char* const scan_lds = (char*)lds + ((kRegroupBins + 11 * (size_t)S) * sizeof(uint32_t) + 15) / 16 * 16;
    WaveScanLds ring;
    ring.k = reinterpret_cast<WaveScanKeys*>(scan_lds) + (t >> 6);
    ring.i = reinterpret_cast<WaveScanIds*>(scan_lds + sizeof(WaveScanKeys) * (size_t)(B / 64)) + (t >> 6);
    KdNode* const staged =
        reinterpret_cast<KdNode*>(scan_lds + (sizeof(WaveScanKeys) + sizeof(WaveScanIds)) * (size_t)(B / 64));
    int64_t next = 0, chunk_end = 0;  // persistent: the claimed tiles not yet taken
    for (bool more = true; more;) {
        int64_t tt = run_tile(blockIdx.x);  // one tile per workgroup
        more = false;
        if (kPersistent) {
            // tiles are claimed kTileChunk at a time: one counter increment
            // per chunk rather than per tile
            if (next >= chunk_end) {
                if (t == 0) s_tile = (int64_t)atomicAdd(counter, (uint32_t)kTileChunk);
                __syncthreads();
                // the same for every lane: kept in scalar registers, with the
                // mesh view derived from it
                next = (int64_t)__builtin_amdgcn_readfirstlane((int)s_tile);
                chunk_end = next + kTileChunk;
                __syncthreads();
            }
            tt = next++;
            more = true;
        }
        if (tt >= ntiles) break;  // uniform across the workgroup
        const Tile T = tiles[tt];
        const MeshView v = arena_view(A.desc[T.mesh], A.node, A.vhead, A.lent, A.seg, A.tri, A.fedge, A.nboff, A.nbrec,
                                      A.seed, A.frec, A.erec);
        // the per-lane tree search reads the top of this mesh's tree from
        // LDS (the previous tile's readers have passed the barrier that ends
        // its last round)
        const KdNode* top = nullptr;
        int32_t ntop = 0;
        if (kWalk == WALK_LANE && ntop_max > 0) {
            ntop = min(ntop_max, v.nv);
            stage_top(v.node, ntop, staged);
            __syncthreads();
            top = staged;
        }
        for (int r0 = 0; r0 < qpl; r0 += group) {
            const int rounds = min(group, qpl - r0);
            if (t < kRegroupBins) hist[t] = 0;
            __syncthreads();
            // nearest vertex of each query of these rounds, kept in LDS
            for (int r = 0; r < rounds; ++r) {
                const int64_t local = (int64_t)(r0 + r) * B + t;
                const int64_t j = (int64_t)T.start + local;
                int64_t i = (local < T.count && j < n) ? (int64_t)perm[j] : -1;
                if (i >= n) i = -1;
                float qx = 0.f, qy = 0.f, qz = 0.f;
                if (i >= 0) {
                    qx = q[3 * i];
                    qy = q[3 * i + 1];
                    qz = q[3 * i + 2];
                }
                const bool fin = finite3(qx, qy, qz);
                ScanCounters c;
                // every lane of the wavefront calls this (see nearest_vertex)
                const Nearest nv = nearest_vertex<kWalk>(v, qx, qy, qz, i >= 0 && fin, c.nodes, c.steps, top, ntop);
                const int bin = (i >= 0 && fin) ? regroup_bin(v, nv.vid) : 0;
                const uint32_t rank = atomicAdd(&hist[bin], 1u);
                const int u = r * B + t;
                col[u] = qx;
                col[S + u] = qy;
                col[2 * S + u] = qz;
                col[3 * S + u] = nv.d2;
                col[4 * S + u] = nv.px;
                col[5 * S + u] = nv.py;
                col[6 * S + u] = nv.pz;
                icol[u] = (int32_t)i;
                icol[S + u] = nv.vid;
                icol[2 * S + u] = (int32_t)(((uint32_t)bin << 24) | rank);
            }
            __syncthreads();
            regroup_scan(hist);
            __syncthreads();
            for (int r = 0; r < rounds; ++r) {
                const int u = r * B + t;
                const uint32_t br = (uint32_t)icol[2 * S + u];
                const uint32_t bin = br >> 24;
                icol[3 * S + (bin ? hist[bin - 1] : 0u) + (br & 0xffffffu)] = u;
            }
            __syncthreads();
            // the list scan, lanes taking the queries in list-length order
            for (int r = 0; r < rounds; ++r) {
                const int u = icol[3 * S + r * B + t];
                const int64_t i = icol[u];
                const float qx = col[u], qy = col[S + u], qz = col[2 * S + u];
                Nearest nv;
                nv.d2 = col[3 * S + u];
                nv.px = col[4 * S + u];
                nv.py = col[5 * S + u];
                nv.pz = col[6 * S + u];
                nv.vid = icol[S + u];
                ScanCounters c;
                const bool fin = finite3(qx, qy, qz);
                // every lane of the wavefront takes part in the scan
                float best;
                int best_kind;
                int32_t best_id;
                wave_scan(v, ring, i >= 0 && fin, qx, qy, qz, nv, best, best_kind, best_id, c);
                if (i < 0) continue;
                const Answer a = fin ? finish_answer(v, qx, qy, qz, nv, best, best_kind, best_id, c) : nonfinite_answer();
                // one 16-byte record per query, (prim, closest point); the
                // write-out (k_batch_split) rebuilds the distance and status
                stage[i] = make_float4(__int_as_float(a.prim), a.sx, a.sy, a.sz);
            }
            __syncthreads();  // the slots are refilled by the next rounds or tile
        }
    }
}

// The tree-walk forms (traversals 1 and 2).
template <int kWalk, bool kPersistent>
__global__ __launch_bounds__(kQueryMaxBlock) void k_batch_query(Arena A, const Tile* __restrict__ tiles,
                                                                int64_t ntiles, uint32_t* counter, int qpl,
                                                                int group, const float* __restrict__ q,
                                                                const int32_t* __restrict__ perm, int64_t n,
                                                                float4* __restrict__ stage, int32_t ntop_max) {
    batch_query<kWalk, kPersistent>(A, tiles, ntiles, counter, qpl, group, q, perm, n, stage, ntop_max);
}

// The Voronoi-walk forms (the default traversal), held to 80 registers so
// that six wavefronts fit on each SIMD.
__global__ __launch_bounds__(kQueryMaxBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_batch_query_walk(
    Arena A, const Tile* __restrict__ tiles, int64_t ntiles, uint32_t* counter, int qpl, int group,
    const float* __restrict__ q, const int32_t* __restrict__ perm, int64_t n, float4* __restrict__ stage,
    int32_t ntop_max) {
    batch_query<WALK_VORONOI, false>(A, tiles, ntiles, counter, qpl, group, q, perm, n, stage, ntop_max);
}
// The persistent form: its tile loop needs more registers; held to 96
// (five wavefronts a SIMD), where it does not spill.
__global__ __launch_bounds__(kQueryMaxBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_query_walk_persistent(
    Arena A, const Tile* __restrict__ tiles, int64_t ntiles, uint32_t* counter, int qpl, int group,
    const float* __restrict__ q, const int32_t* __restrict__ perm, int64_t n, float4* __restrict__ stage,
    int32_t ntop_max) {
    batch_query<WALK_VORONOI, true>(A, tiles, ntiles, counter, qpl, group, q, perm, n, stage, ntop_max);
}

// Tree nodes the batched kernel stages per tile: traversal 1 only.
int32_t batch_top_nodes(const p2m_batch* b) {
    return b->traversal == 1 ? top_nodes(b->lds_levels, INT32_MAX) : 0;
}

void drop_graph(p2m_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

p2m_status hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? P2M_ERR_OOM : P2M_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Work buffers and tile list for a query layout and launch shape.
p2m_status prepare(p2m_batch* b, const int64_t* qoff_host, hipStream_t st) {
    std::vector<int64_t> layout(qoff_host, qoff_host + b->count + 1);
    if (layout[0] != 0) return fail(P2M_ERR_ARG, "q_offsets[0] must be 0");
    for (int32_t k = 0; k < b->count; ++k)
        if (layout[(size_t)k + 1] < layout[(size_t)k]) return fail(P2M_ERR_ARG, "q_offsets must be non-decreasing");
    const int64_t n = layout.back();
    if (n > (int64_t)INT32_MAX) return fail(P2M_ERR_ARG, "more than 2^31-1 queries in one batch");
    const bool same_layout = layout == b->layout;
    if (same_layout && b->tile_block == b->block && b->tile_qpl == b->qpl) return P2M_OK;
    drop_graph(b);
    std::vector<RadixSegTile> stiles;
    std::vector<RadixSegInfo> ssegs;
    radix_segment_tiles(layout, stiles, ssegs);
    RadixPlan plan = radix_plan_segmented(std::max<int64_t>(n, 1), (int64_t)stiles.size(), b->count);
    const int64_t b_stiles = up256((int64_t)sizeof(RadixSegTile) * std::max<size_t>(1, stiles.size()));
    const int64_t b_ssegs = up256((int64_t)sizeof(RadixSegInfo) * std::max<size_t>(1, ssegs.size()));
    const int64_t tsize = (int64_t)b->block * b->qpl;
    std::vector<int64_t> order((size_t)b->count);
    std::iota(order.begin(), order.end(), 0);
    // most work first: queries x log(vertices)
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
        double wx = (double)(layout[(size_t)x + 1] - layout[(size_t)x]) * b->cost[(size_t)x];
        double wy = (double)(layout[(size_t)y + 1] - layout[(size_t)y]) * b->cost[(size_t)y];
        return wx > wy;
    });
    std::vector<Tile> tiles;
    for (int64_t k : order)
        for (int64_t s = layout[(size_t)k]; s < layout[(size_t)k + 1]; s += tsize)
            tiles.push_back(Tile{(int32_t)k, (int32_t)s, (int32_t)std::min(tsize, layout[(size_t)k + 1] - s), 0});
    const int64_t need = up256((int64_t)sizeof(Tile) * std::max<size_t>(1, tiles.size())) + 256 + b_stiles + b_ssegs +
                         up256(plan.bytes) + 16 * std::max<int64_t>(n, 1);
    if (need > b->work_bytes) {
        if (b->work) (void)hipFree(b->work);
        b->work = nullptr;
        b->work_bytes = 0;
        hipError_t e = hipMalloc(&b->work, (size_t)need);
        if (e != hipSuccess) return hip_fail(e, "batch work buffers");
        b->work_bytes = need;
    }
    char* p = (char*)b->work;
    b->tiles = (Tile*)p;
    p += up256((int64_t)sizeof(Tile) * std::max<size_t>(1, tiles.size()));
    b->counter = (uint32_t*)p;
    p += 256;
    b->sort_seg.tiles = (const RadixSegTile*)p;
    p += b_stiles;
    b->sort_seg.segs = (const RadixSegInfo*)p;
    p += b_ssegs;
    b->sort_seg.ntiles = (int64_t)stiles.size();
    b->sort_seg.nseg = (int32_t)ssegs.size();
    b->scratch = p;
    p += up256(plan.bytes);
    b->stage = (float4*)p;
    hipError_t e = hipSuccess;
    if (!tiles.empty())
        e = hipMemcpyAsync(b->tiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !stiles.empty())
        e = hipMemcpyAsync((void*)b->sort_seg.tiles, stiles.data(), sizeof(RadixSegTile) * stiles.size(),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !ssegs.empty())
        e = hipMemcpyAsync((void*)b->sort_seg.segs, ssegs.data(), sizeof(RadixSegInfo) * ssegs.size(),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // host staging goes out of scope
    if (e != hipSuccess) return hip_fail(e, "batch layout upload");
    b->layout = layout;
    b->n = n;
    b->ntiles = (int64_t)tiles.size();
    b->tile_block = b->block;
    b->tile_qpl = b->qpl;
    return P2M_OK;
}

// Enqueue the whole batched query (keys, sort, counter reset, persistent
// kernel, write-out of the staged answers).
p2m_status enqueue(p2m_batch* b, const float* q, int32_t* prim, float* closest, float* dist, uint8_t* status,
                   hipStream_t st) {
    const int64_t n = b->n;
    if (n == 0) return P2M_OK;
    RadixPlan plan = radix_plan_segmented(n, b->sort_seg.ntiles, b->sort_seg.nseg);
    RadixBuffers rb = radix_buffers(plan, b->scratch);
    k_batch_keys<<<(unsigned)b->sort_seg.ntiles, kRadixHistThreads, 0, st>>>(q, b->desc, b->sort_seg, rb.keys[0],
                                                                          rb.counts);
    const int cur = radix_sort_pairs(plan, rb, 0, 24, false, st, &b->sort_seg, true);
    k_reset<<<1, 64, 0, st>>>(b->counter);
    const int64_t run8 = kXcds * kTileRun;
    const int grid = b->persistent ? b->grid : (int)((b->ntiles + run8 - 1) / run8 * run8);
    const Arena A{b->node,  b->vhead, b->lent, b->seg,  b->tri,  b->fedge,
                  b->nboff, b->nbrec, b->seed, b->frec, b->erec, b->desc};
    const int32_t ntop_max = batch_top_nodes(b);
#define P2M_LAUNCH_BATCH(K)                                                                                   \
    K<<<grid, b->block, batch_lds_bytes(b->block, b->qpl, ntop_max), st>>>(A, b->tiles, b->ntiles, b->counter,   \
                                                                         b->qpl, regroup_rounds(b->block, b->qpl), \
                                                                         q, rb.vals[cur], n, b->stage, ntop_max)
    if (b->persistent) {
        if (b->traversal == 1) P2M_LAUNCH_BATCH((k_batch_query<WALK_LANE, true>));
        else if (b->traversal == 2) P2M_LAUNCH_BATCH((k_batch_query<WALK_WAVE, true>));
        else P2M_LAUNCH_BATCH(k_batch_query_walk_persistent);
    } else {
        if (b->traversal == 1) P2M_LAUNCH_BATCH((k_batch_query<WALK_LANE, false>));
        else if (b->traversal == 2) P2M_LAUNCH_BATCH((k_batch_query<WALK_WAVE, false>));
        else P2M_LAUNCH_BATCH(k_batch_query_walk);
    }
#undef P2M_LAUNCH_BATCH
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batched query launch");
    k_batch_split<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(b->stage, q, n, b->sort_seg.segs, b->sort_seg.nseg,
                                                              b->desc, prim, closest, dist, status);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batched answer write-out");
    return P2M_OK;
}

p2m_status set_grid(p2m_batch* b) {
    int dev = b->device, cus = 0, per = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device attribute");
    const void* k = b->traversal == 1   ? (const void*)k_batch_query<WALK_LANE, true>
                    : b->traversal == 2 ? (const void*)k_batch_query<WALK_WAVE, true>
                                        : (const void*)k_batch_query_walk_persistent;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, b->block,
                                                     batch_lds_bytes(b->block, b->qpl, batch_top_nodes(b)));
    if (e != hipSuccess) return hip_fail(e, "occupancy query");
    b->grid = std::max(1, cus * std::max(1, per));
    return P2M_OK;
}

struct Guard {
    int old = -1;
    explicit Guard(int dev) {
        if (hipGetDevice(&old) != hipSuccess) old = -1;
        (void)hipSetDevice(dev);
    }
    ~Guard() {
        if (old >= 0) (void)hipSetDevice(old);
    }
};

}  // namespace

}  // namespace p2m

using namespace p2m;

extern "C" {

p2m_status p2m_batch_create(p2m_mesh* const* meshes, int32_t count, int device, void* stream, p2m_batch** out) {
    if (!out) return fail(P2M_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!meshes || count < 1) return fail(P2M_ERR_ARG, "need at least one mesh");
    // the segmented sort scans 256 digit columns per mesh, one workgroup each
    if (count > (1 << 20)) return fail(P2M_ERR_ARG, "more than 2^20 meshes in one batch");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(P2M_ERR_HIP, "no HIP device");
    if (device < 0 || device >= ndev) return fail(P2M_ERR_ARG, "device index out of range");
    for (int32_t k = 0; k < count; ++k) {
        if (!meshes[k]) return fail(P2M_ERR_ARG, "NULL mesh in the batch");
        if (!meshes[k]->s.precomputed) return fail(P2M_ERR_STATE, "batch mesh not precomputed");
    }
    Guard g(device);
    p2m_batch* b = new p2m_batch();
    b->device = device;
    b->count = count;
    // host staging of the arena
    std::vector<float> node, seg, tri, nbrec, frec, erec;
    std::vector<uint32_t> vhead, nboff;
    std::vector<uint32_t> lent;
    std::vector<int32_t> fedge;
    int64_t seeds = 0;
    std::vector<BatchMesh> desc((size_t)count);
    b->cost.resize((size_t)count);
    for (int32_t k = 0; k < count; ++k) {
        MeshState& s = meshes[k]->s;
        pack_mesh(s);
        BatchMesh& d = desc[(size_t)k];
        d.node = (int64_t)node.size() / 16;
        d.head = (int64_t)vhead.size() / 4;
        d.ent = (int64_t)lent.size() / 4;  // uint4 elements (two entries each)
        d.seg = (int64_t)seg.size() / 4;
        d.tri = (int64_t)tri.size() / 4;
        d.fedge = (int64_t)fedge.size();
        d.nboff = (int64_t)nboff.size();
        d.nbrec = (int64_t)nbrec.size() / 4;
        d.seed = seeds;
        d.frec = (int64_t)frec.size() / 4;
        d.erec = (int64_t)erec.size() / 4;
        d.nv = (int32_t)s.m.nv;
        const MeshView hv = host_view(s);
        d.grid = hv.grid;
        seeds += (int64_t)hv.grid * hv.grid * hv.grid;
        float lo[3], sc[3];
        morton_params(s.dlo, s.dhi, lo, sc);
        for (int c = 0; c < 3; ++c) {
            d.dlo[c] = hv.dlo[c];
            d.dhi[c] = hv.dhi[c];
            d.mlo[c] = lo[c];
            d.msc[c] = sc[c];
            d.gscale[c] = hv.gscale[c];
            d.ctr[c] = hv.ctr[c];
            d.qlo[c] = hv.qlo[c];
            d.qs[c] = hv.qs[c];
        }
        d.mu = hv.mu;
        d.eta = hv.eta;
        node.insert(node.end(), s.pk_node.begin(), s.pk_node.end());
        vhead.insert(vhead.end(), s.pk_vhead.begin(), s.pk_vhead.end());
        lent.insert(lent.end(), s.pk_lent.begin(), s.pk_lent.end());
        seg.insert(seg.end(), s.pk_seg.begin(), s.pk_seg.end());
        tri.insert(tri.end(), s.pk_tri.begin(), s.pk_tri.end());
        fedge.insert(fedge.end(), s.pk_fedge.begin(), s.pk_fedge.end());
        nboff.insert(nboff.end(), s.pk_nboff.begin(), s.pk_nboff.end());
        nbrec.insert(nbrec.end(), s.pk_nbrec.begin(), s.pk_nbrec.end());
        frec.insert(frec.end(), s.pk_frec.begin(), s.pk_frec.end());
        erec.insert(erec.end(), s.pk_erec.begin(), s.pk_erec.end());
        b->cost[(size_t)k] = std::log2((double)s.m.nv + 2.0);
    }
    if (lent.size() / 4 >= (size_t)UINT32_MAX || nbrec.size() / 4 >= (size_t)UINT32_MAX) {
        delete b;
        return fail(P2M_ERR_ARG, "batch tables exceed 2^32 entries");
    }
    constexpr int kArrays = 12;
    const size_t sizes[kArrays] = {4 * node.size(), 4 * vhead.size(), 4 * std::max<size_t>(4, lent.size()),
                                   4 * seg.size(), 4 * tri.size(), 4 * fedge.size(), sizeof(BatchMesh) * desc.size(),
                                   4 * nboff.size(), 4 * std::max<size_t>(4, nbrec.size()),
                                   4 * frec.size(), 4 * std::max<size_t>(4, erec.size()), 16 * (size_t)seeds};
    size_t total = 0;
    for (size_t x : sizes) total += (size_t)up256((int64_t)x);
    hipError_t e = hipMalloc(&b->base, total);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "batch arena");
    }
    b->bytes = (int64_t)total;
    char* p = (char*)b->base;
    void* dst[kArrays];
    for (int i = 0; i < kArrays; ++i) {
        dst[i] = p;
        p += up256((int64_t)sizes[i]);
    }
    b->node = (KdNode*)dst[0];
    b->vhead = (uint4*)dst[1];
    b->lent = (uint4*)dst[2];
    b->seg = (float4*)dst[3];
    b->tri = (float4*)dst[4];
    b->fedge = (int32_t*)dst[5];
    b->desc = (BatchMesh*)dst[6];
    b->nboff = (uint32_t*)dst[7];
    b->nbrec = (float4*)dst[8];
    b->frec = (float4*)dst[9];
    b->erec = (float4*)dst[10];
    b->seed = (float4*)dst[11];
    // the seed grids (last array) are filled on the device below
    const void* src[kArrays - 1] = {node.data(),  vhead.data(), lent.data(), seg.data(),  tri.data(), fedge.data(),
                                    desc.data(), nboff.data(), nbrec.data(), frec.data(), erec.data()};
    const size_t nbytes[kArrays - 1] = {sizes[0], sizes[1], 4 * lent.size(), sizes[3], sizes[4],  sizes[5],
                                        sizes[6], sizes[7], 4 * nbrec.size(), sizes[9], 4 * erec.size()};
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < kArrays - 1 && e == hipSuccess; ++i)
        if (nbytes[i]) e = hipMemcpyAsync(dst[i], src[i], nbytes[i], hipMemcpyHostToDevice, st);
    for (int32_t k = 0; k < count && e == hipSuccess; ++k)
        e = launch_seed_grid(arena_view(desc[(size_t)k], b->node, b->vhead, b->lent, b->seg, b->tri, b->fedge, b->nboff,
                                        b->nbrec, b->seed, b->frec, b->erec),
                             b->seed + desc[(size_t)k].seed, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // staging vectors are local
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        p2m_batch_destroy(b);
        return hip_fail(e, "batch upload");
    }
    p2m_status r = set_grid(b);
    if (r != P2M_OK) {
        p2m_batch_destroy(b);
        return r;
    }
    *out = b;
    return P2M_OK;
}

void p2m_batch_destroy(p2m_batch* b) {
    if (!b) return;
    Guard g(b->device);
    drop_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->work) (void)hipFree(b->work);
    if (b->base) (void)hipFree(b->base);
    delete b;
}

p2m_status p2m_batch_set_shape(p2m_batch* b, int block, int qpl, int traversal) {
    if (!b) return fail(P2M_ERR_ARG, "batch is NULL");
    if (block < 64 || block > kQueryMaxBlock || block % 64) return fail(P2M_ERR_ARG, "block must be 64, 128, 192 or 256");
    if (qpl < 1 || qpl > 16) return fail(P2M_ERR_ARG, "queries per lane must be in [1, 16]");
    if (traversal < 1 || traversal > 3) return fail(P2M_ERR_ARG, "traversal must be 1, 2 or 3");
    Guard g(b->device);
    if (b->block != block || b->qpl != qpl || b->traversal != traversal) drop_graph(b);
    b->block = block;
    b->qpl = qpl;
    b->traversal = traversal;
    return set_grid(b);
}

p2m_status p2m_batch_get_shape(const p2m_batch* b, int* block, int* qpl, int* traversal) {
    if (!b) return fail(P2M_ERR_ARG, "batch is NULL");
    if (block) *block = b->block;
    if (qpl) *qpl = b->qpl;
    if (traversal) *traversal = b->traversal;
    return P2M_OK;
}

p2m_status p2m_batch_set_lds_levels(p2m_batch* b, int levels) {
    if (!b) return fail(P2M_ERR_ARG, "batch is NULL");
    if (levels < 0 || levels > kBatchMaxLdsLevels) return fail(P2M_ERR_ARG, "lds levels must be in [0, 9]");
    Guard g(b->device);
    if (b->lds_levels != levels) drop_graph(b);
    b->lds_levels = levels;
    return set_grid(b);
}

p2m_status p2m_batch_get_lds_levels(const p2m_batch* b, int* levels) {
    if (!b) return fail(P2M_ERR_ARG, "batch is NULL");
    if (levels) *levels = b->lds_levels;
    return P2M_OK;
}

p2m_status p2m_batch_set_schedule(p2m_batch* b, int persistent) {
    if (!b) return fail(P2M_ERR_ARG, "batch is NULL");
    if (persistent != 0 && persistent != 1) return fail(P2M_ERR_ARG, "persistent must be 0 or 1");
    if (b->persistent != persistent) drop_graph(b);
    b->persistent = persistent;
    return P2M_OK;
}

p2m_status p2m_batch_get_schedule(const p2m_batch* b, int* persistent) {
    if (!b) return fail(P2M_ERR_ARG, "batch is NULL");
    if (persistent) *persistent = b->persistent;
    return P2M_OK;
}

p2m_status p2m_batch_query(p2m_batch* b, const float* q, const int64_t* qoff, int32_t* prim, float* closest,
                           float* dist, uint8_t* status, void* stream) {
    if (!b) return fail(P2M_ERR_ARG, "batch is NULL");
    if (!qoff) return fail(P2M_ERR_ARG, "q_offsets is NULL");
    Guard g(b->device);
    hipStream_t st = (hipStream_t)stream;
    p2m_status r = prepare(b, qoff, st);
    if (r != P2M_OK) return r;
    if (b->n == 0) return P2M_OK;
    if (!q || !prim || !closest || !dist) return fail(P2M_ERR_ARG, "NULL query or output pointer");
    const void* ptrs[5] = {q, prim, closest, dist, status};
    const int shape[4] = {b->block, b->qpl, b->traversal, batch_top_nodes(b)};
    if (!b->exec || std::memcmp(ptrs, b->g_ptrs, sizeof(ptrs)) != 0 || std::memcmp(shape, b->g_shape, sizeof(shape)) != 0) {
        drop_graph(b);
        hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "graph capture begin");
        r = enqueue(b, q, prim, closest, dist, status, b->cap_stream);
        hipGraph_t gr = nullptr;
        e = hipStreamEndCapture(b->cap_stream, &gr);
        if (r != P2M_OK) {
            if (gr) (void)hipGraphDestroy(gr);
            return r;
        }
        if (e != hipSuccess) return hip_fail(e, "graph capture end");
        b->graph = gr;
        e = hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(b);
            return hip_fail(e, "graph instantiate");
        }
        std::memcpy(b->g_ptrs, ptrs, sizeof(ptrs));
        std::memcpy(b->g_shape, shape, sizeof(shape));
    }
    hipError_t e = hipGraphLaunch(b->exec, st);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return P2M_OK;
}

p2m_status p2m_batch_order_queries(p2m_batch* b, const float* q, const int64_t* qoff, uint32_t* keys_out,
                                   int32_t* perm_out, void* stream) {
    if (!b) return fail(P2M_ERR_ARG, "batch is NULL");
    if (!qoff) return fail(P2M_ERR_ARG, "q_offsets is NULL");
    Guard g(b->device);
    hipStream_t st = (hipStream_t)stream;
    p2m_status r = prepare(b, qoff, st);
    if (r != P2M_OK) return r;
    const int64_t n = b->n;
    if (n == 0) return P2M_OK;
    if (!q || !keys_out || !perm_out) return fail(P2M_ERR_ARG, "NULL query or output pointer");
    RadixPlan plan = radix_plan_segmented(n, b->sort_seg.ntiles, b->sort_seg.nseg);
    RadixBuffers rb = radix_buffers(plan, b->scratch);
    k_batch_keys<<<(unsigned)b->sort_seg.ntiles, kRadixHistThreads, 0, st>>>(q, b->desc, b->sort_seg, rb.keys[0],
                                                                          rb.counts);
    const int cur = radix_sort_pairs(plan, rb, 0, 24, true, st, &b->sort_seg, true);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(keys_out, rb.keys[cur], sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(perm_out, rb.vals[cur], sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "batch ordering");
    return P2M_OK;
}

p2m_status p2m_batch_query_eager(p2m_batch* b, const float* q, const int64_t* qoff, int32_t* prim, float* closest,
                                 float* dist, uint8_t* status, void* stream) {
    if (!b) return fail(P2M_ERR_ARG, "batch is NULL");
    if (!qoff) return fail(P2M_ERR_ARG, "q_offsets is NULL");
    Guard g(b->device);
    hipStream_t st = (hipStream_t)stream;
    p2m_status r = prepare(b, qoff, st);
    if (r != P2M_OK) return r;
    if (b->n == 0) return P2M_OK;
    if (!q || !prim || !closest || !dist) return fail(P2M_ERR_ARG, "NULL query or output pointer");
    return enqueue(b, q, prim, closest, dist, status, st);
}

p2m_status p2m_batch_autotune(p2m_batch* b, const float* q, const int64_t* qoff, int32_t* prim, float* closest,
                              float* dist, void* stream, int* best_block, int* best_qpl, int* best_traversal) {
    if (!b) return fail(P2M_ERR_ARG, "batch is NULL");
    Guard g(b->device);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(P2M_ERR_HIP, "hipEventCreate");
    const int blocks[3] = {64, 128, 256};
    const int qpls[3] = {1, 2, 4};
    const int travs[3] = {1, 2, 3};
    const int levels[2] = {0, 8};  // staged tree levels, traversal 1 only
    float best = INFINITY;
    int bb = b->block, bq = b->qpl, bt = b->traversal, bv = b->lds_levels;
    p2m_status r = P2M_OK;
    // every (traversal, levels, block, queries per lane); the first error ends the sweep
    for (int k = 0; k < 3 * 2 * 3 * 3 && r == P2M_OK; ++k) {
        const int tv = travs[k / 18], lv = levels[(k / 9) % 2], bl = blocks[(k / 3) % 3], qp = qpls[k % 3];
        if (tv != 1 && lv != 0) continue;
        if ((r = p2m_batch_set_lds_levels(b, lv)) != P2M_OK) break;
        if ((r = p2m_batch_set_shape(b, bl, qp, tv)) != P2M_OK) break;
        float tot = 0.f;
        for (int rep = 0; rep < 3 && r == P2M_OK; ++rep) {
            (void)hipEventRecord(e0, st);
            r = p2m_batch_query_eager(b, q, qoff, prim, closest, dist, nullptr, stream);
            (void)hipEventRecord(e1, st);
            float ms = 0.f;
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                r = fail(P2M_ERR_HIP, "autotune timing");
            if (rep > 0) tot += ms;  // first run warms caches
        }
        if (r == P2M_OK && tot < best) {
            best = tot;
            bb = bl;
            bq = qp;
            bt = tv;
            bv = lv;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != P2M_OK) return r;
    r = p2m_batch_set_lds_levels(b, bv);
    if (r == P2M_OK) r = p2m_batch_set_shape(b, bb, bq, bt);
    if (best_block) *best_block = bb;
    if (best_qpl) *best_qpl = bq;
    if (best_traversal) *best_traversal = bt;
    return r;
}

}  // extern "C"
