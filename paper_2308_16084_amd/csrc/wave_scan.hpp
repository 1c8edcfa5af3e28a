// Wavefront-cooperative list scan (step 3 of the query, Algorithm A.2) for
// the query kernels (device only).
//
// Each lane tests the entry boxes of its own list (Sec. 4.6), four entries
// a step, as the one-query scan does.  The entries whose box holds the
// lane's query are not evaluated there: they go to a ring of the wavefront
// in LDS (one ring for edges, one for faces), and whenever a ring holds two
// wavefronts' worth of candidates, all 64 lanes evaluate 128 of them, two
// each with both loads in flight, each for its owner's query (read from the
// owner lane), and fold the gated value into the owner's minimum with an LDS
// atomic min on the key (value bits, kind, id).  So the forms are evaluated
// with every lane busy, however the hits fall across the lanes, instead of
// once per slot for the whole wavefront whenever any lane hits in it.  The
// least key is the least (value, kind, id) -- vertex before edge before
// face, ids ascending -- the winner of the one-query scan in list order, so
// the answers are those of scan_list.
#pragma once

#include <hip/hip_runtime.h>

#include "query_core.hpp"

namespace p2m {

// Candidates a ring holds: an evaluation takes 128 once a ring holds that
// many, and a slot appends at most 64, so a ring never holds more than 191.
constexpr int kRing = 256;
constexpr uint32_t kEval = 128;
constexpr int kStep = 4;  // entries a lane tests per step

// LDS of one wavefront, in two parts: the owners and the keys (1,024 bytes,
// 8-byte aligned; the query kernels put them in the wavefront's regroup
// slots, free after the regroup), and the candidate ids (2,048 bytes).
struct WaveScanKeys {
    unsigned long long best[64];  // per lane: least key so far
    uint8_t eown[kRing], fown[kRing];
};
struct WaveScanIds {
    uint32_t eid[kRing], fid[kRing];
};

struct WaveScanLds {
    WaveScanKeys* k;
    WaveScanIds* i;
};

__device__ __forceinline__ unsigned long long cand_key(float d, int kind, int32_t id) {
    return ((unsigned long long)__float_as_uint(d) << 32) | (((uint32_t)kind << 30) | (uint32_t)id);
}

// Evaluates up to kEval candidates from the head of a ring, two per lane,
// for their owners' queries; all lanes of the wavefront call it.
template <bool kFace>
__device__ __forceinline__ void ring_eval(const MeshView& m, WaveScanLds L, uint32_t& head, uint32_t& count,
                                          float rx, float ry, float rz, int lane) {
    const uint32_t n = count < kEval ? count : kEval;
    uint32_t id[2];
    int o[2];
    bool mine[2];
    float ox[2], oy[2], oz[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t j = (uint32_t)lane + 64u * (uint32_t)h;
        const uint32_t slot = (head + j) & (kRing - 1);
        mine[h] = j < n;
        id[h] = kFace ? L.i->fid[slot] : L.i->eid[slot];
        o[h] = mine[h] ? (int)(kFace ? L.k->fown[slot] : L.k->eown[slot]) : lane;
        ox[h] = __shfl(rx, o[h]);
        oy[h] = __shfl(ry, o[h]);
        oz[h] = __shfl(rz, o[h]);
    }
    float g[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        g[h] = INFINITY;
        if (mine[h])
            g[h] = kFace ? face_gate_d2(m, (int32_t)id[h], ox[h], oy[h], oz[h])
                         : edge_gate_d2(m, (int32_t)id[h], ox[h], oy[h], oz[h]);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
        if (g[h] < INFINITY) atomicMin(&L.k->best[o[h]], cand_key(g[h], kFace ? KIND_FACE : KIND_EDGE, (int32_t)id[h]));
    __builtin_amdgcn_wave_barrier();
    head += n;
    count -= n;
}

// One run (edges or faces) of every lane's list: entries [k0, k1) of each
// lane (empty for a lane without a query).
template <bool kFace>
__device__ __forceinline__ void wave_run(const MeshView& m, WaveScanLds L, uint32_t k0, uint32_t k1,
                                         const Cell5& qc, float rx, float ry, float rz, int lane,
                                         ScanCounters& cnt) {
    uint32_t head = 0, count = 0;  // wavefront-uniform
    const unsigned long long below = (1ull << lane) - 1ull;
    for (uint32_t k = k0; __any(k < k1); k += kStep) {
        uint32_t id[kStep], bx[kStep];
        bool hit[kStep];
        // kStep entries, kStep / 2 16-byte loads issued together; a load past
        // the run's end re-reads the first and its slots are discarded
#pragma unroll
        for (int u = 0; u < kStep; u += 2) {
            uint4 A = make_uint4(0u, 0u, 0u, 0u);
            if (k < k1) A = m.lent[(k + u < k1 ? k + u : k) >> 1];
            id[u] = A.x;
            bx[u] = A.y;
            id[u + 1] = A.z;
            bx[u + 1] = A.w;
        }
#pragma unroll
        for (int u = 0; u < kStep; ++u) hit[u] = k + u < k1 && in_box5(bx[u], qc);
#pragma unroll
        for (int u = 0; u < kStep; ++u) {
            if (kFace) cnt.face_forms += hit[u];
            else cnt.edge_forms += hit[u];
            const unsigned long long bal = __ballot(hit[u]);
            if (hit[u]) {
                const uint32_t slot = (head + count + (uint32_t)__popcll(bal & below)) & (kRing - 1);
                if (kFace) {
                    L.i->fid[slot] = id[u];
                    L.k->fown[slot] = (uint8_t)lane;
                } else {
                    L.i->eid[slot] = id[u];
                    L.k->eown[slot] = (uint8_t)lane;
                }
            }
            __builtin_amdgcn_wave_barrier();
            count += (uint32_t)__popcll(bal);
            if (count >= kEval) ring_eval<kFace>(m, L, head, count, rx, ry, rz, lane);
        }
    }
    while (count > 0u) ring_eval<kFace>(m, L, head, count, rx, ry, rz, lane);
}

// Step 3 for every lane of the wavefront (all lanes call it; `active`
// false for a lane without a query): the least (gated value, kind, id)
// over v and v's list, as scan_list finds it.
__device__ __forceinline__ void wave_scan(const MeshView& m, WaveScanLds L, bool active, float qx, float qy,
                                          float qz, const Nearest& nv, float& best, int& best_kind,
                                          int32_t& best_id, ScanCounters& cnt) {
    const int lane = (int)(threadIdx.x & 63u);
    const float rx = qx - m.ctr[0], ry = qy - m.ctr[1], rz = qz - m.ctr[2];
    uint32_t e0 = 0, f0 = 0, f1 = 0;
    Cell5 qc = {0u, 0u};
    if (active) {
        const uint4 h0 = m.vhead[2 * nv.vid], h1 = m.vhead[2 * nv.vid + 1];
        e0 = h0.x;
        f0 = h0.y;
        f1 = h0.z;
        qc = list_cell(m, qx, qy, qz, h1);
    }
    L.k->best[lane] = active ? cand_key(nv.d2, KIND_VERTEX, nv.vid) : ~0ull;
    __builtin_amdgcn_wave_barrier();
    wave_run<false>(m, L, e0, f0, qc, rx, ry, rz, lane, cnt);
    wave_run<true>(m, L, f0, f1, qc, rx, ry, rz, lane, cnt);
    cnt.edges += f0 - e0;
    cnt.faces += f1 - f0;
    const unsigned long long key = L.k->best[lane];
    best = __uint_as_float((uint32_t)(key >> 32));
    best_kind = (int)((uint32_t)key >> 30);
    best_id = (int32_t)((uint32_t)key & 0x3FFFFFFFu);
}

}  // namespace p2m
