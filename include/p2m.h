/*
 * p2m.h -- C interface of the MI355X point-to-mesh (P2M) query library.
 *
 * Method: Zong, Xu, Song, Chen, Xin, Wang, Tu, "P2M: A Fast Solver for
 * Querying Distance from Point to Mesh Surface" (ACM TOG; arXiv 2308.16084).
 * Given a triangle mesh with one copy of each vertex (Sec. 4.1), a host
 * precompute builds a KD tree of the vertices and the interception table
 * (Sec. 4; Appendix, Algorithm A.1).  A query then finds the nearest vertex
 * v with the KD tree and tests v and the edges and faces in v's interception
 * list (Algorithm A.2), returning the closest primitive (vertex, edge or
 * face), the closest point and the distance (Sec. 1).
 *
 * Conventions
 *  - No exceptions cross this interface; every call returns a p2m_status and
 *    p2m_last_error() gives a message for the calling thread's last failure.
 *  - "host" pointers are ordinary CPU memory; "dev" pointers are device
 *    memory on the device the mesh was uploaded to (e.g. torch tensors).
 *    Device buffers passed in are owned by the caller and never freed here.
 *    Mesh and batch handles own their host structures and device arenas;
 *    the *_destroy calls free them.
 *  - Device calls are asynchronous and ordered on the caller's stream
 *    (hipStream_t passed as void*; NULL = the null stream).  They do not
 *    synchronise the host, except where stated.
 *  - Primitive codes: prim = type << 30 | id, with type P2M_VERTEX, P2M_EDGE
 *    or P2M_FACE.  Vertex id = input index, face id = input row, edge id =
 *    rank of the undirected pair (min,max) among all face sides sorted
 *    lexicographically (p2m_mesh_edges lists them).
 *  - All coordinates are float32.  The host precompute runs in float64.
 */
#ifndef P2M_H
#define P2M_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    P2M_OK = 0,
    P2M_ERR_ARG = -1,      /* null pointer, negative count, bad option */
    P2M_ERR_MESH = -2,     /* invalid mesh (see p2m_mesh_create) */
    P2M_ERR_STATE = -3,    /* call out of order (e.g. query before upload) */
    P2M_ERR_OOM = -4,      /* host or device allocation failed */
    P2M_ERR_HIP = -5,      /* a HIP runtime call failed */
    P2M_ERR_INTERNAL = -6, /* unexpected internal failure */
    P2M_ERR_IO = -7        /* file could not be read or written */
} p2m_status;

enum { P2M_VERTEX = 0, P2M_EDGE = 1, P2M_FACE = 2, P2M_NONE = 3 };
#define P2M_PRIM_TYPE(p) ((int32_t)((uint32_t)(p) >> 30))
#define P2M_PRIM_ID(p) ((int32_t)((uint32_t)(p)&0x3FFFFFFFu))

/* per-query status bits */
enum { P2M_Q_OUT_OF_DOMAIN = 1, P2M_Q_NONFINITE = 2 };

typedef struct p2m_mesh p2m_mesh;
typedef struct p2m_batch p2m_batch;

/* Interception-table construction modes. */
enum {
    P2M_TABLE_FLOODING = 0,  /* convexity filter + flooding (Sec. 4.4-4.5) */
    P2M_TABLE_ALL_PAIRS = 1, /* convexity filter on every vertex-primitive pair (tiny meshes) */
    P2M_TABLE_EVERYTHING = 2, /* every primitive in every list (tiny meshes; test aid) */
    /* P2M_TABLE_FLOODING with the filter and flooding (Sec. 4.4-4.5,
     * Algorithm 1: the inspection, the bulk of the preprocessing per
     * Table 2) run on the current HIP device, one primitive per wavefront,
     * in FP64 with the host's operations and their order, so the table and
     * its entry boxes are those of P2M_TABLE_FLOODING.  The Voronoi cells
     * are built on the device too, from the Delaunay neighbours (still
     * computed on the host, with exact predicates), with the host's
     * arithmetic.  A primitive whose polytope outgrows 64 corners or whose
     * flood outgrows the visit limit, and a cell of more than 64 corners or
     * neighbours, are finished on the host.  Blocks until done; uses the null
     * stream.  Needs a HIP device; fails with P2M_ERR_HIP otherwise. */
    P2M_TABLE_FLOODING_DEVICE = 3
};

typedef struct {
    /* Query domain D: the box queries are expected in.  Voronoi cells are
     * clipped to D (the paper bounds them with 8 far virtual points, Sec.
     * 4.3 Remark); answers for queries outside D are valid distances to the
     * mesh but need not be the closest and are flagged P2M_Q_OUT_OF_DOMAIN. */
    double domain_lo[3], domain_hi[3];
    int use_default_domain; /* nonzero: D = mesh AABB scaled 10x about its centre */
    int num_threads;        /* host threads for the precompute; 0 = all */
    double margin_rel;      /* conservative margin, times diag(D); 0 = 1e-9 */
    int table_mode;         /* P2M_TABLE_* */
    int device_visit_cap;   /* P2M_TABLE_FLOODING_DEVICE: vertices one
                               primitive's flood may visit on the device
                               before the host takes the primitive over;
                               0 = 512 (the most), 1..512 accepted (small
                               values move work to the host; a test aid) */
} p2m_build_opts;

typedef struct {
    double t_validate, t_kdt, t_delaunay, t_cells, t_flood, t_pack; /* seconds */
    int64_t nv, ne, nf;
    int64_t delaunay_edges, tets, exact_predicates;
    int64_t flood_tests, flood_hits, quick_rejects, skipped_clips;
    int64_t nnz_edges, nnz_faces, max_list;
    double avg_list; /* (nnz_edges + nnz_faces) / nv */
    /* P2M_TABLE_FLOODING_DEVICE: seconds spent uploading, in the inspection
     * kernel and downloading (t_cells: the cells, built on the device);
     * primitives and cells the host finished */
    double t_dev_upload, t_dev_kernel, t_dev_download;
    int64_t device_redo, device_cells_back;
    /* The list statistics of Table 1 (Sec. 5.1), edges and faces apart: the
     * mean list over vertices (Avg^1: avg_edges, avg_faces; their sum is
     * avg_list), the mean weighted by the volume of each vertex's Voronoi
     * cell in D (Avg^2: the list a query uniform in D scans; estimated from
     * one jittered sample in each cell of a 128^3 grid on D and its nearest
     * vertex, deterministic), and the maxima over vertices. */
    double avg_edges, avg_faces, avg_list_volw, avg_edges_volw, avg_faces_volw;
    int64_t max_edges, max_faces;
    /* Vertices taken from the flood queues (Algorithm 1): each primitive's
     * own vertices plus the flood_tests; 0 in the ALL_PAIRS and EVERYTHING
     * modes, which do not flood. */
    int64_t flood_visits;
} p2m_build_stats;

typedef struct {
    int sort_queries;   /* <0 default (on for n >= 2^19 queries, off
                           below, where the ordering costs more than the
                           coherence it brings saves), 0 off, 1 Morton-order
                           the batch: a stable sort by the top 24 bits of
                           the key of p2m_order_queries (8 per axis: a
                           256^3 grid on D).  Answers do not depend on it. */
    int block_size;     /* 0 default (256); else 64, 128, 192 or 256 */
    int profile;        /* nonzero: record HIP events around the ordering and
                           query kernels (read with p2m_query_profile) */
    int traversal;      /* nearest-vertex search: 0 default (3), 1 one
                           KD-tree search per lane, 2 wavefront-coherent
                           KD-tree walk, 3 greedy walk over the Voronoi
                           neighbour graph (the graph Algorithm 1 floods)
                           from a grid seed, exact in D, with the
                           wavefront tree walk for queries outside D; every
                           choice returns each query's exact nearest vertex
                           (equal distances: the smallest id, up to float64
                           rounding of the squared distance) */
    int lds_levels;     /* per-lane KD-tree search (traversal 1): the top
                           lds_levels levels of the tree (2^lds_levels - 1
                           nodes, 64 bytes each) are copied into each
                           workgroup's LDS and read from there; 0 (default):
                           none; at most 9; ignored by the other traversals;
                           the answers do not change */
    int reserved[3];    /* must be 0 */
} p2m_query_opts;

/* ------------------------------------------------------------ host side */

/* Copy a mesh: V host float [nv*3], F host int32 [nf*3].  Rejects (P2M_ERR_MESH)
 * a vertex index out of range, a face that repeats a vertex or has zero area,
 * non-finite coordinates, two vertices with equal coordinates (the problem
 * statement assumes one copy per vertex, Sec. 4.1), nv or nf < 1, or more
 * than 2^30-1 vertices, edges or faces. */
p2m_status p2m_mesh_create(const float* V, int64_t nv, const int32_t* F, int64_t nf, p2m_mesh** out);

/* A mixed set of triangles and segments (Sec. 5.5): as p2m_mesh_create plus
 * free segments S host int32 [ns*2] (vertex index pairs; F may be NULL when
 * nf = 0, S when ns = 0; at least one face or segment).  The edges of the
 * mesh are the distinct vertex pairs of the face sides and the segments,
 * numbered by their (min, max) pair in lexicographic order; a segment that
 * is also a face side is that edge.  Rejects a segment index out of range
 * or a segment that repeats a vertex, besides the checks above. */
p2m_status p2m_mesh_create_mixed(const float* V, int64_t nv, const int32_t* F, int64_t nf, const int32_t* S,
                                 int64_t ns, p2m_mesh** out);
void p2m_mesh_destroy(p2m_mesh* m);

/* Vertex, edge and face counts (any pointer may be NULL). */
p2m_status p2m_mesh_counts(const p2m_mesh* m, int64_t* nv, int64_t* ne, int64_t* nf);

/* Canonical edges: *ne receives the count; pairs (host int32 [ne*2]) may be NULL. */
p2m_status p2m_mesh_edges(const p2m_mesh* m, int64_t* ne, int32_t* pairs);

/* Host precompute (Algorithm A.1 without R-trees): KD tree, Voronoi cells
 * clipped to D, convexity-filtered flooding inspection, CSR table.  Blocks.
 * opts may be NULL (default domain, all threads). */
p2m_status p2m_precompute(p2m_mesh* m, const p2m_build_opts* opts, p2m_build_stats* stats);

/* Inspect the precomputed structures.
 * Table: off host uint32 [2*nv+1], ent host int32 [nnz]; vertex v's edges are
 * ent[off[2v]..off[2v+1]) and its faces ent[off[2v+1]..off[2v+2]).  Pass
 * NULL arrays to read *nnz only.
 * Neighbours: Voronoi neighbours of each vertex, CSR (nb_off int64 [nv+1]).
 * KD tree: node coordinates xyz float [nv*3] and vertex ids vid int32 [nv] in
 * implicit left-balanced order (children of node i: 2i+1, 2i+2). */
p2m_status p2m_mesh_table(const p2m_mesh* m, int64_t* nnz, uint32_t* off, int32_t* ent);
/* Entry boxes of the table (host uint16 [nnz*6], in table order): for each
 * entry (v, p), lower x, y, z then upper x, y, z of a box holding
 * ConvexPoly(v,p) = Cell(v) n Space-perp(p) n D (Sec. 4.6 bounds Region(v,p)
 * <= ConvexPoly(v,p) by its box for the per-list R-tree), in the 16-bit
 * frame of D: u = (x - lo) * 65535 / (hi - lo), rounded outward and clamped
 * to [0, 65535]; lower 65535 and upper 0 on every axis for an empty
 * polytope.  The query tests an entry only when q lies in its box. */
p2m_status p2m_mesh_table_boxes(const p2m_mesh* m, uint16_t* boxes);
p2m_status p2m_mesh_neighbors(const p2m_mesh* m, int64_t* nnz, int64_t* nb_off, int32_t* nb);
p2m_status p2m_mesh_kdtree(const p2m_mesh* m, float* xyz, int32_t* vid);

/* Save / load the mesh with its precomputed structures (versioned binary). */
p2m_status p2m_save(const p2m_mesh* m, const char* path);
p2m_status p2m_load(const char* path, p2m_mesh** out);

/* Plain multi-threaded CPU P2M query over the same structures with the
 * same float32 arithmetic as the device kernel's default traversal (host
 * arrays): Voronoi walk from the grid seed in D, KD-tree search outside D.
 * A reported baseline, never used by the device path.  The first call builds
 * a host copy of the seed grid.  counters (may be NULL) receive sums over
 * queries: [0] nearest-vertex candidates evaluated (walk: neighbour
 * vertices; tree: nodes), [1] edge entries and [2] face entries scanned,
 * [3] walk steps (neighbour lists read), [4] edge and [5] face entries whose
 * box held q (their forms read and tested), [6] queries whose list was
 * scanned a second time because the gated ranking's winner was not
 * provably the closest (see p2m_query) and [7] the exact primitive
 * distances evaluated in those second scans. */
p2m_status p2m_query_host(const p2m_mesh* m, const float* q, int64_t n, int32_t* prim, float* closest,
                          float* dist, uint8_t* status, int num_threads, int64_t counters[8]);

const char* p2m_last_error(void);

/* ---------------------------------------------------------- device side */

/* Copy the mesh structures to device `device` (ordered on stream; returns
 * after the copies are enqueued, host staging is kept until destroy).
 * Requires p2m_precompute (or p2m_load).  *bytes (may be NULL) receives the
 * device arena size. */
p2m_status p2m_upload(p2m_mesh* m, int device, void* stream, int64_t* bytes);

/* P2M query of n points q_dev float [n*3] (Algorithm A.2: nearest vertex,
 * then the gated tests of its interception list, Sec. 4.6 entry boxes
 * first; the winner re-evaluated with the exact closed segment / triangle
 * distance; when that exact distance exceeds the winner's gated value (a
 * face whose foot lies just off it, within the gate margin), a second scan
 * evaluates exactly every candidate that could still be closer, so the
 * answer is the exact minimum over the candidates up to float32 rounding,
 * whatever the gate margin).  Outputs (device): prim int32 [n], closest float [n*3], dist
 * float [n] (in float32, every operation rounded on its own: |q - closest|
 * for a vertex; for an edge or face the point is formed relative to the
 * domain centre and the distance is the length of the vector from q to it,
 * taken before the point is rounded to absolute float32 coordinates, so a
 * mesh far from the origin keeps its accuracy);
 * status uint8 [n] (may be NULL).  For the backward pass, bary
 * float [n*3] and pvid int32 [n*3] (both NULL or both set) receive the
 * closest point's barycentric weights over the primitive's vertices (unused
 * slots: weight 0, id -1).  Non-finite queries give P2M_NONE, NaN distance
 * and P2M_Q_NONFINITE.  n = 0 is a no-op.  Scratch device memory (ordering,
 * and 16 bytes per query of staged answers for an ordered batch, 48 with
 * bary/pvid) is owned
 * by the mesh, grown on demand and reused; concurrent calls on the same
 * mesh from different streams race. */
p2m_status p2m_query(p2m_mesh* m, const float* q_dev, int64_t n, int32_t* prim_dev, float* closest_dev,
                     float* dist_dev, uint8_t* status_dev, float* bary_dev, int32_t* pvid_dev,
                     const p2m_query_opts* opts, void* stream);

/* p2m_query for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same query, arguments, kernels and answers, but the ordering buffers and
 * the staged answers live in a fixed device array of the library (64.3
 * MiB, held by each device the library runs on until the process ends)
 * instead of the mesh's scratch, and the call allocates nothing, on the
 * device or the host.  At most 2^20 queries per call (P2M_ERR_ARG beyond);
 * opts->profile must be 0 (P2M_ERR_ARG: its events would allocate).  The
 * first call on a device looks up that device's copy of the array.  Every
 * call on one device shares that array and it keeps the last call's
 * contents (nothing in it needs to start at zero): calls that overlap on one
 * device, on any streams or meshes, race. */
p2m_status p2m_query_noalloc(p2m_mesh* m, const float* q_dev, int64_t n, int32_t* prim_dev, float* closest_dev,
                             float* dist_dev, uint8_t* status_dev, float* bary_dev, int32_t* pvid_dev,
                             const p2m_query_opts* opts, void* stream);

/* Stage times of the last p2m_query on this mesh that set opts->profile, in
 * milliseconds, from HIP events recorded on the call's stream: ordering
 * (Morton keys + sort), the query kernel, and the pass that writes staged
 * answers to the output arrays (0 for an unordered batch).  Any pointer may
 * be NULL.  Waits for those events. */
p2m_status p2m_query_profile(p2m_mesh* m, float* order_ms, float* query_ms, float* finish_ms);

/* KD-tree nearest vertex only (the first step of Algorithm A.2): vid int32
 * [n] and squared distance d2 float [n] (may be NULL).  traversal as in
 * p2m_query_opts.  Queries are taken in the given order (no ordering step). */
p2m_status p2m_nearest_vertex(p2m_mesh* m, const float* q_dev, int64_t n, int32_t* vid_dev, float* d2_dev,
                              int traversal, void* stream);

/* Query ordering: 30-bit Morton keys of q in D (10 bits per axis, cells
 * floor((q-lo)*1024/(hi-lo)) taken in float32 and clamped to [0,1023]) and
 * their stable sort.  keys_dev uint32 [n] receives the sorted keys, perm_dev
 * int32 [n] the input index of each sorted position. */
p2m_status p2m_order_queries(p2m_mesh* m, const float* q_dev, int64_t n, uint32_t* keys_dev, int32_t* perm_dev,
                             void* stream);

/* Backward of dist w.r.t. the query points and the vertex positions, from
 * the forward's closest, bary and pvid (not in the paper; envelope theorem):
 *   grad_q[i]   = g[i] (q_i - c_i) / d_i            (0 when d_i = 0)
 *   grad_V[k]  += -g[i] w_ik (q_i - c_i) / d_i      (float atomics)
 * grad_dist_dev float [n]; grad_q_dev float [n*3] is overwritten (may be
 * NULL); grad_V_dev float [nv*3] is accumulated into (may be NULL; one row
 * per mesh vertex, 16-byte aligned, else P2M_ERR_ARG: large meshes update
 * it four floats at a time).  closest/dist/bary/pvid are the forward's
 * outputs for the same q. */
p2m_status p2m_query_backward(p2m_mesh* m, const float* q_dev, int64_t n, const float* closest_dev,
                              const float* dist_dev, const float* bary_dev, const int32_t* pvid_dev,
                              const float* grad_dist_dev, float* grad_q_dev, float* grad_V_dev, void* stream);

/* ------------------------------------------------------------- batching */

/* Pack precomputed meshes (not necessarily uploaded) into one device arena
 * on `device` for a single persistent launch over all of them.  The copies
 * are complete when the call returns; the meshes may be destroyed after.
 * count is 1 .. 2^20 (P2M_ERR_ARG beyond). */
p2m_status p2m_batch_create(p2m_mesh* const* meshes, int32_t count, int device, void* stream, p2m_batch** out);
void p2m_batch_destroy(p2m_batch* b);

/* Query all meshes in one persistent launch: q_dev float [N*3] holds the
 * queries of mesh k at rows q_offsets_host[k] .. q_offsets_host[k+1] (host
 * int64 [count+1], q_offsets_host[0] = 0, non-decreasing, N =
 * q_offsets_host[count]).  Outputs (device) as p2m_query, in the same row
 * order; primitive ids are local to each mesh; status_dev uint8 [N] (may be
 * NULL) receives the status bits of each query in its mesh's domain.  The launch sequence
 * (ordering keys and sort, work-counter reset, persistent kernel, write-out
 * of the staged 16-byte answers) is captured into a HIP graph on first use
 * and replayed while the offsets,
 * pointers and launch shape stay the same.  A new offset layout uploads a
 * tile list and waits for that copy.  Calls on one batch must not overlap. */
p2m_status p2m_batch_query(p2m_batch* b, const float* q_dev, const int64_t* q_offsets_host, int32_t* prim_dev,
                           float* closest_dev, float* dist_dev, uint8_t* status_dev, void* stream);

/* The batched query's ordering on its own (the ordering step of
 * p2m_batch_query, not in the paper): each query's key -- the top 24 bits of
 * the 30-bit Morton code of p2m_order_queries, taken in its own mesh's
 * domain -- and a stable sort of each mesh's rows by key, in place (mesh k's
 * rows stay at q_offsets_host[k] .. q_offsets_host[k+1]).  keys_dev uint32
 * [N] receives the sorted keys, perm_dev int32 [N] the input row of each
 * sorted position.  q_dev and q_offsets_host as for p2m_batch_query; calls
 * on one batch must not overlap. */
p2m_status p2m_batch_order_queries(p2m_batch* b, const float* q_dev, const int64_t* q_offsets_host, uint32_t* keys_dev,
                                   int32_t* perm_dev, void* stream);

/* The same work enqueued directly on `stream` (no graph). */
p2m_status p2m_batch_query_eager(p2m_batch* b, const float* q_dev, const int64_t* q_offsets_host, int32_t* prim_dev,
                                 float* closest_dev, float* dist_dev, uint8_t* status_dev, void* stream);

/* Launch shape of the batched kernel: workgroup size (64, 128, 192 or
 * 256), queries per lane in a tile (1..16), nearest-vertex traversal (1, 2
 * or 3 as in p2m_query_opts; 3 when the batch is created). */
p2m_status p2m_batch_set_shape(p2m_batch* b, int block, int queries_per_lane, int traversal);
p2m_status p2m_batch_get_shape(const p2m_batch* b, int* block, int* queries_per_lane, int* traversal);

/* Tree levels the per-lane KD-tree search (traversal 1) reads from LDS:
 * each workgroup copies the top `levels` levels of its tile's mesh's tree
 * (2^levels - 1 nodes, 64 bytes each) into LDS before the search; 0 (when
 * the batch is created) stages none.  0..9 (P2M_ERR_ARG beyond); the answers
 * do not change; the other traversals ignore it. */
p2m_status p2m_batch_set_lds_levels(p2m_batch* b, int levels);
p2m_status p2m_batch_get_lds_levels(const p2m_batch* b, int* levels);

/* Work distribution of the batched kernel: 0 (when the batch is created)
 * launches one workgroup per tile of the largest-first tile list; 1
 * launches as many workgroups as fit on the device, each taking tiles from
 * an atomic counter until the list is exhausted.  Both give the same
 * answers; P2M_ERR_ARG for another value. */
p2m_status p2m_batch_set_schedule(p2m_batch* b, int persistent);
p2m_status p2m_batch_get_schedule(const p2m_batch* b, int* persistent);

/* Time every launch shape in {64,128,256} x {1,2,4} x {1,2,3} on these queries,
 * traversal 1 with 0 and with 8 staged tree levels (p2m_batch_set_lds_levels),
 * (eager launches, two timed runs after a warm-up each) and keep the fastest;
 * the best_* outputs (may be NULL) report it and p2m_batch_get_lds_levels
 * its staged levels.  Synchronises the stream. */
p2m_status p2m_batch_autotune(p2m_batch* b, const float* q_dev, const int64_t* q_offsets_host, int32_t* prim_dev,
                              float* closest_dev, float* dist_dev, void* stream, int* best_block,
                              int* best_queries_per_lane, int* best_traversal);

#ifdef __cplusplus
}
#endif

#endif /* P2M_H */
