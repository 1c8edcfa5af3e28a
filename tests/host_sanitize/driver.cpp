// Drives the host precompute through the C interface, for the sanitizer
// builds of the host sources: every table mode with several threads, the
// table and neighbour readers, save / load, mixed primitive sets and the
// error paths.  Meshes come from binary files written by the test
// (nv, nf, ns as int64, then V float32 [nv*3], F int32 [nf*3], S int32
// [ns*2]).  Exits non-zero on any unexpected status.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "p2m.h"

static int g_fail = 0;

static void expect(p2m_status got, p2m_status want, const char* what) {
    if (got != want) {
        std::fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, p2m_last_error());
        g_fail = 1;
    }
}

struct Mesh {
    std::vector<float> V;
    std::vector<int32_t> F, S;
};

static bool read_mesh(const char* path, Mesh& m) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return false;
    int64_t n[3];
    bool ok = std::fread(n, sizeof(int64_t), 3, f) == 3;
    if (ok) {
        m.V.resize((size_t)(3 * n[0]));
        m.F.resize((size_t)(3 * n[1]));
        m.S.resize((size_t)(2 * n[2]));
        ok = std::fread(m.V.data(), 4, m.V.size(), f) == m.V.size() &&
             std::fread(m.F.data(), 4, m.F.size(), f) == m.F.size() &&
             std::fread(m.S.data(), 4, m.S.size(), f) == m.S.size();
    }
    std::fclose(f);
    return ok;
}

static void run(const Mesh& mm, int mode, int threads, const std::string& tmp) {
    const int64_t nv = (int64_t)mm.V.size() / 3, nf = (int64_t)mm.F.size() / 3, ns = (int64_t)mm.S.size() / 2;
    p2m_mesh* m = nullptr;
    expect(p2m_mesh_create_mixed(mm.V.data(), nv, nf ? mm.F.data() : nullptr, nf, ns ? mm.S.data() : nullptr, ns, &m),
           P2M_OK, "create");
    if (!m) return;
    p2m_build_opts o = {};
    o.use_default_domain = 1;
    o.num_threads = threads;
    o.table_mode = mode;
    p2m_build_stats st;
    expect(p2m_precompute(m, &o, &st), P2M_OK, "precompute");
    int64_t nnz = 0, ne = 0;
    expect(p2m_mesh_table(m, &nnz, nullptr, nullptr), P2M_OK, "table size");
    std::vector<uint32_t> off((size_t)(2 * nv + 1));
    std::vector<int32_t> ent((size_t)(nnz > 0 ? nnz : 1));
    std::vector<uint16_t> box((size_t)(6 * (nnz > 0 ? nnz : 1)));
    expect(p2m_mesh_table(m, &nnz, off.data(), ent.data()), P2M_OK, "table");
    expect(p2m_mesh_table_boxes(m, box.data()), P2M_OK, "boxes");
    expect(p2m_mesh_edges(m, &ne, nullptr), P2M_OK, "edges");
    int64_t nb = 0;
    expect(p2m_mesh_neighbors(m, &nb, nullptr, nullptr), P2M_OK, "neighbours size");
    std::vector<int64_t> nboff((size_t)(nv + 1));
    std::vector<int32_t> nbv((size_t)(nb > 0 ? nb : 1));
    expect(p2m_mesh_neighbors(m, &nb, nboff.data(), nbv.data()), P2M_OK, "neighbours");
    std::vector<float> xyz((size_t)(3 * nv));
    std::vector<int32_t> vid((size_t)nv);
    expect(p2m_mesh_kdtree(m, xyz.data(), vid.data()), P2M_OK, "kdtree");
    const std::string path = tmp + "/mesh.p2m";
    expect(p2m_save(m, path.c_str()), P2M_OK, "save");
    p2m_mesh* l = nullptr;
    expect(p2m_load(path.c_str(), &l), P2M_OK, "load");
    int64_t nnz2 = 0;
    if (l) {
        expect(p2m_mesh_table(l, &nnz2, nullptr, nullptr), P2M_OK, "loaded table");
        if (nnz2 != nnz) {
            std::fprintf(stderr, "loaded table has %lld entries, saved %lld\n", (long long)nnz2, (long long)nnz);
            g_fail = 1;
        }
        p2m_mesh_destroy(l);
    }
    // the device inspection reports its missing device
    p2m_mesh* d = nullptr;
    expect(p2m_mesh_create_mixed(mm.V.data(), nv, nf ? mm.F.data() : nullptr, nf, ns ? mm.S.data() : nullptr, ns, &d),
           P2M_OK, "create for the device mode");
    o.table_mode = P2M_TABLE_FLOODING_DEVICE;
    expect(p2m_precompute(d, &o, &st), P2M_ERR_HIP, "device mode without a device");
    p2m_mesh_destroy(d);
    p2m_mesh_destroy(m);
}

int main(int argc, char** argv) {
    if (argc < 3) {
        std::fprintf(stderr, "usage: driver TMPDIR MESH...\n");
        return 2;
    }
    const std::string tmp = argv[1];
    for (int a = 2; a < argc; ++a) {
        Mesh m;
        if (!read_mesh(argv[a], m)) {
            std::fprintf(stderr, "cannot read %s\n", argv[a]);
            return 2;
        }
        const bool tiny = m.V.size() / 3 <= 200;
        for (int threads : {1, 4}) {
            run(m, P2M_TABLE_FLOODING, threads, tmp);
            if (tiny) {
                run(m, P2M_TABLE_ALL_PAIRS, threads, tmp);
                run(m, P2M_TABLE_EVERYTHING, threads, tmp);
            }
        }
    }
    // error paths
    const float V[9] = {0, 0, 0, 1, 0, 0, 0, 1, 0};
    const int32_t Fbad[3] = {0, 1, 5};
    p2m_mesh* m = nullptr;
    expect(p2m_mesh_create(V, 3, Fbad, 1, &m), P2M_ERR_MESH, "index out of range");
    expect(p2m_load((tmp + "/missing.p2m").c_str(), &m), P2M_ERR_IO, "load of a missing file");
    const int32_t F[3] = {0, 1, 2};
    expect(p2m_mesh_create(V, 3, F, 1, &m), P2M_OK, "one triangle");
    int64_t nnz = 0;
    expect(p2m_mesh_table(m, &nnz, nullptr, nullptr), P2M_ERR_STATE, "table before precompute");
    p2m_build_opts o = {};
    o.domain_hi[0] = -1.0;
    expect(p2m_precompute(m, &o, nullptr), P2M_ERR_ARG, "empty domain");
    p2m_mesh_destroy(m);
    std::printf(g_fail ? "FAILED\n" : "ok\n");
    return g_fail;
}
