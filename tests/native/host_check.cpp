// CPU check of the host code that fedfem_precompute_many's workers run: the
// mesh layout (Morton order, tiles, partial and corner lists, packed ids,
// the per-tile corner count that sizes the fixed-point headroom), the
// worker pool with its per-worker cap on layout threads, and the caching
// device allocator -- built with the HIP runtime calls replaced by host
// stubs (hip_stub.cpp) so that it runs under ThreadSanitizer and
// AddressSanitizer + UndefinedBehaviorSanitizer.
//
// Checks: layout invariants on jittered Kuhn boxes and on a fan of 128
// tetrahedra around one node; layouts built concurrently by the pool (each
// worker also churning the device cache) equal the same layouts built
// serially.  Prints one line per part and exits non-zero on any failure.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fedfem.h"
#include "../../paper_1909_05098_amd/csrc/internal.h"

using namespace fedfem;

namespace {

int g_fail = 0;
std::mutex g_msg_mu;

void fail(const std::string& what) {
    std::lock_guard<std::mutex> lock(g_msg_mu);
    std::fprintf(stderr, "FAIL: %s\n", what.c_str());
    g_fail++;
}

struct Mesh {
    std::vector<double> xyz;
    std::vector<int32_t> tets;
    int64_t N = 0, E = 0;
};

// nx * ny * nz cubes of edge h, six tetrahedra each (all sharing the cube's
// (0,0,0)-(1,1,1) diagonal); interior nodes moved by up to 0.2 h with a
// seeded linear congruential generator.
Mesh kuhn_box(int nx, int ny, int nz, double h, uint64_t seed) {
    Mesh m;
    auto id = [&](int i, int j, int k) { return (int32_t)((k * (ny + 1) + j) * (nx + 1) + i); };
    m.N = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    m.xyz.resize(3 * m.N);
    uint64_t s = seed * 6364136223846793005ULL + 1442695040888963407ULL;
    auto uni = [&] {
        s = s * 6364136223846793005ULL + 1442695040888963407ULL;
        return (double)(s >> 11) / 9007199254740992.0 * 2.0 - 1.0;
    };
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                const bool inner = i > 0 && j > 0 && k > 0 && i < nx && j < ny && k < nz;
                double* p = &m.xyz[3 * id(i, j, k)];
                p[0] = i * h + (inner ? 0.2 * h * uni() : 0.0);
                p[1] = j * h + (inner ? 0.2 * h * uni() : 0.0);
                p[2] = k * h + (inner ? 0.2 * h * uni() : 0.0);
            }
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++)
                for (const auto& p : perm) {
                    int c[3] = {0, 0, 0};
                    m.tets.push_back(id(i, j, k));
                    for (int a = 0; a < 3; a++) {
                        c[p[a]] = 1;
                        m.tets.push_back(id(i + c[0], j + c[1], k + c[2]));
                    }
                }
    m.E = (int64_t)m.tets.size() / 4;
    return m;
}

// nx * ny * nz cubes of edge h as eight-node hexahedra (bottom face
// counter-clockwise, then the top face), interior nodes jittered as above.
Mesh hex_box(int nx, int ny, int nz, double h, uint64_t seed) {
    Mesh m = kuhn_box(nx, ny, nz, h, seed);
    auto id = [&](int i, int j, int k) { return (int32_t)((k * (ny + 1) + j) * (nx + 1) + i); };
    m.tets.clear();
    const int cc[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                          {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
    // each element's corners relabelled by one of the 48 symmetries of the
    // cube (axis permutation and sign flips), so that layouts see every
    // orientation
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    const int bits[8] = {0, 1, 3, 2, 4, 5, 7, 6};
    int corner_of[8];
    for (int a = 0; a < 8; a++) corner_of[bits[a]] = a;
    uint64_t r = seed * 0x9E3779B97F4A7C15ULL + 1;
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                r = r * 6364136223846793005ULL + 1442695040888963407ULL;
                const int p = (int)((r >> 33) % 6), fl = (int)((r >> 40) & 7);
                for (int a = 0; a < 8; a++) {
                    int b = 0;
                    for (int q = 0; q < 3; q++)
                        if (((bits[a] >> q) ^ (fl >> q)) & 1) b |= 1 << perm[p][q];
                    const int* c = cc[corner_of[b]];
                    m.tets.push_back(id(i + c[0], j + c[1], k + c[2]));
                }
            }
    m.E = (int64_t)m.tets.size() / 8;
    return m;
}

// m tetrahedra (0, a_i, b_i, c_i) sharing node 0, each with its own base
// triangle (they overlap; the layout does not need a conforming mesh).
Mesh fan(int m) {
    Mesh f;
    f.N = 1 + 3 * (int64_t)m;
    f.xyz.assign(3 * f.N, 0.0);
    for (int i = 0; i < m; i++)
        for (int c = 0; c < 3; c++) {
            const double a = 2.0 * M_PI * i / m + 2.0 * M_PI * c / 3.0;
            double* p = &f.xyz[3 * (1 + 3 * i + c)];
            p[0] = 1e-3 * std::cos(a);
            p[1] = 1e-3 * std::sin(a);
            p[2] = -5e-5;
        }
    for (int i = 0; i < m; i++) {
        f.tets.push_back(0);
        for (int c = 0; c < 3; c++) f.tets.push_back(1 + 3 * i + c);
    }
    f.E = m;
    return f;
}

bool check_layout(const Layout& L, const std::string& name) {
    const int npe = L.npe;
    auto bad = [&](const char* what) {
        fail(name + ": " + what);
        return false;
    };
    if ((int64_t)L.tile_elem_off.size() != L.T + 1 || L.tile_elem_off[0] != 0 ||
        L.tile_elem_off[L.T] != L.E)
        return bad("tile element offsets");
    if ((int64_t)L.tile_node_off.size() != L.T + 1 || L.tile_node_off[L.T] != L.P)
        return bad("tile node offsets");
    int maxn = 0, maxv = 0;
    std::vector<int> cnt;
    for (int64_t t = 0; t < L.T; t++) {
        const int64_t e0 = L.tile_elem_off[t], e1 = L.tile_elem_off[t + 1];
        const int64_t n0 = L.tile_node_off[t], n1 = L.tile_node_off[t + 1];
        if (e1 <= e0 || e1 - e0 > L.tile_elems) return bad("tile size");
        maxn = std::max<int>(maxn, (int)(n1 - n0));
        for (int64_t p = n0 + 1; p < n1; p++)
            if (L.tile_nodes[p - 1] >= L.tile_nodes[p]) return bad("tile nodes not ascending");
        cnt.assign(n1 - n0, 0);
        for (int64_t e = e0; e < e1; e++)
            for (int c = 0; c < npe; c++) {
                const int loc = L.lconn[npe * e + c];
                if (loc >= n1 - n0) return bad("local id out of range");
                if (L.tile_nodes[n0 + loc] != L.conn[npe * e + c]) return bad("local id");
                maxv = std::max(maxv, ++cnt[loc]);
            }
        for (int x : cnt)
            if (x == 0) return bad("tile node with no corner");
    }
    if (maxn != L.max_tile_nodes) return bad("max_tile_nodes");
    if (maxv != L.max_tile_valence) return bad("max_tile_valence");
    // partial positions: tile t's list starts with its single-tile nodes,
    // numbered consecutively from the running count; positions cover [0, P)
    // once, single-tile nodes at their own index
    // reordered tetrahedral layouts number single-tile nodes first
    const bool single_first = L.reorder && npe == 4;
    if (L.n_int < 0 || L.n_int > L.N || (!single_first && L.n_int != 0)) return bad("n_int");
    if ((int64_t)L.tile_part.size() != 4 * L.T) return bad("tile_part size");
    std::vector<int32_t> ntile(L.N, 0), at(L.P, -1);
    for (int64_t p = 0; p < L.P; p++) ntile[L.tile_nodes[p]]++;
    int64_t ib = 0;
    for (int64_t t = 0; t < L.T; t++) {
        const int64_t n0 = L.tile_node_off[t], m = L.tile_node_off[t + 1] - n0;
        const int32_t* tp = &L.tile_part[4 * t];
        if (tp[0] != ib || tp[3] != ib || tp[1] < 0 || tp[1] > m) return bad("tile_part");
        for (int64_t j = 0; j < m; j++) {
            const int32_t i = L.tile_nodes[n0 + j];
            if ((j < tp[1]) != (i < L.n_int)) return bad("single-tile nodes not first");
            if (j < tp[1] && i != tp[0] + j) return bad("single-tile ids not consecutive");
            if ((i < L.n_int) != (ntile[i] == 1 && single_first)) return bad("n_int split");
            const int64_t pos = j < tp[1] ? tp[0] + j : (int64_t)tp[2] + j;
            if (j >= tp[1] && pos < L.n_int) return bad("shared position in the single range");
            if (pos < 0 || pos >= L.P || at[pos] >= 0) return bad("positions not a permutation");
            at[pos] = i;
        }
        ib += tp[1];
    }
    if (ib != L.n_int) return bad("single-tile count");
    // node-major partial list: each node's positions, ascending tile order
    for (int64_t i = 0; i < L.N; i++) {
        if (i < L.n_int &&
            (L.part_off[i + 1] - L.part_off[i] != 1 || L.pidx[L.part_off[i]] != i))
            return bad("single-tile node not at its index");
        if (L.part_off[i + 1] - L.part_off[i] != ntile[i]) return bad("part_off count");
        for (int64_t k = L.part_off[i]; k < L.part_off[i + 1]; k++) {
            const int32_t p = L.pidx[k];
            if (p < 0 || p >= L.P) return bad("pidx out of range");
            if (at[p] != i) return bad("pidx names another node");
            if (k > L.part_off[i] && L.pidx[k - 1] >= p) return bad("pidx not ascending");
        }
    }
    // caller <-> internal node ids are inverse permutations
    for (int64_t i = 0; i < L.N; i++)
        if (L.nperm[i] < 0 || L.nperm[i] >= L.N || L.ninv[L.nperm[i]] != i)
            return bad("nperm / ninv");
    // node -> element corners, ascending element
    for (int64_t i = 0; i < L.N; i++)
        for (int64_t k = L.ec_off[i]; k < L.ec_off[i + 1]; k++) {
            if (L.conn[L.ec[k]] != i) return bad("ec");
            if (k > L.ec_off[i] && L.ec[k - 1] >= L.ec[k]) return bad("ec order");
        }
    // packed ids decode to lconn
    if (!L.lconn_pk.empty() && npe == 8) {
        if ((int64_t)L.lconn_pk.size() != 10 * L.E) return bad("packed hexahedral size");
        for (int64_t e = 0; e < L.E; e++) {
            uint64_t w;
            uint16_t hw;
            std::memcpy(&w, &L.lconn_pk[8 * e], 8);
            std::memcpy(&hw, &L.lconn_pk[8 * L.E + 2 * e], 2);
            int ids[8];
            for (int c = 0; c < 6; c++) ids[c] = (int)(w >> (10 * c) & 1023);
            ids[6] = (int)(w >> 60) | (hw & 63) << 4;
            ids[7] = hw >> 6;
            for (int c = 0; c < 8; c++)
                if (ids[c] != L.lconn[8 * e + c]) return bad("packed hexahedral ids");
        }
    } else if (!L.lconn_pk.empty()) {
        for (int64_t e = 0; e < L.E; e++) {
            uint32_t w;
            std::memcpy(&w, &L.lconn_pk[4 * e], 4);
            const int hi = L.lconn_pk[4 * L.E + e];
            const int ids[4] = {(int)(w & 1023), (int)(w >> 10 & 1023), (int)(w >> 20 & 1023),
                                (int)(w >> 30) | hi << 2};
            for (int c = 0; c < 4; c++)
                if (ids[c] != L.lconn[4 * e + c]) return bad("packed ids");
        }
    }
    return true;
}

struct Case {
    int nx, ny, nz;
    int reorder, tile, mn;
};

bool same_layout(const Layout& a, const Layout& b) {
    return a.T == b.T && a.P == b.P && a.max_tile_nodes == b.max_tile_nodes &&
           a.max_tile_valence == b.max_tile_valence && a.nperm == b.nperm &&
           a.eperm == b.eperm && a.conn == b.conn && a.tile_elem_off == b.tile_elem_off &&
           a.tile_node_off == b.tile_node_off && a.tile_nodes == b.tile_nodes &&
           a.pidx == b.pidx && a.lconn == b.lconn && a.lconn_pk == b.lconn_pk &&
           a.part_off == b.part_off && a.ec == b.ec && a.n_int == b.n_int &&
           a.tile_part == b.tile_part && a.xyz == b.xyz;
}

// Natural-coordinate bits of hexahedral corner a (bit 0 xi, 1 eta, 2 zeta).
constexpr int kCornerBits[8] = {0, 1, 3, 2, 4, 5, 7, 6};

// The internal mesh is the caller's under the node and element permutations.
// Reordered hexahedra may also have their corners relabelled by a symmetry
// of the reference cube, which must then leave every local axis pointing
// along the positive global axis it is nearest to.
bool same_mesh(const Layout& L, const Mesh& m, const std::string& name) {
    const int npe = L.npe;
    const bool relabel = npe == 8 && L.reorder;
    for (int64_t e = 0; e < L.E; e++) {
        const int32_t* ci = &L.conn[npe * e];
        const int32_t* cc = &m.tets[npe * (int64_t)L.eperm[e]];
        if (!relabel) {
            for (int c = 0; c < npe; c++)
                if (ci[c] != L.ninv[cc[c]]) {
                    fail(name + ": internal connectivity");
                    return false;
                }
            continue;
        }
        // internal corner a holds caller corner from[a]; cube edges (corners
        // one coordinate apart) must stay edges
        int from[8];
        for (int a = 0; a < 8; a++) {
            from[a] = -1;
            for (int b = 0; b < 8; b++)
                if (ci[a] == L.ninv[cc[b]]) from[a] = b;
            if (from[a] < 0) {
                fail(name + ": hexahedron lost a corner");
                return false;
            }
        }
        for (int a = 0; a < 8; a++)
            for (int b = 0; b < 8; b++) {
                const int da = __builtin_popcount(kCornerBits[a] ^ kCornerBits[b]);
                const int db = __builtin_popcount(kCornerBits[from[a]] ^ kCornerBits[from[b]]);
                if (da != db) {
                    fail(name + ": corner relabelling is no cube symmetry");
                    return false;
                }
            }
        for (int k = 0; k < 3; k++) {
            double g = 0.0;  // component k of local axis k
            for (int a = 0; a < 8; a++)
                g += ((kCornerBits[a] >> k & 1) ? 1.0 : -1.0) * L.xyz[3 * (int64_t)ci[a] + k];
            if (!(g > 0.0)) {
                fail(name + ": hexahedron not oriented along the axes");
                return false;
            }
        }
    }
    for (int64_t i = 0; i < L.N; i++)
        for (int a = 0; a < 3; a++)
            if (L.xyz[3 * i + a] != m.xyz[3 * (int64_t)L.nperm[i] + a]) {
                fail(name + ": internal coordinates");
                return false;
            }
    return true;
}

bool build(const Mesh& m, const Case& c, Layout& L, const std::string& name) {
    std::string err;
    if (!build_layout(m.xyz.data(), m.tets.data(), 4, m.N, m.E, c.reorder, c.tile, c.mn, L,
                      err)) {
        fail(name + ": " + err);
        return false;
    }
    pack_lconn(L);
    return same_mesh(L, m, name);
}

}  // namespace

int main() {
    // 1. fan: one tile sees all 128 corners of node 0; 64-element tiles half
    {
        const Mesh f = fan(128);
        for (int tile : {64, 128, 2048}) {
            Layout L;
            std::string err;
            if (!build_layout(f.xyz.data(), f.tets.data(), 4, f.N, f.E, 1, tile, 4 * tile, L,
                              err)) {
                fail("fan: " + err);
                continue;
            }
            pack_lconn(L);
            check_layout(L, "fan");
            const int want = tile < 128 ? tile : 128;
            if (L.max_tile_valence != want)
                fail("fan: max_tile_valence " + std::to_string(L.max_tile_valence) +
                     " != " + std::to_string(want));
        }
        std::printf("fan layout: ok\n");
    }
    // 2. serial layouts of several boxes and options
    const std::vector<Case> cases = {
        {6, 5, 4, 1, 64, 32},      {12, 10, 8, 1, 256, 128},  {12, 10, 8, 0, 256, 1024},
        {20, 16, 12, 1, 1024, 512}, {20, 16, 12, 1, 2048, 1024}, {16, 16, 16, 0, 64, 256},
        {9, 7, 5, 1, 128, 40},     {24, 20, 16, 1, 4096, 2048},
    };
    std::vector<Mesh> meshes;
    std::vector<Layout> ref(cases.size());
    int kuhn_valence = 0;
    for (size_t k = 0; k < cases.size(); k++) {
        const Case& c = cases[k];
        meshes.push_back(kuhn_box(c.nx, c.ny, c.nz, 1e-3, 100 + k));
        const std::string name = "box " + std::to_string(k);
        if (build(meshes[k], c, ref[k], name)) check_layout(ref[k], name);
        kuhn_valence = std::max(kuhn_valence, ref[k].max_tile_valence);
    }
    // an interior lattice node has 24 tetrahedra: no tile can see more
    if (kuhn_valence > 24) fail("Kuhn lattice tile valence above 24");
    // tiles cut again on a built layout (the shrink path) renumber on top
    // of the first numbering
    for (const size_t k : {size_t(1), size_t(3), size_t(2)}) {
        Layout L = ref[k];
        std::string err;
        const std::string name = "rebuilt box " + std::to_string(k);
        if (!build_tiles(L, 128, 64, err)) {
            fail(name + ": " + err);
            continue;
        }
        pack_lconn(L);
        if (check_layout(L, name) && same_mesh(L, meshes[k], name) && L.reorder &&
            L.n_int == 0)
            fail(name + ": no single-tile nodes");
    }
    // hexahedra: packed 10-bit ids when a tile has at most 1024 nodes, u16
    // otherwise
    for (const int tile : {256, 512, 1024}) {
        const Mesh hb = hex_box(22, 18, 14, 1e-3, 7);
        Layout L;
        std::string err;
        if (!build_layout(hb.xyz.data(), hb.tets.data(), 8, hb.N, hb.E, 1, tile, 2 * tile, L,
                          err)) {
            fail("hex box: " + err);
            continue;
        }
        pack_lconn(L);
        check_layout(L, "hex box " + std::to_string(tile));
        same_mesh(L, hb, "hex box " + std::to_string(tile));
        if (L.lconn_pk.empty() != (L.max_tile_nodes > kPackedMaxNodes))
            fail("hex box: packed form chosen wrongly");
        if (L.max_tile_valence > 8) fail("hex box: tile valence above 8");
    }
    std::printf("hexahedral layouts: ok\n");
    std::printf("serial layouts: %zu cases ok (largest tile valence %d)\n", cases.size(),
                kuhn_valence);
    // 3. the same layouts from the worker pool, several times each, with the
    // device cache churned by every worker
    const int32_t n_items = (int32_t)(3 * cases.size());
    std::vector<Layout> got(n_items);
    run_workers(n_items, 8, 2, [&](int32_t j) {
        const size_t k = (size_t)j % cases.size();
        const std::string name = "pool item " + std::to_string(j);
        if (build(meshes[k], cases[k], got[j], name) && !same_layout(got[j], ref[k]))
            fail(name + ": differs from the serial layout");
        std::vector<std::pair<void*, size_t>> blocks;
        for (int r = 0; r < 40; r++) {
            const size_t bytes = 100 + (size_t)((j * 7919 + r * 104729) % 300000);
            void* p = nullptr;
            size_t granted = 0;
            if (cached_malloc(&p, bytes, &granted) != hipSuccess || !p || granted < bytes) {
                fail(name + ": cached_malloc");
                continue;
            }
            std::memset(p, j & 0xff, granted);
            blocks.push_back({p, granted});
            if (r % 3 == 2) {
                cached_free(blocks.front().first, blocks.front().second);
                blocks.erase(blocks.begin());
            }
        }
        for (auto& b : blocks) cached_free(b.first, b.second);
    });
    const size_t released = fedfem_release_cached_memory();
    std::printf("pool: %d layouts equal the serial ones; device cache released %zu bytes\n",
                n_items, released);
    if (g_fail) {
        std::printf("host_check: %d failures\n", g_fail);
        return 1;
    }
    std::printf("host_check: ok\n");
    return 0;
}
