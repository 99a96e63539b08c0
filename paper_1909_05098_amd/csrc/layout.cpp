// Host-side mesh layout: Morton renumbering, element tiles with their local
// node lists, single-tile-first node numbering and the element order inside
// tetrahedral tiles, the hexahedra's corner relabelling, and the node ->
// partial / node -> element-corner lists.  Integer topology (plus the corner
// coordinates that orient hexahedra); all floating-point pre-computation
// runs on the GPU.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "internal.h"

namespace fedfem {

namespace {

// Spread the low 21 bits of v so that bit i lands on bit 3i.
inline uint64_t spread3(uint64_t v) {
    v &= 0x1fffffULL;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

// Stable LSD radix sort of (key, id) pairs by key, 11-bit digits.
void radix_sort_pairs(std::vector<uint64_t>& key, std::vector<int32_t>& id,
                      int key_bits) {
    constexpr int kDigit = 11;
    constexpr uint64_t kMask = (1u << kDigit) - 1;
    const size_t n = key.size();
    std::vector<uint64_t> k2(n);
    std::vector<int32_t> i2(n);
    std::vector<size_t> cnt(size_t(1) << kDigit);
    for (int shift = 0; shift < key_bits; shift += kDigit) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (size_t i = 0; i < n; i++) cnt[(key[i] >> shift) & kMask]++;
        size_t run = 0;
        for (auto& c : cnt) {
            size_t t = c;
            c = run;
            run += t;
        }
        for (size_t i = 0; i < n; i++) {
            size_t pos = cnt[(key[i] >> shift) & kMask]++;
            k2[pos] = key[i];
            i2[pos] = id[i];
        }
        key.swap(k2);
        id.swap(i2);
    }
}

// cap on the host threads one layout build may use (0: up to 16); set per
// calling thread, so that builds already running side by side do not each
// spread over every core
thread_local int tl_layout_threads = 0;

// body(a, b) over [0, n) split across up to 16 host threads (or the calling
// thread's cap); ranges of fewer than `grain` items run on the calling thread
template <typename F>
void parallel_for(int64_t n, F&& body, int64_t grain = 4096) {
    unsigned nt = tl_layout_threads > 0
                      ? (unsigned)tl_layout_threads
                      : std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    nt = (unsigned)std::min<int64_t>(nt, std::max<int64_t>(1, n / std::max<int64_t>(1, grain)));
    if (nt <= 1) {
        body(0, n);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; t++) {
        int64_t a = t * chunk, b = std::min(n, a + chunk);
        if (a >= b) break;
        th.emplace_back([&body, a, b] { body(a, b); });
    }
    for (auto& t : th) t.join();
}

}  // namespace

int set_layout_threads(int n) {
    const int old = tl_layout_threads;
    tl_layout_threads = n < 0 ? 0 : n;
    return old;
}

std::vector<int32_t> morton_order(const double* pts, int64_t n) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) {
            lo[a] = std::min(lo[a], pts[3 * i + a]);
            hi[a] = std::max(hi[a], pts[3 * i + a]);
        }
    double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
    // bits per axis: about 16 cells per point along the curve, at most 21
    int lg = 0;
    while ((int64_t(1) << lg) < std::max<int64_t>(n, 2)) lg++;
    const int bits = std::min(21, (lg + 2) / 3 + 4);
    const double cells = double((1u << bits) - 1);
    const double scale = cells / ext;  // same scale on all axes
    std::vector<uint64_t> key(n);
    std::vector<int32_t> id(n);
    parallel_for(n, [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; i++) {
            uint64_t q[3];
            for (int ax = 0; ax < 3; ax++) {
                double v = (pts[3 * i + ax] - lo[ax]) * scale;
                q[ax] = (uint64_t)std::min(cells, std::max(0.0, v));
            }
            key[i] = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
            id[i] = (int32_t)i;
        }
    }, 16384);
    radix_sort_pairs(key, id, 3 * bits);
    return id;
}

namespace {

// node -> (element, corner) as npe * e + corner, ascending internal element
void node_corners(Layout& L) {
    const int64_t N = L.N, S = (int64_t)L.npe * L.E;
    L.ec_off.assign(N + 1, 0);
    for (int64_t s = 0; s < S; s++) L.ec_off[L.conn[s] + 1]++;
    for (int64_t i = 0; i < N; i++) L.ec_off[i + 1] += L.ec_off[i];
    L.ec.assign(S, 0);
    std::vector<int32_t> fill(L.ec_off.begin(), L.ec_off.end() - 1);
    for (int64_t s = 0; s < S; s++) L.ec[fill[L.conn[s]]++] = (int32_t)s;
}

// Interior-first numbering (reordered tetrahedral layouts).  A node that a
// single tile touches gets its whole load from that tile, so its partial can
// sit at the node's own index and the node pass reads it with no slot lookup.
// Hexahedral layouts keep the curve numbering: there the new order of the
// tile lists cost the element pass more than the node pass gained.  Nodes are renumbered in
// the order the tiles first reach them, single-tile nodes first: tile t's
// single-tile nodes take the ids [int_off[t], int_off[t+1]) in the order of
// its list, the shared nodes follow from n_int on, and nodes of no element
// come last.  Each tile's list is sorted again, which puts its single-tile
// nodes first, and the corners' local ids follow the new order.
void interior_first(Layout& L) {
    const int64_t N = L.N, T = L.T, P = L.P;
    const int npe = L.npe;
    std::vector<int32_t> ntile(N, 0);
    for (int64_t p = 0; p < P; p++) ntile[L.tile_nodes[p]]++;
    std::vector<int32_t> nmap(N, -1);
    int32_t next = 0;
    for (int64_t p = 0; p < P; p++)
        if (ntile[L.tile_nodes[p]] == 1) nmap[L.tile_nodes[p]] = next++;
    L.n_int = next;
    for (int64_t p = 0; p < P; p++)
        if (nmap[L.tile_nodes[p]] < 0) nmap[L.tile_nodes[p]] = next++;
    for (int64_t i = 0; i < N; i++)
        if (nmap[i] < 0) nmap[i] = next++;
    std::vector<int32_t>().swap(ntile);
    // tile lists in ascending new id, corner ids remapped
    parallel_for(T, [&](int64_t a, int64_t b) {
        std::vector<std::pair<int32_t, int32_t>> key;
        std::vector<uint16_t> to;
        for (int64_t t = a; t < b; t++) {
            const int64_t p0 = L.tile_node_off[t], m = L.tile_node_off[t + 1] - p0;
            key.resize(m);
            for (int64_t j = 0; j < m; j++) key[j] = {nmap[L.tile_nodes[p0 + j]], (int32_t)j};
            std::sort(key.begin(), key.end());
            to.resize(m);
            for (int64_t j = 0; j < m; j++) {
                L.tile_nodes[p0 + j] = key[j].first;
                to[key[j].second] = (uint16_t)j;
            }
            const int64_t s0 = (int64_t)npe * L.tile_elem_off[t],
                          s1 = (int64_t)npe * L.tile_elem_off[t + 1];
            for (int64_t s2 = s0; s2 < s1; s2++) L.lconn[s2] = to[L.lconn[s2]];
        }
    }, 4);
    parallel_for((int64_t)npe * L.E, [&](int64_t a, int64_t b) {
        for (int64_t s2 = a; s2 < b; s2++) L.conn[s2] = nmap[L.conn[s2]];
    }, 65536);
    std::vector<int32_t> nperm(N);
    std::vector<double> xyz(3 * N);
    for (int64_t i = 0; i < N; i++) {
        nperm[nmap[i]] = L.nperm[i];
        std::memcpy(&xyz[3 * (int64_t)nmap[i]], &L.xyz[3 * i], 3 * sizeof(double));
    }
    L.nperm.swap(nperm);
    L.xyz.swap(xyz);
    for (int64_t i = 0; i < N; i++) L.ninv[L.nperm[i]] = (int32_t)i;
}

// Where each tile writes its partials and where each node finds them.  Tile
// t's list starts with its ni single-tile nodes (ids n0 .. n0 + ni - 1),
// whose partials go to the positions of the same numbers; the rest of the
// list goes tile-major after all single-tile nodes, at ps + j for list
// position j.  tile_part holds (n0, ni, ps, n0) per tile.  pidx[part_off[i]
// .. part_off[i+1]) lists node i's positions in ascending tile order.
void slot_positions(Layout& L) {
    const int64_t N = L.N, T = L.T, P = L.P;
    L.tile_part.assign(4 * T, 0);
    int64_t ib = 0;
    for (int64_t t = 0; t < T; t++) {
        const int64_t p0 = L.tile_node_off[t], p1 = L.tile_node_off[t + 1];
        int64_t ni = 0;
        while (p0 + ni < p1 && L.tile_nodes[p0 + ni] < L.n_int) ni++;
        L.tile_part[4 * t] = (int32_t)ib;
        L.tile_part[4 * t + 1] = (int32_t)ni;
        L.tile_part[4 * t + 2] = (int32_t)(L.n_int + (p0 - ib) - ni);
        L.tile_part[4 * t + 3] = (int32_t)ib;
        ib += ni;
    }
    L.part_off.assign(N + 1, 0);
    for (int64_t p = 0; p < P; p++) L.part_off[L.tile_nodes[p] + 1]++;
    for (int64_t i = 0; i < N; i++) L.part_off[i + 1] += L.part_off[i];
    L.pidx.assign(P, 0);
    std::vector<int32_t> fill(L.part_off.begin(), L.part_off.end() - 1);
    for (int64_t t = 0; t < T; t++) {
        const int64_t p0 = L.tile_node_off[t], m = L.tile_node_off[t + 1] - p0;
        const int32_t* tp = &L.tile_part[4 * t];
        for (int64_t j = 0; j < m; j++)
            L.pidx[fill[L.tile_nodes[p0 + j]]++] = (int32_t)(j < tp[1] ? tp[0] + j : tp[2] + j);
    }
}

// Element order inside each tile (reordered tetrahedral layouts).  The curve
// order puts neighbouring elements next to each other, so the 64 lanes of one
// accumulation step would hit the same few tile nodes in local memory.  The
// tile's elements are dealt out instead: with ch = ceil(ne / 64), curve
// position l * ch + k moves to the k-th group of 64, lane l, so one step's
// lanes take elements from 64 separate stretches of the tile.  The tile's
// element set, and so its node list, stays the same; sums on the fixed-point
// grid are exact, so the loads do not depend on this order.  undo = true
// restores the curve order of the tiles in L.tile_elem_off.  Hexahedra keep
// the curve order: there one step adds the same corner of 64 neighbouring
// elements, which are distinct nodes spread evenly over the banks, and
// dealing them out would only scatter the banks.
void spread_tiles(Layout& L, bool undo) {
    const int npe = L.npe;
    parallel_for(L.T, [&](int64_t a, int64_t b) {
        std::vector<int32_t> conn, eperm;
        for (int64_t t = a; t < b; t++) {
            const int64_t e0 = L.tile_elem_off[t], ne = L.tile_elem_off[t + 1] - e0;
            const int64_t ch = (ne + 63) / 64;
            conn.assign(L.conn.begin() + npe * e0, L.conn.begin() + npe * (e0 + ne));
            eperm.assign(L.eperm.begin() + e0, L.eperm.begin() + e0 + ne);
            int64_t i = 0;
            for (int64_t k = 0; k < ch; k++)
                for (int64_t l = 0; l < 64; l++) {
                    const int64_t o = l * ch + k;
                    if (o >= ne) continue;
                    // curve position o <-> spread position i
                    const int64_t from = undo ? i : o, to = undo ? o : i;
                    for (int c = 0; c < npe; c++)
                        L.conn[npe * (e0 + to) + c] = conn[npe * from + c];
                    L.eperm[e0 + to] = eperm[from];
                    i++;
                }
        }
    }, 16);
}

}  // namespace

bool build_tiles(Layout& L, int TE, int MN, std::string& err) {
    if (TE < 64 || TE > 8192 || TE % 64) {
        err = "tile_elems must be a multiple of 64 in [64, 8192]";
        return false;
    }
    if (MN < L.npe || MN > L.npe * TE) {
        err = "max_tile_nodes must lie in [nodes per element, nodes per element * tile_elems]";
        return false;
    }
    const int64_t E = L.E, N = L.N;
    const int npe = L.npe;
    if (L.spread) {
        spread_tiles(L, true);
        L.spread = 0;
    }
    L.tile_elems = TE;
    // greedy cut along the element order: close a tile when it holds TE
    // elements or the next element would bring it past MN distinct nodes
    L.tile_elem_off.assign(1, 0);
    {
        std::vector<int32_t> mark(N, -1);
        int32_t t = 0;
        int cnt = 0, ne = 0;
        for (int64_t e = 0; e < E; e++) {
            const int32_t* n = &L.conn[(int64_t)npe * e];
            int nnew = 0;
            for (int c = 0; c < npe; c++) {
                bool dup = false;
                for (int d = 0; d < c; d++) dup |= (n[d] == n[c]);
                if (!dup && mark[n[c]] != t) nnew++;
            }
            if (ne == TE || cnt + nnew > MN) {
                L.tile_elem_off.push_back((int32_t)e);
                t++;
                cnt = 0;
                ne = 0;
                nnew = 0;
                for (int c = 0; c < npe; c++) {
                    bool dup = false;
                    for (int d = 0; d < c; d++) dup |= (n[d] == n[c]);
                    if (!dup) nnew++;
                }
            }
            for (int c = 0; c < npe; c++) mark[n[c]] = t;
            cnt += nnew;
            ne++;
        }
        L.tile_elem_off.push_back((int32_t)E);
    }
    const int64_t T = (int64_t)L.tile_elem_off.size() - 1;
    L.T = T;
    if (L.reorder && npe == 4) {
        spread_tiles(L, false);
        L.spread = 1;
    }
    // pass 1: each tile's distinct nodes in ascending id (a marker array per
    // worker finds them; only the distinct nodes are sorted) and every
    // corner's position in that list
    std::vector<int32_t> uniq((size_t)npe * E);  // tile t's list at npe * tile_elem_off[t]
    std::vector<int32_t> ucount(T), uval(T);
    L.lconn.assign((size_t)npe * E, 0);
    parallel_for(T, [&](int64_t a, int64_t b) {
        std::vector<int32_t> loc(N, -1);
        std::vector<int32_t> cnt;
        for (int64_t t = a; t < b; t++) {
            const int64_t e0 = L.tile_elem_off[t], nc = npe * (L.tile_elem_off[t + 1] - e0);
            const int32_t* c = L.conn.data() + npe * e0;
            int32_t* u = uniq.data() + npe * e0;
            int32_t nu = 0;
            for (int64_t s2 = 0; s2 < nc; s2++)
                if (loc[c[s2]] < 0) {
                    loc[c[s2]] = 0;
                    u[nu++] = c[s2];
                }
            std::sort(u, u + nu);
            for (int32_t i = 0; i < nu; i++) loc[u[i]] = i;
            // corners per tile node: the loads one LDS accumulator sums
            cnt.assign(nu, 0);
            int32_t vmax = 0;
            for (int64_t s2 = 0; s2 < nc; s2++) {
                L.lconn[npe * e0 + s2] = (uint16_t)loc[c[s2]];
                vmax = std::max(vmax, ++cnt[loc[c[s2]]]);
            }
            for (int32_t i = 0; i < nu; i++) loc[u[i]] = -1;
            ucount[t] = nu;
            uval[t] = vmax;
        }
    }, 4);
    L.tile_node_off.assign(T + 1, 0);
    int64_t P = 0;
    int maxn = 0, maxv = 0;
    for (int64_t t = 0; t < T; t++) {
        L.tile_node_off[t] = (int32_t)P;
        P += ucount[t];
        maxn = std::max(maxn, ucount[t]);
        maxv = std::max(maxv, uval[t]);
    }
    L.max_tile_valence = maxv;
    if (P > INT32_MAX) {
        err = "mesh too large for 32-bit partial indices";
        return false;
    }
    L.tile_node_off[T] = (int32_t)P;
    L.P = P;
    L.max_tile_nodes = maxn;
    // pass 2: the tile node lists, packed
    L.tile_nodes.assign(P, 0);
    parallel_for(T, [&](int64_t a, int64_t b) {
        for (int64_t t = a; t < b; t++)
            std::memcpy(L.tile_nodes.data() + L.tile_node_off[t],
                        uniq.data() + npe * (int64_t)L.tile_elem_off[t],
                        sizeof(int32_t) * ucount[t]);
    }, 4);
    if (L.reorder && npe == 4) interior_first(L);
    else L.n_int = 0;
    slot_positions(L);
    node_corners(L);
    return true;
}

void pack_lconn(Layout& L) {
    std::vector<uint8_t>().swap(L.lconn_pk);
    if ((L.npe != 4 && L.npe != 8) || L.max_tile_nodes > kPackedMaxNodes) return;
    const int64_t E = L.E;
    if (L.npe == 8) {
        L.lconn_pk.resize(10 * E);
        uint8_t* words = L.lconn_pk.data();
        uint8_t* high = words + 8 * E;
        parallel_for(E, [&](int64_t a, int64_t b) {
            for (int64_t e = a; e < b; e++) {
                const uint16_t* c = &L.lconn[8 * e];
                uint64_t w = 0;
                for (int k = 0; k < 6; k++) w |= uint64_t(c[k]) << (10 * k);
                w |= uint64_t(c[6] & 15) << 60;
                const uint16_t hw = uint16_t((c[6] >> 4) | (c[7] << 6));
                std::memcpy(words + 8 * e, &w, 8);
                std::memcpy(high + 2 * e, &hw, 2);
            }
        }, 65536);
        return;
    }
    L.lconn_pk.resize(5 * E);
    uint8_t* words = L.lconn_pk.data();
    uint8_t* high = words + 4 * E;
    parallel_for(E, [&](int64_t a, int64_t b) {
        for (int64_t e = a; e < b; e++) {
            const uint16_t* c = &L.lconn[4 * e];
            const uint32_t w = uint32_t(c[0]) | uint32_t(c[1]) << 10 | uint32_t(c[2]) << 20 |
                               uint32_t(c[3] & 3) << 30;
            std::memcpy(words + 4 * e, &w, 4);
            high[e] = uint8_t(c[3] >> 2);
        }
    }, 65536);
}

// Corner relabelling of reordered hexahedral layouts.  Corner a of an
// eight-node element sits at natural coordinates xi_a in {-1, 1}^3 (bit 0 of
// kHexCorner[a] is xi, bit 1 eta, bit 2 zeta; set = +1).  A symmetry of the
// reference cube (an axis permutation with sign flips) relabels the corners
// without changing the element: with one integration point at the centre the
// element matrix depends on |det J| and the node set only.  Each element is
// relabelled so that its local axes g_j = sum_a xi_a,j x_a point along +x,
// +y, +z as far as the 48 symmetries allow.  On a lattice-like mesh the same
// corner of neighbouring elements is then a different node, so one
// accumulation step of the element pass (one corner of 64 elements) does
// not add to the same tile node twice.
constexpr int kHexCorner[8] = {0, 1, 3, 2, 4, 5, 7, 6};

void orient_hexahedra(Layout& L) {
    int corner_of[8];  // natural-coordinate bits -> corner index
    for (int a = 0; a < 8; a++) corner_of[kHexCorner[a]] = a;
    static const int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    parallel_for(L.E, [&](int64_t a0, int64_t b0) {
        for (int64_t e = a0; e < b0; e++) {
            int32_t* c = &L.conn[8 * e];
            double g[3][3] = {};  // g[j] = sum_a xi_a,j x_a
            for (int a = 0; a < 8; a++)
                for (int j = 0; j < 3; j++) {
                    const double s = (kHexCorner[a] >> j & 1) ? 1.0 : -1.0;
                    for (int k = 0; k < 3; k++) g[j][k] += s * L.xyz[3 * (int64_t)c[a] + k];
                }
            // new axis k is old axis perm[k] with sign sg[k]
            int best = 0;
            double best_v = -1.0;
            for (int p = 0; p < 6; p++) {
                double v = 0.0;
                for (int k = 0; k < 3; k++) v += std::fabs(g[kPerm[p][k]][k]);
                if (v > best_v) {
                    best_v = v;
                    best = p;
                }
            }
            int32_t old[8];
            std::memcpy(old, c, sizeof old);
            for (int a = 0; a < 8; a++) {
                int bits = 0;  // old natural coordinates of new corner a
                for (int k = 0; k < 3; k++) {
                    const int j = kPerm[best][k];
                    const bool plus = (kHexCorner[a] >> k & 1) != 0;
                    const bool flip = g[j][k] < 0.0;
                    if (plus != flip) bits |= 1 << j;
                }
                c[a] = old[corner_of[bits]];
            }
        }
    }, 16384);
}

bool build_layout(const double* xyz, const int32_t* conn, int npe, int64_t N, int64_t E,
                  int reorder, int TE, int MN, Layout& L, std::string& err) {
    L = Layout();
    L.N = N;
    L.E = E;
    L.npe = npe;
    L.reorder = reorder;
    if ((int64_t)npe * E > INT32_MAX) {
        err = "mesh too large for 32-bit element-corner indices";
        return false;
    }
    L.nperm.resize(N);
    L.ninv.resize(N);
    L.eperm.resize(E);
    if (reorder) {
        std::thread nodes([&] { L.nperm = morton_order(xyz, N); });
        std::vector<double> cen(3 * E);
        parallel_for(E, [&](int64_t a, int64_t b) {
            for (int64_t e = a; e < b; e++)
                for (int ax = 0; ax < 3; ax++) {
                    double s = 0;
                    for (int c = 0; c < npe; c++)
                        s += xyz[3 * (int64_t)conn[(int64_t)npe * e + c] + ax];
                    cen[3 * e + ax] = s / npe;
                }
        });
        L.eperm = morton_order(cen.data(), E);
        nodes.join();
    } else {
        std::iota(L.nperm.begin(), L.nperm.end(), 0);
        std::iota(L.eperm.begin(), L.eperm.end(), 0);
    }
    for (int64_t i = 0; i < N; i++) L.ninv[L.nperm[i]] = (int32_t)i;
    L.xyz.resize(3 * N);
    for (int64_t i = 0; i < N; i++)
        std::memcpy(&L.xyz[3 * i], xyz + 3 * (int64_t)L.nperm[i], 3 * sizeof(double));
    const int64_t S = (int64_t)npe * E;  // element corners
    L.conn.resize(S);
    for (int64_t e = 0; e < E; e++)
        for (int c = 0; c < npe; c++)
            L.conn[npe * e + c] = L.ninv[conn[(int64_t)npe * L.eperm[e] + c]];
    if (reorder && npe == 8) orient_hexahedra(L);
    return build_tiles(L, TE, MN, err);
}

}  // namespace fedfem
