// Time-stepping kernels for gfx950 (Algorithm 1, time-stepping block).
//
// Element pass (Eq 13, 17): one workgroup per tile of consecutive elements
// (Morton order), R elements per thread.  Each thread first issues the loads
// of its elements' six precomputed coefficients a_ab of A = V_tet B^T B
// (Eq 16) and their four local node ids into registers, so they are in
// flight while the tile's distinct nodes (temperature, and k(T) when
// conductivity depends on temperature) are staged in LDS.  Because every row
// of A sums to zero,
//     F_e,a = k_e sum_{b != a} a_ab (T_b - T_a),
// and with T = hi + lo the difference is formed as (hi_b - hi_a) +
// (lo_b - lo_a), accurate to float precision of the difference itself.
//
// Assembly inside the tile (Eq 11): each corner load is scaled by 2^S
// (exact) and rounded to a 64-bit integer, and the integers are added into
// one LDS accumulator per tile node with integer atomics.  Integer addition
// is associative, so the tile sums are exact and independent of the order in
// which lanes arrive: the step is bit-reproducible without floating-point
// atomics.  S is chosen per scenario so that the largest possible load maps
// below 2^58 (see the pre-computation), leaving 5 bits of headroom for the
// sum; loads are resolved to 2^-S, far below float precision of any load.
// Each tile node's sum, converted back once, is written as one partial at
// its tile-node slot, so every tile writes one contiguous, coalesced run; the
// node pass finds a node's slots through a node-major index.
//
// Node pass (Eq 11, 19): one thread per node adds its partials (gathered
// through the index) in ascending tile order and applies the explicit update
// with lumped capacity, perfusion, metabolic heat and the nodal source.  In the compensated float
// mode T is an interleaved (hi, lo) pair; the increment is added with an
// error-free TwoSum and the rounding error folded into lo (Knuth's TwoSum,
// Dekker's Fast2Sum renormalisation).  Dirichlet nodes (u <= 0) are never
// written: both ping-pong buffers hold T_Gamma.
//
// Block mapping: gfx950 deals workgroups to its 8 XCDs round-robin.  With
// xcd = 1 the kernels remap block b to tile (b % 8) * ceil(T / 8) + b / 8, so
// each XCD (and its L2) works through one contiguous stretch of the Morton
// curve; the node pass maps 256-node blocks the same way.
#include <hip/hip_runtime.h>

#include <mutex>
#include <set>
#include <utility>

#include "internal.h"

namespace fedfem {

namespace {

constexpr float kDivergeLimit = 1.0e4f;
constexpr int kXcds = 8;

template <typename Real>
__device__ __forceinline__ Real clampT(Real T, const Props<Real>& p) {
    return T < p.Tlo ? p.Tlo : (T > p.Thi ? p.Thi : T);
}

// piecewise-linear table (times t, values v, slopes s of n points),
// constant outside its range
template <typename Real>
__device__ __forceinline__ Real tab_eval(const Real* __restrict__ tb, int n, Real x) {
    const Real* t = tb;
    const Real* v = tb + kMaxTab;
    const Real* sl = tb + 2 * kMaxTab;
    if (!(x > t[0])) return v[0];
    int k = 0;
    while (k + 1 < n && t[k + 1] <= x) k++;
    if (k + 1 >= n) return v[n - 1];
    return v[k] + sl[k] * (x - t[k]);
}

// k(T) (Eq 13) and rho(T) c(T) (Eq 19): clamped linear laws or tables
template <typename Real>
__device__ __forceinline__ Real prop_k(Real T, const Props<Real>& p) {
    if (p.nt[0]) return tab_eval(p.tab, p.nt[0], T);
    return p.k0 + p.dk * (clampT(T, p) - p.Tref);
}

template <typename Real>
__device__ __forceinline__ Real prop_rho_c(Real T, const Props<Real>& p) {
    const Real dT = clampT(T, p) - p.Tref;
    const Real rho = p.nt[1] ? tab_eval(p.tab + 3 * kMaxTab, p.nt[1], T) : p.rho0 + p.drho * dT;
    const Real c = p.nt[2] ? tab_eval(p.tab + 6 * kMaxTab, p.nt[2], T) : p.c0 + p.dc * dT;
    return rho * c;
}

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// Nodal state access: FP32C stores float2 (hi, lo), FP64 stores double.
template <typename Real, bool COMP>
struct State;
template <>
struct State<float, true> {
    __device__ static void load(const void* T, int64_t i, float& hi, float& lo) {
        const float2 v = static_cast<const float2*>(T)[i];
        hi = v.x;
        lo = v.y;
    }
    __device__ static void store(void* T, int64_t i, float hi, float lo) {
        static_cast<float2*>(T)[i] = make_float2(hi, lo);
    }
};
template <>
struct State<double, false> {
    __device__ static void load(const void* T, int64_t i, double& hi, double& lo) {
        hi = static_cast<const double*>(T)[i];
        lo = 0.0;
    }
    __device__ static void store(void* T, int64_t i, double hi, double) {
        static_cast<double*>(T)[i] = hi;
    }
};

struct LdsCarve {
    size_t acc, T, Tlo, k, total;
};

// Per tile node: a 64-bit accumulator, T (hi, lo) and k(T).  With COMP the
// T and Tlo regions are used together as one float2 array starting at T.
__host__ __device__ inline LdsCarve carve(int TE, int maxn, int rb, bool comp, bool td) {
    (void)TE;
    LdsCarve c;
    c.acc = 0;
    c.T = align16(c.acc + sizeof(unsigned long long) * (size_t)maxn);
    c.Tlo = align16(c.T + (size_t)rb * maxn);
    c.k = align16(c.Tlo + (comp ? (size_t)rb * maxn : 0));
    c.total = align16(c.k + (td ? (size_t)rb * maxn : 0));
    return c;
}

__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t n) {
    const int64_t per = (n + kXcds - 1) / kXcds;
    return (b % kXcds) * per + b / kXcds;
}

struct TileArgs {
    int64_t E;     // plane stride of the coefficient arrays
    int64_t T;     // number of tiles
    int TE, maxn;  // LDS sizing
    int xcd;       // remap blocks to XCD-contiguous tiles
    const int32_t* tile_elem_off;
    const int32_t* tile_node_off;
    const int32_t* tile_nodes;
    const int4* tile_part;  // per tile: its single-tile nodes and where its partials go
    const void* lconn;  // packed 10-bit ids (lconn_pk) or [4E] u16
    int lconn_pk;
};

// The four tile-local corner ids of one element from its raw connectivity
// record: (word, high byte) of the packed form, or two words of u16 pairs.
__device__ __forceinline__ void corner_ids(uint2 r, bool pk, int (&n)[4]) {
    if (pk) {
        n[0] = (int)(r.x & 1023u);
        n[1] = (int)((r.x >> 10) & 1023u);
        n[2] = (int)((r.x >> 20) & 1023u);
        n[3] = (int)((r.x >> 30) | (r.y << 2));
    } else {
        n[0] = (int)(r.x & 0xffffu);
        n[1] = (int)(r.x >> 16);
        n[2] = (int)(r.y & 0xffffu);
        n[3] = (int)(r.y >> 16);
    }
}

__device__ __forceinline__ long long to_fixed(float f, float scale) {
    return __float2ll_rn(f * scale);
}
__device__ __forceinline__ long long to_fixed(double f, double scale) {
    return __double2ll_rn(f * scale);
}

// Per-element data is read once per step: non-temporal loads keep it from
// displacing the node temperatures and partials in the caches.
template <typename T>
__device__ __forceinline__ T stream_load(const T* p) {
    return __builtin_nontemporal_load(p);
}

// Tile-node temperatures in LDS: FP64 T, or (FP32C) the (hi, lo) pair of a
// node side by side, so that one 64-bit LDS read fetches both.
template <bool COMP, typename Real>
__device__ __forceinline__ void store_T(Real* s_T, int j, Real hi, Real lo) {
    if constexpr (COMP) reinterpret_cast<float2*>(s_T)[j] = make_float2(hi, lo);
    else s_T[j] = hi;
}
template <bool COMP, typename Real>
__device__ __forceinline__ void load_T(const Real* s_T, int j, Real& hi, Real& lo) {
    if constexpr (COMP) {
        const float2 v = reinterpret_cast<const float2*>(s_T)[j];
        hi = v.x;
        lo = v.y;
    } else {
        hi = s_T[j];
        lo = Real(0);
    }
}

// A tile's list starts with its ni single-tile nodes, ids n0 .. n0 + ni - 1;
// list position j writes its partial to pi + j when j < ni, else ps + j.
struct TilePart {
    int pi, ni, ps, n0;
    __device__ __forceinline__ int pos(int j) const { return j < ni ? pi + j : ps + j; }
    // the id is loaded either way (a select, not a branch, so that the load
    // does not make the compiler wait for every load before it)
    __device__ __forceinline__ int node(const TileArgs& a, int p0, int j) const {
        const int g = a.tile_nodes[p0 + j];
        return j < ni ? n0 + j : g;
    }
};
__device__ __forceinline__ TilePart tile_part(const TileArgs& a, int64_t t) {
    const int4 v = a.tile_part[t];
    return TilePart{v.x, v.y, v.z, v.w};
}

// Tile nodes into LDS: temperature, conductivity, zeroed accumulators.  The
// first SJ rounds go out together, list entries (stage_ids) then
// temperatures (lanes past the list load its last node and store nothing),
// so a thread waits for two memory round trips instead of two per round.
// Single-tile nodes' ids follow from the list position.
constexpr int kStageRounds = 2;

// The raw list entries of the first rounds.  The tetrahedral pass issues
// them before its element loads, so that the temperature loads wait for
// these alone.
__device__ __forceinline__ void stage_ids(const TileArgs& a, int p0, int m,
                                          int (&graw)[kStageRounds]) {
#pragma unroll
    for (int u = 0; u < kStageRounds; u++)
        graw[u] = a.tile_nodes[p0 + min((int)threadIdx.x + u * (int)blockDim.x, m - 1)];
}

template <typename Real, bool COMP, bool TD>
__device__ __forceinline__ void stage_tile_nodes(const TileArgs& a, int p0, int m,
                                                 const TilePart& tp,
                                                 const int (&graw)[kStageRounds],
                                                 const void* __restrict__ Tin,
                                                 const Props<Real>& pr, Real* s_T,
                                                 Real* s_k, unsigned long long* s_acc) {
    const int tid = threadIdx.x, bs = blockDim.x;
    constexpr int SJ = kStageRounds;
    {
        int gj[SJ];
#pragma unroll
        for (int u = 0; u < SJ; u++) {
            const int j = min(tid + u * bs, m - 1);
            gj[u] = j < tp.ni ? tp.n0 + j : graw[u];
        }
        Real hj[SJ], lj[SJ];
#pragma unroll
        for (int u = 0; u < SJ; u++) State<Real, COMP>::load(Tin, gj[u], hj[u], lj[u]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < SJ; u++) {
            const int j = tid + u * bs;
            if (j < m) {
                store_T<COMP>(s_T, j, hj[u], lj[u]);
                if (TD) s_k[j] = prop_k(hj[u], pr);
                s_acc[j] = 0ull;
            }
        }
    }
    for (int j = tid + SJ * bs; j < m; j += bs) {
        const int g = tp.node(a, p0, j);
        Real hi, lo;
        State<Real, COMP>::load(Tin, g, hi, lo);
        store_T<COMP>(s_T, j, hi, lo);
        if (TD) s_k[j] = prop_k(hi, pr);
        s_acc[j] = 0ull;
    }
}

template <typename Real, bool COMP, bool TD, int R>
__device__ __forceinline__ void elem_tile(const TileArgs& a, int64_t t,
                                          const Real* __restrict__ coef,
                                          const void* __restrict__ Tin,
                                          Real* __restrict__ partial, const Props<Real>& pr) {
    extern __shared__ __align__(16) unsigned char lds[];
    const LdsCarve c = carve(a.TE, a.maxn, sizeof(Real), COMP, TD);
    unsigned long long* s_acc = reinterpret_cast<unsigned long long*>(lds + c.acc);
    Real* s_T = reinterpret_cast<Real*>(lds + c.T);
    Real* s_k = reinterpret_cast<Real*>(lds + c.k);

    const int tid = threadIdx.x, bs = blockDim.x;
    const int64_t e0 = a.tile_elem_off[t];
    const int ne = (int)(a.tile_elem_off[t + 1] - e0);
    const int p0 = a.tile_node_off[t];
    const int m = a.tile_node_off[t + 1] - p0;
    const TilePart tp = tile_part(a, t);

    // 0. the first rounds' tile-node list entries
    int graw[kStageRounds];
    stage_ids(a, p0, m, graw);
    __builtin_amdgcn_sched_barrier(0);
    // 1. coefficient and local-connectivity loads in flight during staging
    Real cf[R][6];
    uint2 lc[R];
    const bool pk = a.lconn_pk != 0;
    const uint2* glc = static_cast<const uint2*>(a.lconn) + e0;
    const uint32_t* gw = static_cast<const uint32_t*>(a.lconn) + e0;
    const uint8_t* gb = static_cast<const uint8_t*>(a.lconn) + 4 * a.E + e0;
    // (lanes past the tile reload its last element: straight-line loads, so
    // that the staging below waits for the list entries only)
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int el = min(tid + r * bs, ne - 1);
#pragma unroll
        for (int k = 0; k < 6; k++) cf[r][k] = stream_load(&coef[k * a.E + e0 + el]);
        if (pk) {
            lc[r] = make_uint2(stream_load(&gw[el]), gb[el]);
        } else {
            const unsigned long long w = stream_load(
                reinterpret_cast<const unsigned long long*>(glc) + el);
            lc[r] = make_uint2((unsigned)w, (unsigned)(w >> 32));
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    // 2. tile nodes
    stage_tile_nodes<Real, COMP, TD>(a, p0, m, tp, graw, Tin, pr, s_T, s_k, s_acc);
    __syncthreads();
    // 3. element loads, accumulated exactly on the fixed-point grid
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int el = tid + r * bs;
        if (el < ne) {
            int n[4];
            corner_ids(lc[r], pk, n);
            Real h0, h1, h2, h3, l0, l1, l2, l3;
            load_T<COMP>(s_T, n[0], h0, l0);
            load_T<COMP>(s_T, n[1], h1, l1);
            load_T<COMP>(s_T, n[2], h2, l2);
            load_T<COMP>(s_T, n[3], h3, l3);
            Real d01 = h1 - h0, d02 = h2 - h0, d03 = h3 - h0;
            Real d12 = h2 - h1, d13 = h3 - h1, d23 = h3 - h2;
            if (COMP) {
                d01 += l1 - l0;
                d02 += l2 - l0;
                d03 += l3 - l0;
                d12 += l2 - l1;
                d13 += l3 - l1;
                d23 += l3 - l2;
            }
            Real ke;
            if (TD)
                ke = (s_k[n[0]] + s_k[n[1]] + s_k[n[2]] + s_k[n[3]]) * Real(0.25);
            else
                ke = pr.k0;
            const Real g01 = cf[r][0] * d01, g02 = cf[r][1] * d02, g03 = cf[r][2] * d03;
            const Real g12 = cf[r][3] * d12, g13 = cf[r][4] * d13, g23 = cf[r][5] * d23;
            const long long v[4] = {to_fixed(ke * ((g01 + g02) + g03), pr.fxs),
                                    to_fixed(ke * ((g12 + g13) - g01), pr.fxs),
                                    to_fixed(ke * (g23 - (g02 + g12)), pr.fxs),
                                    to_fixed(-ke * ((g03 + g13) + g23), pr.fxs)};
            // rotate the corner order across lanes to spread LDS conflicts
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int cc = (q + tid) & 3;
                atomicAdd(&s_acc[n[cc]], (unsigned long long)v[cc]);
            }
        }
    }
    __syncthreads();
    // 4. one partial per tile node: the single-tile nodes' at their own
    // index, the others' in the tile's run of the tile-major part
    for (int j = tid; j < m; j += bs) partial[tp.pos(j)] = (Real)(long long)s_acc[j] * pr.fxi;
}

template <typename Real, bool COMP, bool TD, int R>
__global__ void __launch_bounds__(1024)
k_elem_loads(TileArgs a, const Real* __restrict__ coef, const void* __restrict__ Tin,
             Real* __restrict__ partial, Props<Real> pr) {
    const int64_t t = a.xcd ? xcd_remap(blockIdx.x, a.T) : (int64_t)blockIdx.x;
    if (t >= a.T) return;
    elem_tile<Real, COMP, TD, R>(a, t, coef, Tin, partial, pr);
}

// Eight-node hexahedra with one integration point (Eq 14, 16, 17).  The
// element is stored as the symmetric 3 x 3 matrix S with
// A_e[a][b] = xi_a^T S xi_b (xi_a in {-1, 1}^3, the corner's natural
// coordinates; entries S00, S11, S22, S01, S02, S12 at coef[k E + e]), so
//     F_e,a = k_e xi_a . (S t),   t = sum_b xi_b (T_b - T_0),
// the differences formed as (hi_b - hi_0) + (lo_b - lo_0) (each component of
// xi sums to zero over the corners, so T_0 drops out of t).  k_e is the mean
// over the eight corners (Eq 13).  Tiles, staging, fixed-point assembly and
// partials are those of the tetrahedral pass; local corner ids are 8 x 10
// bits (tiles of at most 1024 nodes) or 8 x u16.
template <typename Real, bool COMP, bool TD, int R>
__device__ __forceinline__ void elem_tile_hex(const TileArgs& a, int64_t t,
                                              const Real* __restrict__ coef,
                                              const void* __restrict__ Tin,
                                              Real* __restrict__ partial,
                                              const Props<Real>& pr) {
    extern __shared__ __align__(16) unsigned char lds[];
    const LdsCarve c = carve(a.TE, a.maxn, sizeof(Real), COMP, TD);
    unsigned long long* s_acc = reinterpret_cast<unsigned long long*>(lds + c.acc);
    Real* s_T = reinterpret_cast<Real*>(lds + c.T);
    Real* s_k = reinterpret_cast<Real*>(lds + c.k);

    const int tid = threadIdx.x, bs = blockDim.x;
    const int64_t e0 = a.tile_elem_off[t];
    const int ne = (int)(a.tile_elem_off[t + 1] - e0);
    const int p0 = a.tile_node_off[t];
    const int m = a.tile_node_off[t + 1] - p0;
    // hexahedral layouts keep tile-major positions for every tile node
    const TilePart tp{0, 0, p0, 0};

    // 1. coefficient and local-connectivity loads in flight during staging:
    // eight 10-bit ids as a 64-bit word and a 16-bit word (packed), or eight
    // u16 as one 16-byte load
    Real sv[R][6];
    uint4 lc[R];
    const bool pk = a.lconn_pk != 0;
    const uint4* glc = static_cast<const uint4*>(a.lconn) + e0;
    const unsigned long long* gw = static_cast<const unsigned long long*>(a.lconn) + e0;
    const uint16_t* gh = reinterpret_cast<const uint16_t*>(
                             static_cast<const unsigned long long*>(a.lconn) + a.E) + e0;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int el = tid + r * bs;
        if (el < ne) {
#pragma unroll
            for (int k = 0; k < 6; k++) sv[r][k] = stream_load(&coef[k * a.E + e0 + el]);
            if (pk) {
                const unsigned long long w = gw[el];
                lc[r] = make_uint4((unsigned)w, (unsigned)(w >> 32), gh[el], 0u);
            } else {
                lc[r] = glc[el];
            }
        }
    }
    // 2. tile nodes
    int graw[kStageRounds];
    stage_ids(a, p0, m, graw);
    __builtin_amdgcn_sched_barrier(0);  // all list loads before any wait
    stage_tile_nodes<Real, COMP, TD>(a, p0, m, tp, graw, Tin, pr, s_T, s_k, s_acc);
    __syncthreads();
    // 3. element loads, accumulated exactly on the fixed-point grid
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int el = tid + r * bs;
        if (el < ne) {
            int n[8];
            if (pk) {
                const unsigned long long w =
                    (unsigned long long)lc[r].x | ((unsigned long long)lc[r].y << 32);
#pragma unroll
                for (int q = 0; q < 6; q++) n[q] = (int)((w >> (10 * q)) & 1023u);
                n[6] = (int)((w >> 60) | ((lc[r].z & 63u) << 4));
                n[7] = (int)(lc[r].z >> 6);
            } else {
                const unsigned ww[4] = {lc[r].x, lc[r].y, lc[r].z, lc[r].w};
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    n[2 * q] = (int)(ww[q] & 0xffffu);
                    n[2 * q + 1] = (int)(ww[q] >> 16);
                }
            }
            Real h0, l0;
            load_T<COMP>(s_T, n[0], h0, l0);
            Real d[8];
            d[0] = 0;
#pragma unroll
            for (int b = 1; b < 8; b++) {
                Real hb, lb;
                load_T<COMP>(s_T, n[b], hb, lb);
                d[b] = hb - h0;
                if (COMP) d[b] += lb - l0;
            }
            // t = sum_b xi_b d_b, corners in the order of the natural
            // coordinates (-,-,-), (+,-,-), (+,+,-), (-,+,-), then z = +1
            const Real t0 = ((d[1] + d[2]) + (d[5] + d[6])) - ((d[3] + d[4]) + d[7]);
            const Real t1 = ((d[2] + d[3]) + (d[6] + d[7])) - ((d[1] + d[4]) + d[5]);
            const Real t2 = ((d[4] + d[5]) + (d[6] + d[7])) - ((d[1] + d[2]) + d[3]);
            Real ke;
            if (TD) {
                Real ks = 0;
#pragma unroll
                for (int b = 0; b < 8; b++) ks += s_k[n[b]];
                ke = ks * Real(0.125);
            } else {
                ke = pr.k0;
            }
            const Real u0 = ke * ((sv[r][0] * t0 + sv[r][3] * t1) + sv[r][4] * t2);
            const Real u1 = ke * ((sv[r][3] * t0 + sv[r][1] * t1) + sv[r][5] * t2);
            const Real u2 = ke * ((sv[r][4] * t0 + sv[r][5] * t1) + sv[r][2] * t2);
            // F_a = xi_a . u, formed on the fixed-point grid from the three
            // converted components: exact integer sums, so the eight corner
            // loads of an element add up to zero exactly (|u_i| is at most
            // max_a |F_a|, so the scale's bound holds)
            const long long U0 = to_fixed(u0, pr.fxs), U1 = to_fixed(u1, pr.fxs),
                            U2 = to_fixed(u2, pr.fxs);
            const long long P = U0 + U1, M = U0 - U1;
            const long long F[8] = {-P - U2, M - U2, P - U2, -M - U2,
                                    U2 - P, M + U2, P + U2, U2 - M};
#pragma unroll
            for (int q = 0; q < 8; q++) atomicAdd(&s_acc[n[q]], (unsigned long long)F[q]);
        }
    }
    __syncthreads();
    // 4. one partial per tile node, placed as in the tetrahedral pass
    for (int j = tid; j < m; j += bs) partial[tp.pos(j)] = (Real)(long long)s_acc[j] * pr.fxi;
}

template <typename Real, bool COMP, bool TD, int R>
__global__ void __launch_bounds__(1024)
k_elem_loads_hex(TileArgs a, const Real* __restrict__ coef, const void* __restrict__ Tin,
                 Real* __restrict__ partial, Props<Real> pr) {
    const int64_t t = a.xcd ? xcd_remap(blockIdx.x, a.T) : (int64_t)blockIdx.x;
    if (t >= a.T) return;
    elem_tile_hex<Real, COMP, TD, R>(a, t, coef, Tin, partial, pr);
}

// Batched form: the workgroup's tile comes from a list of active tiles and
// its material from the tile's scenario.
template <typename Real, bool COMP, int R>
__global__ void __launch_bounds__(1024)
k_elem_loads_batch(TileArgs a, const int32_t* __restrict__ tile_list,
                   const int32_t* __restrict__ tile_scen, const Real* __restrict__ coef,
                   const void* __restrict__ Tin, Real* __restrict__ partial,
                   const Props<Real>* __restrict__ props) {
    const int64_t t = tile_list[blockIdx.x];
    const Props<Real> pr = props[tile_scen[t]];
    elem_tile<Real, COMP, true, R>(a, t, coef, Tin, partial, pr);
}

// Scheduled source patterns of one step: n_pat patterns [n_pat][N] and this
// step's amplitudes amp[0..n_pat) (none when n_pat == 0).
template <typename Real>
struct Sched {
    const Real* pat;
    const Real* amp;
    int n_pat;
    int64_t N;
};

// Thermal dose of one step (none when acc is null): node i adds
// dt * a * f(T_i) with T_i its temperature at the start of the step;
// model 1 (CEM43): f = 2^(T - 43) at or above 43 C, 4^(T - 43) below;
// model 2 (Arrhenius): f = exp(-b / (T + 273.15)), b = E_a / R_gas.
struct Dose {
    double* acc;
    int model;
    double a, b, dt;
};

__device__ __forceinline__ double dose_rate(const Dose& dz, double T) {
    if (dz.model == 1) return exp2(T >= 43.0 ? T - 43.0 : 2.0 * (T - 43.0)) * dz.a;
    return exp(-dz.b / (T + 273.15)) * dz.a;
}

// NPT nodes per thread (indices at or above N are skipped): their chains of
// dependent loads (node data, slot indices, partials) run side by side.
// Nodes below n_int are single-tile nodes: their one partial sits at their
// own index plus pshift (0 but in batched copies) and is loaded with the
// node's own data.
template <typename Real, bool COMP, int NPT>
__device__ __forceinline__ void node_update(const int64_t (&iv)[NPT], int64_t N, int64_t n_int,
                                            int64_t pshift,
                                            const int32_t* __restrict__ part_off,
                                            const int32_t* __restrict__ pidx,
                                            const Real* __restrict__ partial,
                                            const Real* __restrict__ u,
                                            const Real* __restrict__ q,
                                            const void* __restrict__ Tin, void* __restrict__ Tout,
                                            const Props<Real>& pr, int* __restrict__ flag,
                                            const Sched<Real>& sch, const Dose& dz) {
    // every load that depends only on the node first, so a node waits for
    // three rounds of memory latency: these, the slot indices, the partials
    // (one round for single-tile nodes, whose slot lists are not read).  The
    // loads go out unconditionally, so that none waits on a branch: a node
    // reads the slot offsets or the partial at index 0 where it needs none
    // (one shared cache line per wave).
    Real ui[NPT], q0[NPT], hi[NPT], lo[NPT], fs[NPT];
    int a[NPT], n[NPT];
#pragma unroll
    for (int v = 0; v < NPT; v++) {
        const int64_t i = iv[v] < N ? iv[v] : 0;
        const bool single = i < n_int;
        ui[v] = u[i];
        const int64_t io = single ? 0 : i;
        a[v] = part_off[io];
        n[v] = part_off[io + 1];
        fs[v] = partial[single ? i + pshift : 0];
        q0[v] = q[i];
        State<Real, COMP>::load(Tin, i, hi[v], lo[v]);
    }
#pragma unroll
    for (int v = 0; v < NPT; v++) {
        const bool single = (iv[v] < N ? iv[v] : 0) < n_int;
        n[v] = single ? 0 : n[v] - a[v];
        if (!single) fs[v] = Real(0);
    }
    // the first four slots of every other node, indices then partials
    int pk[NPT][4];
    Real f[NPT][4];
#pragma unroll
    for (int v = 0; v < NPT; v++)
#pragma unroll
        for (int k = 0; k < 4; k++) pk[v][k] = k < n[v] ? pidx[a[v] + k] : -1;
#pragma unroll
    for (int v = 0; v < NPT; v++)
#pragma unroll
        for (int k = 0; k < 4; k++) f[v][k] = pk[v][k] >= 0 ? partial[pk[v][k]] : Real(0);
    // dose at the step's starting temperature, held nodes included
    if (dz.acc) {
#pragma unroll
        for (int v = 0; v < NPT; v++)
            if (iv[v] < N)
                dz.acc[iv[v]] += dz.dt * dose_rate(dz, (double)hi[v] + (double)lo[v]);
    }
#pragma unroll
    for (int v = 0; v < NPT; v++) {
        // Dirichlet nodes (u <= 0) are held at T_Gamma
        if (iv[v] >= N || !(ui[v] > Real(0))) continue;
        // partials added in ascending tile order
        Real F = fs[v];
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (k < n[v]) F += f[v][k];
        for (int k = 4; k < n[v]; k++) F += partial[pidx[a[v] + k]];
        const int64_t i = iv[v];
        Real qi = q0[v];
        for (int p = 0; p < sch.n_pat; p++) qi += sch.amp[p] * sch.pat[p * sch.N + i];
        const Real rc = prop_rho_c(hi[v], pr);
        // heat flow per unit volume [W/m^3]: source and conduction per lumped
        // volume, metabolic heat, perfusion towards T_a
        const Real R = (qi - F) * ui[v] + pr.Qm + pr.wbcb * ((pr.Ta - hi[v]) - lo[v]);
        const Real d = pr.dt * R / rc;
        Real nh, nl = 0;
        if (COMP) {
            // TwoSum(hi, d) = s + err exactly
            const Real s = hi[v] + d;
            const Real bp = s - hi[v];
            const Real err = (hi[v] - (s - bp)) + (d - bp);
            const Real l2 = lo[v] + err;
            // Fast2Sum(s, l2): |s| >= |l2|
            nh = s + l2;
            nl = l2 - (nh - s);
        } else {
            nh = hi[v] + d;
        }
        State<Real, COMP>::store(Tout, i, nh, nl);
        if (!(nh < Real(kDivergeLimit) && nh > -Real(kDivergeLimit))) *flag = 1;
    }
}

constexpr int kNodesPerThread = 1;

// With the XCD remap, blocks wholly below n_int (single-tile nodes only) and
// the others are remapped separately, so that every XCD gets its share of
// each kind.
template <typename Real, bool COMP>
__global__ void __launch_bounds__(256)
k_node_update(int64_t N, int64_t n_int, int xcd, const int32_t* __restrict__ part_off,
              const int32_t* __restrict__ pidx, const Real* __restrict__ partial, const Real* __restrict__ u,
              const Real* __restrict__ q, const void* __restrict__ Tin, void* __restrict__ Tout,
              Props<Real> pr, int* __restrict__ flag, Sched<Real> sch, Dose dz) {
    constexpr int64_t span = 256 * kNodesPerThread;
    const int64_t nb = (N + span - 1) / span;
    int64_t blk = blockIdx.x;
    if (xcd) {
        const int64_t nbf = n_int / span, gf = (nbf + kXcds - 1) / kXcds * kXcds;
        if (blk < gf) {
            blk = xcd_remap(blk, nbf);
            if (blk >= nbf) return;
        } else {
            blk = xcd_remap(blk - gf, nb - nbf);
            if (blk >= nb - nbf) return;
            blk += nbf;
        }
    }
    if (blk >= nb) return;
    int64_t iv[kNodesPerThread];
#pragma unroll
    for (int v = 0; v < kNodesPerThread; v++) iv[v] = blk * span + v * 256 + threadIdx.x;
    node_update<Real, COMP, kNodesPerThread>(iv, N, n_int, 0, part_off, pidx, partial, u, q, Tin,
                                             Tout, pr, flag, sch, dz);
}

// Batched form: 256-node blocks never straddle scenarios; the block comes
// from a list of active blocks, its material and where its single-tile nodes
// end from the block's scenario.
template <typename Real, bool COMP>
__global__ void __launch_bounds__(256)
k_node_update_batch(const int32_t* __restrict__ block_list,
                    const int32_t* __restrict__ block_scen,
                    const int32_t* __restrict__ part_off, const int32_t* __restrict__ pidx,
                    const Real* __restrict__ partial,
                    const Real* __restrict__ u, const Real* __restrict__ q,
                    const void* __restrict__ Tin, void* __restrict__ Tout,
                    const Props<Real>* __restrict__ props,
                    const int2* __restrict__ scen_single, int* __restrict__ flags) {
    const int blk = block_list[blockIdx.x];
    const int sc = block_scen[blk];
    const Props<Real> pr = props[sc];
    const int2 ss = scen_single[sc];
    const int64_t iv[1] = {(int64_t)blk * 256 + threadIdx.x};
    node_update<Real, COMP, 1>(iv, INT64_MAX, ss.x, ss.y, part_off, pidx, partial, u, q, Tin,
                               Tout, pr, flags + sc, Sched<Real>{nullptr, nullptr, 0, 0},
                               Dose{nullptr, 0, 0.0, 0.0, 0.0});
}

TileArgs tile_args(const DevLayout& d) {
    TileArgs a;
    a.E = d.E;
    a.T = d.T;
    a.TE = d.tile_elems;
    a.maxn = d.max_tile_nodes;
    a.xcd = d.xcd;
    a.tile_elem_off = d.tile_elem_off;
    a.tile_node_off = d.tile_node_off;
    a.tile_nodes = d.tile_nodes;
    a.tile_part = reinterpret_cast<const int4*>(d.tile_part);
    a.lconn = d.lconn;
    a.lconn_pk = d.lconn_pk;
    return a;
}

__global__ void k_lconn_unpack(const uint32_t* __restrict__ words, const uint8_t* __restrict__ high,
                               int64_t E, ushort4* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    int n[4];
    corner_ids(make_uint2(words[e], high[e]), true, n);
    out[e] = make_ushort4((unsigned short)n[0], (unsigned short)n[1], (unsigned short)n[2],
                          (unsigned short)n[3]);
}

// Dynamic LDS above 64 KiB must be allowed per kernel.  The attribute is
// process-wide state of the kernel, so it is set once per kernel (to the
// device's LDS limit, enough for every layout) under a lock: rewriting it on
// every launch would race with launches of the same kernel from other host
// threads (precompute of several handles at once).
std::mutex g_lds_mu;
std::set<std::pair<int, const void*>> g_lds_done;  // (device, kernel)

template <typename K>
hipError_t allow_lds(K kern, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    const void* f = reinterpret_cast<const void*>(kern);
    int dev = 0, limit = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_lds_mu);
    if (g_lds_done.count({dev, f})) return hipSuccess;
    e = hipDeviceGetAttribute(&limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    if ((size_t)limit < lds) return hipErrorInvalidValue;
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, limit);
    if (e == hipSuccess) g_lds_done.insert({dev, f});
    return e;
}

template <typename Real, bool COMP, bool TD, int R>
hipError_t launch_elem_r(const DevLayout& d, const Real* coef, const Props<Real>& p,
                         const void* Tin, Real* partial, hipStream_t s) {
    const size_t lds = carve(d.tile_elems, d.max_tile_nodes, sizeof(Real), COMP, TD).total;
    if (d.npe == 8 && d.n_int != 0) return hipErrorInvalidValue;  // tile-major hexahedra only
    auto kern = d.npe == 8 ? k_elem_loads_hex<Real, COMP, TD, R> : k_elem_loads<Real, COMP, TD, R>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    const int64_t grid = d.xcd ? (d.T + kXcds - 1) / kXcds * kXcds : d.T;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(d.threads), lds, s, tile_args(d), coef,
                       Tin, partial, p);
    return hipGetLastError();
}

template <typename Real, bool COMP, bool TD>
hipError_t launch_elem_t(const DevLayout& d, const Real* coef, const Props<Real>& p,
                         const void* Tin, Real* partial, hipStream_t s) {
    switch (elems_per_thread(d)) {
        case 1: return launch_elem_r<Real, COMP, TD, 1>(d, coef, p, Tin, partial, s);
        case 2: return launch_elem_r<Real, COMP, TD, 2>(d, coef, p, Tin, partial, s);
        case 4: return launch_elem_r<Real, COMP, TD, 4>(d, coef, p, Tin, partial, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename Real, bool COMP>
hipError_t launch_node_t(const DevLayout& d, int cur, const Props<Real>& p, int* flag,
                         hipStream_t s, int j) {
    constexpr int64_t span = 256 * kNodesPerThread;
    const int64_t nb = (d.N + span - 1) / span, nbf = d.n_int / span;
    const int64_t grid = d.xcd ? (nbf + kXcds - 1) / kXcds * kXcds +
                                     (nb - nbf + kXcds - 1) / kXcds * kXcds
                               : nb;
    Sched<Real> sch{static_cast<const Real*>(d.pat),
                    d.n_pat ? static_cast<const Real*>(d.amp) + (int64_t)j * d.n_pat : nullptr,
                    d.n_pat, d.N};
    hipLaunchKernelGGL((k_node_update<Real, COMP>), dim3((unsigned)grid), dim3(256), 0, s, d.N,
                       d.n_int, d.xcd, d.part_off, d.pidx, static_cast<const Real*>(d.partial),
                       static_cast<const Real*>(d.u), static_cast<const Real*>(d.q), d.T_[cur],
                       d.T_[1 - cur], p, flag, sch,
                       Dose{d.dose, d.dose_model, d.dose_a, d.dose_b, d.dose_dt});
    return hipGetLastError();
}

template <typename Real, bool COMP, int R>
hipError_t launch_elem_batch_r(const DevLayout& d, const BatchTables& b, int cur, int n_tiles,
                               hipStream_t s) {
    const size_t lds = carve(d.tile_elems, d.max_tile_nodes, sizeof(Real), COMP, true).total;
    auto kern = k_elem_loads_batch<Real, COMP, R>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n_tiles), dim3(d.threads), lds, s, tile_args(d), b.tile_list,
                       b.tile_scen, static_cast<const Real*>(d.coef), d.T_[cur],
                       static_cast<Real*>(d.partial), static_cast<const Props<Real>*>(b.props));
    return hipGetLastError();
}

template <typename Real, bool COMP>
hipError_t launch_elem_batch_t(const DevLayout& d, const BatchTables& b, int cur, int n_tiles,
                               hipStream_t s) {
    switch (elems_per_thread(d)) {
        case 1: return launch_elem_batch_r<Real, COMP, 1>(d, b, cur, n_tiles, s);
        case 2: return launch_elem_batch_r<Real, COMP, 2>(d, b, cur, n_tiles, s);
        case 4: return launch_elem_batch_r<Real, COMP, 4>(d, b, cur, n_tiles, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int elems_per_thread(const DevLayout& d) {
    const int r = (d.tile_elems + d.threads - 1) / d.threads;
    return r <= 1 ? 1 : (r <= 2 ? 2 : (r <= 4 ? 4 : 8));
}

size_t tile_lds_bytes(int TE, int maxn, int rb, bool comp, bool td) {
    return carve(TE, maxn, rb, comp, td).total;
}

hipError_t launch_elem_f32c(const DevLayout& d, int cur, const Props<float>& p, bool td,
                            hipStream_t s) {
    const float* cf = static_cast<const float*>(d.coef);
    float* part = static_cast<float*>(d.partial);
    return td ? launch_elem_t<float, true, true>(d, cf, p, d.T_[cur], part, s)
              : launch_elem_t<float, true, false>(d, cf, p, d.T_[cur], part, s);
}

hipError_t launch_node_f32c(const DevLayout& d, int cur, const Props<float>& p, int* flag,
                            hipStream_t s) {
    return launch_node_t<float, true>(d, cur, p, flag, s, 0);
}

hipError_t launch_elem_f64(const DevLayout& d, int cur, const Props<double>& p, bool td,
                           hipStream_t s) {
    const double* cf = static_cast<const double*>(d.coef);
    double* part = static_cast<double*>(d.partial);
    return td ? launch_elem_t<double, false, true>(d, cf, p, d.T_[cur], part, s)
              : launch_elem_t<double, false, false>(d, cf, p, d.T_[cur], part, s);
}

hipError_t launch_node_f64(const DevLayout& d, int cur, const Props<double>& p, int* flag,
                           hipStream_t s) {
    return launch_node_t<double, false>(d, cur, p, flag, s, 0);
}

hipError_t launch_step_f32c(const DevLayout& d, int cur, const Props<float>& p, bool td,
                            int* flag, hipStream_t s, int j) {
    hipError_t e = launch_elem_f32c(d, cur, p, td, s);
    if (e != hipSuccess) return e;
    return launch_node_t<float, true>(d, cur, p, flag, s, j);
}

hipError_t launch_step_f64(const DevLayout& d, int cur, const Props<double>& p, bool td,
                           int* flag, hipStream_t s, int j) {
    hipError_t e = launch_elem_f64(d, cur, p, td, s);
    if (e != hipSuccess) return e;
    return launch_node_t<double, false>(d, cur, p, flag, s, j);
}

hipError_t launch_geometry_apply(const DevLayout& d, const double* coef64, const double* x,
                                 double* partial, double fx_scale, hipStream_t s) {
    Props<double> p{};
    p.k0 = 1.0;
    p.fxs = fx_scale;
    p.fxi = 1.0 / fx_scale;
    return launch_elem_t<double, false, false>(d, coef64, p, x, partial, s);
}

hipError_t launch_lconn_unpack(const void* packed, int64_t E, uint16_t* out, hipStream_t s) {
    if (E <= 0) return hipSuccess;
    const uint32_t* w = static_cast<const uint32_t*>(packed);
    const uint8_t* hb = static_cast<const uint8_t*>(packed) + 4 * E;
    hipLaunchKernelGGL(k_lconn_unpack, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, s, w, hb, E,
                       reinterpret_cast<ushort4*>(out));
    return hipGetLastError();
}

hipError_t launch_elem_batch(const DevLayout& d, const BatchTables& b, int cur, int n_tiles,
                             int fp32c, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    return fp32c ? launch_elem_batch_t<float, true>(d, b, cur, n_tiles, s)
                 : launch_elem_batch_t<double, false>(d, b, cur, n_tiles, s);
}

hipError_t launch_node_batch(const DevLayout& d, const BatchTables& b, int cur, int n_blocks,
                             int fp32c, int* flags, hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    if (fp32c)
        hipLaunchKernelGGL((k_node_update_batch<float, true>), dim3(n_blocks), dim3(256), 0, s,
                           b.block_list, b.block_scen, d.part_off, d.pidx,
                           static_cast<const float*>(d.partial), static_cast<const float*>(d.u),
                           static_cast<const float*>(d.q), d.T_[cur], d.T_[1 - cur],
                           static_cast<const Props<float>*>(b.props), b.scen_single, flags);
    else
        hipLaunchKernelGGL((k_node_update_batch<double, false>), dim3(n_blocks), dim3(256), 0,
                           s, b.block_list, b.block_scen, d.part_off, d.pidx,
                           static_cast<const double*>(d.partial),
                           static_cast<const double*>(d.u), static_cast<const double*>(d.q),
                           d.T_[cur], d.T_[1 - cur], static_cast<const Props<double>*>(b.props),
                           b.scen_single, flags);
    return hipGetLastError();
}

}  // namespace fedfem
