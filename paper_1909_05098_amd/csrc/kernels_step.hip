// Time-stepping kernels for gfx950 (Algorithm 1, time-stepping block).
//
// Element pass (Eq 13, 17): one workgroup per tile of consecutive elements.
// The tile's distinct nodes are staged in LDS (temperature, and k(T) when the
// conductivity depends on temperature); each thread evaluates whole elements
// with the precomputed off-diagonal entries a_ab of A = V_tet B^T B (Eq 16).
// Because every row of A sums to zero,
//     F_e,a = k_e sum_{b != a} a_ab (T_b - T_a),
// and with T = hi + lo the difference is formed as (hi_b - hi_a) +
// (lo_b - lo_a), which keeps it accurate to float precision of the
// difference itself.  The four corner loads go to LDS; then each tile node
// sums its corners in a fixed order and writes one partial per (tile, node).
//
// Node pass (Eq 11, 19): one thread per node adds its partials in ascending
// tile order (no floating-point atomics, so results are bit-reproducible)
// and applies the explicit update with lumped capacity, perfusion, metabolic
// heat and the nodal source.  In the compensated float mode the increment is
// added to hi with an error-free TwoSum and the rounding error folded into
// lo (Knuth's TwoSum, Dekker's Fast2Sum renormalisation).  Dirichlet nodes
// (u <= 0) are never written: both ping-pong buffers hold T_Gamma.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace fedfem {

namespace {

constexpr float kDivergeLimit = 1.0e4f;

template <typename Real>
__device__ __forceinline__ Real clampT(Real T, const Props<Real>& p) {
    return T < p.Tlo ? p.Tlo : (T > p.Thi ? p.Thi : T);
}

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

struct LdsCarve {
    size_t slot, conn, f, T, Tlo, k, total;
};

__host__ __device__ inline LdsCarve carve(int TE, int maxn, int rb, bool comp, bool td) {
    LdsCarve c;
    c.slot = 0;
    c.conn = align16(c.slot + sizeof(uint16_t) * 4 * (size_t)TE);
    c.f = align16(c.conn + sizeof(uint16_t) * 4 * (size_t)TE);
    c.T = align16(c.f + (size_t)rb * 4 * TE);
    c.Tlo = align16(c.T + (size_t)rb * maxn);
    c.k = align16(c.Tlo + (comp ? (size_t)rb * maxn : 0));
    c.total = align16(c.k + (td ? (size_t)rb * maxn : 0));
    return c;
}

template <typename Real, bool COMP, bool TD>
__device__ __forceinline__ void elem_tile(int64_t E, int TE, int maxn, int64_t t, int64_t e0,
                                          int ne,
                                          const int32_t* __restrict__ tile_node_off,
                                          const int32_t* __restrict__ tile_nodes,
                                          const uint16_t* __restrict__ seg_start,
                                          const uint16_t* __restrict__ slots,
                                          const Real* __restrict__ coef,
                                          const Real* __restrict__ Thi,
                                          const Real* __restrict__ Tlo,
                                          Real* __restrict__ partial, const Props<Real>& pr) {
    extern __shared__ __align__(16) unsigned char lds[];
    const LdsCarve c = carve(TE, maxn, sizeof(Real), COMP, TD);
    uint16_t* s_slot = reinterpret_cast<uint16_t*>(lds + c.slot);
    uint16_t* s_conn = reinterpret_cast<uint16_t*>(lds + c.conn);
    Real* s_f = reinterpret_cast<Real*>(lds + c.f);
    Real* s_T = reinterpret_cast<Real*>(lds + c.T);
    Real* s_Tlo = reinterpret_cast<Real*>(lds + c.Tlo);
    Real* s_k = reinterpret_cast<Real*>(lds + c.k);

    const int tid = threadIdx.x, bs = blockDim.x;
    const int ns = 4 * ne;
    const int p0 = tile_node_off[t];
    const int m = tile_node_off[t + 1] - p0;

    // stage the corner list (4 x u16 per element) and the tile's nodes
    const uint2* gslot = reinterpret_cast<const uint2*>(slots) + e0;
    uint2* sslot2 = reinterpret_cast<uint2*>(s_slot);
    for (int el = tid; el < ne; el += bs) sslot2[el] = gslot[el];
    for (int j = tid; j < m; j += bs) {
        const int g = tile_nodes[p0 + j];
        const Real th = Thi[g];
        s_T[j] = th;
        if (COMP) s_Tlo[j] = Tlo[g];
        if (TD) s_k[j] = pr.k0 + pr.dk * (clampT(th, pr) - pr.Tref);
    }
    __syncthreads();
    // invert the node groups into per-corner local node ids
    for (int j = tid; j < m; j += bs) {
        const int a = seg_start[p0 + j];
        const int b = (j + 1 < m) ? (int)seg_start[p0 + j + 1] : ns;
        for (int k = a; k < b; k++) s_conn[s_slot[k]] = (uint16_t)j;
    }
    __syncthreads();
    // element loads
    const Real* c01 = coef;
    const Real* c02 = coef + E;
    const Real* c03 = coef + 2 * E;
    const Real* c12 = coef + 3 * E;
    const Real* c13 = coef + 4 * E;
    const Real* c23 = coef + 5 * E;
    const uint2* sconn2 = reinterpret_cast<const uint2*>(s_conn);
    for (int el = tid; el < ne; el += bs) {
        const int64_t e = e0 + el;
        const Real a01 = c01[e], a02 = c02[e], a03 = c03[e];
        const Real a12 = c12[e], a13 = c13[e], a23 = c23[e];
        const uint2 cc = sconn2[el];
        const int n0 = cc.x & 0xffff, n1 = cc.x >> 16, n2 = cc.y & 0xffff, n3 = cc.y >> 16;
        const Real h0 = s_T[n0], h1 = s_T[n1], h2 = s_T[n2], h3 = s_T[n3];
        Real d01 = h1 - h0, d02 = h2 - h0, d03 = h3 - h0;
        Real d12 = h2 - h1, d13 = h3 - h1, d23 = h3 - h2;
        if (COMP) {
            const Real l0 = s_Tlo[n0], l1 = s_Tlo[n1], l2 = s_Tlo[n2], l3 = s_Tlo[n3];
            d01 += l1 - l0;
            d02 += l2 - l0;
            d03 += l3 - l0;
            d12 += l2 - l1;
            d13 += l3 - l1;
            d23 += l3 - l2;
        }
        Real ke;
        if (TD)
            ke = (s_k[n0] + s_k[n1] + s_k[n2] + s_k[n3]) * Real(0.25);
        else
            ke = pr.k0;
        const Real g01 = a01 * d01, g02 = a02 * d02, g03 = a03 * d03;
        const Real g12 = a12 * d12, g13 = a13 * d13, g23 = a23 * d23;
        Real* f = s_f + 4 * el;
        f[0] = ke * ((g01 + g02) + g03);
        f[1] = ke * ((g12 + g13) - g01);
        f[2] = ke * (g23 - (g02 + g12));
        f[3] = -ke * ((g03 + g13) + g23);
    }
    __syncthreads();
    // per tile node: fixed-order sum of its corners
    for (int j = tid; j < m; j += bs) {
        const int a = seg_start[p0 + j];
        const int b = (j + 1 < m) ? (int)seg_start[p0 + j + 1] : ns;
        Real s = 0;
        for (int k = a; k < b; k++) s += s_f[s_slot[k]];
        partial[p0 + j] = s;
    }
}

template <typename Real, bool COMP, bool TD>
__global__ void __launch_bounds__(1024)
k_elem_loads(int64_t E, int TE, int maxn, const int32_t* __restrict__ tile_node_off,
             const int32_t* __restrict__ tile_nodes, const uint16_t* __restrict__ seg_start,
             const uint16_t* __restrict__ slots, const Real* __restrict__ coef,
             const Real* __restrict__ Thi, const Real* __restrict__ Tlo,
             Real* __restrict__ partial, Props<Real> pr) {
    const int64_t t = blockIdx.x;
    const int64_t e0 = t * TE;
    const int ne = (int)min<int64_t>(TE, E - e0);
    elem_tile<Real, COMP, TD>(E, TE, maxn, t, e0, ne, tile_node_off, tile_nodes, seg_start,
                              slots, coef, Thi, Tlo, partial, pr);
}

// Batched form: the workgroup's tile comes from a list of active tiles, its
// element range from per-tile offsets, and its material from the tile's
// scenario.
template <typename Real, bool COMP>
__global__ void __launch_bounds__(1024)
k_elem_loads_batch(int64_t E, int TE, int maxn, const int32_t* __restrict__ tile_list,
                   const int32_t* __restrict__ tile_elem_off,
                   const int32_t* __restrict__ tile_scen,
                   const int32_t* __restrict__ tile_node_off,
                   const int32_t* __restrict__ tile_nodes,
                   const uint16_t* __restrict__ seg_start, const uint16_t* __restrict__ slots,
                   const Real* __restrict__ coef, const Real* __restrict__ Thi,
                   const Real* __restrict__ Tlo, Real* __restrict__ partial,
                   const Props<Real>* __restrict__ props) {
    const int64_t t = tile_list[blockIdx.x];
    const int64_t e0 = tile_elem_off[t];
    const int ne = (int)(tile_elem_off[t + 1] - e0);
    const Props<Real> pr = props[tile_scen[t]];
    elem_tile<Real, COMP, true>(E, TE, maxn, t, e0, ne, tile_node_off, tile_nodes, seg_start,
                                slots, coef, Thi, Tlo, partial, pr);
}

template <typename Real, bool COMP>
__device__ __forceinline__ void node_update(int64_t i, const int32_t* __restrict__ part_off,
                                            const int32_t* __restrict__ part_idx,
                                            const Real* __restrict__ partial,
                                            const Real* __restrict__ u,
                                            const Real* __restrict__ q,
                                            const Real* __restrict__ Thi_in,
                                            const Real* __restrict__ Tlo_in,
                                            Real* __restrict__ Thi_out,
                                            Real* __restrict__ Tlo_out, const Props<Real>& pr,
                                            int* __restrict__ flag) {
    const Real ui = u[i];
    if (!(ui > Real(0))) return;  // Dirichlet node: held at T_Gamma
    const int a = part_off[i], b = part_off[i + 1];
    Real F = 0;
    for (int k = a; k < b; k++) F += partial[part_idx[k]];
    const Real hi = Thi_in[i];
    const Real lo = COMP ? Tlo_in[i] : Real(0);
    const Real dT = clampT(hi, pr) - pr.Tref;
    const Real rc = (pr.rho0 + pr.drho * dT) * (pr.c0 + pr.dc * dT);
    // heat flow per unit volume [W/m^3]: source and conduction per lumped
    // volume, metabolic heat, perfusion towards T_a
    const Real R = (q[i] - F) * ui + pr.Qm + pr.wbcb * ((pr.Ta - hi) - lo);
    const Real d = pr.dt * R / rc;
    Real nh, nl;
    if (COMP) {
        // TwoSum(hi, d) = s + err exactly
        const Real s = hi + d;
        const Real bp = s - hi;
        const Real err = (hi - (s - bp)) + (d - bp);
        const Real l2 = lo + err;
        // Fast2Sum(s, l2): |s| >= |l2|
        nh = s + l2;
        nl = l2 - (nh - s);
        Tlo_out[i] = nl;
    } else {
        nh = hi + d;
    }
    Thi_out[i] = nh;
    if (!(nh < Real(kDivergeLimit) && nh > -Real(kDivergeLimit))) *flag = 1;
}

template <typename Real, bool COMP>
__global__ void __launch_bounds__(256)
k_node_update(int64_t N, const int32_t* __restrict__ part_off,
              const int32_t* __restrict__ part_idx, const Real* __restrict__ partial,
              const Real* __restrict__ u, const Real* __restrict__ q,
              const Real* __restrict__ Thi_in, const Real* __restrict__ Tlo_in,
              Real* __restrict__ Thi_out, Real* __restrict__ Tlo_out, Props<Real> pr,
              int* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    node_update<Real, COMP>(i, part_off, part_idx, partial, u, q, Thi_in, Tlo_in, Thi_out,
                            Tlo_out, pr, flag);
}

// Batched form: 256-node blocks never straddle scenarios; the block comes
// from a list of active blocks and its material from the block's scenario.
template <typename Real, bool COMP>
__global__ void __launch_bounds__(256)
k_node_update_batch(const int32_t* __restrict__ block_list,
                    const int32_t* __restrict__ block_scen,
                    const int32_t* __restrict__ part_off, const int32_t* __restrict__ part_idx,
                    const Real* __restrict__ partial, const Real* __restrict__ u,
                    const Real* __restrict__ q, const Real* __restrict__ Thi_in,
                    const Real* __restrict__ Tlo_in, Real* __restrict__ Thi_out,
                    Real* __restrict__ Tlo_out, const Props<Real>* __restrict__ props,
                    int* __restrict__ flags) {
    const int blk = block_list[blockIdx.x];
    const int sc = block_scen[blk];
    const Props<Real> pr = props[sc];
    const int64_t i = (int64_t)blk * 256 + threadIdx.x;
    node_update<Real, COMP>(i, part_off, part_idx, partial, u, q, Thi_in, Tlo_in, Thi_out,
                            Tlo_out, pr, flags + sc);
}

template <typename Real, bool COMP, bool TD>
hipError_t launch_elem_t(const DevLayout& d, const Real* coef, const Props<Real>& p,
                         const Real* Thi, const Real* Tlo, Real* partial,
                         hipStream_t s) {
    const size_t lds = carve(d.tile_elems, d.max_tile_nodes, sizeof(Real), COMP, TD).total;
    auto kern = k_elem_loads<Real, COMP, TD>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)d.T), dim3(d.threads), lds, s, d.E,
                       d.tile_elems, d.max_tile_nodes, d.tile_node_off, d.tile_nodes,
                       d.seg_start, d.slots, coef, Thi, Tlo, partial, p);
    return hipGetLastError();
}

template <typename Real, bool COMP>
hipError_t launch_node_t(const DevLayout& d, int cur, const Props<Real>& p, int* flag,
                         hipStream_t s) {
    const unsigned blocks = (unsigned)((d.N + 255) / 256);
    hipLaunchKernelGGL((k_node_update<Real, COMP>), dim3(blocks), dim3(256), 0, s, d.N,
                       d.part_off, d.part_idx, static_cast<const Real*>(d.partial),
                       static_cast<const Real*>(d.u), static_cast<const Real*>(d.q),
                       static_cast<const Real*>(d.Thi[cur]),
                       static_cast<const Real*>(d.Tlo[cur]),
                       static_cast<Real*>(d.Thi[1 - cur]),
                       static_cast<Real*>(d.Tlo[1 - cur]), p, flag);
    return hipGetLastError();
}

}  // namespace

size_t tile_lds_bytes(int TE, int maxn, int rb, bool comp, bool td) {
    return carve(TE, maxn, rb, comp, td).total;
}

hipError_t launch_elem_f32c(const DevLayout& d, int cur, const Props<float>& p, bool td,
                            hipStream_t s) {
    const float* hi = static_cast<const float*>(d.Thi[cur]);
    const float* lo = static_cast<const float*>(d.Tlo[cur]);
    const float* cf = static_cast<const float*>(d.coef);
    float* part = static_cast<float*>(d.partial);
    return td ? launch_elem_t<float, true, true>(d, cf, p, hi, lo, part, s)
              : launch_elem_t<float, true, false>(d, cf, p, hi, lo, part, s);
}

hipError_t launch_node_f32c(const DevLayout& d, int cur, const Props<float>& p, int* flag,
                            hipStream_t s) {
    return launch_node_t<float, true>(d, cur, p, flag, s);
}

hipError_t launch_elem_f64(const DevLayout& d, int cur, const Props<double>& p, bool td,
                           hipStream_t s) {
    const double* hi = static_cast<const double*>(d.Thi[cur]);
    const double* cf = static_cast<const double*>(d.coef);
    double* part = static_cast<double*>(d.partial);
    return td ? launch_elem_t<double, false, true>(d, cf, p, hi, nullptr, part, s)
              : launch_elem_t<double, false, false>(d, cf, p, hi, nullptr, part, s);
}

hipError_t launch_node_f64(const DevLayout& d, int cur, const Props<double>& p, int* flag,
                           hipStream_t s) {
    return launch_node_t<double, false>(d, cur, p, flag, s);
}

hipError_t launch_step_f32c(const DevLayout& d, int cur, const Props<float>& p, bool td,
                            int* flag, hipStream_t s) {
    hipError_t e = launch_elem_f32c(d, cur, p, td, s);
    if (e != hipSuccess) return e;
    return launch_node_f32c(d, cur, p, flag, s);
}

hipError_t launch_step_f64(const DevLayout& d, int cur, const Props<double>& p, bool td,
                           int* flag, hipStream_t s) {
    hipError_t e = launch_elem_f64(d, cur, p, td, s);
    if (e != hipSuccess) return e;
    return launch_node_f64(d, cur, p, flag, s);
}

hipError_t launch_geometry_apply(const DevLayout& d, const double* coef64, const double* x,
                                 double* partial, hipStream_t s) {
    Props<double> p{};
    p.k0 = 1.0;
    return launch_elem_t<double, false, false>(d, coef64, p, x, nullptr, partial, s);
}

hipError_t launch_elem_batch(const DevLayout& d, const BatchTables& b, int cur, int n_tiles,
                             int fp32c, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    const int rb = fp32c ? 4 : 8;
    const size_t lds = carve(d.tile_elems, d.max_tile_nodes, rb, fp32c != 0, true).total;
    if (fp32c) {
        auto kern = k_elem_loads_batch<float, true>;
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kern, dim3(n_tiles), dim3(d.threads), lds, s, d.E, d.tile_elems,
                           d.max_tile_nodes, b.tile_list, b.tile_elem_off, b.tile_scen,
                           d.tile_node_off, d.tile_nodes, d.seg_start, d.slots,
                           static_cast<const float*>(d.coef),
                           static_cast<const float*>(d.Thi[cur]),
                           static_cast<const float*>(d.Tlo[cur]),
                           static_cast<float*>(d.partial),
                           static_cast<const Props<float>*>(b.props));
    } else {
        auto kern = k_elem_loads_batch<double, false>;
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kern, dim3(n_tiles), dim3(d.threads), lds, s, d.E, d.tile_elems,
                           d.max_tile_nodes, b.tile_list, b.tile_elem_off, b.tile_scen,
                           d.tile_node_off, d.tile_nodes, d.seg_start, d.slots,
                           static_cast<const double*>(d.coef),
                           static_cast<const double*>(d.Thi[cur]),
                           static_cast<const double*>(nullptr),
                           static_cast<double*>(d.partial),
                           static_cast<const Props<double>*>(b.props));
    }
    return hipGetLastError();
}

hipError_t launch_node_batch(const DevLayout& d, const BatchTables& b, int cur, int n_blocks,
                             int fp32c, int* flags, hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    if (fp32c)
        hipLaunchKernelGGL((k_node_update_batch<float, true>), dim3(n_blocks), dim3(256), 0, s,
                           b.block_list, b.block_scen, d.part_off, d.part_idx,
                           static_cast<const float*>(d.partial),
                           static_cast<const float*>(d.u), static_cast<const float*>(d.q),
                           static_cast<const float*>(d.Thi[cur]),
                           static_cast<const float*>(d.Tlo[cur]),
                           static_cast<float*>(d.Thi[1 - cur]),
                           static_cast<float*>(d.Tlo[1 - cur]),
                           static_cast<const Props<float>*>(b.props), flags);
    else
        hipLaunchKernelGGL((k_node_update_batch<double, false>), dim3(n_blocks), dim3(256), 0,
                           s, b.block_list, b.block_scen, d.part_off, d.part_idx,
                           static_cast<const double*>(d.partial),
                           static_cast<const double*>(d.u), static_cast<const double*>(d.q),
                           static_cast<const double*>(d.Thi[cur]),
                           static_cast<const double*>(nullptr),
                           static_cast<double*>(d.Thi[1 - cur]),
                           static_cast<double*>(nullptr),
                           static_cast<const Props<double>*>(b.props), flags);
    return hipGetLastError();
}

}  // namespace fedfem
