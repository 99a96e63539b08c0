// Internal declarations of the FED-FEM gfx950 library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace fedfem {

// ---------------------------------------------------------------------------
// Host-side mesh layout (integer topology only).
//
// Internal numbering: nodes and elements optionally follow a Morton curve.
// Elements are cut into tiles of consecutive elements, each holding at most
// `tile_elems` elements and touching at most `max_tile_nodes` distinct nodes;
// reordered tetrahedral layouts then deal each tile's elements out so that
// neighbouring positions hold elements from separate parts of the tile.
// For every tile the distinct nodes it touches are listed in ascending
// internal id ("tile nodes"), and each element corner stores its node's
// position in that list (lconn, u16).  Each (tile, tile node) pair in
// [tile_node_off[t], tile_node_off[t+1]) produces one partial sum.
// Reordered tetrahedral layouts number the nodes that a single tile touches
// first (ids [0, n_int), grouped by tile): such a node's partial sits at its
// own index.  The other tile nodes' partials follow at [n_int, P), tile-major
// (each tile writes one contiguous run).  tile_part[4t .. 4t+3] =
// (pi, ni, ps, n0): tile t's list starts with its ni single-tile nodes, ids
// n0 .. n0 + ni - 1, and list position j writes position pi + j if j < ni,
// else ps + j (pi = n0 here; batched copies shift ids and positions apart).
// Otherwise n_int = 0, ni = 0 and ps = tile_node_off[t].  Node i
// finds its partials at pidx[part_off[i] .. part_off[i+1]), in ascending tile
// order.
// ---------------------------------------------------------------------------
struct Layout {
    int64_t N = 0, E = 0, T = 0, P = 0;
    int64_t n_int = 0;  // nodes of a single tile: ids [0, n_int)
    int npe = 4;  // nodes per element: 4 (linear tetrahedra) or 8 (hexahedra)
    int reorder = 0;
    int spread = 0;  // elements dealt out inside each tile (see spread_tiles)
    int tile_elems = 0;
    int max_tile_nodes = 0;
    // most corners of one tile on a single node: the number of loads one
    // tile-node accumulator adds (bounds the fixed-point headroom)
    int max_tile_valence = 0;
    std::vector<int32_t> nperm;          // internal -> caller node id
    std::vector<int32_t> ninv;           // caller -> internal node id
    std::vector<int32_t> eperm;          // internal -> caller element id
    std::vector<double> xyz;             // [3N] internal order
    std::vector<int32_t> conn;           // [npe E] internal ids, internal order
    std::vector<int32_t> tile_elem_off;  // [T+1]
    std::vector<int32_t> tile_node_off;  // [T+1]
    std::vector<int32_t> tile_nodes;     // [P]
    std::vector<int32_t> tile_part;      // [4T] (pi, ni, ps, n0) per tile
    std::vector<int32_t> pidx;           // [P] node-major list of partial positions
    std::vector<uint16_t> lconn;         // [npe E] local node id per corner
    std::vector<uint8_t> lconn_pk;       // packed form of lconn (pack_lconn)
    std::vector<int32_t> part_off;       // [N+1] node -> partial positions
    std::vector<int32_t> ec_off;         // [N+1] node -> element corners
    std::vector<int32_t> ec;             // [npe E] npe*e+corner, ascending e
};

// Build the layout.  Returns false with a message on failure.
bool build_layout(const double* xyz, const int32_t* conn, int npe, int64_t N,
                  int64_t E, int reorder, int tile_elems, int max_tile_nodes,
                  Layout& L, std::string& err);

// Tile layout only (used again when tiles must shrink).
bool build_tiles(Layout& L, int tile_elems, int max_tile_nodes,
                 std::string& err);

// Tiles of at most kPackedMaxNodes nodes store their local corner ids in 10
// bits each.  Tetrahedra: 5 bytes per element instead of 8, an array of E
// 32-bit words (ids 0, 1, 2 and the low 2 bits of id 3 at bits 0, 10, 20,
// 30) followed by an array of E bytes (the high 8 bits of id 3).
// Hexahedra: 10 bytes instead of 16, an array of E 64-bit words (ids 0..5
// at bits 0, 10, ..., 50 and the low 4 bits of id 6 at bit 60) followed by
// an array of E 16-bit words (the high 6 bits of id 6, then id 7 at bit 6).
// pack_lconn fills L.lconn_pk when the layout qualifies and clears it
// otherwise.
constexpr int kPackedMaxNodes = 1024;
void pack_lconn(Layout& L);

// Cap the host threads of layout builds made by the calling thread (0: the
// default, up to 16); returns the previous cap.
int set_layout_threads(int n);

// Run fn(0) .. fn(n - 1) on `threads` host workers (the caller among them)
// that take items from one atomic counter; each worker's layout builds use
// at most `inner` host threads (pool.cpp).
void run_workers(int32_t n, int32_t threads, int inner,
                 const std::function<void(int32_t)>& fn);

// Morton (Z-order) permutation of points; returns new -> old.
std::vector<int32_t> morton_order(const double* pts, int64_t n);

// Caching device allocator (devcache.cpp): blocks come from per-device free
// lists when one of the right size class is there; `granted` is the block's
// class size, to be handed back to cached_free once no stream uses it.
hipError_t cached_malloc(void** p, size_t bytes, size_t* granted);
void cached_free(void* p, size_t granted);

// ---------------------------------------------------------------------------
// Material parameters as the kernels see them.
// ---------------------------------------------------------------------------
// fxs = 2^S and fxi = 2^-S scale corner loads to the 64-bit fixed-point
// grid on which a tile sums them exactly (chosen so that the largest
// possible load maps below 2^58).
template <typename Real>
struct Props {
    Real k0, dk, rho0, drho, c0, dc, Tref, Tlo, Thi, wbcb, Ta, Qm, dt;
    Real fxs, fxi;
    // property tables (fedfem_set_property_tables): nt[p] points of property
    // p (0 k, 1 rho, 2 c) at tab + p * 3 * kMaxTab as times, values, slopes;
    // nt[p] == 0 keeps the linear law of that property
    const Real* tab = nullptr;
    int nt[3] = {0, 0, 0};
};
constexpr int kMaxTab = 16;  // FEDFEM_MAX_TABLE

// Device copy of a layout plus the numerical arrays of one precision.
struct DevLayout {
    int64_t N = 0, E = 0, T = 0, P = 0;
    int tile_elems = 0, max_tile_nodes = 0, threads = 256;
    int npe = 4;  // nodes per element: 4 or 8 (coef [6][E] either way)
    int xcd = 0;  // remap blocks so each XCD walks a contiguous stretch
    int32_t* tile_elem_off = nullptr;
    int32_t* tile_node_off = nullptr;
    int32_t* tile_nodes = nullptr;
    int32_t* tile_part = nullptr;  // [4T] (pi, ni, ps, n0), see Layout
    int64_t n_int = 0;             // nodes [0, n_int) read their partial at their index
    int32_t* pidx = nullptr;
    void* lconn = nullptr;     // packed (lconn_pk = 1) or [4E] u16
    int lconn_pk = 0;
    int32_t* part_off = nullptr;
    void* coef = nullptr;      // [6][E] Real: a01 a02 a03 a12 a13 a23, or S (hexahedra)
    void* u = nullptr;         // [N] Real, 1/V_i, or -1 for Dirichlet nodes
    void* q = nullptr;         // [N] Real, active nodal source [W]
    void* T_[2] = {nullptr, nullptr};  // state: float2 (hi, lo) or double
    void* partial = nullptr;   // [P] Real, positions as Layout describes
    // scheduled source patterns (fedfem_set_schedule): node i receives
    // sum_p amp[j][p] pat[p][i] on top of q in the j-th step of a graph chunk
    void* pat = nullptr;       // [n_pat][N] Real
    void* amp = nullptr;       // [512][n_pat] Real, refilled before each chunk
    int n_pat = 0;
    // thermal dose (fedfem_set_dose): every node adds dt * dose_a * f(T) at
    // the start of each step, f the CEM43 or Arrhenius rate shape
    double* dose = nullptr;    // [N], internal node order
    int dose_model = 0;
    double dose_a = 0.0, dose_b = 0.0;
    double dose_dt = 0.0;      // the step the captured launches use
};

// ---------------------------------------------------------------------------
// Kernel launchers (kernels_step.hip).
// ---------------------------------------------------------------------------
size_t tile_lds_bytes(int tile_elems, int max_nodes, int real_bytes, bool comp,
                      bool td);
// Elements per thread of the element kernel, rounded up to 1, 2 or 4 (the
// instantiated counts); 8 means the workgroup is too small for the tile.
int elems_per_thread(const DevLayout& d);
// One explicit step: element loads then nodal update, ping-pong cur -> 1-cur;
// j is the step's position in its graph chunk (row j of the amplitudes).
hipError_t launch_step_f32c(const DevLayout& d, int cur, const Props<float>& p,
                            bool td, int* flag, hipStream_t s, int j = 0);
hipError_t launch_step_f64(const DevLayout& d, int cur, const Props<double>& p,
                           bool td, int* flag, hipStream_t s, int j = 0);
hipError_t launch_elem_f32c(const DevLayout& d, int cur, const Props<float>& p,
                            bool td, hipStream_t s);
hipError_t launch_node_f32c(const DevLayout& d, int cur, const Props<float>& p,
                            int* flag, hipStream_t s);
hipError_t launch_elem_f64(const DevLayout& d, int cur, const Props<double>& p,
                           bool td, hipStream_t s);
hipError_t launch_node_f64(const DevLayout& d, int cur, const Props<double>& p,
                           int* flag, hipStream_t s);
// Batched execution: per-tile element offsets and scenario ids, node blocks
// of 256 that never straddle scenarios, and lists of the active tiles and
// blocks (a prefix of each list is active at any step).
struct BatchTables {
    const int32_t* tile_list = nullptr;      // [T]
    const int32_t* tile_scen = nullptr;      // [T]
    const int32_t* block_list = nullptr;     // [NB]
    const int32_t* block_scen = nullptr;     // [NB]
    const void* props = nullptr;             // Props<Real>[S]
    // per scenario: (node_off + n_int, pbase - node_off): its nodes below the
    // first number are single-tile nodes, whose partial sits at the node's
    // index plus the second
    const int2* scen_single = nullptr;       // [S]
};
// Expand packed corner ids of E elements to [4E] u16.
hipError_t launch_lconn_unpack(const void* packed, int64_t E, uint16_t* out,
                               hipStream_t s);
hipError_t launch_elem_batch(const DevLayout& d, const BatchTables& b, int cur,
                             int n_tiles, int fp32c, hipStream_t s);
hipError_t launch_node_batch(const DevLayout& d, const BatchTables& b, int cur,
                             int n_blocks, int fp32c, int* flags,
                             hipStream_t s);
// Element loads of x with k = 1 (geometry operator sum_e A_e), FP64.
// fx_scale is the fixed-point scale 2^S for loads of x.
hipError_t launch_geometry_apply(const DevLayout& d, const double* coef64,
                                 const double* x, double* partial,
                                 double fx_scale, hipStream_t s);

// ---------------------------------------------------------------------------
// Pre-computation launchers (kernels_pre.hip), all double precision.
// ---------------------------------------------------------------------------
// out[0] (as u64 bits) = max over elements and corners a of sum_b |a_ab|.
hipError_t launch_coef_bound(int64_t E, const double* coef64,
                             unsigned long long* out, hipStream_t s);
// bad receives the smallest caller element id with |det J| <= 1e-12 l^3.
hipError_t launch_geometry(int64_t E, const double* xyz, const int32_t* conn,
                           const int32_t* eperm, double* coef64, double* vol,
                           int32_t* bad, hipStream_t s);
// Hexahedra (Eq 14): coef64 receives W = sqrt(V_e) grad N at the element
// centre, [24][E] (component i of corner a at row 8 i + a).
hipError_t launch_geometry_hex(int64_t E, const double* xyz,
                               const int32_t* conn, const int32_t* eperm,
                               double* coef64, double* vol, int32_t* bad,
                               hipStream_t s);
hipError_t launch_coef_bound_hex(int64_t E, const double* coef64,
                                 unsigned long long* out, hipStream_t s);
hipError_t launch_lump(int64_t N, const int32_t* ec_off, const int32_t* ec,
                       const double* vol, int npe, double* Vi,
                       hipStream_t s);
hipError_t launch_source_nodal(int64_t N, const double* xyz, const double* Vi,
                               int n_src, const double* src, double* q64,
                               hipStream_t s);
hipError_t launch_source_consistent(int64_t N, int64_t E, const double* xyz,
                                    const int32_t* conn, const double* vol,
                                    const int32_t* ec_off, const int32_t* ec,
                                    int n_src, const double* src,
                                    const double* qpts, double* slot64,
                                    double* q64, hipStream_t s);
// The same for eight-node hexahedra (slot holds 8 E corner loads).
hipError_t launch_source_consistent_hex(int64_t N, int64_t E, const double* xyz,
                                        const int32_t* conn, const int32_t* ec_off,
                                        const int32_t* ec, int n_src, const double* src,
                                        double* slot64, double* q64, hipStream_t s);
hipError_t launch_cast_coef(int64_t n, const double* src, float* dst,
                            hipStream_t s);
hipError_t launch_node_init(int64_t N, const double* Vi, const int32_t* is_dir,
                            const double* dirT, double T0, int fp32c, void* u,
                            void* T0buf, void* T1buf, hipStream_t s);
// q (Real, internal order) <- src64[nperm[i]] (caller order) or src64[i].
// Nodal loads of a surface heat flux on triangles (nv 3) or bilinear
// quadrilaterals (nv 4): per-face corner shares, then a fixed-order gather
// over the node -> face-corner list (off, idx).
hipError_t launch_face_loads(int64_t N, int64_t F, int nv, const double* xyz,
                             const int32_t* faces, const double* flux, const int32_t* off,
                             const int32_t* idx, double* slot, double* out, hipStream_t s);
hipError_t launch_set_source(int64_t N, const double* src64,
                             const int32_t* nperm, int fp32c, void* q,
                             hipStream_t s);
// out64[nperm[i]] = q[i] (Real) : internal -> caller order.
hipError_t launch_get_source(int64_t N, const void* q, const int32_t* nperm,
                             int fp32c, double* out64, hipStream_t s);
hipError_t launch_read_T(int64_t N, const void* T, const int32_t* nperm,
                         int fp32c, double* out, hipStream_t s);
// Caller-order raw state: FP32C hi[N] then lo[N] (float), FP64 T[N].
hipError_t launch_state_io(int64_t N, void* T, const int32_t* nperm,
                           int fp32c, void* buf, int to_buf, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);

// Lanczos pieces for the critical step.
hipError_t launch_lanczos_start(int64_t N, const double* Vi,
                                const int32_t* is_dir, double* sc, double* v,
                                double* vprev, double* xs, double* bsum,
                                double* scal, hipStream_t s);
hipError_t launch_lanczos_iter(const DevLayout& d, const double* coef64,
                               double fx_scale, int j, const double* sc,
                               double* v, double* vprev, double* w, double* xs,
                               double* partial, double* bsum, int* counter,
                               double* alpha, double* beta, hipStream_t s);

}  // namespace fedfem
