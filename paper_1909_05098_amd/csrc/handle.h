// Definition of the opaque fedfem_handle (shared by the ABI sources only).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/fedfem.h"
#include "internal.h"

struct fedfem_handle {
    // caller inputs (deep copies)
    int64_t N = 0, E = 0;
    int npe = 4;  // nodes per element: 4 (tetrahedra) or 8 (hexahedra)
    std::vector<double> xyz;
    std::vector<int32_t> tets;  // [npe E] element nodes
    fedfem_materials mat{};
    bool fp32c = true;
    double T0 = 0.0;
    std::vector<int32_t> dir_nodes;
    std::vector<double> dir_T;
    double dt_spec = 0.0;
    fedfem_options opt{};
    // runtime
    int device = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t cap_stream = nullptr;
    hipStream_t stream = nullptr;
    bool precomputed = false;
    bool timing_trial = false;  // autotuner trial: skip the critical-step estimate
    bool broken = false;
    std::string err;
    fedfem::Layout L;
    fedfem::DevLayout d;
    std::vector<std::pair<void*, size_t>> allocs;  // device blocks and their sizes
    int64_t dev_bytes = 0;
    int64_t n_dir = 0;
    std::vector<int32_t> host_isdir;  // internal order
    // device arrays beyond the step layout
    double* d_xyz = nullptr;      // [3N] internal order
    int32_t* d_conn = nullptr;    // [npe E]
    int32_t* d_ec_off = nullptr;  // [N+1]
    int32_t* d_ec = nullptr;      // [npe E]
    double* d_vol = nullptr;      // [E]
    double* d_Vi = nullptr;       // [N]
    int32_t* d_nperm = nullptr;   // [N] internal -> caller
    int32_t* d_isdir = nullptr;   // [N]
    double* d_dirT = nullptr;     // [N]
    double* d_stage = nullptr;    // [N] double staging
    double* d_qpts = nullptr;     // [256][4]
    int32_t* d_flag = nullptr;
    // estimator and time
    int lz_max_iter = 600;
    int lz_iters = 0;
    double lam_geo = 0.0, lam_ritz = 0.0;
    double dt = 0.0, dt_cr = 0.0;
    double a_max = 0.0;          // largest off-diagonal row sum of |A_e|
    double fx_scale = 1.0;       // fixed-point scale of the element loads
    double fx_scale_lz = 1.0;    // same for the Lanczos operator
    double t = 0.0;
    int64_t steps = 0;
    int cur = 0;
    std::map<std::pair<int64_t, int>, hipGraphExec_t> graphs;
    // scheduled source patterns (fedfem_set_schedule); device arrays in d.pat
    // and d.amp, amplitude tables (times, values) per pattern on the host
    std::vector<std::vector<double>> sched_t, sched_a;
    // property tables (fedfem_set_property_tables): points of k, rho, c;
    // empty keeps the material's linear law.  d_tab holds them on the device
    // in the working precision as [3][times, values, slopes][kMaxTab].
    std::vector<double> tab_t[3], tab_v[3];
    void* d_tab = nullptr;
};
