// Batched execution of many independent scenarios (Algorithm 1 applied to
// each) as one captured HIP graph.  The pre-computed layouts of all handles
// are concatenated once; element tiles keep their per-scenario size, node
// ranges are padded to whole 256-node blocks so a node block never mixes
// scenarios.  At run time scenarios are ordered by step count, longest
// first, so the scenarios still running at global step k are a prefix of the
// tile and block lists and every launch covers exactly the active work.
#include <hip/hip_runtime.h>

#include <cmath>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/fedfem.h"
#include "handle.h"
#include "internal.h"

using namespace fedfem;

namespace fedfem {
constexpr int kChains = 2;  // independent lockstep chains in a batched run
}

struct fedfem_batch {
    std::vector<fedfem_handle*> hs;
    int S = 0;
    bool fp32c = true;
    int device = 0;
    hipStream_t stream = nullptr, cap = nullptr;
    DevLayout d;
    std::vector<int64_t> node_off, elem_off, tile_off, pbase;
    std::vector<int32_t> tile_count, block_count;
    int32_t *tile_list = nullptr, *tile_scen = nullptr;
    int32_t *block_list = nullptr, *block_scen = nullptr, *flags = nullptr;
    int32_t* scen_single = nullptr;  // [2S], see BatchTables
    void* props = nullptr;
    std::vector<std::pair<void*, size_t>> allocs;  // device blocks and their sizes
    std::map<std::vector<int64_t>, hipGraphExec_t> graphs;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // the other chains' capture streams, and the events that fork them from
    // cap and join them back
    hipStream_t chain[kChains - 1] = {};
    hipEvent_t ev_fork = nullptr, ev_join[kChains - 1] = {};
    double last_ms = 0.0;
};

namespace {

template <typename T>
hipError_t balloc(fedfem_batch* b, T** p, size_t count) {
    void* q = nullptr;
    size_t granted = 0;
    hipError_t e = cached_malloc(&q, std::max<size_t>(16, count * sizeof(T)), &granted);
    if (e != hipSuccess) return e;
    b->allocs.emplace_back(q, granted);
    *p = static_cast<T*>(q);
    return hipSuccess;
}

template <typename T>
hipError_t bupload(fedfem_batch* b, T** p, const std::vector<T>& v) {
    hipError_t e = balloc(b, p, v.size());
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, b->stream);
}

void destroy_batch(fedfem_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& a : b->allocs) cached_free(a.first, a.second);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (int c = 0; c < kChains - 1; c++) {
        if (b->chain[c]) (void)hipStreamDestroy(b->chain[c]);
        if (b->ev_join[c]) (void)hipEventDestroy(b->ev_join[c]);
    }
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    delete b;
}

template <typename Real>
Props<Real> props_of(const fedfem_handle* h) {
    const fedfem_materials& m = h->mat;
    Props<Real> p;
    p.k0 = (Real)m.k0;
    p.dk = (Real)m.dk_dT;
    p.rho0 = (Real)m.rho0;
    p.drho = (Real)m.drho_dT;
    p.c0 = (Real)m.c0;
    p.dc = (Real)m.dc_dT;
    p.Tref = (Real)m.T_ref;
    p.Tlo = (Real)m.T_lo;
    p.Thi = (Real)m.T_hi;
    p.wbcb = (Real)(m.w_b * m.c_b);
    p.Ta = (Real)m.T_a;
    p.Qm = (Real)m.Q_m;
    p.dt = (Real)h->dt;
    p.fxs = (Real)h->fx_scale;
    p.fxi = (Real)(1.0 / h->fx_scale);
    p.tab = static_cast<const Real*>(h->d_tab);  // the handle's device copy
    for (int k = 0; k < 3; k++) p.nt[k] = h->d_tab ? (int)h->tab_t[k].size() : 0;
    return p;
}

#define BCHK(expr)                                       \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) {                          \
            destroy_batch(b);                            \
            return FEDFEM_E_HIP;                         \
        }                                                \
    } while (0)

#define RCHK(expr)                                       \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return FEDFEM_E_HIP;       \
    } while (0)

}  // namespace

extern "C" {

int fedfem_batch_create(fedfem_handle* const* handles, int32_t n, fedfem_batch** out) {
    if (!out || !handles || n <= 0) return FEDFEM_E_INVALID;
    *out = nullptr;
    for (int j = 0; j < n; j++) {
        const fedfem_handle* h = handles[j];
        if (!h || h->broken) return FEDFEM_E_INVALID;
        if (h->d.n_pat > 0) return FEDFEM_E_STATE;  // schedules run per handle only
        if (h->npe != 4) return FEDFEM_E_STATE;     // batches hold tetrahedral meshes
        if (h->d.dose) return FEDFEM_E_STATE;       // and accumulate no dose
        if (!h->precomputed || !(h->dt > 0)) return FEDFEM_E_NOT_PRECOMPUTED;
        if (h->fp32c != handles[0]->fp32c || h->device != handles[0]->device)
            return FEDFEM_E_INVALID;
        for (int k = 0; k < j; k++)
            if (handles[k] == h) return FEDFEM_E_INVALID;
    }
    fedfem_batch* b = new (std::nothrow) fedfem_batch();
    if (!b) return FEDFEM_E_NOMEM;
    b->hs.assign(handles, handles + n);
    b->S = n;
    b->fp32c = handles[0]->fp32c;
    b->device = handles[0]->device;
    BCHK(hipSetDevice(b->device));
    BCHK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    BCHK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    BCHK(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    for (int c = 0; c < kChains - 1; c++) {
        BCHK(hipStreamCreateWithFlags(&b->chain[c], hipStreamNonBlocking));
        BCHK(hipEventCreateWithFlags(&b->ev_join[c], hipEventDisableTiming));
    }
    BCHK(hipEventCreate(&b->ev0));
    BCHK(hipEventCreate(&b->ev1));
    // offsets
    int64_t Nt = 0, Et = 0, Tt = 0, Pt = 0;
    int maxte = 0, maxn = 0;
    b->node_off.resize(n + 1);
    b->elem_off.resize(n + 1);
    b->tile_off.resize(n + 1);
    b->pbase.resize(n + 1);
    for (int j = 0; j < n; j++) {
        const fedfem_handle* h = handles[j];
        b->node_off[j] = Nt;
        b->elem_off[j] = Et;
        b->tile_off[j] = Tt;
        b->pbase[j] = Pt;
        Nt += (h->N + 255) / 256 * 256;
        Et += h->E;
        Tt += h->d.T;
        Pt += h->d.P;
        maxte = std::max(maxte, h->d.tile_elems);
        maxn = std::max(maxn, h->d.max_tile_nodes);
    }
    b->node_off[n] = Nt;
    b->elem_off[n] = Et;
    b->tile_off[n] = Tt;
    b->pbase[n] = Pt;
    if (Nt > INT32_MAX || 4 * Et > INT32_MAX || Pt > INT32_MAX) {
        destroy_batch(b);
        return FEDFEM_E_INVALID;
    }
    int lds_attr = 0;
    BCHK(hipDeviceGetAttribute(&lds_attr, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device));
    if (tile_lds_bytes(maxte, maxn, b->fp32c ? 4 : 8, b->fp32c, true) > (size_t)lds_attr) {
        destroy_batch(b);
        return FEDFEM_E_INVALID;
    }
    DevLayout& d = b->d;
    d.N = Nt;
    d.E = Et;
    d.T = Tt;
    d.P = Pt;
    d.tile_elems = maxte;
    d.max_tile_nodes = maxn;
    // one workgroup size for every tile: four elements per thread for the
    // largest tiles (layouts tuned with FEDFEM_TUNE_BATCH share it)
    d.threads = std::max(64, std::min(1024, (maxte / 4 + 63) / 64 * 64));
    d.xcd = 0;
    if (elems_per_thread(d) > 4) {
        destroy_batch(b);
        return FEDFEM_E_INVALID;
    }
    // integer tables on the host
    std::vector<int32_t> tno(Tt + 1), tnodes(Pt), poff(Nt + 1, 0), wp(Pt), teo(Tt + 1), tsc(Tt),
        bsc(Nt / 256), tpart(4 * Tt), ssingle(2 * n);
    for (int j = 0; j < n; j++) {
        const fedfem_handle* h = handles[j];
        const Layout& L = h->L;
        const int64_t no = b->node_off[j], to = b->tile_off[j], pb = b->pbase[j],
                      eo = b->elem_off[j];
        for (int64_t t = 0; t < h->d.T; t++) {
            tno[to + t] = (int32_t)(L.tile_node_off[t] + pb);
            teo[to + t] = (int32_t)(eo + L.tile_elem_off[t]);
            tsc[to + t] = j;
            // single-tile node ids shift with the nodes, positions with the
            // partials
            const int32_t* tp = &L.tile_part[4 * t];
            int32_t* bt = &tpart[4 * (to + t)];
            bt[0] = (int32_t)(tp[0] + pb);
            bt[1] = tp[1];
            bt[2] = (int32_t)(tp[2] + pb);
            bt[3] = (int32_t)(tp[3] + no);
        }
        for (int64_t p = 0; p < h->d.P; p++) {
            tnodes[pb + p] = (int32_t)(L.tile_nodes[p] + no);
            wp[pb + p] = (int32_t)(L.pidx[p] + pb);
        }
        const int64_t npad = b->node_off[j + 1] - no;
        for (int64_t i = 0; i < npad; i++)
            poff[no + i] = (int32_t)((i < h->N ? L.part_off[i] : L.part_off[h->N]) + pb);
        for (int64_t k = no / 256; k < b->node_off[j + 1] / 256; k++) bsc[k] = j;
        ssingle[2 * j] = (int32_t)(no + L.n_int);
        ssingle[2 * j + 1] = (int32_t)(pb - no);
    }
    tno[Tt] = (int32_t)Pt;
    teo[Tt] = (int32_t)Et;
    poff[Nt] = (int32_t)Pt;
    BCHK(bupload(b, &d.tile_node_off, tno));
    BCHK(bupload(b, &d.tile_nodes, tnodes));
    BCHK(bupload(b, &d.tile_part, tpart));
    BCHK(bupload(b, &d.part_off, poff));
    BCHK(bupload(b, &d.pidx, wp));
    BCHK(bupload(b, &d.tile_elem_off, teo));
    BCHK(bupload(b, &b->tile_scen, tsc));
    BCHK(bupload(b, &b->block_scen, bsc));
    BCHK(bupload(b, &b->scen_single, ssingle));
    BCHK(balloc(b, &b->tile_list, Tt));
    BCHK(balloc(b, &b->block_list, Nt / 256));
    BCHK(balloc(b, &b->flags, n));
    // numeric arrays
    const size_t rb = b->fp32c ? 4 : 8;
    auto ralloc = [&](void** p, size_t count) {
        unsigned char* q = nullptr;
        hipError_t e = balloc(b, &q, count * rb);
        *p = q;
        return e;
    };
    // corner ids stay packed when every scenario's are; otherwise packed
    // scenarios are expanded to u16 on the device
    d.lconn_pk = 1;
    for (int j = 0; j < n; j++) d.lconn_pk &= handles[j]->d.lconn_pk;
    unsigned char* lc = nullptr;
    BCHK(balloc(b, &lc, (d.lconn_pk ? 5 : 8) * Et));
    d.lconn = lc;
    BCHK(ralloc(&d.coef, 6 * Et));
    BCHK(ralloc(&d.u, Nt));
    BCHK(ralloc(&d.q, Nt));
    BCHK(ralloc(&d.partial, Pt));
    BCHK(ralloc(&b->props, n * (b->fp32c ? sizeof(Props<float>) : sizeof(Props<double>)) / rb + 1));
    for (int k = 0; k < 2; k++) {
        double* tb = nullptr;  // float2 (hi, lo) or double: 8 bytes per node
        BCHK(balloc(b, &tb, Nt));
        d.T_[k] = tb;
    }
    // padding nodes: u = -1 (never updated); copy each scenario's data
    {
        std::vector<unsigned char> neg(Nt * rb);
        if (b->fp32c) {
            std::vector<float> v(Nt, -1.0f);
            std::memcpy(neg.data(), v.data(), Nt * rb);
        } else {
            std::vector<double> v(Nt, -1.0);
            std::memcpy(neg.data(), v.data(), Nt * rb);
        }
        BCHK(hipMemcpyAsync(d.u, neg.data(), Nt * rb, hipMemcpyHostToDevice, b->stream));
        BCHK(hipStreamSynchronize(b->stream));
    }
    for (int j = 0; j < n; j++) {
        const fedfem_handle* h = handles[j];
        const int64_t no = b->node_off[j], eo = b->elem_off[j];
        const unsigned char* hl = static_cast<const unsigned char*>(h->d.lconn);
        if (d.lconn_pk) {
            BCHK(hipMemcpyAsync(lc + 4 * eo, hl, 4 * h->E, hipMemcpyDeviceToDevice, b->stream));
            BCHK(hipMemcpyAsync(lc + 4 * Et + eo, hl + 4 * h->E, h->E, hipMemcpyDeviceToDevice,
                                b->stream));
        } else if (h->d.lconn_pk) {
            BCHK(launch_lconn_unpack(hl, h->E, reinterpret_cast<uint16_t*>(lc) + 4 * eo,
                                     b->stream));
        } else {
            BCHK(hipMemcpyAsync(lc + 8 * eo, hl, 8 * h->E, hipMemcpyDeviceToDevice, b->stream));
        }
        for (int k = 0; k < 6; k++)
            BCHK(hipMemcpyAsync(static_cast<unsigned char*>(d.coef) + (k * Et + eo) * rb,
                                static_cast<const unsigned char*>(h->d.coef) + k * h->E * rb,
                                h->E * rb, hipMemcpyDeviceToDevice, b->stream));
        BCHK(hipMemcpyAsync(static_cast<unsigned char*>(d.u) + no * rb, h->d.u, h->N * rb,
                            hipMemcpyDeviceToDevice, b->stream));
    }
    BCHK(hipStreamSynchronize(b->stream));
    *out = b;
    return FEDFEM_OK;
}

int fedfem_batch_run(fedfem_batch* b, const int64_t* n_steps, const double* const* sources) {
    if (!b || !n_steps) return FEDFEM_E_INVALID;
    const int S = b->S;
    for (int j = 0; j < S; j++) {
        if (n_steps[j] < 0 || n_steps[j] > 100000000) return FEDFEM_E_INVALID;
        const fedfem_handle* h = b->hs[j];
        if (h->broken || !h->precomputed || !(h->dt > 0)) return FEDFEM_E_STATE;
        // a schedule or dose model set after the batch was created would be
        // ignored by the lockstep launches: refuse, as fedfem_batch_create does
        if (h->d.n_pat > 0 || h->d.dose) return FEDFEM_E_STATE;
    }
    // new sources replace the handles' active ones, as in fedfem_step; all
    // are checked before any is taken
    if (sources) {
        for (int j = 0; j < S; j++)
            if (sources[j])
                for (int64_t i = 0; i < b->hs[j]->N; i++)
                    if (!std::isfinite(sources[j][i])) return FEDFEM_E_INVALID;
        for (int j = 0; j < S; j++)
            if (sources[j]) {
                const int rc = fedfem_set_source(b->hs[j], sources[j]);
                if (rc) return rc;
            }
    }
    RCHK(hipSetDevice(b->device));
    DevLayout& d = b->d;
    const size_t rb = b->fp32c ? 4 : 8;
    // Two independent lockstep chains, each over half of the scenarios (by
    // element-steps), so that one chain's node pass and the tail of each
    // launch overlap the other chain's work.  Within a chain, longest first:
    // the active scenarios form a prefix of its lists.
    std::vector<int> ord(S);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int x, int y) { return n_steps[x] > n_steps[y]; });
    std::vector<int> grp[kChains];
    {
        int64_t work[kChains] = {};
        for (int r = 0; r < S; r++) {
            const int j = ord[r];
            int g = 0;
            for (int c = 1; c < kChains; c++)
                if (work[c] < work[g]) g = c;
            grp[g].push_back(j);
            work[g] += (b->elem_off[j + 1] - b->elem_off[j]) * std::max<int64_t>(1, n_steps[j]);
        }
    }
    std::vector<int32_t> tl, bl;
    std::vector<int64_t> tcum[kChains], bcum[kChains];
    int64_t tbase[kChains], bbase[kChains];
    for (int g = 0; g < kChains; g++) {
        tbase[g] = (int64_t)tl.size();
        bbase[g] = (int64_t)bl.size();
        tcum[g].assign(grp[g].size() + 1, 0);
        bcum[g].assign(grp[g].size() + 1, 0);
        for (size_t r = 0; r < grp[g].size(); r++) {
            const int j = grp[g][r];
            for (int64_t t = b->tile_off[j]; t < b->tile_off[j + 1]; t++)
                tl.push_back((int32_t)t);
            for (int64_t k = b->node_off[j] / 256; k < b->node_off[j + 1] / 256; k++)
                bl.push_back((int32_t)k);
            tcum[g][r + 1] = (int64_t)tl.size() - tbase[g];
            bcum[g][r + 1] = (int64_t)bl.size() - bbase[g];
        }
    }
    RCHK(hipMemcpyAsync(b->tile_list, tl.data(), tl.size() * 4, hipMemcpyHostToDevice,
                        b->stream));
    RCHK(hipMemcpyAsync(b->block_list, bl.data(), bl.size() * 4, hipMemcpyHostToDevice,
                        b->stream));
    // per-scenario parameters (dt may have changed since creation)
    if (b->fp32c) {
        std::vector<Props<float>> p(S);
        for (int j = 0; j < S; j++) p[j] = props_of<float>(b->hs[j]);
        RCHK(hipMemcpyAsync(b->props, p.data(), S * sizeof(p[0]), hipMemcpyHostToDevice,
                            b->stream));
    } else {
        std::vector<Props<double>> p(S);
        for (int j = 0; j < S; j++) p[j] = props_of<double>(b->hs[j]);
        RCHK(hipMemcpyAsync(b->props, p.data(), S * sizeof(p[0]), hipMemcpyHostToDevice,
                            b->stream));
    }
    // copy-in of each scenario's state (both buffers) and source
    for (int j = 0; j < S; j++) {
        fedfem_handle* h = b->hs[j];
        const int64_t no = b->node_off[j];
        for (int k = 0; k < 2; k++)
            RCHK(hipMemcpyAsync(static_cast<unsigned char*>(d.T_[k]) + no * 8, h->d.T_[h->cur],
                                h->N * 8, hipMemcpyDeviceToDevice, b->stream));
        RCHK(hipMemcpyAsync(static_cast<unsigned char*>(d.q) + no * rb, h->d.q, h->N * rb,
                            hipMemcpyDeviceToDevice, b->stream));
    }
    RCHK(launch_fill_i32(b->flags, S, 0, b->stream));
    // graph of the whole run
    std::vector<int64_t> key(n_steps, n_steps + S);
    const int64_t nmax = S ? n_steps[ord[0]] : 0;
    hipGraphExec_t ex = nullptr;
    auto it = b->graphs.find(key);
    if (it != b->graphs.end()) {
        ex = it->second;
    } else if (nmax > 0) {
        if (b->graphs.size() >= 4) {
            for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
            b->graphs.clear();
        }
        RCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        hipError_t err = hipEventRecord(b->ev_fork, b->cap);
        bool forked[kChains] = {};
        for (int g = 1; g < kChains && err == hipSuccess; g++)
            if (!grp[g].empty()) {
                err = hipStreamWaitEvent(b->chain[g - 1], b->ev_fork, 0);
                forked[g] = err == hipSuccess;
            }
        for (int g = 0; g < kChains && err == hipSuccess; g++) {
            if (grp[g].empty()) continue;
            hipStream_t cs = g == 0 ? b->cap : b->chain[g - 1];
            BatchTables tb;
            tb.tile_list = b->tile_list + tbase[g];
            tb.tile_scen = b->tile_scen;
            tb.block_list = b->block_list + bbase[g];
            tb.block_scen = b->block_scen;
            tb.props = b->props;
            tb.scen_single = reinterpret_cast<const int2*>(b->scen_single);
            int r = (int)grp[g].size();  // active scenarios of the chain
            const int64_t kmax = n_steps[grp[g][0]];
            for (int64_t k = 0; k < kmax && err == hipSuccess; k++) {
                while (r > 0 && n_steps[grp[g][r - 1]] <= k) r--;
                const int cur = (int)(k & 1);
                err = launch_elem_batch(d, tb, cur, (int)tcum[g][r], b->fp32c, cs);
                if (err == hipSuccess)
                    err = launch_node_batch(d, tb, cur, (int)bcum[g][r], b->fp32c, b->flags, cs);
            }
        }
        // join every forked chain, also after an error, so that the capture
        // ends cleanly
        for (int g = 1; g < kChains; g++)
            if (forked[g]) {
                hipError_t ej = hipEventRecord(b->ev_join[g - 1], b->chain[g - 1]);
                if (ej == hipSuccess) ej = hipStreamWaitEvent(b->cap, b->ev_join[g - 1], 0);
                if (err == hipSuccess) err = ej;
            }
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->cap, &g);
        if (err != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return FEDFEM_E_HIP;
        }
        hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        RCHK(e3);
        b->graphs[key] = ex;
    }
    RCHK(hipEventRecord(b->ev0, b->stream));
    if (ex) RCHK(hipGraphLaunch(ex, b->stream));
    RCHK(hipEventRecord(b->ev1, b->stream));
    // copy-out into each handle's current buffer
    for (int j = 0; j < S; j++) {
        fedfem_handle* h = b->hs[j];
        const int64_t no = b->node_off[j];
        const int fin = (int)(n_steps[j] & 1);
        RCHK(hipMemcpyAsync(h->d.T_[h->cur], static_cast<unsigned char*>(d.T_[fin]) + no * 8,
                            h->N * 8, hipMemcpyDeviceToDevice, b->stream));
    }
    std::vector<int32_t> fl(S);
    RCHK(hipMemcpyAsync(fl.data(), b->flags, S * 4, hipMemcpyDeviceToHost, b->stream));
    RCHK(hipStreamSynchronize(b->stream));
    float ms = 0.0f;
    RCHK(hipEventElapsedTime(&ms, b->ev0, b->ev1));
    b->last_ms = ms;
    int rc = FEDFEM_OK;
    for (int j = 0; j < S; j++) {
        fedfem_handle* h = b->hs[j];
        h->steps += n_steps[j];
        h->t += (double)n_steps[j] * h->dt;
        if (fl[j]) {
            h->err = "temperature left [-1e4, 1e4] degC or NaN in a batched run";
            rc = FEDFEM_E_DIVERGED;
        }
    }
    return rc;
}

int fedfem_batch_last_ms(const fedfem_batch* b, double* ms) {
    if (!b || !ms) return FEDFEM_E_INVALID;
    *ms = b->last_ms;
    return FEDFEM_OK;
}

int fedfem_batch_destroy(fedfem_batch* b) {
    destroy_batch(b);
    return FEDFEM_OK;
}

}  // extern "C"
