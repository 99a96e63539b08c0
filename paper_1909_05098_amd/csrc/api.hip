// C ABI of the FED-FEM gfx950 library: handle lifecycle, pre-computation,
// graph-captured time stepping, sources, read-back and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <system_error>
#include <thread>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <utility>
#include <vector>

#include "../../include/fedfem.h"
#include "handle.h"
#include "internal.h"

using namespace fedfem;

// Tile partials of fedfem_step_static: a fixed device array instead of the
// handle's own buffer, so that call allocates nothing.  Each device holds its
// own copy for the life of the process; host code reaches it only through the
// address hipGetSymbolAddress returns on that device (static_scratch below).
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

int set_err(fedfem_handle* h, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    return code;
}

int hip_fail(fedfem_handle* h, hipError_t e, const char* where) {
    if (h) h->broken = true;
    return set_err(h, FEDFEM_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define HIPCHK(h, expr)                                            \
    do {                                                           \
        hipError_t e_ = (expr);                                    \
        if (e_ != hipSuccess) return hip_fail((h), e_, #expr);     \
    } while (0)

bool finite_all(const double* p, int64_t n) {
    for (int64_t i = 0; i < n; i++)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// Property window bounds of the clamped linear laws (rho c may be quadratic
// in T; its extremum may lie inside the window).
void window_bounds(const fedfem_materials& m, double* kmin, double* kmax, double* rcmin,
                   double* rcmax) {
    std::vector<double> ts = {m.T_lo, m.T_hi};
    const double a = m.drho_dT * m.dc_dT;
    if (a != 0.0) {
        const double b = m.rho0 * m.dc_dT + m.c0 * m.drho_dT;
        const double tv = m.T_ref - b / (2.0 * a);
        if (tv > m.T_lo && tv < m.T_hi) ts.push_back(tv);
    }
    *kmin = 1e300;
    *kmax = -1e300;
    *rcmin = 1e300;
    *rcmax = -1e300;
    for (double T : ts) {
        const double d = T - m.T_ref;
        const double k = m.k0 + m.dk_dT * d;
        const double rc = (m.rho0 + m.drho_dT * d) * (m.c0 + m.dc_dT * d);
        *kmin = std::min(*kmin, k);
        *kmax = std::max(*kmax, k);
        *rcmin = std::min(*rcmin, rc);
        *rcmax = std::max(*rcmax, rc);
    }
}

// Property p (0 k, 1 rho, 2 c) at T: the handle's table if it has one, else
// the material's clamped linear law.
double prop_at(const fedfem_handle* h, int p, double T) {
    const std::vector<double>& t = h->tab_t[p];
    const std::vector<double>& v = h->tab_v[p];
    if (!t.empty()) {
        if (T <= t[0]) return v[0];
        if (T >= t.back()) return v.back();
        size_t k = (size_t)(std::upper_bound(t.begin(), t.end(), T) - t.begin()) - 1;
        return v[k] + (v[k + 1] - v[k]) * (T - t[k]) / (t[k + 1] - t[k]);
    }
    const fedfem_materials& m = h->mat;
    const double d = std::min(std::max(T, m.T_lo), m.T_hi) - m.T_ref;
    return p == 0 ? m.k0 + m.dk_dT * d : (p == 1 ? m.rho0 + m.drho_dT * d : m.c0 + m.dc_dT * d);
}

// Extremes of k and rho c over all temperatures for a handle with tables:
// every property is piecewise linear with breakpoints at its table points
// (or its window ends), so k peaks at a breakpoint and rho c, quadratic
// between consecutive breakpoints, at a breakpoint or a vertex.
void window_bounds_h(const fedfem_handle* h, double* kmin, double* kmax, double* rcmin,
                     double* rcmax) {
    bool any = false;
    for (int p = 0; p < 3; p++) any |= !h->tab_t[p].empty();
    if (!any) return window_bounds(h->mat, kmin, kmax, rcmin, rcmax);
    std::vector<double> ts;
    for (int p = 0; p < 3; p++) {
        if (h->tab_t[p].empty()) {
            ts.push_back(h->mat.T_lo);
            ts.push_back(h->mat.T_hi);
        } else {
            ts.insert(ts.end(), h->tab_t[p].begin(), h->tab_t[p].end());
        }
    }
    std::sort(ts.begin(), ts.end());
    ts.erase(std::unique(ts.begin(), ts.end()), ts.end());
    std::vector<double> cand = ts;
    for (size_t i = 0; i + 1 < ts.size(); i++) {
        const double a = ts[i], b = ts[i + 1];
        const double r0 = prop_at(h, 1, a), r1 = prop_at(h, 1, b);
        const double c0 = prop_at(h, 2, a), c1 = prop_at(h, 2, b);
        const double sr = (r1 - r0) / (b - a), sc = (c1 - c0) / (b - a);
        if (sr * sc != 0.0) {
            const double x = a - (r0 * sc + c0 * sr) / (2.0 * sr * sc);
            if (x > a && x < b) cand.push_back(x);
        }
    }
    *kmin = *rcmin = 1e300;
    *kmax = *rcmax = -1e300;
    for (double T : cand) {
        const double k = prop_at(h, 0, T), rc = prop_at(h, 1, T) * prop_at(h, 2, T);
        *kmin = std::min(*kmin, k);
        *kmax = std::max(*kmax, k);
        *rcmin = std::min(*rcmin, rc);
        *rcmax = std::max(*rcmax, rc);
    }
}

// 2^S with S = 58 - ceil(log2(bound)), kept inside float range: values of
// magnitude <= bound scale below 2^58.
double fixed_scale(double bound) {
    if (!(bound > 0) || !std::isfinite(bound)) return 1.0;
    int S = 58 - (int)std::ceil(std::log2(bound));
    S = std::max(-100, std::min(100, S));
    return std::ldexp(1.0, S);
}

// Largest eigenvalue of the symmetric tridiagonal matrix (a[0..k), b[1..k))
// by Sturm-sequence bisection, and the last component of its unit
// eigenvector by shifted inverse iteration.
void tridiag_top(const std::vector<double>& a, const std::vector<double>& b, int k,
                 double* theta, double* last) {
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < k; i++) {
        const double r = (i > 0 ? std::fabs(b[i]) : 0.0) + (i + 1 < k ? std::fabs(b[i + 1]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    auto count_below = [&](double x) {
        int c = 0;
        double q = a[0] - x;
        if (q < 0) c++;
        for (int i = 1; i < k; i++) {
            if (q == 0.0) q = 1e-300;
            q = (a[i] - x) - b[i] * b[i] / q;
            if (q < 0) c++;
        }
        return c;
    };
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(hi), 1e-300); it++) {
        const double mid = 0.5 * (lo + hi);
        if (count_below(mid) >= k)
            hi = mid;
        else
            lo = mid;
    }
    *theta = hi;
    // inverse iteration with a shift just above theta: (T - s I) y = x
    const double s = hi + 1e-9 * std::max(std::fabs(hi), 1e-300);
    std::vector<double> y(k, 1.0), c(k), d(k);
    for (int rep = 0; rep < 3; rep++) {
        // Thomas algorithm on the (negative definite) shifted matrix
        d[0] = a[0] - s;
        std::vector<double> r = y;
        for (int i = 1; i < k; i++) {
            c[i] = b[i] / d[i - 1];
            d[i] = (a[i] - s) - c[i] * b[i];
            r[i] -= c[i] * r[i - 1];
        }
        y[k - 1] = r[k - 1] / d[k - 1];
        for (int i = k - 2; i >= 0; i--) y[i] = (r[i] - b[i + 1] * y[i + 1]) / d[i];
        double nrm = 0.0;
        for (double v : y) nrm += v * v;
        nrm = std::sqrt(nrm);
        for (double& v : y) v /= nrm;
    }
    *last = y[k - 1];
}

// Quadrature points of the composite source rule: two regular (Bey)
// refinements of the reference tetrahedron, then the symmetric 4-point
// degree-2 rule on each of the 64 children, in barycentric coordinates.
void make_quadrature(std::vector<double>& pts) {
    struct Tet {
        double v[4][4];
    };
    std::vector<Tet> level(1);
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) level[0].v[i][j] = (i == j) ? 1.0 : 0.0;
    // child corner lists over {v0..v3, m01, m02, m03, m12, m13, m23}
    static const int kids[8][4] = {{0, 4, 5, 6}, {4, 1, 7, 8}, {5, 7, 2, 9}, {6, 8, 9, 3},
                                   {4, 5, 6, 8}, {4, 5, 7, 8}, {5, 6, 8, 9}, {5, 7, 8, 9}};
    static const int mids[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    for (int lv = 0; lv < 2; lv++) {
        std::vector<Tet> next;
        for (const Tet& t : level) {
            double P[10][4];
            for (int i = 0; i < 4; i++) std::memcpy(P[i], t.v[i], sizeof(P[i]));
            for (int m = 0; m < 6; m++)
                for (int c = 0; c < 4; c++)
                    P[4 + m][c] = 0.5 * (t.v[mids[m][0]][c] + t.v[mids[m][1]][c]);
            for (int k = 0; k < 8; k++) {
                Tet ch;
                for (int i = 0; i < 4; i++) std::memcpy(ch.v[i], P[kids[k][i]], sizeof(ch.v[i]));
                next.push_back(ch);
            }
        }
        level.swap(next);
    }
    const double wa = (5.0 + 3.0 * std::sqrt(5.0)) / 20.0;
    const double wb = (5.0 - std::sqrt(5.0)) / 20.0;
    pts.clear();
    for (const Tet& t : level)
        for (int q = 0; q < 4; q++)
            for (int c = 0; c < 4; c++) {
                double s = 0.0;
                for (int k = 0; k < 4; k++) s += (k == q ? wa : wb) * t.v[k][c];
                pts.push_back(s);
            }
}

template <typename T>
int dalloc(fedfem_handle* h, T** p, size_t count) {
    void* q = nullptr;
    const size_t bytes = std::max<size_t>(count * sizeof(T), 16);
    size_t granted = 0;
    hipError_t e = cached_malloc(&q, bytes, &granted);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_err(h, FEDFEM_E_NOMEM, "device allocation of %zu bytes failed", bytes);
    }
    h->allocs.emplace_back(q, granted);
    h->dev_bytes += (int64_t)granted;
    *p = static_cast<T*>(q);
    return FEDFEM_OK;
}

// the handle's streams are idle before a block goes back to the cache
void quiesce(fedfem_handle* h) {
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->own_stream && h->own_stream != h->stream) (void)hipStreamSynchronize(h->own_stream);
}

void dfree(fedfem_handle* h, void* p) {
    if (!p) return;
    auto it = std::find_if(h->allocs.begin(), h->allocs.end(),
                           [p](const std::pair<void*, size_t>& a) { return a.first == p; });
    if (it != h->allocs.end()) {
        quiesce(h);
        h->dev_bytes -= (int64_t)it->second;
        cached_free(it->first, it->second);
        h->allocs.erase(it);
    }
}

template <typename T>
int upload(fedfem_handle* h, T** dst, const std::vector<T>& src) {
    int rc = dalloc(h, dst, src.size());
    if (rc) return rc;
    HIPCHK(h, hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice,
                             h->own_stream));
    return FEDFEM_OK;
}

void drop_graphs(fedfem_handle* h) {
    for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
}

Props<float> props_f(const fedfem_handle* h) {
    const fedfem_materials& m = h->mat;
    Props<float> p;
    p.k0 = (float)m.k0;
    p.dk = (float)m.dk_dT;
    p.rho0 = (float)m.rho0;
    p.drho = (float)m.drho_dT;
    p.c0 = (float)m.c0;
    p.dc = (float)m.dc_dT;
    p.Tref = (float)m.T_ref;
    p.Tlo = (float)m.T_lo;
    p.Thi = (float)m.T_hi;
    p.wbcb = (float)(m.w_b * m.c_b);
    p.Ta = (float)m.T_a;
    p.Qm = (float)m.Q_m;
    p.dt = (float)h->dt;
    p.fxs = (float)h->fx_scale;
    p.fxi = (float)(1.0 / h->fx_scale);
    p.tab = static_cast<const float*>(h->d_tab);
    for (int k = 0; k < 3; k++) p.nt[k] = h->d_tab ? (int)h->tab_t[k].size() : 0;
    return p;
}

Props<double> props_d(const fedfem_handle* h) {
    const fedfem_materials& m = h->mat;
    Props<double> p;
    p.k0 = m.k0;
    p.dk = m.dk_dT;
    p.rho0 = m.rho0;
    p.drho = m.drho_dT;
    p.c0 = m.c0;
    p.dc = m.dc_dT;
    p.Tref = m.T_ref;
    p.Tlo = m.T_lo;
    p.Thi = m.T_hi;
    p.wbcb = m.w_b * m.c_b;
    p.Ta = m.T_a;
    p.Qm = m.Q_m;
    p.dt = h->dt;
    p.fxs = h->fx_scale;
    p.fxi = 1.0 / h->fx_scale;
    p.tab = static_cast<const double*>(h->d_tab);
    for (int k = 0; k < 3; k++) p.nt[k] = h->d_tab ? (int)h->tab_t[k].size() : 0;
    return p;
}

hipError_t launch_one_step(fedfem_handle* h, int cur, hipStream_t s, int j) {
    const bool td = h->mat.dk_dT != 0.0 || !h->tab_t[0].empty();
    h->d.dose_dt = h->dt;
    if (h->fp32c) return launch_step_f32c(h->d, cur, props_f(h), td, h->d_flag, s, j);
    return launch_step_f64(h->d, cur, props_d(h), td, h->d_flag, s, j);
}

// Amplitude of a schedule at time x: piecewise linear through (t[k], a[k]),
// constant before the first and after the last point; where times repeat,
// the last point at that time holds from it on.
double sched_amp(const std::vector<double>& t, const std::vector<double>& a, double x) {
    if (x < t[0]) return a[0];
    const size_t k = (size_t)(std::upper_bound(t.begin(), t.end(), x) - t.begin()) - 1;
    if (k + 1 >= t.size()) return a.back();
    return a[k] + (a[k + 1] - a[k]) * (x - t[k]) / (t[k + 1] - t[k]);
}

int get_graph(fedfem_handle* h, int64_t n, int cur, hipGraphExec_t* out) {
    auto key = std::make_pair(n, cur);
    auto it = h->graphs.find(key);
    if (it != h->graphs.end()) {
        *out = it->second;
        return FEDFEM_OK;
    }
    if (h->graphs.size() >= 16) drop_graphs(h);
    HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    int c = cur;
    for (int64_t k = 0; k < n; k++) {
        hipError_t e = launch_one_step(h, c, h->cap_stream, (int)k);
        if (e != hipSuccess) {
            hipGraph_t g;
            (void)hipStreamEndCapture(h->cap_stream, &g);
            return hip_fail(h, e, "kernel launch during capture");
        }
        c ^= 1;
    }
    hipGraph_t g = nullptr;
    HIPCHK(h, hipStreamEndCapture(h->cap_stream, &g));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(h, e, "hipGraphInstantiate");
    h->graphs[key] = ex;
    *out = ex;
    return FEDFEM_OK;
}

int check_handle(fedfem_handle* h, bool need_pre) {
    if (!h) return FEDFEM_E_INVALID;
    if (h->broken) return set_err(h, FEDFEM_E_HIP, "handle unusable after a HIP failure");
    if (need_pre && !h->precomputed)
        return set_err(h, FEDFEM_E_NOT_PRECOMPUTED, "fedfem_precompute has not run");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    return FEDFEM_OK;
}

int lanczos(fedfem_handle* h, const double* coef64) {
    const int64_t N = h->N;
    const int maxit = h->lz_max_iter;
    double *sc, *v, *vprev, *w, *xs, *partial, *bsum, *alpha, *beta, *scal;
    int32_t* counter = nullptr;
    int rc = 0;
    const int64_t nb = (N + 255) / 256;
    if ((rc = dalloc(h, &sc, N)) || (rc = dalloc(h, &v, N)) || (rc = dalloc(h, &vprev, N)) ||
        (rc = dalloc(h, &w, N)) || (rc = dalloc(h, &xs, N)) ||
        (rc = dalloc(h, &partial, h->d.P)) || (rc = dalloc(h, &bsum, nb)) ||
        (rc = dalloc(h, &alpha, maxit + 1)) || (rc = dalloc(h, &beta, maxit + 2)) ||
        (rc = dalloc(h, &scal, 4)) || (rc = dalloc(h, &counter, 1)))
        return rc;
    HIPCHK(h, hipMemsetAsync(beta, 0, sizeof(double) * (maxit + 2), h->own_stream));
    HIPCHK(h, launch_fill_i32(counter, 1, 0, h->own_stream));
    HIPCHK(h, launch_lanczos_start(N, h->d_Vi, h->d_isdir, sc, v, vprev, xs, bsum, scal,
                                   h->own_stream));
    std::vector<double> a(maxit + 1), b(maxit + 2);
    double theta = 0.0, prev = -1.0, last = 0.0;
    int k = 0;
    // the host looks at the coefficients every 8 iterations (one stream
    // synchronisation each); a breakdown (beta ~ 0: the Krylov space is
    // exhausted) inside such a stretch ends the recurrence at its first
    // occurrence, and the coefficients computed after it are ignored
    constexpr int kCheck = 8;
    for (int j = 0; j < maxit; j++) {
        HIPCHK(h, launch_lanczos_iter(h->d, coef64, h->fx_scale_lz, j, sc, v, vprev, w, xs,
                                      partial, bsum, counter, alpha, beta, h->own_stream));
        k = j + 1;
        if (k % kCheck == 0 || k == maxit) {
            HIPCHK(h, hipMemcpyAsync(a.data(), alpha, sizeof(double) * k,
                                     hipMemcpyDeviceToHost, h->own_stream));
            HIPCHK(h, hipMemcpyAsync(b.data(), beta, sizeof(double) * (k + 1),
                                     hipMemcpyDeviceToHost, h->own_stream));
            HIPCHK(h, hipStreamSynchronize(h->own_stream));
            // first breakdown in this stretch, against the largest |alpha| so far
            // (a scale of the operator that is known before its Ritz value)
            double scale = 1e-300;
            for (int m = 0; m < k; m++) scale = std::max(scale, std::fabs(a[m]));
            int kb = k;
            for (int m = k - kCheck + 1; m <= k; m++)
                if (m >= 1 && !(b[m] > 1e-13 * scale)) {
                    kb = m;
                    break;
                }
            tridiag_top(a, b, kb, &theta, &last);
            if (kb < k || std::fabs(theta - prev) <= 1e-11 * theta) {
                k = kb;
                break;
            }
            prev = theta;
        }
    }
    h->lz_iters = k;
    h->lam_ritz = theta;
    h->lam_geo = theta + std::fabs(b[k] * last);
    for (void* p : {(void*)sc, (void*)v, (void*)vprev, (void*)w, (void*)xs, (void*)partial,
                    (void*)bsum, (void*)alpha, (void*)beta, (void*)scal, (void*)counter})
        dfree(h, p);
    return FEDFEM_OK;
}

int release_device(fedfem_handle* h) {
    drop_graphs(h);
    quiesce(h);
    for (auto& a : h->allocs) cached_free(a.first, a.second);
    h->allocs.clear();
    h->dev_bytes = 0;
    h->d = DevLayout();
    h->d_tab = nullptr;
    return FEDFEM_OK;
}

}  // namespace

extern "C" {

const char* fedfem_strerror(int code) {
    switch (code) {
        case FEDFEM_OK: return "ok";
        case FEDFEM_E_INVALID: return "invalid argument";
        case FEDFEM_E_DEGENERATE: return "degenerate element";
        case FEDFEM_E_NOT_PRECOMPUTED: return "not precomputed";
        case FEDFEM_E_UNSTABLE: return "time step not below the critical step";
        case FEDFEM_E_DIVERGED: return "solution diverged";
        case FEDFEM_E_HIP: return "HIP runtime failure";
        case FEDFEM_E_NOMEM: return "out of memory";
        case FEDFEM_E_STATE: return "call not valid in this state";
        case FEDFEM_E_TOO_LARGE: return "problem larger than the static scratch";
        default: return "unknown error";
    }
}

int fedfem_last_error(const fedfem_handle* h, char* buf, size_t len) {
    if (!h || !buf || len == 0) return FEDFEM_E_INVALID;
    std::snprintf(buf, len, "%s", h->err.c_str());
    return FEDFEM_OK;
}

namespace {

// fedfem_create and fedfem_create_hex: elements of npe nodes each
int create_handle(int64_t N, const double* xyz, int64_t E, const int32_t* conn, int npe,
                  const fedfem_materials* mat, const fedfem_bc* bc, fedfem_handle** out) {
    if (!out) return FEDFEM_E_INVALID;
    *out = nullptr;
    if (!mat || !bc) return FEDFEM_E_INVALID;
    if (N < npe || E < 1 || !xyz || !conn || N > INT32_MAX || npe * E > INT32_MAX)
        return FEDFEM_E_INVALID;
    if (!finite_all(xyz, 3 * N)) return FEDFEM_E_INVALID;
    fedfem_handle* h = new (std::nothrow) fedfem_handle();
    if (!h) return FEDFEM_E_NOMEM;
    auto fail = [&](int code) {
        delete h;
        return code;
    };
    try {
        h->N = N;
        h->E = E;
        h->npe = npe;
        h->xyz.assign(xyz, xyz + 3 * N);
        h->tets.assign(conn, conn + npe * E);
        std::vector<uint8_t> used(N, 0);
        for (int64_t s = 0; s < npe * E; s++) {
            const int32_t n = h->tets[s];
            if (n < 0 || n >= N) return fail(FEDFEM_E_INVALID);
            used[n] = 1;
        }
        for (int64_t i = 0; i < N; i++)
            if (!used[i]) return fail(FEDFEM_E_INVALID);
        const fedfem_materials& m = *mat;
        const double vals[] = {m.rho0, m.c0, m.k0, m.drho_dT, m.dc_dT, m.dk_dT, m.T_ref,
                               m.T_lo, m.T_hi, m.w_b, m.c_b, m.T_a, m.Q_m};
        if (!finite_all(vals, 13)) return fail(FEDFEM_E_INVALID);
        if (!(m.T_lo < m.T_hi) || m.w_b < 0 || m.c_b < 0) return fail(FEDFEM_E_INVALID);
        if (m.precision != FEDFEM_FP64 && m.precision != FEDFEM_FP32C)
            return fail(FEDFEM_E_INVALID);
        double kmin, kmax, rcmin, rcmax;
        window_bounds(m, &kmin, &kmax, &rcmin, &rcmax);
        if (!(kmin > 0) || !(rcmin > 0)) return fail(FEDFEM_E_INVALID);
        h->mat = m;
        h->fp32c = (m.precision == FEDFEM_FP32C);
        if (!std::isfinite(bc->T0) || !std::isfinite(bc->dt) || bc->dt == 0.0 ||
            bc->dt <= -1.0 || bc->n_dir < 0 || bc->n_dir > N)
            return fail(FEDFEM_E_INVALID);
        if (bc->n_dir > 0 && (!bc->dir_nodes || !bc->dir_T)) return fail(FEDFEM_E_INVALID);
        h->T0 = bc->T0;
        h->dt_spec = bc->dt;
        std::vector<uint8_t> seen(N, 0);
        for (int64_t k = 0; k < bc->n_dir; k++) {
            const int32_t n = bc->dir_nodes[k];
            if (n < 0 || n >= N || seen[n] || !std::isfinite(bc->dir_T[k]))
                return fail(FEDFEM_E_INVALID);
            seen[n] = 1;
        }
        h->dir_nodes.assign(bc->dir_nodes, bc->dir_nodes + bc->n_dir);
        h->dir_T.assign(bc->dir_T, bc->dir_T + bc->n_dir);
    } catch (const std::bad_alloc&) {
        return fail(FEDFEM_E_NOMEM);
    }
    if (hipGetDevice(&h->device) != hipSuccess) return fail(FEDFEM_E_HIP);
    if (hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking) != hipSuccess)
        return fail(FEDFEM_E_HIP);
    if (hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(h->own_stream);
        return fail(FEDFEM_E_HIP);
    }
    h->stream = h->own_stream;
    h->opt.reorder = 1;
    h->opt.tile_elems = 2048;
    h->opt.threads = 512;
    h->opt.max_tile_nodes = npe == 8 ? 4096 : 1024;
    h->opt.xcd = 0;
    *out = h;
    return FEDFEM_OK;
}

}  // namespace

int fedfem_create(const fedfem_mesh* mesh, const fedfem_materials* mat, const fedfem_bc* bc,
                  fedfem_handle** out) {
    if (!mesh) {
        if (out) *out = nullptr;
        return FEDFEM_E_INVALID;
    }
    return create_handle(mesh->n_nodes, mesh->xyz, mesh->n_tets, mesh->tets, 4, mat, bc, out);
}

int fedfem_create_hex(const fedfem_mesh_hex* mesh, const fedfem_materials* mat,
                      const fedfem_bc* bc, fedfem_handle** out) {
    if (!mesh) {
        if (out) *out = nullptr;
        return FEDFEM_E_INVALID;
    }
    return create_handle(mesh->n_nodes, mesh->xyz, mesh->n_hexes, mesh->hexes, 8, mat, bc, out);
}

int fedfem_set_options(fedfem_handle* h, const fedfem_options* o) {
    if (!h || !o) return FEDFEM_E_INVALID;
    if (h->precomputed) return set_err(h, FEDFEM_E_STATE, "options are fixed after precompute");
    // hexahedra: reordered tiles of up to twice as many nodes as elements
    const bool hex = h->npe == 8;
    const int te = o->tile_elems ? o->tile_elems : 2048;
    const int th = o->threads ? o->threads : std::max(64, std::min(1024, te / 4));
    const int mn = o->max_tile_nodes
                       ? o->max_tile_nodes
                       : (o->reorder ? (hex ? 2 * te : te / 2) : h->npe * te);
    const int r = te / std::max(th, 1);
    if (te < 64 || te > 8192 || te % 64 || th < 64 || th > 1024 || th % 64 || te % th ||
        (r != 1 && r != 2 && r != 4) || mn < h->npe || mn > h->npe * te ||
        (o->reorder != 0 && o->reorder != 1) || (o->xcd != 0 && o->xcd != 1))
        return set_err(h, FEDFEM_E_INVALID, "invalid options");
    h->opt = *o;
    h->opt.tile_elems = te;
    h->opt.threads = th;
    h->opt.max_tile_nodes = mn;
    return FEDFEM_OK;
}

// Wall-clock phases of fedfem_precompute, printed to stderr when the
// environment variable FEDFEM_TRACE is set (diagnostics only).
struct PhaseClock {
    bool on = std::getenv("FEDFEM_TRACE") != nullptr;
    std::chrono::steady_clock::time_point last = std::chrono::steady_clock::now();
    std::string line;
    void mark(const char* name) {
        if (!on) return;
        const auto now = std::chrono::steady_clock::now();
        char buf[64];
        std::snprintf(buf, sizeof buf, " %s %.2f", name,
                      std::chrono::duration<double, std::milli>(now - last).count());
        line += buf;
        last = now;
    }
    void print(int64_t E) const {
        if (on) std::fprintf(stderr, "[fedfem] precompute E=%lld ms:%s\n", (long long)E, line.c_str());
    }
};

int fedfem_precompute(fedfem_handle* h) {
    int rc = check_handle(h, false);
    if (rc) return rc;
    if (h->precomputed) return set_err(h, FEDFEM_E_STATE, "already precomputed");
    release_device(h);
    const int64_t N = h->N, E = h->E;
    PhaseClock clk;
    int lds_attr = 0;
    HIPCHK(h, hipDeviceGetAttribute(&lds_attr, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                    h->device));
    const size_t lds_limit = (size_t)lds_attr;
    Layout& L = h->L;
    std::string err;
    int TE = h->opt.tile_elems;
    try {
        int MN = h->opt.max_tile_nodes;
        if (!build_layout(h->xyz.data(), h->tets.data(), h->npe, N, E, h->opt.reorder, TE, MN,
                          L, err))
            return set_err(h, FEDFEM_E_INVALID, "%s", err.c_str());
        // shrink tiles until the widest kernel (FP64 loads) fits in LDS
        while (tile_lds_bytes(L.tile_elems, L.max_tile_nodes, 8, false, true) > lds_limit) {
            if (L.tile_elems <= 64)
                return set_err(h, FEDFEM_E_INVALID, "tile does not fit in LDS");
            const int te2 = std::max(64, L.tile_elems / 128 * 64);
            MN = std::min(MN, h->npe * te2);
            if (!build_tiles(L, te2, MN, err))
                return set_err(h, FEDFEM_E_INVALID, "%s", err.c_str());
        }
    } catch (const std::bad_alloc&) {
        return set_err(h, FEDFEM_E_NOMEM, "host allocation failed");
    }
    clk.mark("layout");
    hipStream_t s = h->own_stream;
    DevLayout& d = h->d;
    d.N = N;
    d.E = E;
    d.T = L.T;
    d.P = L.P;
    d.n_int = L.n_int;
    d.tile_elems = L.tile_elems;
    d.npe = h->npe;
    d.max_tile_nodes = L.max_tile_nodes;
    d.threads = std::min(h->opt.threads, L.tile_elems);
    while (elems_per_thread(d) > 4 && d.threads < 1024) d.threads *= 2;
    if (elems_per_thread(d) > 4) return set_err(h, FEDFEM_E_INVALID, "tiles too large for the workgroup");
    d.xcd = h->opt.xcd;
    // topology
    try {
        pack_lconn(L);
    } catch (const std::bad_alloc&) {
        return set_err(h, FEDFEM_E_NOMEM, "host allocation failed");
    }
    d.lconn_pk = L.lconn_pk.empty() ? 0 : 1;
    if (d.lconn_pk) {
        uint8_t* p = nullptr;
        if ((rc = upload(h, &p, L.lconn_pk))) return rc;
        d.lconn = p;
    } else {
        uint16_t* p = nullptr;
        if ((rc = upload(h, &p, L.lconn))) return rc;
        d.lconn = p;
    }
    if ((rc = upload(h, &d.tile_elem_off, L.tile_elem_off)) ||
        (rc = upload(h, &d.tile_node_off, L.tile_node_off)) ||
        (rc = upload(h, &d.tile_nodes, L.tile_nodes)) ||
        (rc = upload(h, &d.tile_part, L.tile_part)) ||
        (rc = upload(h, &d.pidx, L.pidx)) || (rc = upload(h, &d.part_off, L.part_off)) ||
        (rc = upload(h, &h->d_ec_off, L.ec_off)) || (rc = upload(h, &h->d_ec, L.ec)) ||
        (rc = upload(h, &h->d_conn, L.conn)) || (rc = upload(h, &h->d_xyz, L.xyz)) ||
        (rc = upload(h, &h->d_nperm, L.nperm)))
        return rc;
    {
        std::vector<int32_t> isd(N, 0);
        std::vector<double> dT(N, 0.0);
        for (size_t k = 0; k < h->dir_nodes.size(); k++) {
            isd[L.ninv[h->dir_nodes[k]]] = 1;
            dT[L.ninv[h->dir_nodes[k]]] = h->dir_T[k];
        }
        h->n_dir = (int64_t)h->dir_nodes.size();
        if ((rc = upload(h, &h->d_isdir, isd)) || (rc = upload(h, &h->d_dirT, dT))) return rc;
        h->host_isdir.swap(isd);
    }
    clk.mark("upload");
    // geometry (Eq 15-16)
    double* coef64 = nullptr;
    int32_t* bad = nullptr;
    int32_t* d_eperm = nullptr;
    if ((rc = upload(h, &d_eperm, L.eperm))) return rc;
    // coefficients per element: the six off-diagonals of A_e (tetrahedra) or
    // the six entries of the 3 x 3 matrix S with A_e[a][b] = xi_a^T S xi_b
    // (hexahedra)
    const int ncoef = 6;
    if ((rc = dalloc(h, &coef64, (size_t)ncoef * E)) || (rc = dalloc(h, &h->d_vol, E)) ||
        (rc = dalloc(h, &bad, 1)) || (rc = dalloc(h, &h->d_Vi, N)) ||
        (rc = dalloc(h, &h->d_flag, 4)) || (rc = dalloc(h, &h->d_stage, N)))
        return rc;
    HIPCHK(h, launch_fill_i32(bad, 1, INT32_MAX, s));
    if (h->npe == 8)
        HIPCHK(h, launch_geometry_hex(E, h->d_xyz, h->d_conn, d_eperm, coef64, h->d_vol, bad, s));
    else
        HIPCHK(h, launch_geometry(E, h->d_xyz, h->d_conn, d_eperm, coef64, h->d_vol, bad, s));
    int32_t hbad = 0;
    HIPCHK(h, hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    dfree(h, bad);
    dfree(h, d_eperm);
    if (hbad != INT32_MAX) {
        release_device(h);
        return set_err(h, FEDFEM_E_DEGENERATE, "degenerate %s %d",
                       h->npe == 8 ? "hexahedron" : "tetrahedron", hbad);
    }
    clk.mark("geometry");
    HIPCHK(h, launch_lump(N, h->d_ec_off, h->d_ec, h->d_vol, h->npe, h->d_Vi, s));
    // fixed-point scales: the largest possible corner load maps below 2^58
    {
        unsigned long long* dbits = nullptr;
        if ((rc = dalloc(h, &dbits, 1))) return rc;
        HIPCHK(h, hipMemsetAsync(dbits, 0, sizeof(unsigned long long), s));
        if (h->npe == 8)
            HIPCHK(h, launch_coef_bound_hex(E, coef64, dbits, s));
        else
            HIPCHK(h, launch_coef_bound(E, coef64, dbits, s));
        unsigned long long bits = 0;
        std::vector<double> Vi(N);
        HIPCHK(h, hipMemcpyAsync(&bits, dbits, sizeof(bits), hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipMemcpyAsync(Vi.data(), h->d_Vi, sizeof(double) * N, hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        dfree(h, dbits);
        double amax;
        std::memcpy(&amax, &bits, sizeof(amax));
        double vmin = 1e300;
        for (int64_t i = 0; i < N; i++)
            if (!h->host_isdir[i]) vmin = std::min(vmin, Vi[i]);
        double kmin, kmax, rcmin, rcmax;
        window_bounds_h(h, &kmin, &kmax, &rcmin, &rcmax);
        // one load maps below 2^58, leaving 5 bits for the sum of up to 32
        // loads in a tile-node accumulator; a node with more corners in one
        // tile (an unstructured fan) lowers the scale until the whole sum
        // stays below 2^63
        const double fan = std::max(1.0, L.max_tile_valence / 32.0);
        // loads: k <= kmax, |T_b - T_a| <= 2e4 (both within the divergence limit)
        h->fx_scale = fixed_scale(kmax * amax * 2.0e4 * fan);
        // Lanczos: |x| <= 1 / sqrt(min free V_i) for a unit vector
        h->fx_scale_lz = fixed_scale(amax * 2.0 / std::sqrt(std::max(vmin, 1e-300)) * fan);
        h->a_max = amax;
    }
    // time-stepping arrays in the chosen precision
    const size_t rb = h->fp32c ? sizeof(float) : sizeof(double);
    auto dalloc_bytes = [&](void** p, size_t count) -> int {
        if (rb == 4) {
            float* f;
            int r = dalloc(h, &f, count);
            *p = f;
            return r;
        }
        double* g;
        int r = dalloc(h, &g, count);
        *p = g;
        return r;
    };
    if (h->fp32c) {
        if ((rc = dalloc_bytes(&d.coef, (size_t)ncoef * E))) return rc;
        HIPCHK(h, launch_cast_coef((int64_t)ncoef * E, coef64, static_cast<float*>(d.coef), s));
    } else {
        d.coef = coef64;
    }
    // nodal state: float2 (hi, lo) or double, 8 bytes per node either way
    if ((rc = dalloc_bytes(&d.u, N)) || (rc = dalloc_bytes(&d.q, N)) ||
        (rc = dalloc_bytes(&d.partial, d.P)))
        return rc;
    for (int b = 0; b < 2; b++) {
        double* tb = nullptr;
        if ((rc = dalloc(h, &tb, N))) return rc;
        d.T_[b] = tb;
    }
    HIPCHK(h, launch_node_init(N, h->d_Vi, h->d_isdir, h->d_dirT, h->T0, h->fp32c, d.u, d.T_[0],
                               d.T_[1], s));
    HIPCHK(h, launch_set_source(N, nullptr, nullptr, h->fp32c, d.q, s));
    // property tables: times, values and slopes in the working precision
    if (!h->tab_t[0].empty() || !h->tab_t[1].empty() || !h->tab_t[2].empty()) {
        std::vector<double> tb(9 * kMaxTab, 0.0);
        for (int p = 0; p < 3; p++) {
            const std::vector<double>& t = h->tab_t[p];
            const std::vector<double>& v = h->tab_v[p];
            for (size_t k = 0; k < t.size(); k++) {
                tb[p * 3 * kMaxTab + k] = t[k];
                tb[p * 3 * kMaxTab + kMaxTab + k] = v[k];
                if (k + 1 < t.size())
                    tb[p * 3 * kMaxTab + 2 * kMaxTab + k] = (v[k + 1] - v[k]) / (t[k + 1] - t[k]);
            }
        }
        if (h->fp32c) {
            std::vector<float> tf(tb.begin(), tb.end());
            float* dt_ = nullptr;
            if ((rc = upload(h, &dt_, tf))) return rc;
            h->d_tab = dt_;
        } else {
            double* dt_ = nullptr;
            if ((rc = upload(h, &dt_, tb))) return rc;
            h->d_tab = dt_;
        }
    }
    clk.mark("scales+init");
    // critical step (Eq 9): top eigenvalue of the geometry pencil on free
    // nodes, bounded over the property window
    if (h->timing_trial) {
        h->lam_geo = h->lam_ritz = 0.0;
        h->lz_iters = 0;
    } else if (h->n_dir < N) {
        rc = lanczos(h, coef64);
        if (rc) return rc;
    } else {
        h->lam_geo = h->lam_ritz = 0.0;
        h->lz_iters = 0;
    }
    clk.mark("lanczos");
    if (h->fp32c) dfree(h, coef64);
    double kmin, kmax, rcmin, rcmax;
    window_bounds_h(h, &kmin, &kmax, &rcmin, &rcmax);
    const double lam = h->lam_geo * kmax / rcmin + h->mat.w_b * h->mat.c_b / rcmin;
    h->dt_cr = lam > 0 ? 2.0 / lam : INFINITY;
    {
        std::vector<double> q;
        make_quadrature(q);
        if ((rc = upload(h, &h->d_qpts, q))) return rc;
    }
    HIPCHK(h, hipStreamSynchronize(s));
    if (h->timing_trial) {
        // kernels are timed only; any positive step keeps them well defined
        h->dt = 1e-9;
        h->dt_cr = INFINITY;
    } else if (h->dt_spec > 0) {
        if (!(h->dt_spec < h->dt_cr)) {
            h->dt = 0.0;
            h->precomputed = true;
            return set_err(h, FEDFEM_E_UNSTABLE, "dt %.9g is not below dt_cr %.9g", h->dt_spec,
                           h->dt_cr);
        }
        h->dt = h->dt_spec;
    } else {
        if (!std::isfinite(h->dt_cr)) {
            h->precomputed = true;
            return set_err(h, FEDFEM_E_INVALID, "no finite critical step: give dt > 0");
        }
        h->dt = -h->dt_spec * h->dt_cr;
    }
    h->t = 0.0;
    h->steps = 0;
    h->cur = 0;
    h->precomputed = true;
    clk.mark("finish");
    clk.print(E);
    // host copies of the big arrays are no longer needed
    std::vector<double>().swap(L.xyz);
    std::vector<int32_t>().swap(L.conn);
    std::vector<uint16_t>().swap(L.lconn);
    std::vector<uint8_t>().swap(L.lconn_pk);
    std::vector<int32_t>().swap(L.ec);
    return FEDFEM_OK;
}

int fedfem_precompute_many(fedfem_handle* const* handles, int32_t n, int32_t threads,
                           int32_t* rcs) {
    if (!handles || n < 0 || threads < 0) return FEDFEM_E_INVALID;
    {
        std::unordered_set<const fedfem_handle*> seen;
        for (int32_t j = 0; j < n; j++)
            if (!handles[j] || !seen.insert(handles[j]).second) return FEDFEM_E_INVALID;
    }
    std::vector<int> res(n, FEDFEM_OK);
    const int cores = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    int32_t nt = threads;
    if (nt == 0) {
        const char* env = std::getenv("FEDFEM_PRECOMPUTE_THREADS");
        nt = env ? std::atoi(env) : 0;
        if (nt <= 0) nt = cores;
    }
    nt = std::max<int32_t>(1, std::min(nt, n));
    // each worker's layout builds share the cores with the other workers'
    const int inner = std::max(1, cores / nt);
    run_workers(n, nt, inner, [&](int32_t j) { res[j] = fedfem_precompute(handles[j]); });
    int first = FEDFEM_OK;
    for (int32_t j = 0; j < n; j++) {
        if (rcs) rcs[j] = res[j];
        if (first == FEDFEM_OK && res[j] != FEDFEM_OK) first = res[j];
    }
    return first;
}

int fedfem_set_property_tables(fedfem_handle* h, int32_t n_k, const double* T_k,
                               const double* k, int32_t n_rho, const double* T_rho,
                               const double* rho, int32_t n_c, const double* T_c,
                               const double* c) {
    if (!h) return FEDFEM_E_INVALID;
    if (h->precomputed) return set_err(h, FEDFEM_E_STATE, "tables must be set before precompute");
    const int32_t n[3] = {n_k, n_rho, n_c};
    const double* ts[3] = {T_k, T_rho, T_c};
    const double* vs[3] = {k, rho, c};
    static const char* names[3] = {"k", "rho", "c"};
    for (int p = 0; p < 3; p++) {
        if (n[p] < 0 || n[p] > FEDFEM_MAX_TABLE || (n[p] > 0 && (!ts[p] || !vs[p])))
            return set_err(h, FEDFEM_E_INVALID, "table %s: bad point count or NULL", names[p]);
        if (!finite_all(ts[p], n[p]) || !finite_all(vs[p], n[p]))
            return set_err(h, FEDFEM_E_INVALID, "table %s: non-finite entry", names[p]);
        for (int32_t j = 0; j < n[p]; j++) {
            if (!(vs[p][j] > 0.0))
                return set_err(h, FEDFEM_E_INVALID, "table %s: values must be positive", names[p]);
            if (j > 0 && !(ts[p][j] > ts[p][j - 1]))
                return set_err(h, FEDFEM_E_INVALID, "table %s: temperatures must increase",
                               names[p]);
        }
    }
    for (int p = 0; p < 3; p++) {
        h->tab_t[p].assign(ts[p], ts[p] + n[p]);
        h->tab_v[p].assign(vs[p], vs[p] + n[p]);
    }
    return FEDFEM_OK;
}

int fedfem_set_schedule(fedfem_handle* h, int32_t n_patterns, const double* patterns,
                        const int32_t* n_points, const double* times, const double* amps) {
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (n_patterns < 0 || n_patterns > FEDFEM_MAX_PATTERNS)
        return set_err(h, FEDFEM_E_INVALID, "n_patterns must lie in [0, %d]", FEDFEM_MAX_PATTERNS);
    if (n_patterns > 0 && (!patterns || !n_points || !times || !amps))
        return set_err(h, FEDFEM_E_INVALID, "NULL schedule array");
    const int64_t N = h->N;
    std::vector<std::vector<double>> st(n_patterns), sa(n_patterns);
    int64_t off = 0;
    for (int p = 0; p < n_patterns; p++) {
        const int32_t m = n_points[p];
        if (m < 1 || m > (1 << 20)) return set_err(h, FEDFEM_E_INVALID, "pattern %d: bad point count", p);
        if (!finite_all(times + off, m) || !finite_all(amps + off, m))
            return set_err(h, FEDFEM_E_INVALID, "pattern %d: non-finite schedule", p);
        for (int32_t k = 1; k < m; k++)
            if (times[off + k] < times[off + k - 1])
                return set_err(h, FEDFEM_E_INVALID, "pattern %d: times decrease", p);
        st[p].assign(times + off, times + off + m);
        sa[p].assign(amps + off, amps + off + m);
        off += m;
        if (!finite_all(patterns + (int64_t)p * N, N))
            return set_err(h, FEDFEM_E_INVALID, "pattern %d: non-finite loads", p);
    }
    hipStream_t s = h->stream;
    drop_graphs(h);  // captured steps hold the pattern pointers
    dfree(h, h->d.pat);
    dfree(h, h->d.amp);
    h->d.pat = h->d.amp = nullptr;
    h->d.n_pat = 0;
    h->sched_t.clear();
    h->sched_a.clear();
    if (n_patterns == 0) return FEDFEM_OK;
    const size_t rb = h->fp32c ? sizeof(float) : sizeof(double);
    char* pat = nullptr;
    char* amp = nullptr;
    if ((rc = dalloc(h, &pat, rb * (size_t)n_patterns * N)) ||
        (rc = dalloc(h, &amp, rb * 512 * (size_t)n_patterns)))
        return rc;
    for (int p = 0; p < n_patterns; p++) {
        HIPCHK(h, hipMemcpyAsync(h->d_stage, patterns + (int64_t)p * N, sizeof(double) * N,
                                 hipMemcpyHostToDevice, s));
        HIPCHK(h, launch_set_source(N, h->d_stage, h->d_nperm, h->fp32c,
                                    pat + rb * (size_t)p * N, s));
    }
    HIPCHK(h, hipStreamSynchronize(s));
    h->d.pat = pat;
    h->d.amp = amp;
    h->d.n_pat = n_patterns;
    h->sched_t.swap(st);
    h->sched_a.swap(sa);
    return FEDFEM_OK;
}

int fedfem_set_dose(fedfem_handle* h, int32_t model, double a, double b) {
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (model == FEDFEM_DOSE_ARRHENIUS && !(a > 0 && std::isfinite(a) && b >= 0 && std::isfinite(b)))
        return set_err(h, FEDFEM_E_INVALID, "Arrhenius dose needs A > 0 and E_a >= 0, finite");
    if (model != FEDFEM_DOSE_OFF && model != FEDFEM_DOSE_CEM43 && model != FEDFEM_DOSE_ARRHENIUS)
        return set_err(h, FEDFEM_E_INVALID, "unknown dose model %d", model);
    drop_graphs(h);  // captured steps hold the dose pointer and constants
    DevLayout& d = h->d;
    if (model == FEDFEM_DOSE_OFF) {
        dfree(h, d.dose);
        d.dose = nullptr;
        d.dose_model = 0;
        return FEDFEM_OK;
    }
    if (!d.dose && (rc = dalloc(h, &d.dose, h->N))) return rc;
    HIPCHK(h, hipMemsetAsync(d.dose, 0, sizeof(double) * h->N, h->stream));
    d.dose_model = model;
    // CEM43: minutes per second; Arrhenius: A and E_a / R_gas
    d.dose_a = model == FEDFEM_DOSE_CEM43 ? 1.0 / 60.0 : a;
    d.dose_b = model == FEDFEM_DOSE_CEM43 ? 0.0 : b / 8.314462618;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return FEDFEM_OK;
}

int fedfem_read_dose(fedfem_handle* h, double* out) {
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (!out) return FEDFEM_E_INVALID;
    if (!h->d.dose) return set_err(h, FEDFEM_E_STATE, "no dose model is set");
    hipStream_t s = h->stream;
    HIPCHK(h, launch_get_source(h->N, h->d.dose, h->d_nperm, 0, h->d_stage, s));
    HIPCHK(h, hipMemcpyAsync(out, h->d_stage, sizeof(double) * h->N, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    return FEDFEM_OK;
}

// Surface-flux loads on faces of nv corners (3: triangles of a tetrahedral
// mesh, 4: quadrilaterals of a hexahedral one), gathered in ascending face
// order and returned in caller node order.
static int flux_loads_nv(fedfem_handle* h, int nv, int64_t n_faces, const int32_t* faces,
                         const double* flux, double* out) {
    int rc = check_handle(h, true);
    if (rc) return rc;
    const int64_t N = h->N;
    if (h->npe != (nv == 3 ? 4 : 8))
        return set_err(h, FEDFEM_E_INVALID, nv == 3
                           ? "triangle flux loads need a tetrahedral mesh"
                           : "quadrilateral flux loads need a hexahedral mesh");
    if (n_faces < 0 || n_faces > INT32_MAX / nv || !out || (n_faces > 0 && (!faces || !flux)))
        return set_err(h, FEDFEM_E_INVALID, "bad flux arguments");
    if (!finite_all(flux, n_faces)) return set_err(h, FEDFEM_E_INVALID, "non-finite flux");
    std::vector<int32_t> fi((size_t)nv * n_faces);
    for (int64_t f = 0; f < n_faces; f++) {
        for (int c = 0; c < nv; c++) {
            const int32_t v = faces[nv * f + c];
            if (v < 0 || v >= N) return set_err(h, FEDFEM_E_INVALID, "face %lld: bad node id", (long long)f);
            fi[nv * f + c] = h->L.ninv[v];
            for (int d = 0; d < c; d++)
                if (faces[nv * f + d] == v)
                    return set_err(h, FEDFEM_E_INVALID, "face %lld repeats a node", (long long)f);
        }
    }
    if (n_faces == 0) {
        std::fill(out, out + N, 0.0);
        return FEDFEM_OK;
    }
    // node -> face corners (nv f + c), ascending face order
    std::vector<int32_t> foff(N + 1, 0), fidx((size_t)nv * n_faces);
    for (size_t k = 0; k < fi.size(); k++) foff[fi[k] + 1]++;
    for (int64_t i = 0; i < N; i++) foff[i + 1] += foff[i];
    {
        std::vector<int32_t> fill(foff.begin(), foff.end() - 1);
        for (size_t k = 0; k < fi.size(); k++) fidx[fill[fi[k]]++] = (int32_t)k;
    }
    std::vector<double> fl(flux, flux + n_faces);
    hipStream_t s = h->stream;
    int32_t *d_faces = nullptr, *d_off = nullptr, *d_idx = nullptr;
    double *d_flux = nullptr, *d_slot = nullptr;
    if ((rc = upload(h, &d_faces, fi)) || (rc = upload(h, &d_off, foff)) ||
        (rc = upload(h, &d_idx, fidx)) || (rc = upload(h, &d_flux, fl)) ||
        (rc = dalloc(h, &d_slot, (size_t)nv * n_faces)))
        return rc;
    HIPCHK(h, hipStreamSynchronize(h->own_stream));  // uploads ran there
    HIPCHK(h, launch_face_loads(N, n_faces, nv, h->d_xyz, d_faces, d_flux, d_off, d_idx, d_slot,
                                h->d_stage, s));
    std::vector<double> tmp(N);
    HIPCHK(h, hipMemcpyAsync(tmp.data(), h->d_stage, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    for (int64_t i = 0; i < N; i++) out[h->L.nperm[i]] = tmp[i];
    for (void* p : {(void*)d_faces, (void*)d_off, (void*)d_idx, (void*)d_flux, (void*)d_slot})
        dfree(h, p);
    return FEDFEM_OK;
}

int fedfem_flux_loads(fedfem_handle* h, int64_t n_faces, const int32_t* faces, const double* flux,
                      double* out) {
    return flux_loads_nv(h, 3, n_faces, faces, flux, out);
}

int fedfem_flux_loads_quad(fedfem_handle* h, int64_t n_faces, const int32_t* faces,
                           const double* flux, double* out) {
    return flux_loads_nv(h, 4, n_faces, faces, flux, out);
}

int fedfem_set_source(fedfem_handle* h, const double* source) {
    int rc = check_handle(h, true);
    if (rc) return rc;
    hipStream_t s = h->stream;
    if (source) {
        if (!finite_all(source, h->N)) return set_err(h, FEDFEM_E_INVALID, "non-finite source");
        HIPCHK(h, hipMemcpyAsync(h->d_stage, source, sizeof(double) * h->N,
                                 hipMemcpyHostToDevice, s));
        HIPCHK(h, launch_set_source(h->N, h->d_stage, h->d_nperm, h->fp32c, h->d.q, s));
    } else {
        HIPCHK(h, launch_set_source(h->N, nullptr, nullptr, h->fp32c, h->d.q, s));
    }
    HIPCHK(h, hipStreamSynchronize(s));
    return FEDFEM_OK;
}

int fedfem_set_gaussian_sources(fedfem_handle* h, int32_t n_src, const double* params,
                                int32_t mode) {
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (n_src < 0 || n_src > 4096 || (n_src > 0 && !params) ||
        (mode != FEDFEM_SOURCE_NODAL && mode != FEDFEM_SOURCE_CONSISTENT))
        return set_err(h, FEDFEM_E_INVALID, "bad source arguments");
    for (int k = 0; k < n_src; k++) {
        if (!finite_all(params + 5 * k, 5) || !(params[5 * k + 3] > 0))
            return set_err(h, FEDFEM_E_INVALID, "bad Gaussian source %d", k);
    }
    hipStream_t s = h->stream;
    if (n_src == 0) return fedfem_set_source(h, nullptr);
    double* dsrc = nullptr;
    if ((rc = dalloc(h, &dsrc, 5 * (size_t)n_src))) return rc;
    HIPCHK(h, hipMemcpyAsync(dsrc, params, sizeof(double) * 5 * n_src, hipMemcpyHostToDevice, s));
    if (mode == FEDFEM_SOURCE_NODAL) {
        HIPCHK(h, launch_source_nodal(h->N, h->d_xyz, h->d_Vi, n_src, dsrc, h->d_stage, s));
    } else {
        double* slot = nullptr;
        if ((rc = dalloc(h, &slot, (size_t)h->npe * h->E))) {
            dfree(h, dsrc);
            return rc;
        }
        if (h->npe == 8)
            HIPCHK(h, launch_source_consistent_hex(h->N, h->E, h->d_xyz, h->d_conn, h->d_ec_off,
                                                   h->d_ec, n_src, dsrc, slot, h->d_stage, s));
        else
            HIPCHK(h, launch_source_consistent(h->N, h->E, h->d_xyz, h->d_conn, h->d_vol,
                                               h->d_ec_off, h->d_ec, n_src, dsrc, h->d_qpts,
                                               slot, h->d_stage, s));
        HIPCHK(h, hipStreamSynchronize(s));
        dfree(h, slot);
    }
    HIPCHK(h, launch_set_source(h->N, h->d_stage, nullptr, h->fp32c, h->d.q, s));
    HIPCHK(h, hipStreamSynchronize(s));
    dfree(h, dsrc);
    return FEDFEM_OK;
}

int fedfem_read_source(fedfem_handle* h, double* out) {
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (!out) return FEDFEM_E_INVALID;
    hipStream_t s = h->stream;
    HIPCHK(h, launch_get_source(h->N, h->d.q, h->d_nperm, h->fp32c, h->d_stage, s));
    HIPCHK(h, hipMemcpyAsync(out, h->d_stage, sizeof(double) * h->N, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    return FEDFEM_OK;
}

int fedfem_step(fedfem_handle* h, int64_t n_steps, const double* source) {
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (n_steps < 0) return set_err(h, FEDFEM_E_INVALID, "negative step count");
    if (!(h->dt > 0)) return set_err(h, FEDFEM_E_UNSTABLE, "no valid time step");
    if (source && (rc = fedfem_set_source(h, source))) return rc;
    if (n_steps == 0) return FEDFEM_OK;
    hipStream_t s = h->stream;
    HIPCHK(h, launch_fill_i32(h->d_flag, 1, 0, s));
    // amplitudes of the scheduled patterns at the start of every step of
    // this call, in the working precision; each chunk's rows are copied in
    // before its graph runs (stream order keeps the previous chunk's reads)
    const int P = h->d.n_pat;
    std::vector<float> amp32;
    std::vector<double> amp64;
    if (P > 0) {
        const size_t cnt = (size_t)n_steps * P;
        if (h->fp32c) amp32.resize(cnt); else amp64.resize(cnt);
        for (int64_t k = 0; k < n_steps; k++) {
            const double x = h->t + (double)k * h->dt;
            for (int p = 0; p < P; p++) {
                const double v = sched_amp(h->sched_t[p], h->sched_a[p], x);
                if (h->fp32c) amp32[k * P + p] = (float)v; else amp64[k * P + p] = v;
            }
        }
    }
    int64_t done = 0;
    while (done < n_steps) {
        const int64_t chunk = std::min<int64_t>(n_steps - done, 512);
        hipGraphExec_t ex;
        if ((rc = get_graph(h, chunk, h->cur, &ex))) return rc;
        if (P > 0) {
            const void* src = h->fp32c ? (const void*)(amp32.data() + done * P)
                                       : (const void*)(amp64.data() + done * P);
            const size_t rb = h->fp32c ? sizeof(float) : sizeof(double);
            HIPCHK(h, hipMemcpyAsync(h->d.amp, src, (size_t)chunk * P * rb,
                                     hipMemcpyHostToDevice, s));
        }
        HIPCHK(h, hipGraphLaunch(ex, s));
        if (chunk & 1) h->cur ^= 1;
        done += chunk;
    }
    int32_t flag = 0;
    HIPCHK(h, hipMemcpyAsync(&flag, h->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    h->steps += n_steps;
    h->t += (double)n_steps * h->dt;
    if (flag) return set_err(h, FEDFEM_E_DIVERGED, "temperature left [-1e4, 1e4] degC or NaN");
    return FEDFEM_OK;
}

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// This device's copy of `scratch`, looked up once per device (the handle's
// device is current: check_handle made it so).
int static_scratch(fedfem_handle* h, void** out) {
    if (h->device < 0 || h->device >= kMaxDevices)
        return set_err(h, FEDFEM_E_INVALID, "device %d beyond the static scratch table", h->device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    void*& p = g_scratch_ptr[h->device];
    if (!p) {
        void* q = nullptr;
        hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(h, e, "hipGetSymbolAddress(scratch)");
        p = q;
    }
    *out = p;
    return FEDFEM_OK;
}

}  // namespace

int fedfem_step_static(fedfem_handle* h, int64_t n_steps, const double* source) {
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (n_steps < 0) return set_err(h, FEDFEM_E_INVALID, "negative step count");
    if (!(h->dt > 0)) return set_err(h, FEDFEM_E_UNSTABLE, "no valid time step");
    if (h->d.n_pat > 0)
        return set_err(h, FEDFEM_E_STATE,
                       "fedfem_step_static does not apply source schedules (fedfem_step does)");
    const size_t need = (size_t)h->d.P * (h->fp32c ? sizeof(float) : sizeof(double));
    if (need > kStaticScratchBytes)
        return set_err(h, FEDFEM_E_TOO_LARGE,
                       "the tile partials need %zu bytes; the static scratch holds %zu", need,
                       kStaticScratchBytes);
    void* buf = nullptr;
    if ((rc = static_scratch(h, &buf))) return rc;
    if (source && (rc = fedfem_set_source(h, source))) return rc;
    if (n_steps == 0) return FEDFEM_OK;
    hipStream_t s = h->stream;
    // the step kernels of fedfem_step, launched one by one; every tile writes
    // all of its partials before the node pass reads them, so the scratch
    // needs no clearing between calls
    DevLayout d = h->d;
    d.partial = buf;
    d.dose_dt = h->dt;
    const bool td = h->mat.dk_dT != 0.0 || !h->tab_t[0].empty();
    HIPCHK(h, launch_fill_i32(h->d_flag, 1, 0, s));
    if (h->fp32c) {
        const Props<float> p = props_f(h);
        for (int64_t k = 0; k < n_steps; k++) {
            HIPCHK(h, launch_step_f32c(d, h->cur, p, td, h->d_flag, s, 0));
            h->cur ^= 1;
        }
    } else {
        const Props<double> p = props_d(h);
        for (int64_t k = 0; k < n_steps; k++) {
            HIPCHK(h, launch_step_f64(d, h->cur, p, td, h->d_flag, s, 0));
            h->cur ^= 1;
        }
    }
    int32_t flag = 0;
    HIPCHK(h, hipMemcpyAsync(&flag, h->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    h->steps += n_steps;
    h->t += (double)n_steps * h->dt;
    if (flag) return set_err(h, FEDFEM_E_DIVERGED, "temperature left [-1e4, 1e4] degC or NaN");
    return FEDFEM_OK;
}

int fedfem_prepare(fedfem_handle* h, int64_t n_steps) {
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (n_steps < 0) return set_err(h, FEDFEM_E_INVALID, "negative step count");
    if (!(h->dt > 0)) return set_err(h, FEDFEM_E_UNSTABLE, "no valid time step");
    for (int parity = 0; parity < 2; parity++) {
        int c = parity;
        int64_t left = n_steps;
        while (left > 0) {
            const int64_t chunk = std::min<int64_t>(left, 512);
            hipGraphExec_t ex;
            if ((rc = get_graph(h, chunk, c, &ex))) return rc;
            if (chunk & 1) c ^= 1;
            left -= chunk;
        }
    }
    return FEDFEM_OK;
}

int fedfem_time_kernels(fedfem_handle* h, int64_t n_steps, double* elem_ms, double* node_ms) {
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (n_steps <= 0 || n_steps > 10000 || !elem_ms || !node_ms)
        return set_err(h, FEDFEM_E_INVALID, "bad arguments");
    if (h->d.n_pat > 0)
        return set_err(h, FEDFEM_E_STATE, "kernel timing does not apply source schedules");
    if (!(h->dt > 0)) return set_err(h, FEDFEM_E_UNSTABLE, "no valid time step");
    hipStream_t s = h->stream;
    hipEvent_t ev[3];
    for (auto& e : ev) HIPCHK(h, hipEventCreate(&e));
    const bool td = h->mat.dk_dT != 0.0 || !h->tab_t[0].empty();
    // every launch starts from the current state: the element pass rewrites
    // the partials and the node pass the other ping-pong buffer (both
    // scratch between steps), and a dose goes to the staging buffer, so the
    // state, the clock and the accumulated dose stay as they were
    DevLayout d = h->d;
    d.dose_dt = h->dt;
    if (d.dose) d.dose = h->d_stage;
    const int c = h->cur;
    HIPCHK(h, hipEventRecord(ev[0], s));
    for (int64_t k = 0; k < n_steps; k++) {
        if (h->fp32c) HIPCHK(h, launch_elem_f32c(d, c, props_f(h), td, s));
        else HIPCHK(h, launch_elem_f64(d, c, props_d(h), td, s));
    }
    HIPCHK(h, hipEventRecord(ev[1], s));
    for (int64_t k = 0; k < n_steps; k++) {
        if (h->fp32c) HIPCHK(h, launch_node_f32c(d, c, props_f(h), h->d_flag, s));
        else HIPCHK(h, launch_node_f64(d, c, props_d(h), h->d_flag, s));
    }
    HIPCHK(h, hipEventRecord(ev[2], s));
    HIPCHK(h, hipStreamSynchronize(s));
    float a = 0, b = 0;
    HIPCHK(h, hipEventElapsedTime(&a, ev[0], ev[1]));
    HIPCHK(h, hipEventElapsedTime(&b, ev[1], ev[2]));
    for (auto& e : ev) (void)hipEventDestroy(e);
    *elem_ms = a / n_steps;
    *node_ms = b / n_steps;
    return FEDFEM_OK;
}

int fedfem_read_T(fedfem_handle* h, double* T_out) {
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (!T_out) return FEDFEM_E_INVALID;
    hipStream_t s = h->stream;
    HIPCHK(h, launch_read_T(h->N, h->d.T_[h->cur], h->d_nperm, h->fp32c, h->d_stage, s));
    HIPCHK(h, hipMemcpyAsync(T_out, h->d_stage, sizeof(double) * h->N, hipMemcpyDeviceToHost,
                             s));
    HIPCHK(h, hipStreamSynchronize(s));
    return FEDFEM_OK;
}

int fedfem_read_T_device(fedfem_handle* h, double* d_out) {
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (!d_out) return FEDFEM_E_INVALID;
    hipStream_t s = h->stream;
    HIPCHK(h, launch_read_T(h->N, h->d.T_[h->cur], h->d_nperm, h->fp32c, d_out, s));
    HIPCHK(h, hipStreamSynchronize(s));
    return FEDFEM_OK;
}

int fedfem_get_dt(const fedfem_handle* h, double* dt, double* dt_cr) {
    if (!h) return FEDFEM_E_INVALID;
    if (!h->precomputed) return FEDFEM_E_NOT_PRECOMPUTED;
    if (dt) *dt = h->dt;
    if (dt_cr) *dt_cr = h->dt_cr;
    return FEDFEM_OK;
}

int fedfem_get_time(const fedfem_handle* h, double* t, int64_t* steps) {
    if (!h) return FEDFEM_E_INVALID;
    if (t) *t = h->t;
    if (steps) *steps = h->steps;
    return FEDFEM_OK;
}

int fedfem_set_dt(fedfem_handle* h, double dt) {
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (!(dt > 0) || !(dt < h->dt_cr))
        return set_err(h, FEDFEM_E_UNSTABLE, "dt %.9g outside (0, %.9g)", dt, h->dt_cr);
    if (dt != h->dt) drop_graphs(h);
    h->dt = dt;
    return FEDFEM_OK;
}

int fedfem_set_stream(fedfem_handle* h, void* stream) {
    if (!h) return FEDFEM_E_INVALID;
    h->stream = stream ? static_cast<hipStream_t>(stream) : h->own_stream;
    return FEDFEM_OK;
}

int fedfem_state_bytes(const fedfem_handle* h, size_t* bytes) {
    if (!h || !bytes) return FEDFEM_E_INVALID;
    *bytes = (size_t)h->N * (h->fp32c ? 2 * sizeof(float) : sizeof(double));
    return FEDFEM_OK;
}

int fedfem_read_state(fedfem_handle* h, void* buf, double* t, int64_t* steps) {
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (!buf) return FEDFEM_E_INVALID;
    size_t bytes = 0;
    fedfem_state_bytes(h, &bytes);
    hipStream_t s = h->stream;
    HIPCHK(h, launch_state_io(h->N, h->d.T_[h->cur], h->d_nperm, h->fp32c, h->d_stage, 1, s));
    HIPCHK(h, hipMemcpyAsync(buf, h->d_stage, bytes, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    if (t) *t = h->t;
    if (steps) *steps = h->steps;
    return FEDFEM_OK;
}

int fedfem_write_state(fedfem_handle* h, const void* buf, double t, int64_t steps) {
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (!buf || !std::isfinite(t) || steps < 0) return FEDFEM_E_INVALID;
    size_t bytes = 0;
    fedfem_state_bytes(h, &bytes);
    hipStream_t s = h->stream;
    HIPCHK(h, hipMemcpyAsync(h->d_stage, buf, bytes, hipMemcpyHostToDevice, s));
    for (int b = 0; b < 2; b++)
        HIPCHK(h, launch_state_io(h->N, h->d.T_[b], h->d_nperm, h->fp32c, h->d_stage, 0, s));
    HIPCHK(h, hipStreamSynchronize(s));
    h->t = t;
    h->steps = steps;
    return FEDFEM_OK;
}

int fedfem_get_info(const fedfem_handle* h, fedfem_info* info) {
    if (!h || !info) return FEDFEM_E_INVALID;
    std::memset(info, 0, sizeof(*info));
    info->n_nodes = h->N;
    info->n_tets = h->E;
    info->n_dirichlet = (int64_t)h->dir_nodes.size();
    info->precision = h->mat.precision;
    info->reorder = h->opt.reorder;
    if (!h->precomputed) return FEDFEM_E_NOT_PRECOMPUTED;
    info->n_tiles = h->d.T;
    info->n_partials = h->d.P;
    info->max_tile_nodes = h->d.max_tile_nodes;
    info->tile_elems = h->d.tile_elems;
    info->threads = h->d.threads;
    info->device_bytes = h->dev_bytes;
    info->lambda_geometry = h->lam_geo;
    info->lanczos_iterations = h->lz_iters;
    info->max_tile_valence = h->L.max_tile_valence;
    info->fixed_point_shift = std::ilogb(h->fx_scale);
    info->n_single_tile_nodes = (int32_t)h->d.n_int;
    return FEDFEM_OK;
}

int fedfem_autotune(fedfem_handle* h, const char* cache_path, int32_t flags,
                    fedfem_options* chosen) {
    if (!h || (flags & ~FEDFEM_TUNE_BATCH)) return FEDFEM_E_INVALID;
    const bool batch = (flags & FEDFEM_TUNE_BATCH) != 0;
    if (h->precomputed) return set_err(h, FEDFEM_E_STATE, "autotune must run before precompute");
    int rc = check_handle(h, false);
    if (rc) return rc;
    char key[128];
    // tetrahedral keys keep their earlier form; hexahedral ones say so
    std::snprintf(key, sizeof(key), "f%d_prec%d_td%d_e%d%s", flags, h->mat.precision,
                  (h->mat.dk_dT != 0.0 || !h->tab_t[0].empty()) ? 1 : 0,
                  (int)std::lround(4.0 * std::log2((double)h->E)), h->npe == 8 ? "_hex" : "");
    fedfem_options best{};
    bool found = false;
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "r")) {
            char k[128];
            fedfem_options o{};
            while (std::fscanf(f, "%127s %d %d %d %d %d", k, &o.reorder, &o.tile_elems,
                               &o.threads, &o.max_tile_nodes, &o.xcd) == 6)
                if (std::strcmp(k, key) == 0) {
                    best = o;
                    found = true;
                }
            std::fclose(f);
        }
    }
    if (!found) {
        struct Build {
            int reorder, te;
        };
        const Build all[] = {{1, 1024}, {1, 2048}, {1, 4096}, {0, 1024}};
        // hexahedra touch about one node per element: smaller tiles
        const Build all_hex[] = {{1, 512}, {1, 1024}, {1, 2048}, {0, 512}};
        const Build for_batch[] = {{1, 1024}, {1, 2048}};
        const Build* builds = batch ? for_batch : (h->npe == 8 ? all_hex : all);
        const int n_builds = batch ? 2 : 4;
        double best_ms = 1e300;
        fedfem_mesh mesh{h->N, h->xyz.data(), h->E, h->tets.data()};
        fedfem_mesh_hex mesh_hex{h->N, h->xyz.data(), h->E, h->tets.data()};
        fedfem_bc bc{h->T0, (int64_t)h->dir_nodes.size(), h->dir_nodes.data(), h->dir_T.data(),
                     -0.5};
        for (int bi = 0; bi < n_builds; bi++) {
            const Build& bd = builds[bi];
            if (bd.te > 64 && (int64_t)bd.te > 8 * h->E) continue;  // tiny meshes
            fedfem_handle* t = nullptr;
            rc = h->npe == 8 ? fedfem_create_hex(&mesh_hex, &h->mat, &bc, &t)
                             : fedfem_create(&mesh, &h->mat, &bc, &t);
            if (rc) return set_err(h, rc, "autotune");
            t->timing_trial = true;
            fedfem_options o{};
            o.reorder = bd.reorder;
            o.tile_elems = bd.te;
            if ((rc = fedfem_set_options(t, &o)) || (rc = fedfem_precompute(t))) {
                fedfem_destroy(t);
                if (rc == FEDFEM_E_HIP) return hip_fail(h, hipErrorUnknown, "autotune trial");
                continue;  // e.g. the tile does not fit: skip the candidate
            }
            const int te = t->d.tile_elems;
            // 4, 2 and 1 elements per thread
            const int ths[3] = {std::max(64, std::min(1024, te / 4)),
                                std::max(64, std::min(1024, te / 2)),
                                std::max(64, std::min(1024, te))};
            for (int ti = 0; ti < (batch ? 1 : 3); ti++)
                for (int xcd = 0; xcd < (batch ? 1 : 2); xcd++) {
                    if (ti > 0 && ths[ti] == ths[ti - 1]) continue;  // capped at 1024
                    t->d.threads = ths[ti];
                    t->d.xcd = xcd;
                    if (elems_per_thread(t->d) > 4) continue;
                    double e1, n1;
                    if ((rc = fedfem_time_kernels(t, 3, &e1, &n1)) ||
                        (rc = fedfem_time_kernels(t, 10, &e1, &n1))) {
                        fedfem_destroy(t);
                        return set_err(h, rc, "autotune timing failed");
                    }
                    if (e1 + n1 < best_ms) {
                        best_ms = e1 + n1;
                        best = fedfem_options{};
                        best.reorder = bd.reorder;
                        best.tile_elems = te;
                        best.threads = ths[ti];
                        best.max_tile_nodes = t->opt.max_tile_nodes;
                        best.xcd = xcd;
                    }
                }
            fedfem_destroy(t);
        }
        if (best_ms == 1e300) return set_err(h, FEDFEM_E_INVALID, "no autotune candidate ran");
        if (cache_path) {
            if (FILE* f = std::fopen(cache_path, "a")) {
                std::fprintf(f, "%s %d %d %d %d %d\n", key, best.reorder, best.tile_elems,
                             best.threads, best.max_tile_nodes, best.xcd);
                std::fclose(f);
            }
        }
    }
    if ((rc = fedfem_set_options(h, &best))) return rc;
    if (chosen) *chosen = h->opt;
    return FEDFEM_OK;
}

int fedfem_destroy(fedfem_handle* h) {
    if (!h) return FEDFEM_OK;
    (void)hipSetDevice(h->device);
    if (h->own_stream) (void)hipStreamSynchronize(h->own_stream);
    release_device(h);
    if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    delete h;
    return FEDFEM_OK;
}

}  // extern "C"
