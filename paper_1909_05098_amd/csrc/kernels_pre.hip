// Pre-computation kernels for gfx950, double precision (Algorithm 1,
// pre-computation block; Eq 15-16; Sec 2.3.4-2.3.5), plus the small
// gather/scatter kernels that move nodal data between the caller's node
// order and the internal one.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace fedfem {

namespace {

constexpr int kBlock = 256;
// grids up to this many blocks finish their dot products in their last block
constexpr unsigned kFusedSumBlocks = 256;

inline unsigned blocks_for(int64_t n, int bs = kBlock) {
    return (unsigned)((n + bs - 1) / bs);
}

// Element geometry.  With edge vectors e_k = x_k - x_0 (the Jacobian's
// columns), the rows of J^-1 are (e2 x e3, e3 x e1, e1 x e2) / det J, which
// are the gradients of N_1..N_3; grad N_0 = -(sum of the others).  The
// element matrix A = V_tet B^T B (Eq 15-16) has zero row sums, so its six
// off-diagonal entries a_ab = V grad N_a . grad N_b define it.
__global__ void k_geometry(int64_t E, const double* __restrict__ xyz,
                           const int32_t* __restrict__ conn, const int32_t* __restrict__ eperm,
                           double* __restrict__ coef, double* __restrict__ vol,
                           int32_t* __restrict__ bad) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double p[4][3];
    for (int c = 0; c < 4; c++) {
        const int64_t n = conn[4 * e + c];
        p[c][0] = xyz[3 * n];
        p[c][1] = xyz[3 * n + 1];
        p[c][2] = xyz[3 * n + 2];
    }
    double ed[3][3];
    for (int k = 0; k < 3; k++)
        for (int a = 0; a < 3; a++) ed[k][a] = p[k + 1][a] - p[0][a];
    auto cross = [](const double* u, const double* v, double* w) {
        w[0] = u[1] * v[2] - u[2] * v[1];
        w[1] = u[2] * v[0] - u[0] * v[2];
        w[2] = u[0] * v[1] - u[1] * v[0];
    };
    double g[4][3];
    cross(ed[1], ed[2], g[1]);
    cross(ed[2], ed[0], g[2]);
    cross(ed[0], ed[1], g[3]);
    const double det = ed[0][0] * g[1][0] + ed[0][1] * g[1][1] + ed[0][2] * g[1][2];
    double l2max = 0.0;
    for (int a = 0; a < 4; a++)
        for (int b = a + 1; b < 4; b++) {
            const double dx = p[a][0] - p[b][0], dy = p[a][1] - p[b][1],
                         dz = p[a][2] - p[b][2];
            l2max = fmax(l2max, dx * dx + dy * dy + dz * dz);
        }
    const double lmax = sqrt(l2max);
    if (!(fabs(det) > 1e-12 * lmax * lmax * lmax)) {
        atomicMin(bad, eperm[e]);  // smallest caller element id
        for (int k = 0; k < 6; k++) coef[k * E + e] = 0.0;
        vol[e] = 0.0;
        return;
    }
    const double inv = 1.0 / det;
    for (int k = 1; k < 4; k++)
        for (int a = 0; a < 3; a++) g[k][a] *= inv;
    for (int a = 0; a < 3; a++) g[0][a] = -(g[1][a] + g[2][a] + g[3][a]);
    const double V = fabs(det) / 6.0;
    vol[e] = V;
    const int pa[6] = {0, 0, 0, 1, 1, 2};
    const int pb[6] = {1, 2, 3, 2, 3, 3};
    for (int k = 0; k < 6; k++) {
        const double* u = g[pa[k]];
        const double* v = g[pb[k]];
        coef[k * E + e] = V * (u[0] * v[0] + u[1] * v[1] + u[2] * v[2]);
    }
}

// Geometry of the eight-node hexahedron with one integration point at its
// centre (Eq 14, 16).  Corner a sits at natural coordinates xi_a in
// {-1, 1}^3 (bottom face counter-clockwise, then the top face), so at the
// centre dN_a/dxi = xi_a / 8 and M[j][i] = dx_i/dxi_j = sum_a xi_a,j x_a,i / 8.
// Then grad_x N_a = M^-1 grad_xi N_a and V_e = 8 |det M|.  Every corner's
// gradient is the same 3 x 3 map applied to its xi_a, so A_e = V_e B^T B
// factors as A_e[a][b] = xi_a^T S xi_b with S = (V_e / 64) M^-T M^-1 (3 x 3,
// symmetric).  The element is stored as the six entries of S, at
// coef[k E + e] in the order S00, S11, S22, S01, S02, S12.
__constant__ double kHexNat[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                     {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

__global__ void k_geometry_hex(int64_t E, const double* __restrict__ xyz,
                               const int32_t* __restrict__ conn, const int32_t* __restrict__ eperm,
                               double* __restrict__ coef, double* __restrict__ vol,
                               int32_t* __restrict__ bad) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double p[8][3];
    for (int c = 0; c < 8; c++) {
        const int64_t n = conn[8 * e + c];
        p[c][0] = xyz[3 * n];
        p[c][1] = xyz[3 * n + 1];
        p[c][2] = xyz[3 * n + 2];
    }
    double M[3][3];
    for (int j = 0; j < 3; j++)
        for (int i = 0; i < 3; i++) {
            double sum = 0.0;
            for (int a = 0; a < 8; a++) sum += kHexNat[a][j] * p[a][i];
            M[j][i] = 0.125 * sum;
        }
    // cofactors: Minv = adj(M) / det
    double C[3][3];
    C[0][0] = M[1][1] * M[2][2] - M[1][2] * M[2][1];
    C[0][1] = M[1][2] * M[2][0] - M[1][0] * M[2][2];
    C[0][2] = M[1][0] * M[2][1] - M[1][1] * M[2][0];
    C[1][0] = M[0][2] * M[2][1] - M[0][1] * M[2][2];
    C[1][1] = M[0][0] * M[2][2] - M[0][2] * M[2][0];
    C[1][2] = M[0][1] * M[2][0] - M[0][0] * M[2][1];
    C[2][0] = M[0][1] * M[1][2] - M[0][2] * M[1][1];
    C[2][1] = M[0][2] * M[1][0] - M[0][0] * M[1][2];
    C[2][2] = M[0][0] * M[1][1] - M[0][1] * M[1][0];
    const double det = M[0][0] * C[0][0] + M[0][1] * C[0][1] + M[0][2] * C[0][2];
    double l2max = 0.0;
    for (int a = 0; a < 8; a++)
        for (int b = a + 1; b < 8; b++) {
            const double dx = p[a][0] - p[b][0], dy = p[a][1] - p[b][1],
                         dz = p[a][2] - p[b][2];
            l2max = fmax(l2max, dx * dx + dy * dy + dz * dz);
        }
    const double lmax = sqrt(l2max);
    if (!(fabs(det) > 1e-12 * lmax * lmax * lmax)) {
        atomicMin(bad, eperm[e]);  // smallest caller element id
        for (int k = 0; k < 6; k++) coef[k * E + e] = 0.0;
        vol[e] = 0.0;
        return;
    }
    const double V = 8.0 * fabs(det);
    vol[e] = V;
    // grad N_a = Minv xi_a / 8 with Minv[i][j] = C[j][i] / det, so
    // A_ab = V grad N_a . grad N_b = xi_a^T S xi_b with the symmetric
    //   S_jk = V / (64 det^2) sum_i C[j][i] C[k][i] = sum_i C[j][i] C[k][i] / (8 |det|)
    const double f = 1.0 / V;
    auto cc = [&](int j, int k) {
        return f * (C[j][0] * C[k][0] + C[j][1] * C[k][1] + C[j][2] * C[k][2]);
    };
    coef[0 * E + e] = cc(0, 0);
    coef[1 * E + e] = cc(1, 1);
    coef[2 * E + e] = cc(2, 2);
    coef[3 * E + e] = cc(0, 1);
    coef[4 * E + e] = cc(0, 2);
    coef[5 * E + e] = cc(1, 2);
}

// Lumped nodal volume: each element gives an equal share of its volume to
// each of its npe nodes (Sec 2.3.4), summed in ascending element order.
__global__ void k_lump(int64_t N, const int32_t* __restrict__ off,
                       const int32_t* __restrict__ ec, const double* __restrict__ vol, int npe,
                       double* __restrict__ Vi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double share = 1.0 / npe;  // 1/4 or 1/8: exact
    double s = 0.0;
    for (int k = off[i]; k < off[i + 1]; k++) s += share * vol[ec[k] / npe];
    Vi[i] = s;
}

__device__ inline double gauss_at(const double* x, const double* g) {
    const double dx = x[0] - g[0], dy = x[1] - g[1], dz = x[2] - g[2];
    return g[4] * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * g[3] * g[3]));
}

__global__ void k_source_nodal(int64_t N, const double* __restrict__ xyz,
                               const double* __restrict__ Vi, int n_src,
                               const double* __restrict__ src, double* __restrict__ q) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double s = 0.0;
    for (int k = 0; k < n_src; k++) s += gauss_at(xyz + 3 * i, src + 5 * k);
    q[i] = s * Vi[i];
}

// Consistent nodal heat flow: per element, the 256-point composite rule in
// barycentric coordinates of the element with its corners taken in
// lexicographic coordinate order; N_c at a point is its c-th barycentric
// coordinate.  Elements whose bounding sphere is beyond 8 sigma of a source
// get nothing from it.
// Consistent nodal source on hexahedra: Q_a = integral over the element of
// the Gaussian densities times N_a, by the 4 x 4 x 4 tensor Gauss-Legendre
// rule on the trilinear map (weight |det J(xi)| at each point).  Nodes and
// weights of the 4-point rule are the published ones (Abramowitz and
// Stegun, Table 25.4).  An element is skipped for a source when it lies
// wholly beyond 8 sigma, as for tetrahedra; slot[8 e + a] receives corner a.
__constant__ double kGL4x[4] = {-0.8611363115940525752, -0.3399810435848562648,
                                0.3399810435848562648, 0.8611363115940525752};
__constant__ double kGL4w[4] = {0.3478548451374538574, 0.6521451548625461426,
                                0.6521451548625461426, 0.3478548451374538574};

__global__ void k_source_elem_hex(int64_t E, const double* __restrict__ xyz,
                                  const int32_t* __restrict__ conn, int n_src,
                                  const double* __restrict__ src, double* __restrict__ slot) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double p[8][3];
    double cen[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < 8; c++) {
        const int64_t n = conn[8 * e + c];
        for (int a = 0; a < 3; a++) {
            p[c][a] = xyz[3 * n + a];
            cen[a] += 0.125 * p[c][a];
        }
    }
    double r2 = 0.0;
    for (int c = 0; c < 8; c++) {
        const double dx = p[c][0] - cen[0], dy = p[c][1] - cen[1], dz = p[c][2] - cen[2];
        r2 = fmax(r2, dx * dx + dy * dy + dz * dz);
    }
    const double rad = sqrt(r2);
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < n_src; k++) {
        const double* g = src + 5 * k;
        const double dx = cen[0] - g[0], dy = cen[1] - g[1], dz = cen[2] - g[2];
        if (sqrt(dx * dx + dy * dy + dz * dz) - rad > 8.0 * g[3]) continue;
        for (int qi = 0; qi < 64; qi++) {
            const double q[3] = {kGL4x[qi & 3], kGL4x[(qi >> 2) & 3], kGL4x[qi >> 4]};
            const double wq = kGL4w[qi & 3] * kGL4w[(qi >> 2) & 3] * kGL4w[qi >> 4];
            double N[8], x[3] = {0.0, 0.0, 0.0}, J[3][3] = {};
            for (int a = 0; a < 8; a++) {
                const double f0 = 1.0 + kHexNat[a][0] * q[0], f1 = 1.0 + kHexNat[a][1] * q[1],
                             f2 = 1.0 + kHexNat[a][2] * q[2];
                N[a] = 0.125 * f0 * f1 * f2;
                const double d[3] = {0.125 * kHexNat[a][0] * f1 * f2,
                                     0.125 * kHexNat[a][1] * f0 * f2,
                                     0.125 * kHexNat[a][2] * f0 * f1};
                for (int i = 0; i < 3; i++) {
                    x[i] += N[a] * p[a][i];
                    for (int j = 0; j < 3; j++) J[j][i] += d[j] * p[a][i];
                }
            }
            const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                               J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                               J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
            const double f = wq * fabs(det) * gauss_at(x, g);
            for (int a = 0; a < 8; a++) acc[a] += f * N[a];
        }
    }
    for (int a = 0; a < 8; a++) slot[8 * e + a] = acc[a];
}

__global__ void k_source_elem(int64_t E, const double* __restrict__ xyz,
                              const int32_t* __restrict__ conn,
                              const double* __restrict__ vol, int n_src,
                              const double* __restrict__ src,
                              const double* __restrict__ qpts, double* __restrict__ slot) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double p[4][3];
    int ord[4];
    for (int c = 0; c < 4; c++) {
        const int64_t n = conn[4 * e + c];
        p[c][0] = xyz[3 * n];
        p[c][1] = xyz[3 * n + 1];
        p[c][2] = xyz[3 * n + 2];
        ord[c] = c;
    }
    // rank corners by (x, y, z)
    for (int i = 0; i < 4; i++)
        for (int j = i + 1; j < 4; j++) {
            const double* u = p[ord[i]];
            const double* v = p[ord[j]];
            const bool later = u[0] > v[0] || (u[0] == v[0] && (u[1] > v[1] ||
                                                (u[1] == v[1] && u[2] > v[2])));
            if (later) {
                const int t = ord[i];
                ord[i] = ord[j];
                ord[j] = t;
            }
        }
    double cen[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < 4; c++)
        for (int a = 0; a < 3; a++) cen[a] += 0.25 * p[c][a];
    double r2 = 0.0;
    for (int c = 0; c < 4; c++) {
        const double dx = p[c][0] - cen[0], dy = p[c][1] - cen[1], dz = p[c][2] - cen[2];
        r2 = fmax(r2, dx * dx + dy * dy + dz * dz);
    }
    const double rad = sqrt(r2);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < n_src; k++) {
        const double* g = src + 5 * k;
        const double dx = cen[0] - g[0], dy = cen[1] - g[1], dz = cen[2] - g[2];
        if (sqrt(dx * dx + dy * dy + dz * dz) - rad > 8.0 * g[3]) continue;
        for (int qi = 0; qi < 256; qi++) {
            const double* b = qpts + 4 * qi;
            double x[3];
            for (int a = 0; a < 3; a++)
                x[a] = b[0] * p[ord[0]][a] + b[1] * p[ord[1]][a] + b[2] * p[ord[2]][a] +
                       b[3] * p[ord[3]][a];
            const double f = gauss_at(x, g);
            for (int r = 0; r < 4; r++) acc[r] += f * b[r];
        }
    }
    for (int r = 0; r < 4; r++) slot[4 * e + ord[r]] = acc[r] * vol[e] / 256.0;
}

__global__ void k_gather_slots(int64_t N, const int32_t* __restrict__ off,
                               const int32_t* __restrict__ ec,
                               const double* __restrict__ slot, double* __restrict__ q) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double s = 0.0;
    for (int k = off[i]; k < off[i + 1]; k++) s += slot[ec[k]];
    q[i] = s;
}

// Nodal loads of a surface heat flux (Eq 4): triangle f with flux q_f [W/m^2]
// gives each of its corners q_f |f| / 3 (the integral of q_f N_i over the
// face for linear N_i); slot[3 f + c] holds corner c's share.
__global__ void k_face_loads(int64_t F, const double* __restrict__ xyz,
                             const int32_t* __restrict__ faces, const double* __restrict__ flux,
                             double* __restrict__ slot) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const double* a = xyz + 3 * (int64_t)faces[3 * f];
    const double* b = xyz + 3 * (int64_t)faces[3 * f + 1];
    const double* c = xyz + 3 * (int64_t)faces[3 * f + 2];
    const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    const double n[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2],
                         u[0] * v[1] - u[1] * v[0]};
    const double area = 0.5 * sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const double share = flux[f] * area / 3.0;
    for (int k = 0; k < 3; k++) slot[3 * f + k] = share;
}

// The same for bilinear quadrilaterals (corners in order around the face):
// corner a receives the integral of the flux times its bilinear shape
// function, by the 2 x 2 Gauss-Legendre rule (nodes +-1/sqrt(3), weights 1)
// with the area element |x_s x x_t| of the bilinear map.
__global__ void k_face_loads_quad(int64_t F, const double* __restrict__ xyz,
                                  const int32_t* __restrict__ faces,
                                  const double* __restrict__ flux, double* __restrict__ slot) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const double sa[4] = {-1.0, 1.0, 1.0, -1.0}, ta[4] = {-1.0, -1.0, 1.0, 1.0};
    double p[4][3];
    for (int c = 0; c < 4; c++)
        for (int i = 0; i < 3; i++) p[c][i] = xyz[3 * (int64_t)faces[4 * f + c] + i];
    const double g = 1.0 / sqrt(3.0);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int qi = 0; qi < 4; qi++) {
        const double s = (qi & 1) ? g : -g, t = (qi & 2) ? g : -g;
        double xs[3] = {0.0, 0.0, 0.0}, xt[3] = {0.0, 0.0, 0.0}, N[4];
        for (int c = 0; c < 4; c++) {
            N[c] = 0.25 * (1.0 + sa[c] * s) * (1.0 + ta[c] * t);
            const double ds = 0.25 * sa[c] * (1.0 + ta[c] * t);
            const double dt = 0.25 * ta[c] * (1.0 + sa[c] * s);
            for (int i = 0; i < 3; i++) {
                xs[i] += ds * p[c][i];
                xt[i] += dt * p[c][i];
            }
        }
        const double n0 = xs[1] * xt[2] - xs[2] * xt[1], n1 = xs[2] * xt[0] - xs[0] * xt[2],
                     n2 = xs[0] * xt[1] - xs[1] * xt[0];
        const double dA = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
        for (int c = 0; c < 4; c++) acc[c] += flux[f] * dA * N[c];
    }
    for (int c = 0; c < 4; c++) slot[4 * f + c] = acc[c];
}

// Largest row sum of |A_e| off the diagonal over all elements (for the
// fixed-point scale of the element loads).  Positive doubles order like
// their bit patterns, so an integer max over the bits is exact.
__global__ void k_coef_bound(int64_t E, const double* __restrict__ coef,
                             unsigned long long* __restrict__ out) {
    __shared__ double sh[kBlock];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double r = 0.0;
    if (e < E) {
        double a[6];
        for (int k = 0; k < 6; k++) a[k] = fabs(coef[k * E + e]);
        r = fmax(fmax(a[0] + a[1] + a[2], a[0] + a[3] + a[4]),
                 fmax(a[1] + a[3] + a[5], a[2] + a[4] + a[5]));
    }
    sh[threadIdx.x] = r;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(sh[0]));
}

// The same bound for hexahedra, with A_e[a][b] = xi_a^T S xi_b.
__global__ void k_coef_bound_hex(int64_t E, const double* __restrict__ coef,
                                 unsigned long long* __restrict__ out) {
    __shared__ double sh[kBlock];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double r = 0.0;
    if (e < E) {
        const double c[6] = {coef[e], coef[E + e], coef[2 * E + e],
                             coef[3 * E + e], coef[4 * E + e], coef[5 * E + e]};
        const double S[3][3] = {{c[0], c[3], c[4]}, {c[3], c[1], c[5]}, {c[4], c[5], c[2]}};
        for (int a = 0; a < 8; a++) {
            double Sx[3];
            for (int i = 0; i < 3; i++)
                Sx[i] = S[i][0] * kHexNat[a][0] + S[i][1] * kHexNat[a][1] + S[i][2] * kHexNat[a][2];
            double row = 0.0;
            for (int b = 0; b < 8; b++)
                if (b != a)
                    row += fabs(Sx[0] * kHexNat[b][0] + Sx[1] * kHexNat[b][1] +
                                Sx[2] * kHexNat[b][2]);
            r = fmax(r, row);
        }
    }
    sh[threadIdx.x] = r;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(sh[0]));
}

__global__ void k_cast(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

__global__ void k_node_init(int64_t N, const double* __restrict__ Vi,
                            const int32_t* __restrict__ is_dir, const double* __restrict__ dirT,
                            double T0, int fp32c, void* __restrict__ u, void* __restrict__ T0buf,
                            void* __restrict__ T1buf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const bool d = is_dir[i] != 0;
    const double T = d ? dirT[i] : T0;
    if (fp32c) {
        static_cast<float*>(u)[i] = d ? -1.0f : (float)(1.0 / Vi[i]);
        const float hi = (float)T;
        const float2 v = make_float2(hi, (float)(T - (double)hi));
        static_cast<float2*>(T0buf)[i] = v;
        static_cast<float2*>(T1buf)[i] = v;
    } else {
        static_cast<double*>(u)[i] = d ? -1.0 : 1.0 / Vi[i];
        static_cast<double*>(T0buf)[i] = T;
        static_cast<double*>(T1buf)[i] = T;
    }
}

template <typename Real>
__global__ void k_set_source(int64_t N, const double* __restrict__ src,
                             const int32_t* __restrict__ nperm, Real* __restrict__ q) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    q[i] = (Real)(src ? src[nperm ? nperm[i] : i] : 0.0);
}

template <typename Real>
__global__ void k_get_source(int64_t N, const Real* __restrict__ q,
                             const int32_t* __restrict__ nperm, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    out[nperm[i]] = (double)q[i];
}

__global__ void k_read_T(int64_t N, const void* __restrict__ T, const int32_t* __restrict__ nperm,
                         int fp32c, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (fp32c) {
        const float2 v = static_cast<const float2*>(T)[i];
        out[nperm[i]] = (double)v.x + (double)v.y;
    } else {
        out[nperm[i]] = static_cast<const double*>(T)[i];
    }
}

__global__ void k_state_io(int64_t N, void* __restrict__ T, const int32_t* __restrict__ nperm,
                           int fp32c, void* __restrict__ buf, int to_buf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t o = nperm[i];
    if (fp32c) {
        float2* t = static_cast<float2*>(T);
        float* b = static_cast<float*>(buf);
        if (to_buf) {
            const float2 v = t[i];
            b[o] = v.x;
            b[N + o] = v.y;
        } else {
            t[i] = make_float2(b[o], b[N + o]);
        }
    } else {
        double* t = static_cast<double*>(T);
        double* b = static_cast<double*>(buf);
        if (to_buf)
            b[o] = t[i];
        else
            t[i] = b[o];
    }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---- Lanczos on B = S K S, S = diag(1/sqrt(V_i)) on free nodes, 0 else ----

__device__ inline double block_sum(double v, double* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    return sh[0];
}

// Block partial s of a grid-wide sum.  With a counter (small grids) the
// last block to finish adds all partials in a fixed order into out[0] (or
// its square root, op 1) and returns the counter to zero for the next
// launch; without one (large grids, where every block's atomic on the one
// counter would queue at L2) the partials are left for k_reduce.
__device__ inline void grid_sum(double s, double* __restrict__ bsum, int* __restrict__ counter,
                                double* __restrict__ out, int op, double* sh) {
    __shared__ int last;
    if (!counter) {
        if (threadIdx.x == 0) bsum[blockIdx.x] = s;
        return;
    }
    if (threadIdx.x == 0) {
        bsum[blockIdx.x] = s;
        __threadfence();
        last = atomicAdd(counter, 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double t = 0.0;
    for (int k = threadIdx.x; k < (int)gridDim.x; k += blockDim.x)
        t += __hip_atomic_load(&bsum[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    t = block_sum(t, sh);
    if (threadIdx.x == 0) {
        out[0] = op ? sqrt(t) : t;
        atomicExch(counter, 0);
    }
}

__device__ inline double hash_unit(uint64_t x) {
    // splitmix64 finaliser, mapped to [-1, 1)
    x += 0x9e3779b97f4a7c15ULL;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
    x ^= x >> 31;
    return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void k_lz_init(int64_t N, const double* __restrict__ Vi,
                          const int32_t* __restrict__ is_dir, double* __restrict__ sc,
                          double* __restrict__ v, double* __restrict__ bsum) {
    __shared__ double sh[kBlock];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double vv = 0.0;
    if (i < N) {
        const bool d = is_dir[i] != 0;
        sc[i] = d ? 0.0 : 1.0 / sqrt(Vi[i]);
        vv = d ? 0.0 : hash_unit((uint64_t)i);
        v[i] = vv;
    }
    const double s = block_sum(vv * vv, sh);
    if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

// out[0] = sum of in[0..n) (op 0), or sqrt of it (op 1); fixed order.
__global__ void k_reduce(const double* __restrict__ in, int64_t n, double* __restrict__ out,
                         int op) {
    __shared__ double sh[1024];
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) s += in[k];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[0] = op ? sqrt(s) : s;
}

__global__ void k_lz_scale(int64_t N, const double* __restrict__ norm, const double* __restrict__ sc,
                           double* __restrict__ v, double* __restrict__ vprev,
                           double* __restrict__ xs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double nv = norm[0];
    const double x = nv > 0.0 ? v[i] / nv : 0.0;
    v[i] = x;
    vprev[i] = 0.0;
    xs[i] = sc[i] * x;
}

__global__ void k_lz_w(int64_t N, const int32_t* __restrict__ part_off,
                       const int32_t* __restrict__ pidx, const double* __restrict__ partial,
                       const double* __restrict__ sc, const double* __restrict__ v,
                       const double* __restrict__ vprev, const double* __restrict__ beta_j,
                       double* __restrict__ w, double* __restrict__ bsum, int* __restrict__ counter,
                       double* __restrict__ alpha_j) {
    __shared__ double sh[kBlock];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double prod = 0.0;
    if (i < N) {
        double F = 0.0;
        for (int k = part_off[i]; k < part_off[i + 1]; k++) F += partial[pidx[k]];
        const double wi = sc[i] * F - beta_j[0] * vprev[i];
        w[i] = wi;
        prod = v[i] * wi;
    }
    grid_sum(block_sum(prod, sh), bsum, counter, alpha_j, 0, sh);
}

__global__ void k_lz_orth(int64_t N, const double* __restrict__ alpha_j,
                          const double* __restrict__ v, double* __restrict__ w,
                          double* __restrict__ bsum, int* __restrict__ counter,
                          double* __restrict__ beta_next) {
    __shared__ double sh[kBlock];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double sq = 0.0;
    if (i < N) {
        const double wi = w[i] - alpha_j[0] * v[i];
        w[i] = wi;
        sq = wi * wi;
    }
    grid_sum(block_sum(sq, sh), bsum, counter, beta_next, 1, sh);
}

__global__ void k_lz_next(int64_t N, const double* __restrict__ beta_next,
                          const double* __restrict__ sc, const double* __restrict__ w,
                          double* __restrict__ v, double* __restrict__ vprev,
                          double* __restrict__ xs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double b = beta_next[0];
    const double x = b > 1e-300 ? w[i] / b : 0.0;
    vprev[i] = v[i];
    v[i] = x;
    xs[i] = sc[i] * x;
}

}  // namespace

hipError_t launch_geometry(int64_t E, const double* xyz, const int32_t* conn,
                           const int32_t* eperm, double* coef64, double* vol, int32_t* bad,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_geometry, dim3(blocks_for(E)), dim3(kBlock), 0, s, E, xyz, conn, eperm,
                       coef64, vol, bad);
    return hipGetLastError();
}

hipError_t launch_geometry_hex(int64_t E, const double* xyz, const int32_t* conn,
                               const int32_t* eperm, double* coef64, double* vol, int32_t* bad,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_geometry_hex, dim3(blocks_for(E)), dim3(kBlock), 0, s, E, xyz, conn,
                       eperm, coef64, vol, bad);
    return hipGetLastError();
}

hipError_t launch_lump(int64_t N, const int32_t* ec_off, const int32_t* ec, const double* vol,
                       int npe, double* Vi, hipStream_t s) {
    hipLaunchKernelGGL(k_lump, dim3(blocks_for(N)), dim3(kBlock), 0, s, N, ec_off, ec, vol, npe,
                       Vi);
    return hipGetLastError();
}

hipError_t launch_source_nodal(int64_t N, const double* xyz, const double* Vi, int n_src,
                               const double* src, double* q64, hipStream_t s) {
    hipLaunchKernelGGL(k_source_nodal, dim3(blocks_for(N)), dim3(kBlock), 0, s, N, xyz, Vi,
                       n_src, src, q64);
    return hipGetLastError();
}

hipError_t launch_source_consistent(int64_t N, int64_t E, const double* xyz,
                                    const int32_t* conn, const double* vol,
                                    const int32_t* ec_off, const int32_t* ec, int n_src,
                                    const double* src, const double* qpts, double* slot64,
                                    double* q64, hipStream_t s) {
    hipLaunchKernelGGL(k_source_elem, dim3(blocks_for(E, 128)), dim3(128), 0, s, E, xyz, conn,
                       vol, n_src, src, qpts, slot64);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather_slots, dim3(blocks_for(N)), dim3(kBlock), 0, s, N, ec_off, ec,
                       slot64, q64);
    return hipGetLastError();
}

hipError_t launch_source_consistent_hex(int64_t N, int64_t E, const double* xyz,
                                        const int32_t* conn, const int32_t* ec_off,
                                        const int32_t* ec, int n_src, const double* src,
                                        double* slot64, double* q64, hipStream_t s) {
    hipLaunchKernelGGL(k_source_elem_hex, dim3(blocks_for(E, 128)), dim3(128), 0, s, E, xyz, conn,
                       n_src, src, slot64);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather_slots, dim3(blocks_for(N)), dim3(kBlock), 0, s, N, ec_off, ec,
                       slot64, q64);
    return hipGetLastError();
}

hipError_t launch_face_loads(int64_t N, int64_t F, int nv, const double* xyz,
                             const int32_t* faces, const double* flux, const int32_t* off,
                             const int32_t* idx, double* slot, double* out, hipStream_t s) {
    if (nv == 4)
        hipLaunchKernelGGL(k_face_loads_quad, dim3(blocks_for(F)), dim3(kBlock), 0, s, F, xyz,
                           faces, flux, slot);
    else
        hipLaunchKernelGGL(k_face_loads, dim3(blocks_for(F)), dim3(kBlock), 0, s, F, xyz, faces,
                           flux, slot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather_slots, dim3(blocks_for(N)), dim3(kBlock), 0, s, N, off, idx, slot,
                       out);
    return hipGetLastError();
}

hipError_t launch_coef_bound(int64_t E, const double* coef64, unsigned long long* out,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_coef_bound, dim3(blocks_for(E)), dim3(kBlock), 0, s, E, coef64, out);
    return hipGetLastError();
}

hipError_t launch_coef_bound_hex(int64_t E, const double* coef64, unsigned long long* out,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_coef_bound_hex, dim3(blocks_for(E)), dim3(kBlock), 0, s, E, coef64,
                       out);
    return hipGetLastError();
}

hipError_t launch_cast_coef(int64_t n, const double* src, float* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_cast, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, src, dst);
    return hipGetLastError();
}

hipError_t launch_node_init(int64_t N, const double* Vi, const int32_t* is_dir,
                            const double* dirT, double T0, int fp32c, void* u, void* T0buf,
                            void* T1buf, hipStream_t s) {
    hipLaunchKernelGGL(k_node_init, dim3(blocks_for(N)), dim3(kBlock), 0, s, N, Vi, is_dir, dirT,
                       T0, fp32c, u, T0buf, T1buf);
    return hipGetLastError();
}

hipError_t launch_set_source(int64_t N, const double* src64, const int32_t* nperm, int fp32c,
                             void* q, hipStream_t s) {
    if (fp32c)
        hipLaunchKernelGGL(k_set_source<float>, dim3(blocks_for(N)), dim3(kBlock), 0, s, N,
                           src64, nperm, (float*)q);
    else
        hipLaunchKernelGGL(k_set_source<double>, dim3(blocks_for(N)), dim3(kBlock), 0, s, N,
                           src64, nperm, (double*)q);
    return hipGetLastError();
}

hipError_t launch_get_source(int64_t N, const void* q, const int32_t* nperm, int fp32c,
                             double* out64, hipStream_t s) {
    if (fp32c)
        hipLaunchKernelGGL(k_get_source<float>, dim3(blocks_for(N)), dim3(kBlock), 0, s, N,
                           (const float*)q, nperm, out64);
    else
        hipLaunchKernelGGL(k_get_source<double>, dim3(blocks_for(N)), dim3(kBlock), 0, s, N,
                           (const double*)q, nperm, out64);
    return hipGetLastError();
}

hipError_t launch_read_T(int64_t N, const void* T, const int32_t* nperm, int fp32c,
                         double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_read_T, dim3(blocks_for(N)), dim3(kBlock), 0, s, N, T, nperm, fp32c, out);
    return hipGetLastError();
}

hipError_t launch_state_io(int64_t N, void* T, const int32_t* nperm, int fp32c, void* buf,
                           int to_buf, hipStream_t s) {
    hipLaunchKernelGGL(k_state_io, dim3(blocks_for(N)), dim3(kBlock), 0, s, N, T, nperm, fp32c,
                       buf, to_buf);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_lanczos_start(int64_t N, const double* Vi, const int32_t* is_dir, double* sc,
                                double* v, double* vprev, double* xs, double* bsum,
                                double* scal, hipStream_t s) {
    const unsigned nb = blocks_for(N);
    hipLaunchKernelGGL(k_lz_init, dim3(nb), dim3(kBlock), 0, s, N, Vi, is_dir, sc, v, bsum);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, s, bsum, (int64_t)nb, scal, 1);
    hipLaunchKernelGGL(k_lz_scale, dim3(nb), dim3(kBlock), 0, s, N, scal, sc, v, vprev, xs);
    return hipGetLastError();
}

hipError_t launch_lanczos_iter(const DevLayout& d, const double* coef64, double fx_scale, int j,
                               const double* sc, double* v, double* vprev, double* w,
                               double* xs, double* partial, double* bsum, int* counter,
                               double* alpha, double* beta, hipStream_t s) {
    const unsigned nb = blocks_for(d.N);
    hipError_t e = launch_geometry_apply(d, coef64, xs, partial, fx_scale, s);
    if (e != hipSuccess) return e;
    // alpha_j = v . w and beta_j+1 = |w - alpha_j v|: on small grids summed
    // by the last block of the kernel that forms the products, on large ones
    // by a separate one-block kernel
    int* ctr = nb <= kFusedSumBlocks ? counter : nullptr;
    hipLaunchKernelGGL(k_lz_w, dim3(nb), dim3(kBlock), 0, s, d.N, d.part_off, d.pidx, partial, sc, v,
                       vprev, beta + j, w, bsum, ctr, alpha + j);
    if (!ctr)
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, s, bsum, (int64_t)nb, alpha + j, 0);
    hipLaunchKernelGGL(k_lz_orth, dim3(nb), dim3(kBlock), 0, s, d.N, alpha + j, v, w, bsum, ctr,
                       beta + j + 1);
    if (!ctr)
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, s, bsum, (int64_t)nb, beta + j + 1,
                           1);
    hipLaunchKernelGGL(k_lz_next, dim3(nb), dim3(kBlock), 0, s, d.N, beta + j + 1, sc, w, v,
                       vprev, xs);
    return hipGetLastError();
}

}  // namespace fedfem
